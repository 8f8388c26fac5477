"""Distilled student: judge/fallback logic (CPU, with the oracle standing in
for both networks) and GPU training with the library's loss gradient."""
import numpy as np
import pytest

from paper_2107_11311_amd import inputs as I
from paper_2107_11311_amd import student as ST


class _HostState:
    def __init__(self, pos, vel):
        self.pos = pos.copy()
        self.vel = vel.copy()

    def save(self):
        return (self.pos.copy(), self.vel.copy())

    def restore(self, ck):
        self.pos, self.vel = ck[0].copy(), ck[1].copy()


def _oracle_runner(orc, model, s, dt):
    def run(state, k):
        state.pos, state.vel, _, _, F = orc.md_vv(model, state.pos, state.vel, s.species, model.masses,
                                                  s.box, s.pbc, dt, k)
        return F
    return run


def _oracle_forces(orc, model, s):
    def f(state):
        return orc.energy_forces(model, state.pos, s.species, s.box, s.pbc)[2]
    return f


def test_judge_accepts_good_student_and_replaces_bad_one(orc):
    teacher = I.load_model("water64")
    s = I.make_system("water64")
    v = I.maxwell_boltzmann(teacher.masses[s.species], 300.0, 1)
    dt = 5e-4
    # a student identical to the teacher passes every check
    st = _HostState(s.pos, v)
    rep = ST.md_with_judge(_oracle_runner(orc, teacher, s, dt), _oracle_runner(orc, teacher, s, dt),
                           _oracle_forces(orc, teacher, s), st, 6, 3, 3e-2)
    assert rep.fallbacks == 0 and rep.chunks == 2 and max(rep.rmse_per_chunk) < 1e-12
    # a corrupted student trips the judge in every chunk; the teacher redoes the
    # chunks, so the trajectory equals the teacher's own
    bad = teacher.with_params(teacher.flat_params() * 1.5)
    st = _HostState(s.pos, v)
    rep = ST.md_with_judge(_oracle_runner(orc, bad, s, dt), _oracle_runner(orc, teacher, s, dt),
                           _oracle_forces(orc, teacher, s), st, 6, 3, 3e-2)
    assert rep.fallbacks == 2 and min(rep.rmse_per_chunk) > 3e-2
    ref = _HostState(s.pos, v)
    _oracle_runner(orc, teacher, s, dt)(ref, 3)
    _oracle_runner(orc, teacher, s, dt)(ref, 3)
    np.testing.assert_allclose(st.pos, ref.pos, atol=1e-12)
    np.testing.assert_allclose(st.vel, ref.vel, atol=1e-9)


def test_restricted_teacher_is_a_function_of_the_smaller_descriptor(orc):
    """A model restricted to orders (3, 2) computes, through the oracle, what
    the same networks give on the (3, 2)-order descriptor with the kept
    first-layer columns (so a student of those orders can represent it)."""
    nr, na, rr, ra = 6, 4, 5.0, 3.5
    D = 2 * (nr + 1 + na + 1)
    g = np.random.default_rng(8)
    nets = []
    for t in range(2):
        n = I.xavier_net([D, 7, 5, 1], 40 + 10 * t)
        n.shift = g.normal(size=D)
        n.scale = g.uniform(0.2, 1.0, size=D)
        nets.append(n)
    m = I.ModelSpec(2, I.default_type_weights(2), np.array([I.MASS["H"], I.MASS["O"]]), nr, rr, na, ra, nets)
    r = ST.restrict_to_orders(m, 3, 2)
    T1, T2 = nr + 1, nr + na + 2
    keep = [0, 1, 2, 3, T1, T1 + 1, T1 + 2]
    keep = keep + [T2 + k for k in keep]
    small_nets = []
    for n in m.nets:
        k = I.NetSpec([n.W[0][:, keep], *n.W[1:]], list(n.b), list(n.act), n.shift[keep], n.scale[keep],
                      n.e_offset)
        small_nets.append(k)
    small = I.ModelSpec(2, m.type_weight, m.masses, 3, rr, 2, ra, small_nets)
    s = I.water_box(12, 21)
    E1, Ea1, F1 = orc.energy_forces(r, s.pos, s.species, s.box, s.pbc)
    E0, Ea0, F0 = orc.energy_forces(small, s.pos, s.species, s.box, s.pbc)
    assert abs(E1 - E0) <= 1e-12 * abs(E0)
    np.testing.assert_allclose(F1, F0, rtol=0, atol=1e-12)
    # and it is not the unrestricted model
    E2, _, _ = orc.energy_forces(m, s.pos, s.species, s.box, s.pbc)
    assert abs(E2 - E0) > 1e-3 * abs(E0)


@pytest.mark.gpu
def test_student_training_improves_forces():
    import torch
    from paper_2107_11311_amd import aenet as A
    A.load()
    teacher_m = I.load_model("water64")
    s = I.make_system("water64")
    v = I.maxwell_boltzmann(teacher_m.masses[s.species], 300.0, 2)
    teacher = A.Context(teacher_m, "fp64", skin=0.5)
    snaps = ST.generate_snapshots(teacher, s, v, 160, 4, 2.5e-4)
    assert torch.isfinite(snaps.forces).all()
    stud_m = I.load_model("student")
    student = A.Context(stud_m, "fp32", skin=0.5)
    test_idx = np.arange(140, 160)
    rmse0 = ST.force_rmse(student, snaps, test_idx)
    res = ST.train(student, snaps, np.arange(0, 140), steps=400, batch=4, lr=3e-3, lr_final=3e-4)
    rmse1 = ST.force_rmse(student, snaps, test_idx)
    print(f"student force rmse: untrained {rmse0:.4f} trained {rmse1:.4f} eV/A "
          f"({res.steps} steps, {res.seconds:.1f} s)")
    assert np.isfinite(rmse1) and rmse1 < 0.7 * rmse0
