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


def test_sub_network_teacher_is_the_small_network(orc):
    """The distillation teacher (a network of the full shape reduced to a
    network of the student's shape on the student's descriptor components)
    computes, through the oracle, what the small network computes on the
    small descriptor."""
    nr, na, rr, ra = 6, 4, 5.0, 3.5
    D = 2 * (nr + 1 + na + 1)
    g = np.random.default_rng(18)
    nets = []
    for t in range(2):
        n = I.xavier_net([D, 9, 8, 1], 60 + 10 * t)
        n.shift = g.normal(size=D)
        n.scale = g.uniform(0.2, 1.0, size=D)
        nets.append(n)
    m = I.ModelSpec(2, I.default_type_weights(2), np.array([I.MASS["H"], I.MASS["O"]]), nr, rr, na, ra, nets)
    r = I.sub_network(m, 3, 2, [5, 4])
    T1, T2 = nr + 1, nr + na + 2
    keep = [0, 1, 2, 3, T1, T1 + 1, T1 + 2]
    keep = keep + [T2 + k for k in keep]
    small_nets = [I.NetSpec([n.W[0][:5][:, keep], n.W[1][:4, :5], n.W[2][:, :4]], [n.b[0][:5], n.b[1][:4], n.b[2]],
                            list(n.act), n.shift[keep], n.scale[keep], n.e_offset) for n in m.nets]
    small = I.ModelSpec(2, m.type_weight, m.masses, 3, rr, 2, ra, small_nets)
    s = I.water_box(12, 22)
    E1, _, F1 = orc.energy_forces(r, s.pos, s.species, s.box, s.pbc)
    E0, _, F0 = orc.energy_forces(small, s.pos, s.species, s.box, s.pbc)
    assert abs(E1 - E0) <= 1e-12 * abs(E0)
    np.testing.assert_allclose(F1, F0, rtol=0, atol=1e-12)


@pytest.mark.gpu
def test_student_meets_bar_and_beats_teacher_md():
    """The distilled student end to end on the GPU: teacher MD on water4096
    gives snapshots, the student (orders 6/2, 20-16-16-1) is trained by the
    library's kernels (device Adam, then full-batch L-BFGS), its force RMSE
    against the teacher on held-out snapshots is within 3e-2 eV/A (teacher
    force RMS 1 eV/A), and MD with the student under the teacher's judge
    (every 50 steps) keeps every chunk and runs faster than the teacher alone."""
    import time
    import torch
    from paper_2107_11311_amd import aenet as A
    A.load()
    teacher_m = I.load_model("student_teacher")
    stud_m = I.load_model("student")
    s = I.make_system("water4096")
    v = I.maxwell_boltzmann(teacher_m.masses[s.species], 300.0, 2)
    dt = 2.5e-4
    teacher = A.Context(teacher_m, "fp64", skin=0.5)
    snaps = ST.generate_snapshots(teacher, s, v, 800, 4, dt)
    assert torch.isfinite(snaps.forces).all()
    student = A.Context(stud_m, "fp32", skin=0.5)
    test_idx = np.arange(740, 800, 6)
    train_idx = np.arange(0, 730)
    rmse0 = ST.force_rmse(student, snaps, test_idx)
    res = ST.train(student, snaps, train_idx, steps=600, batch=4, lr=3e-3, lr_final=3e-4)
    res = ST.polish_lbfgs(student, snaps, train_idx[::60], 12000, res=res, log=lambda m: None, target=1e-4)
    rmse1 = ST.force_rmse(student, snaps, test_idx)
    rms = float(torch.sqrt((snaps.forces[test_idx].to(torch.float64) ** 2).mean()).item())
    print(f"student force rmse: untrained {rmse0:.4f} trained {rmse1:.4f} eV/A (teacher rms {rms:.3f}; "
          f"Adam {res.seconds:.1f} s, L-BFGS {res.lbfgs_iterations} iterations {res.lbfgs_seconds:.1f} s)")
    assert rmse1 <= 3e-2
    del snaps
    # production MD from the snapshot run's start: student + judge vs teacher alone
    trained = A.Context(stud_m.with_params(res.params), "fp32", skin=0.5)
    st = ST.DeviceState(s, v)
    judge = dict(rmse=st.rmse(teacher))
    ST.md_with_judge(st.runner(trained, dt), st.runner(teacher, dt), st.forces(teacher), st, 50, 50, 3e-2, **judge)
    torch.cuda.synchronize()
    st = ST.DeviceState(s, v)
    t0 = time.perf_counter()
    rep = ST.md_with_judge(st.runner(trained, dt), st.runner(teacher, dt), st.forces(teacher), st, 400, 50, 3e-2,
                           rmse=st.rmse(teacher))
    torch.cuda.synchronize()
    t_student = time.perf_counter() - t0
    st = ST.DeviceState(s, v)
    st.runner(teacher, dt)(st, 50)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st.runner(teacher, dt)(st, 400)
    torch.cuda.synchronize()
    t_teacher = time.perf_counter() - t0
    print(f"judge: {rep.fallbacks} fallbacks in {rep.chunks} chunks, rmse {np.round(rep.rmse_per_chunk, 4)}; "
          f"400 steps: student+judge {t_student:.3f} s, teacher {t_teacher:.3f} s")
    assert rep.fallbacks == 0 and max(rep.rmse_per_chunk) <= 3e-2
    assert t_student < t_teacher
