"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

FP64 mode must reproduce the oracle's descriptors, energies and forces to
rounding: relative energy error <= 1e-10 and force RMSE <= 1e-10 x the force
RMS (the FP64 bar of the method statement); descriptors to 1e-12 relative.
"""
import numpy as np
import pytest

from paper_2107_11311_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def A():
    from paper_2107_11311_amd import aenet
    aenet.load()
    return aenet


def rel_rmse(a, b):
    return float(np.sqrt(np.mean((a - b) ** 2)) / max(np.sqrt(np.mean(b ** 2)), 1e-300))


def small_model(S=2, nr=5, na=3, rr=5.0, ra=3.5, hidden=(9, 7), seed=3, tw=None):
    typed = nr + 1 + na + 1
    D = 2 * typed if S > 1 else typed
    g = np.random.default_rng(seed)
    nets = []
    for t in range(S):
        n = I.xavier_net([D, *hidden, 1], seed + 10 * t)
        n.shift = g.normal(size=D)
        n.scale = g.uniform(0.2, 1.0, size=D)
        n.e_offset = float(g.normal())
        nets.append(n)
    tw = I.default_type_weights(S) if tw is None else np.asarray(tw, float)
    return I.ModelSpec(S, tw, np.array([I.MASS["H"], I.MASS["O"], I.MASS["Si"]][:S]), nr, rr, na, ra, nets)


def check_ef(A, orc, model, s, precision="fp64", skin=0.0, tol_e=1e-10, tol_f=1e-10):
    ctx = A.Context(model, precision, skin=skin)
    E, Ea, F = ctx.energy_forces(s.pos, s.species, s.box, s.pbc)
    E0, Ea0, F0 = orc.energy_forces(model, s.pos, s.species, s.box, s.pbc)
    de = abs(E - E0) / abs(E0)
    df = rel_rmse(F, F0)
    dea = float(np.abs(Ea - Ea0).max() / np.abs(Ea0).max())
    # element-wise: the largest error of any force component against the
    # largest force component (a single wrong component cannot hide in a norm)
    dmax = float(np.abs(F - F0).max() / np.abs(F0).max())
    print(f"{precision}: rel dE={de:.3e} rel F rmse={df:.3e} max|dF|/max|F|={dmax:.3e} rel dE_atom={dea:.3e}")
    assert de <= tol_e, f"energy rel err {de:.3e}"
    assert df <= tol_f, f"force rel rmse {df:.3e}"
    assert dmax <= (1.0 if precision == "fp64" else 10.0) * tol_f, f"force max rel err {dmax:.3e}"
    assert dea <= 10 * tol_e, f"atom energy rel err {dea:.3e}"
    ctx.close()
    return E, F


def test_descriptors_water64(A, orc):
    m = I.load_model("water64")
    s = I.make_system("water64")
    ctx = A.Context(m, "fp64")
    G = ctx.descriptors(s.pos, s.species, s.box, s.pbc)
    G0 = orc.descriptors(m, s.pos, s.species, s.box, s.pbc)
    np.testing.assert_allclose(G, G0, rtol=1e-12, atol=1e-12 * np.abs(G0).max())


def test_energy_forces_water64(A, orc):
    check_ef(A, orc, I.load_model("water64"), I.make_system("water64"))


@pytest.mark.parametrize("n_mol", [8, 20])
def test_small_box_images(A, orc, n_mol):
    """Edges shorter than twice the cutoff: several images of one atom are neighbours."""
    s = I.water_box(n_mol, 900 + n_mol)
    m = small_model(nr=6, na=2, rr=min(6.5, s.box[0] * 0.99), ra=4.0)
    assert s.box[0] < 2 * m.radial_cutoff
    check_ef(A, orc, m, s)


def test_open_cluster_three_species(A, orc):
    g = np.random.default_rng(5)
    pos = I.rsa(60, 14.0, 1.6, 77) + 30.0
    sp = g.integers(0, 3, size=60).astype(np.int32)
    s = I.System(pos, sp, np.array([80.0, 80.0, 80.0]), np.zeros(3, dtype=np.uint8))
    m = small_model(S=3, nr=4, na=2, rr=5.0, ra=4.0, tw=(1.0, 2.0, 3.0))
    check_ef(A, orc, m, s)


def test_mixed_periodicity(A, orc):
    s = I.water_box(30, 31)
    s.pbc = np.array([1, 0, 1], dtype=np.uint8)
    s.pos[:, 1] += 5.0
    s.box = s.box.copy()
    s.box[1] = s.box[1] + 10.0
    check_ef(A, orc, small_model(nr=5, na=3, rr=4.5, ra=3.5), s)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_degenerate_systems(A, orc, precision):
    """The degenerate cases of the method, against the oracle: an isolated
    atom and one atom in the smallest periodic box allowed (no neighbours:
    G = 0, the energy is the network's value at the shifted origin and the
    force is exactly zero); an open dimer (radial terms only, one angular
    neighbour each and so no pairs; the two forces exact negatives); a pair
    at exactly the radial cutoff (f_c(R) = 0: no contribution); and a
    collinear trimer (cos theta = -1 at the centre, the end of the
    Chebyshev domain)."""
    m = small_model(nr=5, na=3, rr=4.5, ra=3.5)
    rl = max(m.radial_cutoff, m.angular_cutoff) + 0.5
    open_box = np.array([60.0, 60.0, 60.0])
    no_pbc = np.zeros(3, dtype=np.uint8)
    cases = {
        "isolated": I.System(np.array([[30.0, 30.0, 30.0]]), np.array([0], np.int32), open_box, no_pbc),
        "periodic_single": I.System(np.array([[1.0, 2.0, 3.0]]), np.array([1], np.int32),
                                    np.array([rl, rl, rl]), np.ones(3, dtype=np.uint8)),
        "dimer": I.System(np.array([[30.0, 30.0, 30.0], [31.2, 30.9, 30.4]]), np.array([0, 1], np.int32),
                          open_box, no_pbc),
        "at_cutoff": I.System(np.array([[30.0, 30.0, 30.0], [30.0 + m.radial_cutoff, 30.0, 30.0],
                                        [30.0, 31.1, 30.0]]), np.array([0, 1, 1], np.int32), open_box, no_pbc),
        "collinear": I.System(np.array([[28.6, 30.0, 30.0], [30.0, 30.0, 30.0], [31.3, 30.0, 30.0]]),
                              np.array([1, 0, 1], np.int32), open_box, no_pbc),
    }
    tol = 1e-10 if precision == "fp64" else 1e-5
    for name, sy in cases.items():
        ctx = A.Context(m, precision, skin=0.5)
        E, Ea, F = ctx.energy_forces(sy.pos, sy.species, sy.box, sy.pbc)
        ctx.close()
        E0, Ea0, F0 = orc.energy_forces(m, sy.pos, sy.species, sy.box, sy.pbc)
        fs = max(float(np.abs(F0).max()), 1.0)
        print(f"{name} {precision}: E {E:.12f} oracle {E0:.12f} max|dF| {np.abs(F - F0).max():.2e}")
        assert abs(E - E0) <= tol * max(abs(E0), 1.0), name
        assert np.abs(Ea - Ea0).max() <= tol * max(float(np.abs(Ea0).max()), 1.0), name
        assert np.abs(F - F0).max() <= tol * fs, name
        if name in ("isolated", "periodic_single"):
            assert np.all(F == 0.0), name
        if name == "dimer":
            assert np.array_equal(F[0], -F[1]), name


def test_skin_does_not_change_results(A, orc):
    s = I.make_system("water64")
    m = I.load_model("water64")
    E0, F0 = check_ef(A, orc, m, s, skin=0.0)
    E1, F1 = check_ef(A, orc, m, s, skin=0.5)
    de = abs(E1 - E0) / abs(E0)
    df = float(np.abs(F1 - F0).max() / np.abs(F0).max())
    assert de <= 1e-12, de
    assert df <= 1e-12, df


def test_deterministic_bitwise(A):
    s = I.make_system("water64")
    ctx = A.Context(I.load_model("water64"), "fp64")
    r1 = ctx.energy_forces(s.pos, s.species, s.box, s.pbc)
    r2 = ctx.energy_forces(s.pos, s.species, s.box, s.pbc)
    assert r1[0] == r2[0]
    assert np.array_equal(r1[1], r2[1]) and np.array_equal(r1[2], r2[2])


def test_md_matches_oracle(A, orc):
    s = I.water_box(32, 55)
    m = small_model(nr=5, na=3, rr=4.5, ra=3.5)
    # normalise the force scale so dynamics stay tame
    v = I.maxwell_boltzmann(m.masses[s.species], 300.0, 3)
    ctx = A.Context(m, "fp64", skin=0.4)
    p1, v1, ep, ek, F = ctx.md_step(s.pos, v, s.species, s.box, s.pbc, 2.5e-4, 10)
    p0, v0, ep0, ek0, F0 = orc.md_vv(m, s.pos, v, s.species, m.masses, s.box, s.pbc, 2.5e-4, 10)
    dp = float(np.abs((p1 - p0 + s.box / 2) % s.box - s.box / 2).max())
    dv = float(np.abs(v1 - v0).max())
    dep = abs(ep - ep0) / abs(ep0)
    dek = abs(ek - ek0) / abs(ek0)
    print(f"md: dpos={dp:.3e} dvel={dv:.3e} rel dEpot={dep:.3e} rel dEkin={dek:.3e}")
    assert dp < 1e-10, dp
    assert dv < 1e-8, dv
    assert dep <= 1e-10, dep
    assert dek <= 1e-10, dek


def test_error_paths(A):
    s = I.make_system("water64")
    ctx = A.Context(I.load_model("water64"), "fp64")
    bad = s.species.copy()
    bad[3] = 7
    with pytest.raises(A.AenetError) as e:
        ctx.energy_forces(s.pos, bad, s.box, s.pbc)
    assert e.value.code == A.AENET_E_SPECIES
    with pytest.raises(A.AenetError) as e:
        ctx.energy_forces(s.pos, s.species, s.box * 0.4, s.pbc)
    assert e.value.code == A.AENET_E_BOX
    p = s.pos.copy()
    p[5, 1] = np.nan
    with pytest.raises(A.AenetError) as e:
        ctx.energy_forces(p, s.species, s.box, s.pbc)
    assert e.value.code == A.AENET_E_NONFINITE
    p = s.pos.copy()
    p[7] = p[8]
    with pytest.raises(A.AenetError) as e:
        ctx.energy_forces(p, s.species, s.box, s.pbc)
    assert e.value.code == A.AENET_E_OVERLAP
    # the context still works after errors
    E, _, _ = ctx.energy_forces(s.pos, s.species, s.box, s.pbc)
    assert np.isfinite(E)
    # two atoms 1e-9 A apart are distinct (no overlap error), also where the
    # per-cell list kernel sees them coincide in FP32 (27 atoms per cell here)
    w = I.water_box(256, 71)
    c2 = A.Context(small_model(nr=5, na=3, rr=4.5, ra=3.5), "fp64", skin=0.5)
    for base in (c2, ctx):
        sy = w if base is c2 else s
        p = sy.pos.copy()
        p[7] = p[8] + np.array([1e-9, 0.0, 0.0])
        E, _, F = base.energy_forces(p, sy.species, sy.box, sy.pbc)
        assert np.isfinite(E) and np.all(np.isfinite(F))
        p[7] = p[8]
        with pytest.raises(A.AenetError) as e:
            base.energy_forces(p, sy.species, sy.box, sy.pbc)
        assert e.value.code == A.AENET_E_OVERLAP
    c2.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16"])
def test_fused_forward_network_is_bitwise_the_two_kernels(A, precision):
    """Descriptors + networks in one kernel per 16-atom tile give the bits of
    the separate kernels: water64 (full tiles and a partial one per species)
    and a three-species cluster (short tiles at every species boundary)."""
    g = np.random.default_rng(5)
    pos = I.rsa(60, 14.0, 1.6, 77) + 30.0
    sp = g.integers(0, 3, size=60).astype(np.int32)
    s3 = I.System(pos, sp, np.array([80.0, 80.0, 80.0]), np.zeros(3, dtype=np.uint8))
    m3 = small_model(S=3, nr=4, na=2, rr=5.0, ra=4.0, tw=(1.0, 2.0, 3.0))
    cases = [("water64", I.load_model("water64"), I.make_system("water64")), ("cluster3", m3, s3)]
    for name, m, s in cases:
        out = []
        for fused in (True, False):
            ctx = A.Context(m, precision)
            ctx.set_fused(fused)
            out.append(ctx.energy_forces(s.pos, s.species, s.box, s.pbc))
            ctx.close()
        (E1, Ea1, F1), (E0, Ea0, F0) = out
        assert E1 == E0, name
        assert np.array_equal(Ea1, Ea0) and np.array_equal(F1, F0), name


@pytest.mark.parametrize("hidden", [(), (9,), (9, 7, 5), (40, 7), (9, 40, 33)])
def test_network_shapes(A, orc, hidden):
    """Every network depth (1..4 weight layers) and hidden widths on both
    sides of 32 (the network tile keeps narrower operand fragments when all
    hidden layers are at most 32 wide) against the oracle, through the fused
    kernel and through the separate network kernel, whose results agree
    bitwise."""
    m = small_model(nr=5, na=3, rr=4.5, ra=3.5, hidden=hidden)
    s = I.make_system("water64")
    E0, Ea0, F0 = orc.energy_forces(m, s.pos, s.species, s.box, s.pbc)
    out = []
    for fused in (True, False):
        ctx = A.Context(m, "fp64")
        ctx.set_fused(fused)
        E, Ea, F = ctx.energy_forces(s.pos, s.species, s.box, s.pbc)
        ctx.close()
        assert abs(E - E0) / abs(E0) <= 1e-10, (hidden, fused)
        assert rel_rmse(F, F0) <= 1e-10, (hidden, fused)
        out.append((E, Ea, F))
    assert out[0][0] == out[1][0] and np.array_equal(out[0][2], out[1][2]), hidden


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_virial_matches_oracle(A, orc, precision):
    """The virial (-dE/d strain, summed over every entry's gradient) of a
    periodic water box, a three-species open cluster and a small box with
    many images against the oracle; energy and forces unchanged by asking
    for it."""
    g = np.random.default_rng(5)
    pos = I.rsa(60, 14.0, 1.6, 77) + 30.0
    sp = g.integers(0, 3, size=60).astype(np.int32)
    s3 = I.System(pos, sp, np.array([80.0, 80.0, 80.0]), np.zeros(3, dtype=np.uint8))
    m3 = small_model(S=3, nr=4, na=2, rr=5.0, ra=4.0, tw=(1.0, 2.0, 3.0))
    cases = [("water64", I.load_model("water64"), I.make_system("water64")), ("cluster3", m3, s3),
             ("water20", None, I.water_box(20, 920))]
    tol = 1e-10 if precision == "fp64" else 1e-5
    for name, m, s in cases:
        if m is None:  # a box smaller than twice the cutoff: entries through many images
            m = small_model(nr=6, na=2, rr=min(6.5, s.box[0] * 0.99), ra=4.0)
        E0, F0, W0 = orc.energy_forces_virial(m, s.pos, s.species, s.box, s.pbc)
        ctx = A.Context(m, precision)
        E, F, W = ctx.energy_forces_virial(s.pos, s.species, s.box, s.pbc)
        E1, _, F1 = ctx.energy_forces(s.pos, s.species, s.box, s.pbc)
        ctx.close()
        scale = np.abs(W0).max()
        print(f"{name} {precision}: |W| {scale:.3e} max dW {np.abs(W - W0).max():.3e}")
        assert np.abs(W - W0).max() <= tol * scale, name
        assert E == E1 and np.array_equal(F, F1), name
        assert abs(E - E0) <= tol * abs(E0), name


def test_nonfinite_device_input(A):
    """A NaN in device-resident positions is reported, not computed with."""
    import torch
    s = I.make_system("water64")
    ctx = A.Context(I.load_model("water64"), "fp64")
    p = torch.from_numpy(s.pos.copy()).to("cuda:0")
    p[11, 2] = float("nan")
    F = torch.zeros_like(p)
    et = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    with pytest.raises(A.AenetError) as e:
        ctx.energy_forces_dev(p, s.species, s.box, s.pbc, et, None, F)
    assert e.value.code == A.AENET_E_NONFINITE
    E, _, _ = ctx.energy_forces(s.pos, s.species, s.box, s.pbc)
    assert np.isfinite(E)


def test_capacity_retry_forces(A):
    """Rows far too short for the first build: the build overflows, the rows
    grow and the build is redone, with the same result as estimated rows."""
    m = I.load_model("water64")
    s = I.make_system("water64")
    E0, Ea0, F0 = A.Context(m, "fp64").energy_forces(s.pos, s.species, s.box, s.pbc)
    ctx = A.Context(m, "fp64")
    ctx.set_capacity(12, 6)
    E1, Ea1, F1 = ctx.energy_forces(s.pos, s.species, s.box, s.pbc)
    st = ctx.stats()
    assert st["n_capacity_retries"] >= 1 and st["row_capacity"] > 12 and st["ang_capacity"] > 6
    assert abs(E1 - E0) <= 1e-13 * abs(E0)
    np.testing.assert_allclose(Ea1, Ea0, rtol=0, atol=1e-13)
    np.testing.assert_allclose(F1, F0, rtol=0, atol=1e-12)
    with pytest.raises(A.AenetError) as e:
        ctx.set_capacity(8, 9)
    assert e.value.code == A.AENET_E_INVALID


def test_capacity_retry_md(A):
    """Rows sized to exactly the first configuration: as atoms move, a later
    build overflows inside an MD chunk; the chunk is redone from its
    checkpoint with longer rows and the trajectory stays on the one run with
    estimated rows."""
    # with this seed the largest angular shell (42 entries within R_a + skin
    # at the start) has grown by step 7 and stays above 42 (checked with the
    # oracle's MD), so the build at step 10 at the latest overflows and the
    # chunk of steps 1..10 is redone
    m = I.load_model("water64")
    s = I.make_system("water64")
    v = I.maxwell_boltzmann(m.masses[s.species], 600.0, 12)
    probe = A.Context(m, "fp64", skin=0.3)
    probe.energy_forces(s.pos, s.species, s.box, s.pbc)
    st0 = probe.stats()
    ref = A.Context(m, "fp64", skin=0.3)
    ref.set_rebuild_every(10)
    p0, v0, ep0, ek0, _ = ref.md_step(s.pos, v, s.species, s.box, s.pbc, 5e-4, 40)
    ctx = A.Context(m, "fp64", skin=0.3)
    ctx.set_rebuild_every(10)
    ctx.set_capacity(st0["max_neighbors"], st0["max_angular"])
    p1, v1, ep1, ek1, _ = ctx.md_step(s.pos, v, s.species, s.box, s.pbc, 5e-4, 40)
    st = ctx.stats()
    dp = float(np.abs((p1 - p0 + s.box / 2) % s.box - s.box / 2).max())
    dv = float(np.abs(v1 - v0).max() / np.abs(v0).max())
    print(f"capacity retry md: retries={st['n_capacity_retries']} rows {st0['max_neighbors']}->"
          f"{st['row_capacity']} ang {st0['max_angular']}->{st['ang_capacity']} dpos={dp:.3e} dvel={dv:.3e}")
    assert st["n_capacity_retries"] >= 1
    assert dp < 1e-9 and dv < 1e-9
    assert abs(ep1 + ek1 - ep0 - ek0) < 1e-10 * abs(ep0 + ek0)


def test_empty_input(A):
    ctx = A.Context(I.load_model("water64"), "fp64")
    E, Ea, F = ctx.energy_forces(np.zeros((0, 3)), np.zeros(0, np.int32), [12.42] * 3, (1, 1, 1))
    assert E == 0.0 and Ea.size == 0 and F.size == 0


def test_md_long_with_rebuilds(A, orc):
    """120 steps with a small skin: many device-triggered and forced rebuilds
    (wrap + new list) must leave the trajectory on the oracle's (which
    rebuilds every step)."""
    m = I.load_model("water64")
    s = I.make_system("water64")
    v = I.maxwell_boltzmann(m.masses[s.species], 300.0, 9)
    ctx = A.Context(m, "fp64", skin=0.2)
    ctx.set_rebuild_every(7)
    p1, v1, ep, ek, F = ctx.md_step(s.pos, v, s.species, s.box, s.pbc, 5e-4, 120)
    st = ctx.stats()
    p0, v0, ep0, ek0, F0 = orc.md_vv(m, s.pos, v, s.species, m.masses, s.box, s.pbc, 5e-4, 120)
    dp = float(np.abs((p1 - p0 + s.box / 2) % s.box - s.box / 2).max())
    dv = float(np.abs(v1 - v0).max() / np.abs(v0).max())
    de = abs(ep + ek - ep0 - ek0) / abs(ep0 + ek0)
    print(f"md120: rebuilds={st['n_rebuilds']} dpos={dp:.3e} rel dvel={dv:.3e} rel dE={de:.3e}")
    assert st["n_rebuilds"] > 120 // 7
    assert dp < 1e-8, dp
    assert dv < 1e-8, dv
    assert de < 1e-10, de


def test_md_cell_bins_matches_oracle(A, orc):
    """MD on a box of 4 x 4 x 4 list cells (the per-cell row kernel with the
    integrator's cell bins, every stencil cell distinct) and a small skin, so
    the list is rebuilt often: the trajectory stays on the oracle's."""
    s = I.water_box(256, 71)
    m = small_model(nr=5, na=3, rr=4.5, ra=3.5)
    v = I.maxwell_boltzmann(m.masses[s.species], 300.0, 8)
    ctx = A.Context(m, "fp64", skin=0.15)
    ctx.set_rebuild_every(12)
    p1, v1, ep, ek, F = ctx.md_step(s.pos, v, s.species, s.box, s.pbc, 5e-4, 40)
    st = ctx.stats()
    p0, v0, ep0, ek0, F0 = orc.md_vv(m, s.pos, v, s.species, m.masses, s.box, s.pbc, 5e-4, 40)
    dp = float(np.abs((p1 - p0 + s.box / 2) % s.box - s.box / 2).max())
    dv = float(np.abs(v1 - v0).max() / np.abs(v0).max())
    de = abs(ep + ek - ep0 - ek0) / abs(ep0 + ek0)
    print(f"md cell bins: atoms={s.pos.shape[0]} box={s.box[0]:.2f} rebuilds={st['n_rebuilds']} "
          f"dpos={dp:.3e} rel dvel={dv:.3e} rel dE={de:.3e}")
    assert s.box[0] / (4.5 + 0.15) >= 4  # at least 4 cells per axis
    assert st["n_rebuilds"] > 40 // 12
    assert dp < 1e-9, dp
    assert dv < 1e-9, dv
    assert de < 1e-10, de


def test_capacity_retry_md_cell_bins(A):
    """A capacity retry inside an MD chunk on the per-cell path (cell bins
    filled by the integrator): the redone chunk ends where the run with
    estimated rows ends."""
    s = I.water_box(256, 71)
    m = small_model(nr=5, na=3, rr=4.5, ra=3.5)
    v = I.maxwell_boltzmann(m.masses[s.species], 600.0, 13)
    probe = A.Context(m, "fp64", skin=0.3)
    probe.energy_forces(s.pos, s.species, s.box, s.pbc)
    st0 = probe.stats()
    ref = A.Context(m, "fp64", skin=0.3)
    ref.set_rebuild_every(10)
    p0, v0, ep0, ek0, _ = ref.md_step(s.pos, v, s.species, s.box, s.pbc, 5e-4, 40)
    ctx = A.Context(m, "fp64", skin=0.3)
    ctx.set_rebuild_every(10)
    ctx.set_capacity(st0["max_neighbors"], st0["max_angular"])
    p1, v1, ep1, ek1, _ = ctx.md_step(s.pos, v, s.species, s.box, s.pbc, 5e-4, 40)
    st = ctx.stats()
    dp = float(np.abs((p1 - p0 + s.box / 2) % s.box - s.box / 2).max())
    dv = float(np.abs(v1 - v0).max() / np.abs(v0).max())
    print(f"capacity retry md (cell bins): retries={st['n_capacity_retries']} rows {st0['max_neighbors']}->"
          f"{st['row_capacity']} ang {st0['max_angular']}->{st['ang_capacity']} dpos={dp:.3e} dvel={dv:.3e}")
    assert st["n_capacity_retries"] >= 1
    assert dp < 1e-9 and dv < 1e-9
    assert abs(ep1 + ek1 - ep0 - ek0) < 1e-10 * abs(ep0 + ek0)


def _filling_cell_system():
    """272 O atoms in a 10.5 A periodic box of 2 x 2 x 2 list cells (5.25 A
    at R_list = 5.0 A): 120 on a grid in cell (0, 0, 0), 20 in each other
    cell, and 12 just beyond the face x = 5.25 A of cell (0, 0, 0), moving
    into it at 30 A/ps.  The mean cell count plans the per-cell row kernel;
    cell (0, 0, 0) passes its 128 atoms about ten steps in."""
    g = np.random.default_rng(21)
    L = 10.5
    c = L / 2
    a, b = c / 5, c / 3
    pts = [(a * (i + 0.5), a * (j + 0.5), a * (k + 0.5)) for i in range(5) for j in range(5) for k in range(5)][:120]
    for cx in range(2):
        for cy in range(2):
            for cz in range(2):
                if cx == cy == cz == 0:
                    continue
                pts += [(cx * c + b * (i + 0.5), cy * c + b * (j + 0.5), cz * c + b * (k + 0.5))
                        for i in range(3) for j in range(3) for k in range(3)][:20]
    n0 = len(pts)
    pts += [(c + 0.12, 0.6 + 1.2 * j, 0.7 + 1.6 * k) for j in range(4) for k in range(3)]
    pos = np.array(pts) + g.uniform(-0.05, 0.05, size=(len(pts), 3))
    return I.System(pos, np.ones(len(pts), np.int32), np.array([L, L, L]), np.ones(3, dtype=np.uint8)), n0


def test_md_cell_bin_overflow_falls_back(A, orc):
    """A list cell that fills beyond the per-cell row kernel's 128 atoms
    inside an MD chunk (the integrator's cell bins overflow at a build): the
    chunk is redone from its start on the per-atom row kernels, and the run
    ends where the oracle's velocity Verlet does."""
    m = small_model(nr=5, na=3, rr=4.5, ra=3.5)
    s, n0 = _filling_cell_system()
    v = I.maxwell_boltzmann(m.masses[s.species], 300.0, 5)
    v[n0:, 0] = -30.0
    ctx = A.Context(m, "fp64", skin=0.5)
    ctx.set_rebuild_every(5)
    p1, v1, ep, ek, F = ctx.md_step(s.pos, v, s.species, s.box, s.pbc, 5e-4, 20)
    st = ctx.stats()
    ctx.close()
    p0, v0, ep0, ek0, F0 = orc.md_vv(m, s.pos, v, s.species, m.masses, s.box, s.pbc, 5e-4, 20)
    in0 = int(np.all(p0 % s.box < s.box / 2, axis=1).sum())
    dp = float(np.abs((p1 - p0 + s.box / 2) % s.box - s.box / 2).max())
    dv = float(np.abs(v1 - v0).max() / np.abs(v0).max())
    dF = float(np.abs(F - F0).max() / np.abs(F0).max())
    print(f"cell (0,0,0) ends with {in0} atoms; retries {st['n_capacity_retries']}, builds {st['n_rebuilds']}; "
          f"dpos {dp:.2e} dvel {dv:.2e} max|dF|/max|F| {dF:.2e}")
    assert in0 > 128
    assert st["n_capacity_retries"] >= 1
    assert dp <= 1e-9 and dv <= 1e-9 and dF <= 1e-9
    assert abs(ep + ek - ep0 - ek0) <= 1e-10 * abs(ep0 + ek0)


def test_md_resume_is_bitwise(A):
    """100 steps == 50 steps + (positions, velocities) handed back + 50 steps."""
    m = I.load_model("water64")
    s = I.make_system("water64")
    v = I.maxwell_boltzmann(m.masses[s.species], 300.0, 4)
    ctx = A.Context(m, "fp64", skin=0.3)
    ctx.set_rebuild_every(25)
    pa, va, epa, eka, _ = ctx.md_step(s.pos, v, s.species, s.box, s.pbc, 5e-4, 100)
    pb, vb, _, _, _ = ctx.md_step(s.pos, v, s.species, s.box, s.pbc, 5e-4, 50)
    pb, vb, epb, ekb, _ = ctx.md_step(pb, vb, s.species, s.box, s.pbc, 5e-4, 50)
    assert np.array_equal(pa, pb) and np.array_equal(va, vb)
    assert epa == epb and eka == ekb


def test_nve_energy_error_scales_dt2(A):
    """Velocity Verlet on the GPU: the total-energy error over a fixed time
    falls by about 4x when dt is halved."""
    m = I.load_model("water64")
    s = I.make_system("water64")
    v = I.maxwell_boltzmann(m.masses[s.species], 300.0, 5)
    ctx = A.Context(m, "fp64", skin=0.3)

    def max_dev(dt, nsteps, every):
        p, vv = s.pos, v
        _, _, ep0, ek0, _ = ctx.md_step(p, vv, s.species, s.box, s.pbc, dt, 0)
        dev = 0.0
        for _ in range(nsteps // every):
            p, vv, ep, ek, _ = ctx.md_step(p, vv, s.species, s.box, s.pbc, dt, every)
            dev = max(dev, abs(ep + ek - ep0 - ek0))
        return dev

    d1 = max_dev(5e-4, 40, 2)
    d2 = max_dev(2.5e-4, 80, 4)
    print(f"nve: max |dE| {d1:.3e} (dt 0.5 fs) {d2:.3e} (dt 0.25 fs) ratio {d1 / d2:.2f}")
    assert 2.5 < d1 / d2 < 5.5


def test_md_continuation_detects_changed_state(A):
    """A call that continues from the state the last call left (positions
    handed back unchanged) reuses its forces and list; a call whose positions
    were changed by the caller, or that follows new parameters, starts over
    and gives what a fresh context gives from the same inputs."""
    m = I.load_model("water64")
    s = I.make_system("water64")
    v = I.maxwell_boltzmann(m.masses[s.species], 300.0, 6)
    dt = 5e-4

    def fresh(model, p, vv, steps):
        c = A.Context(model, "fp64", skin=0.3)
        out = c.md_step(p, vv, s.species, s.box, s.pbc, dt, steps)
        c.close()
        return out

    ctx = A.Context(m, "fp64", skin=0.3)
    p1, v1, _, _, _ = ctx.md_step(s.pos, v, s.species, s.box, s.pbc, dt, 7)
    # velocities rescaled (a thermostat): positions unchanged, state continues
    p2, v2, e2, k2, F2 = ctx.md_step(p1, 0.9 * v1, s.species, s.box, s.pbc, dt, 6)
    q2, w2, f2, l2, G2 = fresh(m, p1, 0.9 * v1, 6)
    assert np.abs(p2 - q2).max() <= 1e-10 and np.abs(v2 - w2).max() <= 1e-8 * np.abs(w2).max()
    assert abs(e2 - f2) <= 1e-10 * abs(f2)
    # one atom moved by the caller: the forces of the new positions are used
    p3 = p2.copy()
    p3[5] += np.array([0.05, -0.03, 0.02])
    r3, u3, e3, _, F3 = ctx.md_step(p3, v2, s.species, s.box, s.pbc, dt, 4)
    q3, w3, f3, _, G3 = fresh(m, p3, v2, 4)
    assert np.abs(r3 - q3).max() <= 1e-10 and abs(e3 - f3) <= 1e-10 * abs(f3)
    np.testing.assert_allclose(F3, G3, rtol=0, atol=1e-10 * np.abs(G3).max())
    # new parameters: the kept forces belong to the old network
    m2 = m.with_params(1.1 * m.flat_params())
    ctx.set_params(m2.flat_params())
    r4, u4, e4, _, F4 = ctx.md_step(r3, u3, s.species, s.box, s.pbc, dt, 3)
    q4, w4, f4, _, G4 = fresh(m2, r3, u3, 3)
    assert np.abs(r4 - q4).max() <= 1e-10 and abs(e4 - f4) <= 1e-10 * abs(f4)
    np.testing.assert_allclose(F4, G4, rtol=0, atol=1e-10 * np.abs(G4).max())
    # zero steps on an unchanged state returns it as it is
    r5, u5, e5, _, F5 = ctx.md_step(r4, u4, s.species, s.box, s.pbc, dt, 0)
    assert np.array_equal(r5, r4) and np.array_equal(u5, u4) and e5 == e4
    np.testing.assert_array_equal(F5, F4)
    # a changed state found after the first of several chunks (the call goes
    # on as if it continued and is redone from the caller's inputs)
    ctx.set_rebuild_every(3)
    p6 = r5.copy()
    p6[7] += np.array([0.02, 0.01, -0.04])
    r6, u6, e6, _, F6 = ctx.md_step(p6, u5, s.species, s.box, s.pbc, dt, 8)
    q6, w6, f6, _, G6 = fresh(m2, p6, u5, 8)
    assert np.abs(r6 - q6).max() <= 1e-10 and abs(e6 - f6) <= 1e-10 * abs(f6)
    np.testing.assert_allclose(F6, G6, rtol=0, atol=1e-10 * np.abs(G6).max())
    # ... and with zero steps: the forces of the caller's positions
    p7 = r6.copy()
    p7[3] -= np.array([0.01, 0.02, 0.0])
    r7, u7, e7, _, F7 = ctx.md_step(p7, u6, s.species, s.box, s.pbc, dt, 0)
    q7, w7, f7, _, G7 = fresh(m2, p7, u6, 0)
    assert np.abs(r7 - q7).max() <= 1e-12 and abs(e7 - f7) <= 1e-10 * abs(f7)
    np.testing.assert_allclose(F7, G7, rtol=0, atol=1e-10 * np.abs(G7).max())
    ctx.close()


def test_md_continuation_dev_buffer_changed_in_place(A):
    """A device caller that edits the position buffer the last call wrote:
    the call goes on as if the state were kept, finds it stale with the
    first chunk's status words, discards that chunk and starts over; the
    result is what a fresh context gives from the same inputs (several
    chunks, and zero steps)."""
    import torch
    m = I.load_model("water64")
    s = I.make_system("water64")
    dev = torch.device("cuda:0")
    v = I.maxwell_boltzmann(m.masses[s.species], 300.0, 6)
    dt = 5e-4
    n = len(s.pos)
    ctx = A.Context(m, "fp64", skin=0.3)
    ctx.set_rebuild_every(3)
    pos = torch.from_numpy(s.pos.copy()).to(dev)
    vel = torch.from_numpy(v.copy()).to(dev)
    ep = torch.zeros(1, dtype=torch.float64, device=dev)
    ek = torch.zeros(1, dtype=torch.float64, device=dev)
    F = torch.zeros(n, 3, dtype=torch.float64, device=dev)
    ctx.md_step_dev(pos, vel, s.species, s.box, s.pbc, dt, 4, ep, ek, F)
    for steps in (8, 0):
        pos[7] += torch.tensor([0.02, 0.01, -0.04], dtype=torch.float64, device=dev)
        p_in, v_in = pos.cpu().numpy(), vel.cpu().numpy()
        ctx.md_step_dev(pos, vel, s.species, s.box, s.pbc, dt, steps, ep, ek, F)
        torch.cuda.synchronize()
        ref = A.Context(m, "fp64", skin=0.3)
        q, w, e0, k0, G = ref.md_step(p_in, v_in, s.species, s.box, s.pbc, dt, steps)
        ref.close()
        p1, v1, F1 = pos.cpu().numpy(), vel.cpu().numpy(), F.cpu().numpy()
        dp = float(np.abs((p1 - q + s.box / 2) % s.box - s.box / 2).max())
        print(f"{steps} steps: dpos {dp:.2e} dE {abs(ep.item() - e0) / abs(e0):.2e}")
        assert dp <= 1e-10 and np.abs(v1 - w).max() <= 1e-8 * np.abs(w).max()
        assert abs(ep.item() - e0) <= 1e-10 * abs(e0) and abs(ek.item() - k0) <= 1e-10 * abs(k0)
        np.testing.assert_allclose(F1, G, rtol=0, atol=1e-10 * np.abs(G).max())
    ctx.close()


def test_md_continuation_error_leaves_outputs(A):
    """A device call that would continue from the kept state but gets a
    non-finite velocity fails with AENET_E_NONFINITE and writes nothing to
    the caller's buffers; the next call starts over."""
    import torch
    m = I.load_model("water64")
    s = I.make_system("water64")
    dev = torch.device("cuda:0")
    v = I.maxwell_boltzmann(m.masses[s.species], 300.0, 6)
    ctx = A.Context(m, "fp64", skin=0.3)
    pos = torch.from_numpy(s.pos.copy()).to(dev)
    vel = torch.from_numpy(v.copy()).to(dev)
    n = len(s.pos)
    ep = torch.zeros(1, dtype=torch.float64, device=dev)
    ek = torch.zeros(1, dtype=torch.float64, device=dev)
    F = torch.zeros(n, 3, dtype=torch.float64, device=dev)
    ctx.md_step_dev(pos, vel, s.species, s.box, s.pbc, 5e-4, 4, ep, ek, F)
    torch.cuda.synchronize()
    vel[11, 1] = float("nan")
    before = (pos.clone(), vel.clone(), ep.clone(), ek.clone(), F.clone())
    with pytest.raises(A.AenetError) as e:
        ctx.md_step_dev(pos, vel, s.species, s.box, s.pbc, 5e-4, 3, ep, ek, F)
    assert e.value.code == A.AENET_E_NONFINITE
    torch.cuda.synchronize()
    for a, b in zip((pos, vel, ep, ek, F), before):
        assert torch.equal(a, b) or (torch.isnan(a).any() and torch.equal(torch.nan_to_num(a), torch.nan_to_num(b)))
    vel[11, 1] = 0.0
    ctx.md_step_dev(pos, vel, s.species, s.box, s.pbc, 5e-4, 3, ep, ek, F)
    torch.cuda.synchronize()
    assert torch.isfinite(pos).all() and torch.isfinite(F).all()
    ctx.close()


def _dense_lisio_box():
    n = int(round(0.0964 * 17.0 ** 3))
    return I.amorphous_box(n, (n // 3, n // 6, n - n // 3 - n // 6), 17.0, 4242)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_factorised_angular_matches_oracle(A, orc, precision, tol):
    """The angular terms of Eq. 6 by the addition theorem (forced) against
    the oracle's pair sums: water64 (angular order 4), a three-species open
    cluster with weights 1, 2, 3 (order 2), a small box with several images
    of one atom, and the dense Li/Si/O box (order 6, ~110 angular
    neighbours); descriptors element by element, energies and forces to the
    bars of each precision."""
    g = np.random.default_rng(5)
    pos = I.rsa(60, 14.0, 1.6, 77) + 30.0
    sp = g.integers(0, 3, size=60).astype(np.int32)
    cluster = I.System(pos, sp, np.array([80.0, 80.0, 80.0]), np.zeros(3, dtype=np.uint8))
    small = I.water_box(8, 908)
    cases = [("water64", I.load_model("water64"), I.make_system("water64")),
             ("cluster3", small_model(S=3, nr=4, na=2, rr=5.0, ra=4.0, tw=(1.0, 2.0, 3.0)), cluster),
             ("images", small_model(nr=5, na=3, rr=min(6.5, small.box[0] * 0.99), ra=4.0), small),
             ("lisio_dense", I.load_model("lisio120k"), _dense_lisio_box())]
    for name, m, s in cases:
        ctx = A.Context(m, precision)
        ctx.set_angular_method("factorised")
        E, Ea, F = ctx.energy_forces(s.pos, s.species, s.box, s.pbc)
        G = ctx.descriptors(s.pos, s.species, s.box, s.pbc)
        ctx.close()
        E0, Ea0, F0, G0 = orc.energy_forces(m, s.pos, s.species, s.box, s.pbc, want_G=True)
        dG = float(np.abs(G - G0).max() / np.abs(G0).max())
        de = abs(E - E0) / abs(E0)
        df = rel_rmse(F, F0)
        dmax = float(np.abs(F - F0).max() / np.abs(F0).max())
        print(f"{name} {precision}: max|dG|/max|G| {dG:.2e} rel dE {de:.2e} rel F rmse {df:.2e} max {dmax:.2e}")
        assert dG <= (1e-12 if precision == "fp64" else 1e-5), name
        assert de <= (1e-10 if precision == "fp64" else 1e-5), name
        assert df <= tol and dmax <= (1.0 if precision == "fp64" else 10.0) * tol, name


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_crowded_pair_path_matches_oracle(A, orc, precision, tol):
    """The pair sums of Eq. 6 on the dense Li/Si/O box, where the angular
    shells (~110 entries) exceed a wavefront and the force pass visits each
    unordered pair once with the partner's sums accumulated in LDS: energy
    and forces, element by element, against the oracle."""
    m = I.load_model("lisio120k")
    s = _dense_lisio_box()
    ctx = A.Context(m, precision)
    ctx.set_angular_method("pairs")
    E, Ea, F = ctx.energy_forces(s.pos, s.species, s.box, s.pbc)
    st = ctx.stats()
    ctx.close()
    assert st["max_angular"] > 64, st
    E0, Ea0, F0 = orc.energy_forces(m, s.pos, s.species, s.box, s.pbc)
    de = abs(E - E0) / abs(E0)
    dmax = float(np.abs(F - F0).max() / np.abs(F0).max())
    print(f"{precision}: rel dE {de:.2e} rel F rmse {rel_rmse(F, F0):.2e} max {dmax:.2e}")
    assert de <= tol and rel_rmse(F, F0) <= tol and dmax <= (1.0 if precision == "fp64" else 10.0) * tol


def test_factorised_and_pair_paths_agree(A):
    """On the dense Li/Si/O box the two evaluations of the angular terms give
    the same energies and forces to rounding, and MD over both agrees."""
    m = I.load_model("lisio120k")
    s = _dense_lisio_box()
    out = {}
    for method in ("pairs", "factorised"):
        ctx = A.Context(m, "fp64", skin=0.5)
        ctx.set_angular_method(method)
        out[method] = ctx.energy_forces(s.pos, s.species, s.box, s.pbc)
        v = I.maxwell_boltzmann(m.masses[s.species], 300.0, 3)
        out[method + "_md"] = ctx.md_step(s.pos, v, s.species, s.box, s.pbc, 1e-3, 8)
        ctx.close()
    (E1, Ea1, F1), (E2, Ea2, F2) = out["pairs"], out["factorised"]
    assert abs(E1 - E2) <= 1e-12 * abs(E1)
    assert np.abs(F1 - F2).max() <= 1e-12 * np.abs(F1).max()
    p1, p2 = out["pairs_md"][0], out["factorised_md"][0]
    assert np.abs((p1 - p2 + s.box / 2) % s.box - s.box / 2).max() <= 1e-10
