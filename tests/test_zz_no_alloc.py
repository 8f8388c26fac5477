"""The no-allocation entry point (aenet_energy_forces_noalloc) against the
entry point it mirrors (aenet_energy_forces_dev), through the C ABI: the same
energies and forces bit for bit on two calls in a row (the second on a
smaller structure, so the shared workspace holds the first call's contents),
agreement with the FP64 oracle, a clear error for a structure that does not
fit the workspace, and the context's own entry points unaffected."""
import numpy as np
import pytest

from paper_2107_11311_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def A():
    from paper_2107_11311_amd import aenet
    aenet.load()
    return aenet


def _run(torch, ctx, s, noalloc):
    dev = torch.device("cuda:0")
    n = len(s.pos)
    pos = torch.from_numpy(s.pos.copy()).to(dev)
    e = torch.zeros(1, dtype=torch.float64, device=dev)
    ea = torch.zeros(n, dtype=torch.float64, device=dev)
    F = torch.zeros(n, 3, dtype=torch.float64, device=dev)
    call = ctx.energy_forces_noalloc if noalloc else ctx.energy_forces_dev
    call(pos, s.species, s.box, s.pbc, e, ea, F)
    torch.cuda.synchronize()
    return e.item(), ea.cpu().numpy(), F.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_matches_dev_entry_point(A, orc, precision):
    import torch
    m = I.load_model("water64")
    cases = [I.make_system("water64"), I.water_box(20, 4321)]   # 192 atoms, then 60
    ctx = A.Context(m, precision)
    ref = A.Context(m, precision)
    for s in cases:
        E1, Ea1, F1 = _run(torch, ctx, s, True)
        E0, Ea0, F0 = _run(torch, ref, s, False)
        print(f"{precision} n={len(s.pos)}: E noalloc {E1:.15g} dev {E0:.15g}")
        assert E1 == E0
        assert np.array_equal(Ea1, Ea0) and np.array_equal(F1, F0)
        Eo, _, Fo = orc.energy_forces(m, s.pos, s.species, s.box, s.pbc)
        tol = 1e-10 if precision == "fp64" else 1e-5
        assert abs(E1 - Eo) <= tol * abs(Eo)
        assert np.sqrt(np.mean((F1 - Fo) ** 2)) <= tol * max(1.0, np.sqrt(np.mean(Fo ** 2)))
    # the context's own entry point after the no-allocation calls
    s = cases[0]
    E2, Ea2, F2 = _run(torch, ctx, s, False)
    E0, Ea0, F0 = _run(torch, ref, s, False)
    assert E2 == E0 and np.array_equal(F2, F0)
    ctx.close()
    ref.close()


def test_noalloc_rejects_structures_beyond_the_workspace(A):
    import torch
    m = I.load_model("water4096")
    s = I.make_system("water4096")   # 12,288 atoms: rows alone exceed 64 MiB
    ctx = A.Context(m, "fp64")
    with pytest.raises(A.AenetError) as e:
        _run(torch, ctx, s, True)
    assert e.value.code == A.AENET_E_INVALID and "workspace" in str(e.value)
    # still usable, by both entry points
    s2 = I.make_system("water64")
    m2 = I.load_model("water64")
    ctx2 = A.Context(m2, "fp64")
    E1, _, F1 = _run(torch, ctx2, s2, True)
    E0, _, F0 = _run(torch, ctx2, s2, False)
    assert E1 == E0 and np.array_equal(F1, F0)
    ctx.close()
    ctx2.close()


def test_noalloc_first_then_larger_dev_call(A):
    """A fresh context whose first call is the no-allocation one, then the
    context's own entry point on a larger structure, then the no-allocation
    one again: every per-call buffer the no-allocation call used is the
    workspace's and goes back afterwards, so the context's own buffers grow
    from nothing and the results match a context that never used the
    workspace."""
    import torch
    m = I.load_model("water64")
    small, large = I.water_box(20, 4321), I.make_system("water64")
    ctx = A.Context(m, "fp64")
    ref = A.Context(m, "fp64")
    for s, noalloc in ((small, True), (large, False), (large, True), (small, False)):
        E1, Ea1, F1 = _run(torch, ctx, s, noalloc)
        E0, Ea0, F0 = _run(torch, ref, s, False)
        print(f"n={len(s.pos)} noalloc={noalloc}: E {E1:.15g} ref {E0:.15g}")
        assert E1 == E0 and np.array_equal(Ea1, Ea0) and np.array_equal(F1, F0)
    ctx.close()
    ref.close()
