"""Full-size workloads, reduced-precision modes and the training-loss gradient
on the GPU, against the FP64 oracle.

Bars (method statement): FP64 energy within 1e-10 relative; force RMSE
<= 1e-5 eV/A (FP32 networks and descriptors) and <= 5e-3 eV/A (BF16 network
operands); the models are scaled so the oracle's force RMS on frame 0 is
1 eV/A.  Loss gradient: oracle to 1e-9 relative, central finite differences
(h = 1e-5, FP64) to 1e-6 relative.
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


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def water4096_ref(orc):
    m = I.load_model("water4096")
    s = I.make_system("water4096")
    E, Ea, F = orc.energy_forces(m, s.pos, s.species, s.box, s.pbc)
    return m, s, E, Ea, F


@pytest.mark.parametrize("prec,tol", [("fp64", None), ("fp32", 1e-5), ("bf16", 5e-3)])
def test_water4096_full_size(A, water4096_ref, prec, tol):
    m, s, E0, Ea0, F0 = water4096_ref
    ctx = A.Context(m, prec, skin=0.5)  # the benchmark's configuration
    E, Ea, F = ctx.energy_forces(s.pos, s.species, s.box, s.pbc)
    rmse = float(np.sqrt(np.mean((F - F0) ** 2)))
    rms = float(np.sqrt(np.mean(F0 ** 2)))
    de = abs(E - E0) / abs(E0)
    dea = float(np.abs(Ea - Ea0).max())
    print(f"water4096 {prec}: force rmse {rmse:.3e} eV/A (rms {rms:.3f}), rel dE {de:.3e}, max dE_atom {dea:.3e} eV")
    if prec == "fp64":
        assert de <= 1e-10, de
        assert rmse <= 1e-10 * rms, rmse
    else:
        assert rmse <= tol, rmse


@pytest.fixture(scope="module")
def lisio_sample(orc):
    m = I.load_model("lisio120k")
    s = I.make_system("lisio120k")
    sel = np.random.default_rng(11).choice(s.pos.shape[0], 10, replace=False)
    Es, Fs, Gs = orc.energy_forces_subset(m, s.pos, s.species, s.box, s.pbc, sel)
    return m, s, sel, Es, Fs, Gs


@pytest.mark.parametrize("prec,tol", [("fp64", None), ("bf16", 5e-3)])
def test_lisio120k_sampled(A, lisio_sample, prec, tol):
    """120,000-atom three-species box at full size, checked on sampled atoms."""
    m, s, sel, Es, Fs, Gs = lisio_sample
    ctx = A.Context(m, prec, skin=0.5)
    E, Ea, F = ctx.energy_forces(s.pos, s.species, s.box, s.pbc)
    dF = F[sel] - Fs
    rmse = float(np.sqrt(np.mean(dF ** 2)))
    dea = float(np.abs(Ea[sel] - Es).max())
    print(f"lisio120k {prec}: sampled force rmse {rmse:.3e} eV/A, max dE_atom {dea:.3e} eV")
    if prec == "fp64":
        assert rmse <= 1e-10 * float(np.sqrt(np.mean(Fs ** 2))), rmse
        assert dea <= 1e-10 * float(np.abs(Es).max()), dea
        np.testing.assert_allclose(F.sum(0), 0.0, atol=1e-8 * np.abs(F).sum() / len(F))
    else:
        assert rmse <= tol, rmse


# ---------------------------------------------------------------- training loss (a10)
def _batch(n_boxes, sizes=None):
    sizes = sizes or I.batch_sizes()[:: max(1, 256 // n_boxes)][:n_boxes]
    boxes = [I.water_box(nm, I.seed_for(3, 0) + 7 * k) for k, nm in enumerate(sizes)]
    offs = np.concatenate([[0], np.cumsum([len(b.pos) for b in boxes])]).astype(np.int64)
    pos = np.vstack([b.pos for b in boxes])
    sp = np.concatenate([b.species for b in boxes])
    bx = np.vstack([b.box for b in boxes])
    return boxes, offs, pos, sp, bx


def _refs(orc, ref_model, boxes):
    er, fr = [], []
    for b in boxes:
        E, _, F = orc.energy_forces(ref_model, b.pos, b.species, b.box, b.pbc)
        er.append(E)
        fr.append(F)
    return np.array(er), np.vstack(fr)


def _gpu_loss_grad(ctx, torch_dev, offs, pos, sp, bx, er, fr, lam=1.0):
    torch, dev = torch_dev
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    grad = torch.zeros(ctx.n_params(), dtype=torch.float64, device=dev)
    ctx.loss_grad_dev(offs, torch.from_numpy(pos).to(dev), sp, bx, (1, 1, 1),
                      torch.from_numpy(er).to(dev), torch.from_numpy(fr).to(dev), lam, loss, grad)
    torch.cuda.synchronize()
    return loss.item(), grad.cpu().numpy()


@pytest.fixture(scope="module")
def small_batch(orc):
    m = I.load_model("water4096")
    ref = I.load_model("water4096_ref")
    boxes, offs, pos, sp, bx = _batch(3, sizes=[64, 70, 81])
    er, fr = _refs(orc, ref, boxes)
    return m, boxes, offs, pos, sp, bx, er, fr


def test_loss_grad_matches_oracle(A, orc, torch_dev, small_batch):
    m, boxes, offs, pos, sp, bx, er, fr = small_batch
    ctx = A.Context(m, "fp64")
    L, g = _gpu_loss_grad(ctx, torch_dev, offs, pos, sp, bx, er, fr)
    L0, g0 = orc.loss_grad(m, offs, pos, sp, bx, (1, 1, 1), er, fr, 1.0)
    dl = abs(L - L0) / abs(L0)
    dg = float(np.abs(g - g0).max() / np.abs(g0).max())
    print(f"loss {L:.12e} oracle {L0:.12e} rel {dl:.2e}; grad max rel {dg:.2e}")
    assert dl <= 1e-10, dl
    assert dg <= 1e-9, dg


def test_loss_grad_finite_differences(A, torch_dev, small_batch):
    m, boxes, offs, pos, sp, bx, er, fr = small_batch
    ctx = A.Context(m, "fp64")
    p0 = ctx.get_params()
    _, g = _gpu_loss_grad(ctx, torch_dev, offs, pos, sp, bx, er, fr)
    h = 1e-5
    rng = np.random.default_rng(3)
    idx = list(rng.choice(len(p0), 10, replace=False)) + [len(p0) // 2 - 1, len(p0) - 1]
    worst = 0.0
    for k in idx:
        pp = p0.copy(); pp[k] += h
        ctx.set_params(pp)
        Lp, _ = _gpu_loss_grad(ctx, torch_dev, offs, pos, sp, bx, er, fr)
        pp = p0.copy(); pp[k] -= h
        ctx.set_params(pp)
        Lm, _ = _gpu_loss_grad(ctx, torch_dev, offs, pos, sp, bx, er, fr)
        fd = (Lp - Lm) / (2 * h)
        err = abs(fd - g[k]) / max(abs(fd), 1e-3 * np.abs(g).max())
        worst = max(worst, err)
    ctx.set_params(p0)
    print(f"finite-difference max rel err {worst:.2e}")
    assert worst <= 1e-6, worst


def test_loss_grad_full_batch_is_mean_of_structures(A, orc, torch_dev):
    """The 256-box, 221,184-atom batch in one launch equals the average of the
    per-structure gradients (linearity of the loss), and sampled structures
    match the oracle."""
    m = I.load_model("water4096")
    ref = I.load_model("water4096_ref")
    boxes, offs, pos, sp, bx = _batch(256, sizes=I.batch_sizes())
    assert offs[-1] == 221184
    ctx = A.Context(m, "fp64")
    # reference energies/forces from the second network, computed on the GPU in FP64
    # for the full batch (the oracle checks three sampled structures below)
    ctx_ref = A.Context(ref, "fp64")
    torch, dev = torch_dev
    e_ref = torch.zeros(256, dtype=torch.float64, device=dev)
    f_ref = torch.zeros(len(pos), 3, dtype=torch.float64, device=dev)
    ctx_ref.energy_forces_batch_dev(offs, torch.from_numpy(pos).to(dev), sp, bx, (1, 1, 1), e_ref, None, f_ref)
    torch.cuda.synchronize()
    er, fr = e_ref.cpu().numpy(), f_ref.cpu().numpy()
    L, g = _gpu_loss_grad(ctx, torch_dev, offs, pos, sp, bx, er, fr)
    acc_L, acc_g = 0.0, np.zeros_like(g)
    for k in range(256):
        a, b = offs[k], offs[k + 1]
        Lk, gk = _gpu_loss_grad(ctx, torch_dev, np.array([0, b - a]), pos[a:b], sp[a:b], bx[k:k + 1],
                                er[k:k + 1], fr[a:b])
        acc_L += Lk / 256
        acc_g += gk / 256
    assert abs(L - acc_L) <= 1e-12 * abs(L)
    assert float(np.abs(g - acc_g).max()) <= 1e-11 * float(np.abs(g).max())
    for k in (0, 128, 255):
        a, b = offs[k], offs[k + 1]
        E0, _, F0 = orc.energy_forces(ref, pos[a:b], sp[a:b], bx[k], (1, 1, 1))
        assert abs(E0 - er[k]) <= 1e-10 * abs(E0)
        Lk, gk = _gpu_loss_grad(ctx, torch_dev, np.array([0, b - a]), pos[a:b], sp[a:b], bx[k:k + 1],
                                er[k:k + 1], fr[a:b])
        L0, g0 = orc.loss_grad(m, [0, b - a], pos[a:b], sp[a:b], bx[k:k + 1], (1, 1, 1), er[k:k + 1],
                               fr[a:b], 1.0)
        assert abs(Lk - L0) <= 1e-10 * abs(L0)
        assert float(np.abs(gk - g0).max()) <= 1e-9 * float(np.abs(g0).max())


# ---------------------------------------------------------------- L-BFGS training (Sec. II C)
@pytest.mark.parametrize("lam", [0.0, 1.0])
def test_lbfgs_fit(A, orc, torch_dev, small_batch, lam):
    """Full-batch L-BFGS on the library's cost (energy only, the objective of
    Eq. 7, and energy+force): its first evaluation is the oracle's cost, and
    the optimiser lowers it by an order of magnitude within 40 iterations."""
    from paper_2107_11311_amd import train
    m, boxes, offs, pos, sp, bx, er, fr = small_batch
    ctx = A.Context(m, "fp64")
    L0, _ = orc.loss_grad(m, offs, pos, sp, bx, (1, 1, 1), er, fr, lam)
    r = train.fit_lbfgs(ctx, offs, pos, sp, bx, (1, 1, 1), er, fr if lam > 0 else None, lambda_f=lam,
                        maxiter=40)
    print(f"lambda_f={lam}: loss {r.loss0:.4e} -> {r.loss:.4e} in {r.iterations} iterations, "
          f"{r.evaluations} evaluations, {1e3 * r.seconds / max(r.evaluations, 1):.2f} ms each; "
          f"|grad| {r.grad_norm0:.3e} -> {r.grad_norm:.3e}")
    assert abs(r.loss0 - L0) <= 1e-10 * abs(L0)
    assert r.loss <= 0.1 * r.loss0
    assert np.array_equal(ctx.get_params(), r.params)
    ctx.close()


# ---------------------------------------------------------------- NVT (weak coupling)
def test_nvt_berendsen_matches_oracle_chunks(A, orc, torch_dev):
    """Velocity-Verlet chunks on the GPU with a Berendsen velocity scale after
    each chunk against the oracle's velocity Verlet under the same coupling:
    the temperatures seen, the scale factors and the final state agree, and
    every scale factor pulls toward the target."""
    from paper_2107_11311_amd import thermostat as TH
    torch, dev = torch_dev
    m = I.load_model("water64")
    s = I.make_system("water64")
    v0 = I.maxwell_boltzmann(m.masses[s.species], 900.0, 21)
    dt, chunk, n_chunks, T0, tau = 5e-4, 5, 4, 300.0, 0.01
    ctx = A.Context(m, "fp64", skin=0.5)
    pos = torch.from_numpy(s.pos.copy()).to(dev)
    vel = torch.from_numpy(v0.copy()).to(dev)
    tr = TH.nvt_berendsen(ctx, pos, vel, s.species, s.box, s.pbc, dt, n_chunks, chunk, T0, tau)
    ctx.close()
    p, v = s.pos.copy(), v0.copy()
    n = len(p)
    for k in range(n_chunks):
        p, v, ep, ek, _ = orc.md_vv(m, p, v, s.species, m.masses, s.box, s.pbc, dt, chunk)
        # T with 3N - 3 degrees of freedom (zero total momentum) and the
        # weak-coupling scale sqrt(1 + (t/tau)(T0/T - 1)) of Berendsen et al.
        # (1984) over the chunk's time t, written out here
        t_now = 2.0 * ek / ((3 * n - 3) * 8.617333262e-5)
        lam = np.sqrt(1.0 + (chunk * dt / tau) * (T0 / t_now - 1.0))
        v = v * lam
        assert abs(tr.temperatures[k] - t_now) <= 1e-9 * t_now, k
        assert abs(tr.lambdas[k] - lam) <= 1e-9, k
    L = np.asarray(s.box)
    dp = pos.cpu().numpy() - p
    dp -= L * np.round(dp / L)
    assert np.abs(dp).max() <= 1e-8
    np.testing.assert_allclose(vel.cpu().numpy(), v, atol=1e-8 * np.abs(v).max())
    # every coupling step pulls toward the target (the random-weight network
    # itself keeps heating the box, so T need not fall)
    assert all((t > T0) == (lam < 1.0) for t, lam in zip(tr.temperatures, tr.lambdas))
