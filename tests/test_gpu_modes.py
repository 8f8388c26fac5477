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


def _dense_lisio(L, seed):
    """A three-species amorphous box at the 120k workload's density (0.0964
    atoms/A^3, Li:Si:O = 2:1:3, minimum distance 1.6 A) with edge L."""
    n = int(round(0.0964 * L ** 3))
    counts = (n // 3, n // 6, n - n // 3 - n // 6)
    return I.amorphous_box(n, counts, L, seed)


@pytest.mark.parametrize("L,path", [(17.0, "cell"), (18.0, "cell_wide"), (19.0, "atom")])
def test_lisio_dense_md(A, orc, L, path):
    """MD at the 120k workload's density, orders and cutoffs (18 / 8.0 A, 6 /
    6.5 A) in boxes of 2 x 2 x 2 list cells: about 59 atoms per cell at
    L = 17 A (the per-cell row kernel), 70 at 18 A (the per-cell kernel with
    its cells sorted in two halves of 64) and 83 at 19 A (more than the
    per-cell kernel is planned for: the per-atom row kernels and the reverse
    search), each inside md_step, with about 111 angular neighbours, so the
    force pass takes its crowded-shell path.  12 steps of 1 fs with a build
    forced every 4 steps and rows that start too short (a capacity retry),
    against the oracle's velocity Verlet, element by element."""
    m = I.load_model("lisio120k")
    s = _dense_lisio(L, 4242)
    n = len(s.pos)
    per_cell = n / 8  # 2 x 2 x 2 cells of >= 8.5 A
    # the host plans the per-cell kernel while 1.5 x the mean cell count + 8
    # stays within its 128 atoms
    assert {"cell": per_cell < 64, "cell_wide": 64 < per_cell and 1.5 * per_cell + 8 <= 128,
            "atom": 1.5 * per_cell + 8 > 128}[path], per_cell
    v = I.maxwell_boltzmann(m.masses[s.species], 300.0, 17)
    ctx = A.Context(m, "fp64", skin=0.5)
    ctx.set_rebuild_every(4)
    ctx.set_capacity(160, 80)
    p1, v1, ep, ek, F = ctx.md_step(s.pos, v, s.species, s.box, s.pbc, 1e-3, 12)
    st = ctx.stats()
    p0, v0, ep0, ek0, F0 = orc.md_vv(m, s.pos, v, s.species, m.masses, s.box, s.pbc, 1e-3, 12)
    dp = float(np.abs((p1 - p0 + s.box / 2) % s.box - s.box / 2).max())
    dv = float(np.abs(v1 - v0).max() / np.abs(v0).max())
    dF = float(np.abs(F - F0).max() / np.abs(F0).max())
    print(f"lisio dense {path} n={n}: dpos {dp:.2e} dvel {dv:.2e} max|dF|/max|F| {dF:.2e} rel dEpot "
          f"{abs(ep - ep0) / abs(ep0):.2e}; rows {st['max_neighbors']} / angular {st['max_angular']}, "
          f"builds {st['n_rebuilds']}, capacity retries {st['n_capacity_retries']}")
    assert st["max_angular"] > 64 and st["n_capacity_retries"] >= 1 and st["n_rebuilds"] >= 4
    assert dp <= 1e-10 and dv <= 1e-10 and dF <= 1e-10
    assert abs(ep - ep0) <= 1e-10 * abs(ep0) and abs(ek - ek0) <= 1e-10 * abs(ek0)
    ctx.close()


def test_lisio120k_bf16_trajectory_sampled(A, orc, torch_dev):
    """The 120,000-atom workload as specified: BF16 networks, 200 MD steps of
    1 fs.  At steps 0, 100 and 200 the GPU forces on 96 sampled atoms are
    compared with the oracle's at the same positions (RMSE bar 5e-3 eV/A);
    at step 0 the FP64 path is checked on the same atoms element by element."""
    import os
    torch, dev = torch_dev
    m = I.load_model("lisio120k")
    s = I.make_system("lisio120k")
    n = len(s.pos)
    v = I.maxwell_boltzmann(m.masses[s.species], 300.0, I.seed_for(2, 2))
    ctx = A.Context(m, "bf16", skin=0.5)
    pos = torch.from_numpy(s.pos.copy()).to(dev)
    vel = torch.from_numpy(v.copy()).to(dev)
    F = torch.zeros(n, 3, dtype=torch.float64, device=dev)
    frames = []
    for steps in (0, 100, 100):
        ctx.md_step_dev(pos, vel, s.species, s.box, s.pbc, 1e-3, steps, None, None, F)
        torch.cuda.synchronize()
        frames.append((pos.cpu().numpy(), F.cpu().numpy()))
    ctx.close()
    workers = min(16, os.cpu_count() or 1)
    g = np.random.default_rng(12)
    for k, (p, Fg) in enumerate(frames):
        sel = g.choice(n, 96, replace=False)
        _, Fo, _ = orc.energy_forces_subset_parallel(m, p, s.species, s.box, s.pbc, sel, workers)
        rmse = float(np.sqrt(np.mean((Fg[sel] - Fo) ** 2)))
        print(f"lisio120k bf16 step {100 * k}: sampled force rmse {rmse:.3e} eV/A "
              f"(rms {np.sqrt(np.mean(Fo ** 2)):.3f})")
        assert rmse <= 5e-3, (k, rmse)
        if k == 0:
            c64 = A.Context(m, "fp64", skin=0.5)
            _, _, F64 = c64.energy_forces(p, s.species, s.box, s.pbc)
            c64.close()
            assert np.abs(F64[sel] - Fo).max() <= 1e-10 * np.abs(Fo).max()


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


# ---------------------------------------------------------------- NPT (weak coupling, virial pressure)
def test_npt_berendsen_matches_oracle_chunks(A, orc, torch_dev):
    """Velocity-Verlet chunks on the GPU with a Berendsen temperature and
    pressure coupling after each chunk (pressure from the kinetic energy and
    the GPU virial) against the oracle's velocity Verlet and virial under the
    same couplings, written out here: pressures, volumes and the final state
    agree."""
    from paper_2107_11311_amd import thermostat as TH
    torch, dev = torch_dev
    m = I.load_model("water64")
    s = I.make_system("water64")
    v0 = I.maxwell_boltzmann(m.masses[s.species], 300.0, 23)
    dt, chunk, n_chunks = 5e-4, 5, 4
    T0, tau_t, P0, tau_p, beta = 300.0, 0.05, 1.0, 0.05, 4.5e-5
    ctx = A.Context(m, "fp64", skin=0.3)
    pos = torch.from_numpy(s.pos.copy()).to(dev)
    vel = torch.from_numpy(v0.copy()).to(dev)
    box = s.box.copy()
    tr = TH.npt_berendsen(ctx, pos, vel, s.species, box, s.pbc, dt, n_chunks, chunk, T0, tau_t, P0, tau_p, beta)
    ctx.close()
    p, v, L = s.pos.copy(), v0.copy(), s.box.copy()
    n = len(p)
    ev_a3_bar = 1.602176634e-19 / 1e-30 / 1e5
    for k in range(n_chunks):
        p, v, ep, ek, _ = orc.md_vv(m, p, v, s.species, m.masses, L, s.pbc, dt, chunk)
        _, _, W = orc.energy_forces_virial(m, p, s.species, L, s.pbc)
        P = (2.0 * ek + np.trace(W)) / (3.0 * np.prod(L)) * ev_a3_bar
        T = 2.0 * ek / ((3 * n - 3) * 8.617333262e-5)
        lam = np.sqrt(1.0 + (chunk * dt / tau_t) * (T0 / T - 1.0))
        mu = (1.0 - beta * chunk * dt / tau_p * (P0 - P)) ** (1.0 / 3.0)
        v, p, L = v * lam, p * mu, L * mu
        assert abs(tr.pressures[k] - P) <= 1e-8 * abs(P) + 1e-6, (k, tr.pressures[k], P)
        assert abs(tr.volumes[k] - np.prod(L)) <= 1e-12 * np.prod(L), k
    print(f"npt: pressures {np.round(tr.pressures, 1)} bar, volumes {np.round(tr.volumes, 3)} A^3")
    assert abs(tr.volumes[-1] - np.prod(s.box)) > 1e-3 * np.prod(s.box)   # the box did move
    np.testing.assert_allclose(box, L, rtol=1e-13)
    dp = pos.cpu().numpy() - p
    dp -= L * np.round(dp / L)
    assert np.abs(dp).max() <= 1e-8
    np.testing.assert_allclose(vel.cpu().numpy(), v, atol=1e-8 * np.abs(v).max())


# ---------------------------------------------------------------- Monte Carlo and analyses on GPU data
def test_metropolis_gpu_energies_match_oracle(A, orc):
    """Energy-only Monte Carlo on water64: the GPU (force pass skipped) and the
    oracle, given the same single-atom moves and uniform numbers, take the
    same decisions and end in the same state."""
    from paper_2107_11311_amd import mc
    m = I.load_model("water64")
    s = I.make_system("water64")
    rng = np.random.default_rng(31)
    trials, n = 40, len(s.pos)
    moves = np.zeros((trials, n, 3))
    moves[np.arange(trials), rng.integers(0, n, size=trials)] = rng.uniform(-0.06, 0.06, size=(trials, 3))
    u = rng.uniform(size=trials)
    ctx = A.Context(m, "fp64")
    xg, tg = mc.metropolis(mc.gpu_energy(ctx, s.species, s.box, s.pbc), s.pos, 300.0, moves, u, s.box, s.pbc)
    xo, to = mc.metropolis(lambda p: orc.energy_forces(m, p, s.species, s.box, s.pbc)[0], s.pos, 300.0, moves,
                           u, s.box, s.pbc)
    print(f"mc: acceptance {tg.acceptance:.2f}")
    assert tg.accepted == to.accepted and 0 < sum(tg.accepted) < trials
    assert np.array_equal(xg, xo)
    np.testing.assert_allclose(tg.energies, to.energies, rtol=1e-10)
    ctx.close()


def test_msd_from_gpu_md_frames(A, orc):
    """The diffusion analysis on frames written by the GPU MD (positions
    wrapped by the library) equals the analysis of the oracle's trajectory."""
    from paper_2107_11311_amd import analysis as AN
    m = I.load_model("water64")
    s = I.make_system("water64")
    v = I.maxwell_boltzmann(m.masses[s.species], 300.0, 8)
    ctx = A.Context(m, "fp64", skin=0.3)
    pg, vg, po, vo = s.pos, v, s.pos, v
    fg, fo = [s.pos], [s.pos]
    for _ in range(8):
        pg, vg, _, _, _ = ctx.md_step(pg, vg, s.species, s.box, s.pbc, 5e-4, 5)
        po, vo, _, _, _ = orc.md_vv(m, po, vo, s.species, m.masses, s.box, s.pbc, 5e-4, 5)
        fg.append(pg)
        fo.append(po)
    ctx.close()
    mg = AN.msd(AN.unwrap(np.array(fg), s.box))
    mo = AN.msd(AN.unwrap(np.array(fo), s.box))
    assert mg[-1] > 1e-3
    np.testing.assert_allclose(mg, mo, rtol=1e-7, atol=1e-12)
