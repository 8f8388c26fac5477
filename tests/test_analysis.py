"""Diffusion analysis (Eqs. 8 and 9): a random walk of known diffusion
coefficient, wrapped into a periodic box, recovered through unwrapping and
the MSD slope; the finite-size correction and the 1/L extrapolation against
closed forms."""
import numpy as np

from paper_2107_11311_amd import analysis as AN


def test_random_walk_recovers_diffusion_coefficient():
    rng = np.random.default_rng(4)
    D, dt, T, N = 0.23, 0.05, 400, 500          # A^2/ps, ps, frames, walkers
    steps = rng.normal(scale=np.sqrt(2 * D * dt), size=(T - 1, N, 3))
    x0 = rng.uniform(0, 20.0, size=(N, 3))
    traj = np.concatenate([x0[None], x0 + np.cumsum(steps, axis=0)])
    box = np.array([20.0, 20.0, 20.0])
    wrapped = traj - box * np.floor(traj / box)
    un = AN.unwrap(wrapped, box)
    np.testing.assert_allclose(un, traj, atol=1e-9)
    m = AN.msd(un, max_lag=100)
    assert m[0] == 0.0
    d = AN.diffusion_coefficient(m, dt)
    assert abs(d - D) / D < 0.05, d
    # an open axis is not unwrapped
    un2 = AN.unwrap(traj, box, pbc=(1, 1, 0))
    np.testing.assert_allclose(un2, traj, atol=1e-9)


def test_msd_of_ballistic_motion():
    """Uniform motion r = r0 + v t: MSD(k) = |v|^2 (k dt)^2 exactly."""
    v = np.array([0.3, -0.2, 0.1])
    t = np.arange(50) * 0.1
    traj = np.zeros((50, 3, 3)) + t[:, None, None] * v
    m = AN.msd(traj)
    np.testing.assert_allclose(m, (v @ v) * (np.arange(50) * 0.1) ** 2, rtol=1e-12, atol=1e-15)


def test_eq9_constant_is_the_cubic_lattice_sum():
    """The constant xi of Eq. 9 is the lattice sum of the simple cubic
    lattice (the periodic Oseen tensor's leading term has the same sum as a
    1/r interaction with a uniform background): computed here by Ewald
    summation, independent of the splitting parameter."""
    from scipy.special import erfc
    vals = []
    for alpha in (1.5, 2.0, 3.0):
        n = np.arange(-6, 7)
        X, Y, Z = np.meshgrid(n, n, n, indexing="ij")
        r = np.sqrt(X ** 2 + Y ** 2 + Z ** 2).ravel()
        r = r[r > 0]
        k2 = (X ** 2 + Y ** 2 + Z ** 2).ravel()
        k2 = k2[k2 > 0]
        psi = (np.sum(erfc(alpha * r) / r) + np.sum(np.exp(-np.pi ** 2 * k2 / alpha ** 2) / (np.pi * k2))
               - 2 * alpha / np.sqrt(np.pi) - np.pi / alpha ** 2)
        vals.append(-psi)
    assert max(vals) - min(vals) < 1e-12
    assert abs(vals[0] - AN.XI_CUBIC) < 1e-6


def test_finite_size_correction_closed_form():
    # water near 300 K: eta = 0.89 mPa s, L = 30 A
    d_inf = AN.finite_size_correction(0.20, 30.0, 300.0, 0.89e-3)
    corr = 2.837297 * 1.380649e-23 * 300.0 / (6 * np.pi * 0.89e-3 * 30e-10)  # m^2/s
    assert abs(d_inf - (0.20 + corr * 1e8)) < 1e-12
    assert 0.02 < corr * 1e8 < 0.03


def test_extrapolation_to_infinite_size():
    L = np.array([12.4, 15.6, 19.7, 24.8, 31.3])
    d = 0.25 - 0.9 / L
    d_inf, slope = AN.extrapolate_infinite(L, d)
    assert abs(d_inf - 0.25) < 1e-12 and abs(slope + 0.9) < 1e-10


def test_gliding_average_against_direct_means():
    """Every entry is the plain mean of its window; a constant stays constant
    and a straight line is returned at the window centres."""
    rng = np.random.default_rng(7)
    x = rng.normal(size=37)
    for w in (1, 4, 37):
        g = AN.gliding_average(x, w)
        assert g.size == x.size - w + 1
        np.testing.assert_allclose(g, [x[k - w + 1:k + 1].mean() for k in range(w - 1, x.size)], atol=1e-13)
    np.testing.assert_allclose(AN.gliding_average(np.full(10, -3.25), 4), -3.25, atol=1e-15)
    t = np.arange(20.0)
    np.testing.assert_allclose(AN.gliding_average(2.0 * t + 1.0, 5), 2.0 * (t[4:] - 2.0) + 1.0, atol=1e-12)


def test_metropolis_samples_boltzmann_harmonic():
    """Energy-only Metropolis on independent harmonic degrees of freedom
    E = k/2 sum x^2 samples the Boltzmann distribution: <x^2> = k_B T / k;
    a move that lowers the energy is always accepted."""
    from paper_2107_11311_amd import mc
    rng = np.random.default_rng(3)
    k, T = 2.0, 300.0
    kT = mc.KB_EV * T
    n, trials = 64, 6000
    moves = np.zeros((trials, n, 3))
    which = rng.integers(0, n, size=trials)
    moves[np.arange(trials), which] = rng.uniform(-0.15, 0.15, size=(trials, 3))
    u = rng.uniform(size=trials)

    def energy(p):
        return 0.5 * k * float(np.sum(p * p))

    x, tr = mc.metropolis(energy, np.zeros((n, 3)), T, moves, u)
    assert 0.3 < tr.acceptance < 0.95
    x2, tr2 = mc.metropolis(energy, x, T, moves, u)
    # a second run from equilibrium: average of x^2 over the run
    xs = x.copy()
    acc = []
    for d, uu in zip(moves, u):
        y = xs + d
        if energy(y) <= energy(xs) or uu < np.exp(-(energy(y) - energy(xs)) / kT):
            xs = y
        acc.append(np.mean(xs * xs))
    np.testing.assert_allclose(x2, xs, atol=1e-15)
    assert abs(np.mean(acc) / (kT / k) - 1.0) < 0.15
    down = mc.metropolis(energy, np.full((n, 3), 0.1), T, [np.full((n, 3), -0.05)], [0.999999])[1]
    assert down.accepted == [True]
