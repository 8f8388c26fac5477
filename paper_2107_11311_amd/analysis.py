"""Trajectory analysis of the paper's applications (Sec. IV): the diffusion
coefficient of water from the mean-square displacement (Eq. 8), its
finite-size correction (Eq. 9) and the direct extrapolation of D(L) against
1/L; and the gliding average of the potential energy used to follow the
equilibration of the Li_xSi nanoparticles.  Host-side numpy over frames written by the MD entry points (positions
in the caller's order, wrapped into the box on list rebuilds).

Units: positions in A, times in ps, D in A^2/ps, viscosity in Pa s,
temperature in K.
"""
import numpy as np

XI_CUBIC = 2.837297          # the constant of Eq. 9 for a cubic periodic cell
KB_J = 1.380649e-23          # Boltzmann constant, J/K
M2S_TO_A2PS = 1e8            # 1 m^2/s = 1e20 A^2 / 1e12 ps


def unwrap(frames, box, pbc=(1, 1, 1)):
    """Frames [T, N, 3] of wrapped positions -> continuous trajectories: each
    frame-to-frame displacement is taken at its minimum image along the
    periodic axes (frames must be close enough that no atom moves half a box
    between two of them)."""
    x = np.asarray(frames, dtype=np.float64)
    L = np.asarray(box, dtype=np.float64)
    per = np.asarray(pbc, dtype=bool)
    d = np.diff(x, axis=0)
    d[..., per] -= L[per] * np.round(d[..., per] / L[per])
    out = np.empty_like(x)
    out[0] = x[0]
    out[1:] = x[0] + np.cumsum(d, axis=0)
    return out


def msd(traj, sel=None, max_lag=None):
    """Mean-square displacement <|r(t0 + k) - r(t0)|^2> over the selected atoms
    and every time origin t0, for lags k = 0 .. max_lag (frames)."""
    x = np.asarray(traj, dtype=np.float64)
    if sel is not None:
        x = x[:, sel]
    T = x.shape[0]
    max_lag = T - 1 if max_lag is None else min(max_lag, T - 1)
    out = np.zeros(max_lag + 1)
    for k in range(1, max_lag + 1):
        out[k] = np.mean(np.sum((x[k:] - x[:-k]) ** 2, axis=-1))
    return out


def diffusion_coefficient(msd_values, dt_frame, fit_from=0.2, fit_to=1.0):
    """D = (1/6) d<|r(t) - r(0)|^2>/dt (Eq. 8): the least-squares slope of the
    MSD over the window [fit_from, fit_to] of the lag range, divided by 6."""
    m = np.asarray(msd_values, dtype=np.float64)
    n = m.size - 1
    k0, k1 = int(round(fit_from * n)), int(round(fit_to * n))
    k = np.arange(k0, k1 + 1)
    slope = np.polyfit(k * dt_frame, m[k], 1)[0]
    return slope / 6.0


def finite_size_correction(d_l, box_length, temperature, viscosity, xi=XI_CUBIC):
    """D(inf) = D(L) + xi k_B T / (6 pi eta L) (Eq. 9), D in A^2/ps, L in A,
    eta in Pa s."""
    corr_m2s = xi * KB_J * temperature / (6.0 * np.pi * viscosity * box_length * 1e-10)
    return d_l + corr_m2s * M2S_TO_A2PS


def extrapolate_infinite(box_lengths, d_values):
    """The infinite-size diffusion coefficient by the straight-line fit of
    D(L) against 1/L (the paper's direct extrapolation): (D(inf), slope)."""
    inv = 1.0 / np.asarray(box_lengths, dtype=np.float64)
    slope, intercept = np.polyfit(inv, np.asarray(d_values, dtype=np.float64), 1)
    return intercept, slope


def gliding_average(values, window: int):
    """Trailing moving average: out[k] = mean(values[k - window + 1 .. k]) for
    k >= window - 1 (len(values) - window + 1 entries), the smoothed energy
    curve of an equilibration run."""
    x = np.asarray(values, dtype=np.float64)
    if window < 1 or window > x.size:
        raise ValueError("window must be 1..len(values)")
    c = np.concatenate([[0.0], np.cumsum(x)])
    return (c[window:] - c[:-window]) / window
