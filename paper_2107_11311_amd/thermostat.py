"""Constant-temperature (and constant-pressure) MD by weak coupling to a heat bath (the NVT runs of
the paper's applications, Sec. IV): velocity-Verlet chunks of `chunk` steps
on the GPU (aenet_md_step_dev), after each of which the velocities are scaled
by lambda = sqrt(1 + (chunk dt / tau) (T0 / T - 1)) with T the kinetic
temperature at the end of the chunk (Berendsen coupling applied per chunk,
so the device loop runs undisturbed between couplings).

T = 2 E_kin / ((3 N - 3) k_B): the centre-of-mass momentum is zero at the
start (Maxwell-Boltzmann initialisation) and stays zero (forces sum to zero,
and the scaling keeps it), so 3 of the 3N degrees of freedom carry no kinetic
energy.  Positions and velocities are torch tensors on the device, updated
in place; the caller's atom order.
"""
from dataclasses import dataclass, field
from typing import List

import numpy as np

KB_EV = 8.617333262e-5  # Boltzmann constant, eV/K


def kinetic_temperature(e_kin: float, n_atoms: int) -> float:
    """T (K) of n_atoms with zero total momentum and kinetic energy e_kin (eV)."""
    return 2.0 * e_kin / (max(3 * n_atoms - 3, 1) * KB_EV)


def berendsen_lambda(t_now: float, t_target: float, dt_chunk: float, tau: float) -> float:
    """The velocity scale of one coupling step (never below 0)."""
    return float(np.sqrt(max(0.0, 1.0 + (dt_chunk / tau) * (t_target / t_now - 1.0))))


@dataclass
class NvtTrace:
    temperatures: List[float] = field(default_factory=list)   # K, before each coupling
    e_pot: List[float] = field(default_factory=list)          # eV
    lambdas: List[float] = field(default_factory=list)


def nvt_berendsen(ctx, pos, vel, species, box, pbc, dt_ps: float, n_chunks: int, chunk: int,
                  t_target: float, tau_ps: float) -> NvtTrace:
    import torch
    n = pos.shape[0]
    ep = torch.zeros(1, dtype=torch.float64, device=pos.device)
    ek = torch.zeros(1, dtype=torch.float64, device=pos.device)
    tr = NvtTrace()
    for _ in range(n_chunks):
        ctx.md_step_dev(pos, vel, species, box, pbc, dt_ps, chunk, ep, ek)
        t_now = kinetic_temperature(ek.item(), n)
        lam = berendsen_lambda(t_now, t_target, chunk * dt_ps, tau_ps)
        vel.mul_(lam)
        tr.temperatures.append(t_now)
        tr.e_pot.append(ep.item())
        tr.lambdas.append(lam)
    return tr


EV_PER_A3_IN_BAR = 1.602176634e6  # 1 eV/A^3 = 1.602176634e-19 J / 1e-30 m^3 = 1.602e11 Pa


def pressure_bar(e_kin: float, virial_trace: float, volume: float) -> float:
    """Instantaneous pressure (bar) from the kinetic energy (eV), the trace of
    the virial W = -dE/d(strain) (eV) and the volume (A^3):
    P = (2 E_kin + tr W) / (3 V)."""
    return (2.0 * e_kin + virial_trace) / (3.0 * volume) * EV_PER_A3_IN_BAR


def berendsen_mu(p_now: float, p_target: float, dt_chunk: float, tau: float, compressibility: float) -> float:
    """Isotropic coordinate scale of one weak pressure coupling step:
    mu = (1 - (compressibility t / tau) (P0 - P))^(1/3) (Berendsen et al., 1984)."""
    return float((1.0 - compressibility * dt_chunk / tau * (p_target - p_now)) ** (1.0 / 3.0))


@dataclass
class NptTrace:
    temperatures: List[float] = field(default_factory=list)   # K, before each coupling
    pressures: List[float] = field(default_factory=list)      # bar, before each coupling
    volumes: List[float] = field(default_factory=list)        # A^3, after each coupling
    e_pot: List[float] = field(default_factory=list)
    lambdas: List[float] = field(default_factory=list)
    mus: List[float] = field(default_factory=list)


def npt_berendsen(ctx, pos, vel, species, box, pbc, dt_ps: float, n_chunks: int, chunk: int,
                  t_target: float, tau_t_ps: float, p_target_bar: float, tau_p_ps: float,
                  compressibility_per_bar: float) -> NptTrace:
    """Constant-pressure, constant-temperature MD by weak coupling (the
    pressure conditions of the MD cycle, Fig. 1): velocity-Verlet chunks on
    the GPU; after each chunk the pressure from the kinetic energy and the
    virial of the configuration (aenet_energy_forces_virial_dev), then the
    velocities scaled by the temperature coupling and the positions and the
    box edges by the isotropic pressure-coupling factor mu.  Periodic axes
    only are scaled.  `box` (numpy [3]) is updated in place."""
    import torch
    n = pos.shape[0]
    dev = pos.device
    ep = torch.zeros(1, dtype=torch.float64, device=dev)
    ek = torch.zeros(1, dtype=torch.float64, device=dev)
    W = torch.zeros(9, dtype=torch.float64, device=dev)
    per = np.asarray(pbc).reshape(3) != 0
    tr = NptTrace()
    for _ in range(n_chunks):
        ctx.md_step_dev(pos, vel, species, box, pbc, dt_ps, chunk, ep, ek)
        ctx.energy_forces_virial_dev(pos, species, box, pbc, None, None, W)
        e_kin = ek.item()
        vol = float(np.prod(box))
        p_now = pressure_bar(e_kin, float(W[0] + W[4] + W[8]), vol)
        t_now = kinetic_temperature(e_kin, n)
        lam = berendsen_lambda(t_now, t_target, chunk * dt_ps, tau_t_ps)
        mu = berendsen_mu(p_now, p_target_bar, chunk * dt_ps, tau_p_ps, compressibility_per_bar)
        vel.mul_(lam)
        scale = torch.tensor([mu if a else 1.0 for a in per], dtype=torch.float64, device=dev)
        pos.mul_(scale)
        box[per] *= mu
        tr.temperatures.append(t_now)
        tr.pressures.append(p_now)
        tr.volumes.append(float(np.prod(box)))
        tr.e_pot.append(ep.item())
        tr.lambdas.append(lam)
        tr.mus.append(mu)
    return tr
