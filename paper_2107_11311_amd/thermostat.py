"""Constant-temperature MD by weak coupling to a heat bath (the NVT runs of
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
