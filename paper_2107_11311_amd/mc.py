"""Energy-only Metropolis Monte Carlo with the ANN potential (the paper's
sampling through TINKER includes Monte Carlo, Sec. III; Monte Carlo needs
only energies, Fig. 1 with the propagation step replaced by a trial move and
its acceptance test).

Each trial displaces the configuration by a given move (numpy [n, 3]; a
single-atom move is one non-zero row), evaluates the energy on the GPU with
the force pass skipped (aenet_energy_forces with no force or per-atom
output), and accepts with probability min(1, exp(-(E_trial - E) / k_B T)).
The random numbers are inputs: the moves and one uniform number in [0, 1)
per trial, so a run is reproducible and can be replayed against any other
energy function.
"""
from dataclasses import dataclass, field
from typing import List

import numpy as np

KB_EV = 8.617333262e-5  # Boltzmann constant, eV/K


@dataclass
class McTrace:
    accepted: List[bool] = field(default_factory=list)
    energies: List[float] = field(default_factory=list)   # energy after each trial (eV)

    @property
    def acceptance(self) -> float:
        return float(np.mean(self.accepted)) if self.accepted else 0.0


def metropolis(energy, pos, temperature: float, moves, uniforms, wrap_box=None, pbc=(1, 1, 1)):
    """Runs len(moves) trials from pos (not modified).  energy(pos) -> eV.
    Positions on periodic axes are wrapped into [0, L) after a move when
    wrap_box is given.  Returns (final positions, McTrace)."""
    beta = 1.0 / (KB_EV * temperature)
    x = np.array(pos, dtype=np.float64, copy=True)
    e = energy(x)
    tr = McTrace()
    per = np.asarray(pbc).reshape(3) != 0
    for d, u in zip(moves, uniforms):
        y = x + d
        if wrap_box is not None:
            L = np.asarray(wrap_box, dtype=np.float64)
            y[:, per] -= L[per] * np.floor(y[:, per] / L[per])
        ey = energy(y)
        ok = bool(u < np.exp(-beta * (ey - e))) if ey > e else True
        if ok:
            x, e = y, ey
        tr.accepted.append(ok)
        tr.energies.append(e)
    return x, tr


def gpu_energy(ctx, species, box, pbc):
    """energy(pos) for metropolis(): the library's energy-only evaluation."""
    return lambda p: ctx.energy(p, species, box, pbc)
