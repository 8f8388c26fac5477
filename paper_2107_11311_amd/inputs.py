"""Seeded synthetic inputs shared by the GPU path, the oracle and the benchmark.

This module holds no arithmetic of the method itself (no descriptor, network,
force or integrator code): only random structures, random network weights and
random velocities, plus the plain data containers that describe a model.  Both
the oracle (through duck typing) and the GPU binding accept these containers.

Workload shapes follow the paper's systems (its data sets and trained
potentials are not available, so these stand in for them):
  * liquid water at 1 g/cm^3 with rigid-geometry H2O (O-H 0.96 A,
    H-O-H 104.5 deg), boxes of 64 to 333,334 molecules; the paper's default
    water network is 52-25-25-1 and its reduced one has a 20-dimensional
    descriptor (Sec. IV, model-complexity study);
  * an amorphous three-species Li/Si/O-like random packing standing in for the
    paper's amorphous LiSi.
Masses of H and O are the values of the paper's LAMMPS example (Sec. III).
Every generator takes an explicit seed (numpy PCG64).
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SEED_BASE = 20210723
MASS = {"H": 1.007825, "O": 15.999491, "Li": 6.941, "Si": 28.0855}
WATER_MOL_VOLUME = 18.01528 / 6.02214076e23 * 1e24  # A^3 per H2O at 1 g/cm^3
KAPPA = 9648.533215665  # (eV/amu) in A^2/ps^2
KB_EV = 8.617333262e-5  # eV/K
ACT_LINEAR, ACT_TANH = 0, 1
_GOLDEN = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tests", "golden")


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def seed_for(config: int, stream: int) -> int:
    return SEED_BASE + 100 * int(config) + int(stream)


# --------------------------------------------------------------------------
# Model containers
# --------------------------------------------------------------------------

@dataclass
class NetSpec:
    W: List[np.ndarray]            # W[l]: [out, in]
    b: List[np.ndarray]            # b[l]: [out]
    act: List[int]                 # per layer, ACT_TANH / ACT_LINEAR
    shift: Optional[np.ndarray] = None
    scale: Optional[np.ndarray] = None
    e_offset: float = 0.0

    @property
    def widths(self):
        return [self.W[0].shape[1]] + [w.shape[0] for w in self.W]

    def n_params(self) -> int:
        return int(sum(w.size + b.size for w, b in zip(self.W, self.b)))


@dataclass
class ModelSpec:
    n_species: int
    type_weight: np.ndarray
    masses: np.ndarray
    radial_order: int
    radial_cutoff: float
    angular_order: int
    angular_cutoff: float
    nets: List[NetSpec] = field(default_factory=list)
    species_names: List[str] = field(default_factory=list)

    @property
    def D(self) -> int:
        typed = self.radial_order + 1 + self.angular_order + 1
        return 2 * typed if self.n_species > 1 else typed

    def n_params(self) -> int:
        return sum(n.n_params() for n in self.nets)

    def flat_params(self) -> np.ndarray:
        return np.concatenate([np.concatenate([np.concatenate([w.ravel(), b.ravel()])
                                               for w, b in zip(n.W, n.b)]) for n in self.nets])

    def with_params(self, flat: np.ndarray) -> "ModelSpec":
        """Copy with all weights/biases replaced from the flat vector."""
        flat = np.asarray(flat, dtype=np.float64)
        nets = []
        off = 0
        for n in self.nets:
            W, b = [], []
            for w, bb in zip(n.W, n.b):
                W.append(flat[off:off + w.size].reshape(w.shape).copy()); off += w.size
                b.append(flat[off:off + bb.size].copy()); off += bb.size
            nets.append(NetSpec(W, b, list(n.act), n.shift, n.scale, n.e_offset))
        assert off == flat.size
        return ModelSpec(self.n_species, self.type_weight, self.masses, self.radial_order,
                         self.radial_cutoff, self.angular_order, self.angular_cutoff, nets,
                         list(self.species_names))


def default_type_weights(n_species: int) -> np.ndarray:
    """Centred integer species weights: (-1, +1) for two species, (-1, 0, +1) for three."""
    return np.arange(n_species, dtype=np.float64) - (n_species - 1) / 2.0


def xavier_net(widths, seed: int, act_hidden=ACT_TANH) -> NetSpec:
    """Glorot/Xavier-uniform weights, U(-0.1, 0.1) biases; one stream per layer."""
    W, b, act = [], [], []
    for l in range(len(widths) - 1):
        g = rng(seed + l)
        fan_in, fan_out = widths[l], widths[l + 1]
        lim = np.sqrt(6.0 / (fan_in + fan_out))
        W.append(g.uniform(-lim, lim, size=(fan_out, fan_in)))
        b.append(g.uniform(-0.1, 0.1, size=fan_out))
        act.append(act_hidden if l < len(widths) - 2 else ACT_LINEAR)
    return NetSpec(W, b, act)


# --------------------------------------------------------------------------
# Structures
# --------------------------------------------------------------------------

def rsa(n: int, box: float, dmin: float, seed: int) -> np.ndarray:
    """Random sequential addition of n points in a periodic cube: a uniform
    candidate is kept iff no kept point lies closer than dmin (minimum image).
    Candidates are drawn in batches; within a batch they are taken in draw order,
    so the result is an ordinary sequential RSA realisation of the seeded stream."""
    from scipy.spatial import cKDTree
    g = rng(seed)
    kept = np.zeros((0, 3))
    acc_rate = 1.0
    while kept.shape[0] < n:
        need = n - kept.shape[0]
        batch = int(min(max(256, 2.0 * need / max(acc_rate, 1e-3)), 2_000_000))
        cand = g.uniform(0.0, box, size=(batch, 3))
        cand = np.where(cand >= box, 0.0, cand)
        if kept.shape[0]:
            d, _ = cKDTree(kept, boxsize=box).query(cand, k=1, distance_upper_bound=dmin)
            cand = cand[~(d < dmin)]
        if cand.shape[0]:
            pairs = cKDTree(cand, boxsize=box).query_pairs(dmin, output_type="ndarray")
            keep = np.ones(cand.shape[0], dtype=bool)
            if pairs.size:
                pairs = np.sort(pairs, axis=1)
                order = np.lexsort((pairs[:, 0], pairs[:, 1]))
                pairs = pairs[order]
                # sequential: b is dropped if it conflicts with a kept earlier a
                for a, b in pairs:
                    if keep[a] and keep[b]:
                        keep[b] = False
            cand = cand[keep]
        acc_rate = max(cand.shape[0] / batch, 1e-4)
        kept = np.vstack([kept, cand[:need]])
    return kept


def random_rotations(n: int, g: np.random.Generator) -> np.ndarray:
    """n uniformly distributed rotation matrices (normalised Gaussian quaternions)."""
    q = g.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z); R[:, 0, 1] = 2 * (x * y - z * w); R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w); R[:, 1, 1] = 1 - 2 * (x * x + z * z); R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w); R[:, 2, 1] = 2 * (y * z + x * w); R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def wrap(pos: np.ndarray, box) -> np.ndarray:
    box = np.asarray(box, dtype=np.float64).reshape(1, 3)
    w = pos - box * np.floor(pos / box)
    return np.where(w >= box, w - box, w)


def water_box_length(n_mol: int) -> float:
    return float((n_mol * WATER_MOL_VOLUME) ** (1.0 / 3.0))


@dataclass
class System:
    pos: np.ndarray        # [n,3] A, wrapped into [0, L)
    species: np.ndarray    # [n] int32
    box: np.ndarray        # [3] A
    pbc: np.ndarray        # [3] uint8


def water_box(n_mol: int, seed: int, box: Optional[float] = None, d_oo: float = 2.5,
              r_oh: float = 0.96, angle_deg: float = 104.5) -> System:
    """n_mol rigid H2O, O by RSA (min O-O image distance d_oo), uniform random
    orientations.  Atom order per molecule: O, H, H.  Species: H = 0, O = 1."""
    L = water_box_length(n_mol) if box is None else float(box)
    O = rsa(n_mol, L, d_oo, seed)
    half = np.deg2rad(angle_deg) / 2.0
    local = np.array([[r_oh * np.sin(half), 0.0, r_oh * np.cos(half)],
                      [-r_oh * np.sin(half), 0.0, r_oh * np.cos(half)]])
    R = random_rotations(n_mol, rng(seed + 1))
    H = O[:, None, :] + np.einsum("nij,kj->nki", R, local)
    pos = np.empty((n_mol, 3, 3))
    pos[:, 0] = O
    pos[:, 1:] = H
    pos = wrap(pos.reshape(-1, 3), [L, L, L])
    species = np.tile(np.array([1, 0, 0], dtype=np.int32), n_mol)
    return System(pos, species, np.array([L, L, L]), np.ones(3, dtype=np.uint8))


def amorphous_box(n: int, counts, box: float, seed: int, dmin: float = 1.6) -> System:
    """n sites by RSA (min pair distance dmin), species by a random permutation
    with the given per-species counts."""
    assert sum(counts) == n
    pos = rsa(n, box, dmin, seed)
    sp = np.concatenate([np.full(c, t, dtype=np.int32) for t, c in enumerate(counts)])
    sp = rng(seed + 1).permutation(sp).astype(np.int32)
    return System(pos, sp, np.array([box, box, box], dtype=np.float64), np.ones(3, dtype=np.uint8))


def maxwell_boltzmann(masses_per_atom: np.ndarray, T: float, seed: int) -> np.ndarray:
    """Velocities (A/ps): Gaussian per component with variance kB T kappa / m,
    zero centre-of-mass momentum, rescaled to exactly T with 3N-3 degrees of freedom."""
    m = np.asarray(masses_per_atom, dtype=np.float64)
    g = rng(seed)
    v = g.normal(size=(m.size, 3)) * np.sqrt(KB_EV * T * KAPPA / m)[:, None]
    v -= (m[:, None] * v).sum(0) / m.sum()
    ke = 0.5 * (m[:, None] * v * v).sum() / KAPPA
    dof = 3 * m.size - 3
    Tcur = 2.0 * ke / (dof * KB_EV)
    return v * np.sqrt(T / Tcur)


# --------------------------------------------------------------------------
# The workloads
# --------------------------------------------------------------------------

WATER = dict(species_names=["H", "O"], masses=[MASS["H"], MASS["O"]])
LISIO = dict(species_names=["Li", "Si", "O"], masses=[MASS["Li"], MASS["Si"], MASS["O"]])

CONFIGS = {
    # 64 H2O, single energy+forces call
    "water64": dict(cfg=0, kind="water", n_mol=64, radial=(10, 6.0), angular=(4, 4.0),
                    hidden=(20, 20), skin=0.0, **WATER),
    # 4096 H2O, 1000 NVE steps of 0.25 fs at 300 K
    "water4096": dict(cfg=1, kind="water", n_mol=4096, radial=(16, 6.5), angular=(8, 4.0),
                      hidden=(25, 25), skin=0.5, dt_fs=0.25, steps=1000, T=300.0, **WATER),
    # 120,000-site amorphous Li/Si/O 2:1:3, 200 steps of 1 fs
    "lisio120k": dict(cfg=2, kind="amorphous", n=120000, counts=(40000, 20000, 60000),
                      box=107.575, radial=(18, 8.0), angular=(6, 6.5), hidden=(40, 40), skin=0.5,
                      dt_fs=1.0, steps=200, T=300.0, **LISIO),
    # 256 water boxes of 64..512 H2O for the loss gradient (network of water4096)
    "waterbatch256": dict(cfg=3, kind="water_batch", n_boxes=256, radial=(16, 6.5),
                          angular=(8, 4.0), hidden=(25, 25), skin=0.0, **WATER),
    # distilled student: orders 6 / 2 (D = 20), 20-16-16-1; 333,334 H2O MD
    "student": dict(cfg=4, kind="water", n_mol=333334, radial=(6, 6.5), angular=(2, 4.0),
                    hidden=(16, 16), skin=0.5, dt_fs=0.25, steps=500, T=300.0, **WATER),
}


def batch_sizes(n_boxes: int = 256):
    """Molecule counts 64 + round(448 k / 255), k = 0..255 (64..512 H2O)."""
    return [64 + int(np.floor(448.0 * k / (n_boxes - 1) + 0.5)) for k in range(n_boxes)]


def make_system(name: str, seed_offset: int = 0) -> System:
    c = CONFIGS[name]
    if c["kind"] == "water":
        return water_box(c["n_mol"], seed_for(c["cfg"], 0) + seed_offset)
    if c["kind"] == "amorphous":
        return amorphous_box(c["n"], c["counts"], c["box"], seed_for(c["cfg"], 0) + seed_offset)
    raise ValueError(name)


def make_batch(name: str = "waterbatch256", n_boxes: Optional[int] = None):
    """List of water Systems with the uneven sizes of the batch workload."""
    c = CONFIGS[name]
    sizes = batch_sizes(c["n_boxes"])
    if n_boxes is not None:
        sizes = sizes[:n_boxes]
    return [water_box(nm, seed_for(c["cfg"], 0) + 7 * k) for k, nm in enumerate(sizes)]


def raw_model(name: str, net_seed_offset: int = 0, type_weight=None) -> ModelSpec:
    """Model of a workload with seeded Xavier weights and no input normalisation."""
    c = CONFIGS[name]
    S = len(c["species_names"])
    nr, rr = c["radial"]
    na, ra = c["angular"]
    tw = default_type_weights(S) if type_weight is None else np.asarray(type_weight, dtype=np.float64)
    typed = nr + 1 + na + 1
    D = 2 * typed if S > 1 else typed
    widths = [D, *c["hidden"], 1]
    nets = [xavier_net(widths, seed_for(c["cfg"], 10 + 10 * t) + net_seed_offset) for t in range(S)]
    return ModelSpec(S, tw, np.asarray(c["masses"], dtype=np.float64), nr, rr, na, ra, nets,
                     list(c["species_names"]))


def apply_normalisation(model: ModelSpec, norm: dict) -> ModelSpec:
    """Attach per-species input shift/scale and the output-layer scale factor
    (stored model files)."""
    nets = []
    for t, n in enumerate(model.nets):
        W = [w.copy() for w in n.W]
        W[-1] = W[-1] * float(norm["out_scale"])
        nets.append(NetSpec(W, [b.copy() for b in n.b], list(n.act),
                            np.asarray(norm["shift"][t], dtype=np.float64),
                            np.asarray(norm["scale"][t], dtype=np.float64), n.e_offset))
    return ModelSpec(model.n_species, model.type_weight, model.masses, model.radial_order,
                     model.radial_cutoff, model.angular_order, model.angular_cutoff, nets,
                     list(model.species_names))


def sub_network(model: ModelSpec, radial_order: int, angular_order: int, hidden) -> ModelSpec:
    """A copy of a model whose networks keep only a smaller network inside
    them: the first-layer weights of descriptor components up to the given
    orders (the components of a descriptor with those orders and the same
    cutoffs) and the first hidden[l] units of each hidden layer; every other
    weight is set to zero (biases of dropped units too).  Its energy is then
    exactly a network of the smaller shape on the smaller descriptor."""
    NR, NA = model.radial_order, model.angular_order
    T1, T2 = NR + 1, NR + NA + 2
    keep = [a for a in range(NR + 1) if a <= radial_order] + [T1 + a for a in range(NA + 1) if a <= angular_order]
    if model.n_species > 1:
        keep = keep + [T2 + k for k in keep]
    cols = np.zeros(model.D, dtype=bool)
    cols[keep] = True
    nets = []
    for n in model.nets:
        W = [w.copy() for w in n.W]
        b = [x.copy() for x in n.b]
        W[0][:, ~cols] = 0.0
        for l, h in enumerate(hidden):
            W[l][h:, :] = 0.0
            b[l][h:] = 0.0
            W[l + 1][:, h:] = 0.0
        nets.append(NetSpec(W, b, list(n.act), n.shift, n.scale, n.e_offset))
    return ModelSpec(model.n_species, model.type_weight, model.masses, model.radial_order, model.radial_cutoff,
                     model.angular_order, model.angular_cutoff, nets, list(model.species_names))


def model_file(tag: str) -> str:
    return os.path.join(_GOLDEN, f"model_{tag}.json")


def load_model(tag: str) -> ModelSpec:
    """The normalised model of a workload: seeded weights + the stored
    normalisation file (written once by tests/golden/make_models.py)."""
    with open(model_file(tag)) as f:
        norm = json.load(f)
    m = raw_model(norm["config"], int(norm.get("net_seed_offset", 0)))
    sub = norm.get("sub_network")
    if sub:
        m = sub_network(m, sub["radial_order"], sub["angular_order"], sub["hidden"])
    return apply_normalisation(m, norm)
