"""ctypes wrapper of the FP64 CPU oracle (aenet_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use it to define the expected results of the ANN-potential
hot path (descriptors of Sec. II B, Eqs. 3-6; atomic networks of Sec. II A,
Eqs. 1-2; forces, MD and the training loss).  The GPU library never imports,
links or calls anything here, and this module imports nothing from the GPU
package.

Models are passed duck-typed: any object with the attributes n_species,
type_weight, radial_order, radial_cutoff, angular_order, angular_cutoff and
nets (each net with W, b, act, shift, scale, e_offset) works.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "aenet_oracle.c")
_LIB = os.path.join(_HERE, "libaenet_oracle.so")

ACT_LINEAR = 0
ACT_TANH = 1
KAPPA = 9648.533215665  # (eV/amu) in A^2/ps^2
KB_EV = 8.617333262e-5  # Boltzmann constant, eV/K

_codes = {0: "ok", -1: "invalid", -4: "overlap", -7: "nomem", -8: "capacity"}


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle error {code} ({_codes.get(code, '?')})")
        self.code = code


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C99, -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-fPIC", "-shared",
                               "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        L.orc_chebyshev.argtypes = [C.c_int, C.c_double, dp, dp]
        L.orc_chebyshev.restype = None
        L.orc_cutoff.argtypes = [C.c_double, C.c_double, dp, dp]
        L.orc_cutoff.restype = None
        L.orc_descriptor_dim.argtypes = [C.c_int, C.c_int, C.c_int]
        L.orc_net_eval.argtypes = [C.POINTER(_Net), dp, dp, dp]
        L.orc_neighbors.argtypes = [C.c_int, dp, dp, ip, C.c_double, C.c_int, ip, ip, ip]
        L.orc_descriptors.argtypes = [C.POINTER(_Model), C.c_int, dp, ip, dp, ip, dp]
        L.orc_energy_forces.argtypes = [C.POINTER(_Model), C.c_int, dp, ip, dp, ip, dp, dp, dp, dp]
        L.orc_energy_forces_virial.argtypes = [C.POINTER(_Model), C.c_int, dp, ip, dp, ip, dp, dp, dp, dp, dp]
        L.orc_forces_dense.argtypes = [C.POINTER(_Model), C.c_int, dp, ip, dp, ip, dp]
        L.orc_energy_forces_subset.argtypes = [C.POINTER(_Model), C.c_int, dp, ip, dp, ip, C.c_int, ip,
                                               dp, dp, dp]
        L.orc_md_vv.argtypes = [C.POINTER(_Model), C.c_int, dp, dp, ip, dp, dp, ip, C.c_double,
                                C.c_int, dp, dp, dp]
        L.orc_loss.argtypes = [C.POINTER(_Model), C.c_int, ip, dp, ip, dp, ip, dp, dp, C.c_double, C.c_int, dp]
        L.orc_loss_grad.argtypes = [C.POINTER(_Model), C.c_int, ip, dp, ip, dp, ip, dp, dp,
                                    C.c_double, C.c_int, dp, dp]
        _lib = L
    return _lib


class _Net(C.Structure):
    _fields_ = [("n_layers", C.c_int), ("widths", C.POINTER(C.c_int)), ("act", C.POINTER(C.c_int)),
                ("params", C.POINTER(C.c_double)), ("shift", C.POINTER(C.c_double)),
                ("scale", C.POINTER(C.c_double)), ("e_offset", C.c_double)]


class _Model(C.Structure):
    _fields_ = [("n_species", C.c_int), ("type_weight", C.POINTER(C.c_double)),
                ("radial_order", C.c_int), ("radial_cutoff", C.c_double),
                ("angular_order", C.c_int), ("angular_cutoff", C.c_double),
                ("nets", C.POINTER(_Net))]


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int)) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def flat_params(net) -> np.ndarray:
    """Parameters of one net in the oracle layout: W[0], b[0], W[1], b[1], ..."""
    parts = []
    for W, b in zip(net.W, net.b):
        parts.append(np.asarray(W, dtype=np.float64).ravel())
        parts.append(np.asarray(b, dtype=np.float64).ravel())
    return np.concatenate(parts)


class _Packed:
    """ctypes view of a model; keeps every numpy buffer alive."""

    def __init__(self, model, params_override=None):
        S = int(model.n_species)
        self.keep = []
        self.nets = (_Net * S)()
        off = 0
        for t, net in enumerate(model.nets):
            widths = _i32([np.asarray(net.W[0]).shape[1]] + [np.asarray(W).shape[0] for W in net.W])
            act = _i32(net.act)
            if params_override is not None:
                n = int(sum(np.asarray(W).size + np.asarray(b).size for W, b in zip(net.W, net.b)))
                params = _f64(params_override[off:off + n])
                off += n
            else:
                params = _f64(flat_params(net))
            shift = _f64(net.shift) if net.shift is not None else None
            scale = _f64(net.scale) if net.scale is not None else None
            self.keep += [widths, act, params, shift, scale]
            self.nets[t] = _Net(len(net.W), _ip(widths), _ip(act), _dp(params), _dp(shift),
                                _dp(scale), float(net.e_offset))
        tw = _f64(model.type_weight)
        self.keep.append(tw)
        self.model = _Model(S, _dp(tw), int(model.radial_order), float(model.radial_cutoff),
                            int(model.angular_order), float(model.angular_cutoff), self.nets)

    @property
    def ptr(self):
        return C.byref(self.model)


def _check(code):
    if code != 0:
        raise OracleError(code)


def _geom(pos, box, pbc):
    pos = _f64(pos).reshape(-1, 3)
    box = _f64(box).reshape(3)
    pbc = _i32(np.asarray(pbc, dtype=np.int32).reshape(3))
    return pos, box, pbc


def chebyshev(order: int, x: float):
    T = np.zeros(order + 1)
    dT = np.zeros(order + 1)
    lib().orc_chebyshev(order, float(x), _dp(T), _dp(dT))
    return T, dT


def cutoff(r: float, rc: float):
    fc = C.c_double()
    dfc = C.c_double()
    lib().orc_cutoff(float(r), float(rc), C.byref(fc), C.byref(dfc))
    return fc.value, dfc.value


def descriptor_dim(n_species, radial_order, angular_order) -> int:
    return lib().orc_descriptor_dim(n_species, radial_order, angular_order)


def net_eval(net, G):
    """(E, dE/dG) of one atomic network at descriptor G."""
    widths = _i32([np.asarray(net.W[0]).shape[1]] + [np.asarray(W).shape[0] for W in net.W])
    act = _i32(net.act)
    params = _f64(flat_params(net))
    shift = _f64(net.shift) if net.shift is not None else None
    scale = _f64(net.scale) if net.scale is not None else None
    cn = _Net(len(net.W), _ip(widths), _ip(act), _dp(params), _dp(shift), _dp(scale),
              float(net.e_offset))
    G = _f64(G)
    E = C.c_double()
    g = np.zeros_like(G)
    _check(lib().orc_net_eval(C.byref(cn), _dp(G), C.byref(E), _dp(g)))
    return E.value, g


def neighbors(pos, box, pbc, cutoff_radius, cap=None):
    """Brute-force neighbour lists: list over atoms of (j [k], shift [k,3])."""
    pos, box, pbc = _geom(pos, box, pbc)
    n = pos.shape[0]
    if cap is None:
        cap = 64
    while True:
        counts = np.zeros(n, dtype=np.int32)
        nj = np.zeros(n * cap, dtype=np.int32)
        ns = np.zeros(n * cap * 3, dtype=np.int32)
        code = lib().orc_neighbors(n, _dp(pos), _dp(box), _ip(pbc), float(cutoff_radius), cap,
                                   _ip(counts), _ip(nj), _ip(ns))
        if code == -8:
            cap = int(counts.max()) + 1
            continue
        _check(code)
        nj = nj.reshape(n, cap)
        ns = ns.reshape(n, cap, 3)
        return [(nj[i, :counts[i]].copy(), ns[i, :counts[i]].copy()) for i in range(n)]


def descriptors(model, pos, species, box, pbc):
    pos, box, pbc = _geom(pos, box, pbc)
    sp = _i32(species)
    pk = _Packed(model)
    D = descriptor_dim(model.n_species, model.radial_order, model.angular_order)
    G = np.zeros((pos.shape[0], D))
    _check(lib().orc_descriptors(pk.ptr, pos.shape[0], _dp(pos), _ip(sp), _dp(box), _ip(pbc), _dp(G)))
    return G


def energy_forces(model, pos, species, box, pbc, want_G=False):
    """(E_total, E_atom [n], F [n,3]) (+ G [n,D] if want_G)."""
    pos, box, pbc = _geom(pos, box, pbc)
    sp = _i32(species)
    pk = _Packed(model)
    n = pos.shape[0]
    D = descriptor_dim(model.n_species, model.radial_order, model.angular_order)
    E = C.c_double()
    Ea = np.zeros(n)
    F = np.zeros((n, 3))
    G = np.zeros((n, D)) if want_G else None
    _check(lib().orc_energy_forces(pk.ptr, n, _dp(pos), _ip(sp), _dp(box), _ip(pbc), C.byref(E),
                                   _dp(Ea), _dp(F), _dp(G)))
    if want_G:
        return E.value, Ea, F, G
    return E.value, Ea, F


def energy_forces_virial(model, pos, species, box, pbc):
    """(E_total, F [n,3], W [3,3]): the virial W_ab = -dE/d eps_ab under the
    homogeneous strain r -> (1 + eps) r, by the chain rule over every
    neighbour entry's gradient (the definition the strain derivative of the
    energy reduces to for a function of the entries' displacement vectors)."""
    pos, box, pbc = _geom(pos, box, pbc)
    sp = _i32(species)
    pk = _Packed(model)
    n = pos.shape[0]
    E = C.c_double()
    F = np.zeros((n, 3))
    W = np.zeros((3, 3))
    _check(lib().orc_energy_forces_virial(pk.ptr, n, _dp(pos), _ip(sp), _dp(box), _ip(pbc), C.byref(E),
                                          None, _dp(F), None, _dp(W)))
    return E.value, F, W


def energy_forces_subset(model, pos, species, box, pbc, sel):
    """(E_atom [k], F [k,3], G [k,D]) of the selected atoms only."""
    pos, box, pbc = _geom(pos, box, pbc)
    sp = _i32(species)
    sel = _i32(sel)
    pk = _Packed(model)
    D = descriptor_dim(model.n_species, model.radial_order, model.angular_order)
    E = np.zeros(sel.size)
    F = np.zeros((sel.size, 3))
    G = np.zeros((sel.size, D))
    _check(lib().orc_energy_forces_subset(pk.ptr, pos.shape[0], _dp(pos), _ip(sp), _dp(box), _ip(pbc),
                                          sel.size, _ip(sel), _dp(E), _dp(F), _dp(G)))
    return E, F, G


def _subset_worker(args):
    model, pos, species, box, pbc, sel = args
    build()
    return energy_forces_subset(model, pos, species, box, pbc, sel)


def energy_forces_subset_parallel(model, pos, species, box, pbc, sel, workers=None):
    """energy_forces_subset with the selected atoms split over worker
    processes (each runs the single-threaded oracle on its share); for sampled
    checks of large structures.  Spawned processes: nothing of the calling
    process (a GPU runtime, for instance) is inherited."""
    import concurrent.futures as cf
    import multiprocessing as mp
    sel = np.asarray(sel)
    workers = max(1, min(workers or 8, sel.size))
    parts = [p for p in np.array_split(sel, workers) if p.size]
    with cf.ProcessPoolExecutor(max_workers=len(parts), mp_context=mp.get_context("spawn")) as ex:
        out = list(ex.map(_subset_worker, [(model, pos, species, box, pbc, p) for p in parts]))
    return (np.concatenate([o[0] for o in out]), np.vstack([o[1] for o in out]),
            np.vstack([o[2] for o in out]))


def forces_dense(model, pos, species, box, pbc):
    pos, box, pbc = _geom(pos, box, pbc)
    sp = _i32(species)
    pk = _Packed(model)
    F = np.zeros((pos.shape[0], 3))
    _check(lib().orc_forces_dense(pk.ptr, pos.shape[0], _dp(pos), _ip(sp), _dp(box), _ip(pbc), _dp(F)))
    return F


def md_vv(model, pos, vel, species, masses, box, pbc, dt, n_steps):
    """Velocity Verlet; returns (pos, vel, e_pot, e_kin, F) of the final state."""
    pos, box, pbc = _geom(pos, box, pbc)
    pos = pos.copy()
    vel = _f64(vel).reshape(-1, 3).copy()
    sp = _i32(species)
    ms = _f64(masses)
    pk = _Packed(model)
    ep = C.c_double()
    ek = C.c_double()
    F = np.zeros_like(pos)
    _check(lib().orc_md_vv(pk.ptr, pos.shape[0], _dp(pos), _dp(vel), _ip(sp), _dp(ms), _dp(box),
                           _ip(pbc), float(dt), int(n_steps), C.byref(ep), C.byref(ek), _dp(F)))
    return pos, vel, ep.value, ek.value, F


def _batch_args(offsets, pos, species, boxes, pbc, e_ref, f_ref):
    return (_i32(offsets), _f64(pos).reshape(-1, 3), _i32(species), _f64(boxes).reshape(-1, 3),
            _i32(np.asarray(pbc, dtype=np.int32).reshape(3)), _f64(e_ref), _f64(f_ref).reshape(-1, 3))


LOSS_MEAN_PER_ATOM, LOSS_EQ7 = 0, 1


def loss(model, offsets, pos, species, boxes, pbc, e_ref, f_ref, lambda_f, params=None, form=LOSS_MEAN_PER_ATOM):
    off, pos, sp, boxes, pbc, e_ref, f_ref = _batch_args(offsets, pos, species, boxes, pbc, e_ref, f_ref)
    pk = _Packed(model, params)
    out = C.c_double()
    _check(lib().orc_loss(pk.ptr, len(off) - 1, _ip(off), _dp(pos), _ip(sp), _dp(boxes), _ip(pbc),
                          _dp(e_ref), _dp(f_ref), float(lambda_f), int(form), C.byref(out)))
    return out.value


def n_params(model) -> int:
    return int(sum(np.asarray(W).size + np.asarray(b).size for net in model.nets
                   for W, b in zip(net.W, net.b)))


def loss_grad(model, offsets, pos, species, boxes, pbc, e_ref, f_ref, lambda_f, params=None,
              form=LOSS_MEAN_PER_ATOM):
    off, pos, sp, boxes, pbc, e_ref, f_ref = _batch_args(offsets, pos, species, boxes, pbc, e_ref, f_ref)
    pk = _Packed(model, params)
    out = C.c_double()
    grad = np.zeros(n_params(model))
    _check(lib().orc_loss_grad(pk.ptr, len(off) - 1, _ip(off), _dp(pos), _ip(sp), _dp(boxes),
                               _ip(pbc), _dp(e_ref), _dp(f_ref), float(lambda_f), int(form), C.byref(out),
                               _dp(grad)))
    return out.value, grad


def all_params(model) -> np.ndarray:
    return np.concatenate([flat_params(net) for net in model.nets])
