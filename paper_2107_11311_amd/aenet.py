"""Python binding of the GPU library (include/aenet_gpu.h) through ctypes.

Argument marshalling only: every step of the hot path runs in the HIP
library.  Host-pointer calls take numpy arrays; the *_dev calls take torch
tensors on the GPU (PyTorch is used only for device memory and streams).
If the library is not built, load() raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaenet_gpu.so")

AENET_OK, AENET_E_INVALID, AENET_E_SPECIES, AENET_E_BOX = 0, -1, -2, -3
AENET_E_OVERLAP, AENET_E_NONFINITE, AENET_E_DEVICE, AENET_E_OOM = -4, -5, -6, -7
AENET_FP64, AENET_FP32, AENET_BF16 = 0, 1, 2
AENET_LOSS_MEAN_PER_ATOM, AENET_LOSS_EQ7 = 0, 1
ANGULAR_METHODS = {"auto": 0, "pairs": 1, "factorised": 2}
PRECISIONS = {"fp64": AENET_FP64, "fp32": AENET_FP32, "bf16": AENET_BF16}
STATUS_NAMES = {0: "AENET_OK", -1: "AENET_E_INVALID", -2: "AENET_E_SPECIES", -3: "AENET_E_BOX",
                -4: "AENET_E_OVERLAP", -5: "AENET_E_NONFINITE", -6: "AENET_E_DEVICE", -7: "AENET_E_OOM"}

# every entry point declared in include/aenet_gpu.h
EXPORTS = ["aenet_setup", "aenet_destroy", "aenet_last_error", "aenet_descriptor_dim", "aenet_n_params",
           "aenet_get_params", "aenet_set_params", "aenet_supported_orders", "aenet_energy_forces",
           "aenet_energy_forces_virial", "aenet_energy_forces_virial_dev", "aenet_energy_forces_dev", "aenet_energy_forces_noalloc",
           "aenet_energy_forces_batch_dev", "aenet_descriptors",
           "aenet_md_step", "aenet_md_step_dev", "aenet_loss_grad_dev", "aenet_loss_grad", "aenet_set_loss_form",
           "aenet_set_params_dev", "aenet_adam_step_dev", "aenet_rms_diff_dev", "aenet_get_stats",
           "aenet_set_rebuild_every", "aenet_set_capacity", "aenet_set_fused", "aenet_set_angular_method", "aenet_set_profiling", "aenet_get_kernel_times"]
KERNEL_CLASSES = ["neighbor", "desc_fwd", "network", "desc_bwd", "force_gather", "integrate", "fwd_network"]


class AenetError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class _Net(C.Structure):
    _fields_ = [("n_layers", C.c_int), ("widths", C.POINTER(C.c_int)), ("act", C.POINTER(C.c_int)),
                ("W", C.POINTER(C.POINTER(C.c_double))), ("b", C.POINTER(C.POINTER(C.c_double))),
                ("in_shift", C.POINTER(C.c_double)), ("in_scale", C.POINTER(C.c_double)),
                ("e_offset", C.c_double)]


class _Model(C.Structure):
    _fields_ = [("n_species", C.c_int), ("mass_amu", C.POINTER(C.c_double)),
                ("type_weight", C.POINTER(C.c_double)), ("radial_order", C.c_int),
                ("radial_cutoff", C.c_double), ("angular_order", C.c_int),
                ("angular_cutoff", C.c_double), ("nets", C.POINTER(_Net)), ("precision", C.c_int),
                ("skin", C.c_double), ("device", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("n_rebuilds", C.c_int64), ("n_capacity_retries", C.c_int64), ("row_capacity", C.c_int),
                ("ang_capacity", C.c_int), ("max_neighbors", C.c_int), ("max_angular", C.c_int),
                ("rebuild_every", C.c_int), ("deterministic", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_u8p = C.POINTER(C.c_uint8)
_i64p = C.POINTER(C.c_int64)
_vp = C.c_void_p


def load(path: str = LIB_PATH):
    """Loads the HIP library (built by __graft_entry__.build / build_lib.build)."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build the HIP library first (python __graft_entry__.py)")
    # PyTorch ships its own HIP runtime; it only starts if it initialises the
    # device before the library's runtime does, so let it go first when present.
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()
    except ImportError:
        pass
    L = C.CDLL(path)
    ctxp = C.c_void_p
    L.aenet_setup.argtypes = [C.POINTER(_Model), C.POINTER(ctxp)]
    L.aenet_destroy.argtypes = [ctxp]
    L.aenet_destroy.restype = None
    L.aenet_last_error.argtypes = [ctxp]
    L.aenet_last_error.restype = C.c_char_p
    L.aenet_descriptor_dim.argtypes = [ctxp]
    L.aenet_n_params.argtypes = [ctxp]
    L.aenet_n_params.restype = C.c_int64
    L.aenet_get_params.argtypes = [ctxp, _dp]
    L.aenet_set_params.argtypes = [ctxp, _dp]
    L.aenet_supported_orders.argtypes = [_ip, C.c_int]
    L.aenet_energy_forces.argtypes = [ctxp, C.c_int64, _dp, _ip, _dp, _u8p, _dp, _dp, _dp]
    L.aenet_energy_forces_virial.argtypes = [ctxp, C.c_int64, _dp, _ip, _dp, _u8p, _dp, _dp, _dp]
    L.aenet_energy_forces_virial_dev.argtypes = [ctxp, C.c_int64, _vp, _ip, _dp, _u8p, _vp, _vp, _vp, _vp]
    L.aenet_energy_forces_dev.argtypes = [ctxp, C.c_int64, _vp, _ip, _dp, _u8p, _vp, _vp, _vp, _vp]
    L.aenet_energy_forces_noalloc.argtypes = [ctxp, C.c_int64, _vp, _ip, _dp, _u8p, _vp, _vp, _vp, _vp]
    L.aenet_energy_forces_batch_dev.argtypes = [ctxp, C.c_int, _i64p, _vp, _ip, _dp, _u8p, _vp, _vp,
                                                _vp, _vp]
    L.aenet_descriptors.argtypes = [ctxp, C.c_int64, _dp, _ip, _dp, _u8p, _dp]
    L.aenet_md_step.argtypes = [ctxp, C.c_int64, _dp, _dp, _ip, _dp, _u8p, C.c_double, C.c_int, _dp,
                                _dp, _dp]
    L.aenet_md_step_dev.argtypes = [ctxp, C.c_int64, _vp, _vp, _ip, _dp, _u8p, C.c_double, C.c_int,
                                    _vp, _vp, _vp, _vp]
    L.aenet_loss_grad_dev.argtypes = [ctxp, C.c_int, _i64p, _vp, _ip, _dp, _u8p, _vp, _vp, C.c_double,
                                      _vp, _vp, _vp]
    L.aenet_loss_grad.argtypes = [ctxp, C.c_int, _i64p, _dp, _ip, _dp, _u8p, _dp, _dp, C.c_double, _dp, _dp]
    L.aenet_set_loss_form.argtypes = [ctxp, C.c_int]
    L.aenet_set_params_dev.argtypes = [ctxp, _vp, _vp]
    L.aenet_rms_diff_dev.argtypes = [ctxp, C.c_int64, _vp, _vp, _vp, _vp]
    L.aenet_adam_step_dev.argtypes = [C.c_int64, _vp, _vp, _vp, _vp, C.c_double, C.c_double, C.c_double,
                                      C.c_double, C.c_int64, _vp]
    L.aenet_get_stats.argtypes = [ctxp, C.POINTER(Stats)]
    L.aenet_set_rebuild_every.argtypes = [ctxp, C.c_int]
    L.aenet_set_capacity.argtypes = [ctxp, C.c_int, C.c_int]
    L.aenet_set_fused.argtypes = [ctxp, C.c_int]
    L.aenet_set_angular_method.argtypes = [ctxp, C.c_int]
    L.aenet_set_profiling.argtypes = [ctxp, C.c_int]
    L.aenet_get_kernel_times.argtypes = [ctxp, _dp, _i64p]
    for name in EXPORTS:
        if name not in ("aenet_destroy", "aenet_last_error", "aenet_descriptor_dim", "aenet_n_params",
                        "aenet_supported_orders"):
            getattr(L, name).restype = C.c_int
    L.aenet_descriptor_dim.restype = C.c_int
    L.aenet_supported_orders.restype = C.c_int
    if path == LIB_PATH:
        _lib = L
    return L


def adam_step_dev(params, grad, m, v, lr, beta1=0.9, beta2=0.999, eps=1e-8, step=1, stream=None):
    """aenet_adam_step_dev: one Adam update of float64 device tensors in place."""
    L = load()
    n = int(params.numel())
    code = L.aenet_adam_step_dev(n, _dev(params), _dev(grad), _dev(m), _dev(v), float(lr), float(beta1),
                                 float(beta2), float(eps), int(step), _stream(stream))
    if code != AENET_OK:
        raise AenetError(code, "aenet_adam_step_dev")


def supported_orders():
    L = load()
    buf = (C.c_int32 * 128)()
    k = L.aenet_supported_orders(buf, 64)
    return [(buf[2 * i], buf[2 * i + 1]) for i in range(k)]


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _ptr(a, t=_dp):
    return a.ctypes.data_as(t) if a is not None else None


def _dev(t):
    """Device pointer of a torch tensor (None -> NULL)."""
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(int(stream))


def _box(box, pbc):
    box = _f64(np.broadcast_to(np.asarray(box, dtype=np.float64), (3,)))
    pbc = np.ascontiguousarray(np.asarray(pbc if pbc is not None else (1, 1, 1)).reshape(3) != 0,
                               dtype=np.uint8)
    return box, pbc


class Context:
    """An aenet_ctx: one model on one GPU (the calls of include/aenet_gpu.h)."""

    def __init__(self, model, precision="fp64", skin: float = 0.0, device: int = 0):
        L = load()
        self.model = model
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        keep = []
        S = model.n_species
        nets = (_Net * S)()
        for t, net in enumerate(model.nets):
            widths = _i32([net.W[0].shape[1]] + [w.shape[0] for w in net.W])
            act = _i32(net.act)
            Ws = [_f64(w) for w in net.W]
            bs = [_f64(b) for b in net.b]
            Wp = (_dp * len(Ws))(*[_ptr(w) for w in Ws])
            bp = (_dp * len(bs))(*[_ptr(b) for b in bs])
            sh = _f64(net.shift) if net.shift is not None else None
            sc = _f64(net.scale) if net.scale is not None else None
            keep += [widths, act, Ws, bs, Wp, bp, sh, sc]
            nets[t] = _Net(len(net.W), _ptr(widths, _ip), _ptr(act, _ip), Wp, bp, _ptr(sh), _ptr(sc),
                           float(net.e_offset))
        masses = _f64(model.masses) if getattr(model, "masses", None) is not None else None
        tw = _f64(model.type_weight)
        keep += [masses, tw]
        m = _Model(S, _ptr(masses), _ptr(tw), int(model.radial_order), float(model.radial_cutoff),
                   int(model.angular_order), float(model.angular_cutoff), nets, self.precision,
                   float(skin), int(device))
        h = C.c_void_p()
        code = L.aenet_setup(C.byref(m), C.byref(h))
        if code != AENET_OK:
            raise AenetError(code, L.aenet_last_error(None).decode())
        self._h = h
        self._lib = L
        self.D = L.aenet_descriptor_dim(h)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.aenet_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, code):
        if code != AENET_OK:
            raise AenetError(code, self._lib.aenet_last_error(self._h).decode())

    # -------------------------------------------------------------- parameters
    def n_params(self) -> int:
        return int(self._lib.aenet_n_params(self._h))

    def get_params(self) -> np.ndarray:
        p = np.zeros(self.n_params())
        self._check(self._lib.aenet_get_params(self._h, _ptr(p)))
        return p

    def set_params(self, p) -> None:
        p = _f64(p)
        assert p.size == self.n_params()
        self._check(self._lib.aenet_set_params(self._h, _ptr(p)))

    def set_params_dev(self, p, stream=None) -> None:
        """aenet_set_params_dev: parameters from a float64 device tensor."""
        assert p.numel() == self.n_params() and p.is_contiguous()
        self._check(self._lib.aenet_set_params_dev(self._h, _dev(p), _stream(stream)))

    def rms_diff_dev(self, a, b, out, stream=None) -> None:
        """aenet_rms_diff_dev: out[0] = sqrt(mean((a - b)^2)) of float64 device tensors."""
        assert a.numel() == b.numel() and a.is_contiguous() and b.is_contiguous()
        self._check(self._lib.aenet_rms_diff_dev(self._h, int(a.numel()), _dev(a), _dev(b), _dev(out),
                                                 _stream(stream)))

    def set_loss_form(self, form: int) -> None:
        """AENET_LOSS_MEAN_PER_ATOM (default) or AENET_LOSS_EQ7 for the loss-gradient calls."""
        self._check(self._lib.aenet_set_loss_form(self._h, int(form)))

    def stats(self) -> dict:
        s = Stats()
        self._check(self._lib.aenet_get_stats(self._h, C.byref(s)))
        return s.as_dict()

    def set_rebuild_every(self, k: int) -> None:
        self._check(self._lib.aenet_set_rebuild_every(self._h, int(k)))

    def set_fused(self, on: bool) -> None:
        """Descriptor forward pass and networks in one kernel (default) or two."""
        self._check(self._lib.aenet_set_fused(self._h, 1 if on else 0))

    def set_angular_method(self, method: str) -> None:
        """'auto', 'pairs' (Eq. 6 as a pair sum) or 'factorised' (addition theorem)."""
        self._check(self._lib.aenet_set_angular_method(self._h, ANGULAR_METHODS[method]))

    def set_capacity(self, row: int, ang: int) -> None:
        """Starting neighbour-row capacities (0, 0: estimate from the density)."""
        self._check(self._lib.aenet_set_capacity(self._h, int(row), int(ang)))

    def set_profiling(self, on: bool) -> None:
        self._check(self._lib.aenet_set_profiling(self._h, 1 if on else 0))

    def kernel_times(self) -> dict:
        """{class: (total ms, launches)} since the last call (HIP events on the launch stream)."""
        ms = np.zeros(len(KERNEL_CLASSES))
        nl = np.zeros(len(KERNEL_CLASSES), dtype=np.int64)
        self._check(self._lib.aenet_get_kernel_times(self._h, _ptr(ms), _ptr(nl, _i64p)))
        return {k: (float(ms[i]), int(nl[i])) for i, k in enumerate(KERNEL_CLASSES)}

    # -------------------------------------------------------------- host-pointer calls
    def energy_forces(self, pos, species, box, pbc=(1, 1, 1)):
        """aenet_energy_forces: (E_total, E_atom [n], F [n,3]) from host arrays."""
        pos = _f64(pos).reshape(-1, 3)
        sp = _i32(species)
        box, pbc = _box(box, pbc)
        n = pos.shape[0]
        e = C.c_double()
        ea = np.zeros(n)
        F = np.zeros((n, 3))
        self._check(self._lib.aenet_energy_forces(self._h, n, _ptr(pos), _ptr(sp, _ip), _ptr(box),
                                                  _ptr(pbc, _u8p), C.byref(e), _ptr(ea), _ptr(F)))
        return e.value, ea, F

    def energy(self, pos, species, box, pbc=(1, 1, 1)) -> float:
        """aenet_energy_forces with no per-atom or force output: the force
        pass is skipped (energy-only evaluation, e.g. for Monte Carlo)."""
        pos = _f64(pos).reshape(-1, 3)
        sp = _i32(species)
        box, pbc = _box(box, pbc)
        e = C.c_double()
        self._check(self._lib.aenet_energy_forces(self._h, pos.shape[0], _ptr(pos), _ptr(sp, _ip), _ptr(box),
                                                  _ptr(pbc, _u8p), C.byref(e), None, None))
        return e.value

    def energy_forces_virial(self, pos, species, box, pbc=(1, 1, 1)):
        """aenet_energy_forces_virial: (E_total, F [n,3], W [3,3]) from host arrays."""
        pos = _f64(pos).reshape(-1, 3)
        sp = _i32(species)
        box, pbc = _box(box, pbc)
        n = pos.shape[0]
        e = C.c_double()
        F = np.zeros((n, 3))
        W = np.zeros((3, 3))
        self._check(self._lib.aenet_energy_forces_virial(self._h, n, _ptr(pos), _ptr(sp, _ip), _ptr(box),
                                                         _ptr(pbc, _u8p), C.byref(e), _ptr(F), _ptr(W)))
        return e.value, F, W

    def descriptors(self, pos, species, box, pbc=(1, 1, 1)):
        pos = _f64(pos).reshape(-1, 3)
        sp = _i32(species)
        box, pbc = _box(box, pbc)
        G = np.zeros((pos.shape[0], self.D))
        self._check(self._lib.aenet_descriptors(self._h, pos.shape[0], _ptr(pos), _ptr(sp, _ip), _ptr(box),
                                                _ptr(pbc, _u8p), _ptr(G)))
        return G

    def md_step(self, pos, vel, species, box, pbc, dt_ps: float, n_steps: int):
        """aenet_md_step: returns (pos, vel, e_pot, e_kin, F) after n_steps."""
        pos = _f64(pos).reshape(-1, 3).copy()
        vel = _f64(vel).reshape(-1, 3).copy()
        sp = _i32(species)
        box, pbc = _box(box, pbc)
        ep, ek = C.c_double(), C.c_double()
        F = np.zeros_like(pos)
        self._check(self._lib.aenet_md_step(self._h, pos.shape[0], _ptr(pos), _ptr(vel), _ptr(sp, _ip),
                                            _ptr(box), _ptr(pbc, _u8p), float(dt_ps), int(n_steps),
                                            C.byref(ep), C.byref(ek), _ptr(F)))
        return pos, vel, ep.value, ek.value, F

    def loss_grad(self, offsets, pos, species, boxes, pbc, e_ref, f_ref, lambda_f):
        """aenet_loss_grad: (loss, grad [n_params]) from host arrays."""
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        pos = _f64(pos).reshape(-1, 3)
        sp = _i32(species)
        bx = _f64(boxes).reshape(-1, 3)
        _, pbc = _box(bx[0], pbc)
        er = _f64(e_ref)
        fr = _f64(f_ref).reshape(-1, 3)
        loss = C.c_double()
        grad = np.zeros(self.n_params())
        self._check(self._lib.aenet_loss_grad(self._h, len(off) - 1, _ptr(off, _i64p), _ptr(pos), _ptr(sp, _ip),
                                              _ptr(bx), _ptr(pbc, _u8p), _ptr(er), _ptr(fr), float(lambda_f),
                                              C.byref(loss), _ptr(grad)))
        return loss.value, grad

    # -------------------------------------------------------------- device calls (torch tensors)
    def energy_forces_dev(self, pos, species, box, pbc=(1, 1, 1), e_total=None, e_atom=None,
                          forces=None, stream=None):
        sp = _i32(species)
        box, pbc = _box(box, pbc)
        self._check(self._lib.aenet_energy_forces_dev(self._h, int(pos.shape[0]), _dev(pos), _ptr(sp, _ip),
                                                      _ptr(box), _ptr(pbc, _u8p), _dev(e_total), _dev(e_atom),
                                                      _dev(forces), _stream(stream)))

    def energy_forces_virial_dev(self, pos, species, box, pbc=(1, 1, 1), e_total=None, forces=None,
                                 virial=None, stream=None):
        """aenet_energy_forces_virial_dev: virial (device [9] or [3, 3]) required."""
        sp = _i32(species)
        box, pbc = _box(box, pbc)
        self._check(self._lib.aenet_energy_forces_virial_dev(self._h, int(pos.shape[0]), _dev(pos), _ptr(sp, _ip),
                                                             _ptr(box), _ptr(pbc, _u8p), _dev(e_total),
                                                             _dev(forces), _dev(virial), _stream(stream)))

    def energy_forces_noalloc(self, pos, species, box, pbc=(1, 1, 1), e_total=None, e_atom=None,
                              forces=None, stream=None):
        """aenet_energy_forces_noalloc: as energy_forces_dev, temporaries in the
        library's fixed per-GPU workspace (no device allocation in the call)."""
        sp = _i32(species)
        box, pbc = _box(box, pbc)
        self._check(self._lib.aenet_energy_forces_noalloc(self._h, int(pos.shape[0]), _dev(pos), _ptr(sp, _ip),
                                                          _ptr(box), _ptr(pbc, _u8p), _dev(e_total),
                                                          _dev(e_atom), _dev(forces), _stream(stream)))

    def energy_forces_batch_dev(self, offsets, pos, species, boxes, pbc=(1, 1, 1), e_struct=None,
                                e_atom=None, forces=None, stream=None):
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        sp = _i32(species)
        bx = _f64(boxes).reshape(-1, 3)
        _, pbc = _box(bx[0], pbc)
        self._check(self._lib.aenet_energy_forces_batch_dev(
            self._h, len(off) - 1, _ptr(off, _i64p), _dev(pos), _ptr(sp, _ip), _ptr(bx), _ptr(pbc, _u8p),
            _dev(e_struct), _dev(e_atom), _dev(forces), _stream(stream)))

    def md_step_dev(self, pos, vel, species, box, pbc, dt_ps, n_steps, e_pot=None, e_kin=None,
                    forces=None, stream=None):
        sp = _i32(species)
        box, pbc = _box(box, pbc)
        self._check(self._lib.aenet_md_step_dev(self._h, int(pos.shape[0]), _dev(pos), _dev(vel), _ptr(sp, _ip),
                                                _ptr(box), _ptr(pbc, _u8p), float(dt_ps), int(n_steps),
                                                _dev(e_pot), _dev(e_kin), _dev(forces), _stream(stream)))

    def loss_grad_dev(self, offsets, pos, species, boxes, pbc, e_ref, f_ref, lambda_f, loss, grad,
                      stream=None):
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        sp = _i32(species)
        bx = _f64(boxes).reshape(-1, 3)
        _, pbc = _box(bx[0], pbc)
        self._check(self._lib.aenet_loss_grad_dev(
            self._h, len(off) - 1, _ptr(off, _i64p), _dev(pos), _ptr(sp, _ip), _ptr(bx), _ptr(pbc, _u8p),
            _dev(e_ref), _dev(f_ref), float(lambda_f), _dev(loss), _dev(grad), _stream(stream)))
