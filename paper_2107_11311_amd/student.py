"""Distilled student potential: data from teacher MD, training with the
library's loss-gradient kernels, and MD with the teacher as judge and fallback.

The paper shows that shrinking the descriptor of its water potential from 52
to 20 dimensions makes MD about three times faster at some cost in accuracy
(Sec. IV, model-complexity study).  Here the smaller network is obtained by
distillation: it is trained on configurations, energies and forces produced by
MD with the full network, and during production MD the full network re-checks
the student's forces every few steps and takes over when they drift.

Everything numerical runs through the C ABI (teacher MD, student energies and
forces, the loss gradient by double back-propagation, the Adam update and the
repacking of the parameters); torch only holds device buffers and gathers the
snapshots of a mini-batch.  The final full-batch L-BFGS polish runs SciPy's
optimiser on the host over the same GPU cost and gradient.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np


@dataclass
class Snapshots:
    pos: "object"          # torch [S, N, 3] float64 (device)
    forces: "object"       # torch [S, N, 3] float32 (device)
    energy: "object"       # torch [S] float64 (device)
    species: np.ndarray
    box: np.ndarray
    pbc: np.ndarray
    seconds: float = 0.0


def generate_snapshots(teacher, system, vel0, n_snap: int, stride: int, dt_ps: float,
                       device="cuda:0") -> Snapshots:
    """Runs NVE MD with the teacher context and stores every stride-th state."""
    import torch
    dev = torch.device(device)
    n = system.pos.shape[0]
    pos = torch.from_numpy(np.ascontiguousarray(system.pos, dtype=np.float64)).to(dev)
    vel = torch.from_numpy(np.ascontiguousarray(vel0, dtype=np.float64)).to(dev)
    P = torch.empty((n_snap, n, 3), dtype=torch.float64, device=dev)
    Fs = torch.empty((n_snap, n, 3), dtype=torch.float32, device=dev)
    Es = torch.empty((n_snap,), dtype=torch.float64, device=dev)
    F = torch.empty((n, 3), dtype=torch.float64, device=dev)
    ep = torch.zeros(1, dtype=torch.float64, device=dev)
    t0 = time.perf_counter()
    for k in range(n_snap):
        teacher.md_step_dev(pos, vel, system.species, system.box, system.pbc, dt_ps, stride, ep, None, F)
        P[k].copy_(pos)
        Fs[k].copy_(F)
        Es[k:k + 1].copy_(ep)
    torch.cuda.synchronize()
    return Snapshots(P, Fs, Es, system.species, system.box, system.pbc, time.perf_counter() - t0)


def restrict_to_orders(model, nr: int, na: int):
    """A copy of a model whose networks ignore every descriptor component of
    radial order above nr or angular order above na (their first-layer
    weights set to zero): its energy is a function of the descriptor of a
    model with orders nr / na and the same cutoffs.  Serves as a teacher that
    such a student can represent."""
    import copy
    out = copy.deepcopy(model)
    NR, NA = model.radial_order, model.angular_order
    T1, T2 = NR + 1, NR + NA + 2
    keep = [a for a in range(NR + 1) if a <= nr] + [T1 + a for a in range(NA + 1) if a <= na]
    if model.n_species > 1:
        keep = keep + [T2 + k for k in keep]
    mask = np.zeros(model.D, dtype=bool)
    mask[keep] = True
    for net in out.nets:
        net.W[0] = np.where(mask[None, :], net.W[0], 0.0)
    return out


@dataclass
class TrainResult:
    params: np.ndarray
    losses: List[float] = field(default_factory=list)
    seconds: float = 0.0
    steps: int = 0
    lbfgs_iterations: int = 0
    lbfgs_seconds: float = 0.0


def _batch_args(snaps: Snapshots, batch: int):
    n = snaps.pos.shape[1]
    offs = np.arange(batch + 1, dtype=np.int64) * n
    species = np.tile(snaps.species, batch)
    boxes = np.tile(np.asarray(snaps.box, dtype=np.float64).reshape(1, 3), (batch, 1))
    return offs, species, boxes


def train(student, snaps: Snapshots, train_idx: np.ndarray, steps: int, batch: int, lr: float,
          lambda_f: float = 1.0, seed: int = 0, lr_final: Optional[float] = None,
          log_every: int = 0, log: Callable[[str], None] = print) -> TrainResult:
    """Adam on mini-batches of snapshots, entirely on the device: the gradient
    of the energy+force loss from aenet_loss_grad_dev (double
    back-propagation), the update by aenet_adam_step_dev, the new parameters
    repacked by aenet_set_params_dev; parameters, moments and gradients never
    leave the GPU.  The learning rate falls geometrically from lr to lr_final."""
    import torch
    from . import aenet as A
    dev = snaps.pos.device
    rng = np.random.default_rng(seed)
    n = snaps.pos.shape[1]
    p = torch.from_numpy(student.get_params()).to(dev)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    grad = torch.zeros_like(p)
    offs, species, boxes = _batch_args(snaps, batch)
    res = TrainResult(p.cpu().numpy())
    t0 = time.perf_counter()
    lr_final = lr if lr_final is None else lr_final
    for it in range(steps):
        idx = torch.from_numpy(rng.choice(train_idx, size=batch, replace=False)).to(dev)
        pos = snaps.pos.index_select(0, idx).reshape(batch * n, 3)
        f_ref = snaps.forces.index_select(0, idx).reshape(batch * n, 3).to(torch.float64)
        e_ref = snaps.energy.index_select(0, idx)
        student.loss_grad_dev(offs, pos, species, boxes, snaps.pbc, e_ref, f_ref, lambda_f, loss, grad)
        a = lr * (lr_final / lr) ** (it / max(steps - 1, 1))
        A.adam_step_dev(p, grad, m, v, a, 0.9, 0.999, 1e-8, it + 1)
        student.set_params_dev(p)
        if log_every and (it % log_every == 0 or it == steps - 1):
            res.losses.append(loss.item())
            log(f"adam step {it} loss {res.losses[-1]:.4e} lr {a:.2e}")
    torch.cuda.synchronize()
    res.params = p.cpu().numpy()
    res.seconds = time.perf_counter() - t0
    res.steps = steps
    return res


def polish_lbfgs(student, snaps: Snapshots, idx: np.ndarray, maxiter: int, lambda_f: float = 1.0,
                 res: Optional[TrainResult] = None, log: Callable[[str], None] = print,
                 target: float = 0.0) -> TrainResult:
    """Full-batch L-BFGS (the paper's optimiser, Sec. II C) over the snapshots
    idx, starting from the student's current parameters; every cost and
    gradient evaluation is aenet_loss_grad_dev over the whole set."""
    import torch
    from .train import fit_lbfgs
    n = snaps.pos.shape[1]
    k = len(idx)
    offs, species, boxes = _batch_args(snaps, k)
    sel = torch.from_numpy(np.asarray(idx, dtype=np.int64)).to(snaps.pos.device)
    pos = snaps.pos.index_select(0, sel).reshape(k * n, 3).cpu().numpy()
    f_ref = snaps.forces.index_select(0, sel).reshape(k * n, 3).to(torch.float64).cpu().numpy()
    e_ref = snaps.energy.index_select(0, sel).cpu().numpy()
    r = fit_lbfgs(student, offs, pos, species, boxes, snaps.pbc, e_ref, f_ref, lambda_f=lambda_f,
                  maxiter=maxiter, history=20, log_every=250, log=log, target=target)
    log(f"lbfgs: loss {r.loss0:.4e} -> {r.loss:.4e} in {r.iterations} iterations ({r.seconds:.1f} s)")
    out = res if res is not None else TrainResult(r.params)
    out.params = r.params
    out.losses.append(r.loss)
    out.lbfgs_iterations = r.iterations
    out.lbfgs_seconds = r.seconds
    return out


def force_rmse(ctx, snaps: Snapshots, idx) -> float:
    """Force RMSE (eV/A) of a context against the stored teacher forces."""
    import torch
    dev = snaps.pos.device
    n = snaps.pos.shape[1]
    F = torch.empty((n, 3), dtype=torch.float64, device=dev)
    acc, cnt = 0.0, 0
    for k in idx:
        ctx.energy_forces_dev(snaps.pos[k], snaps.species, snaps.box, snaps.pbc, None, None, F)
        d = F - snaps.forces[k].to(torch.float64)
        acc += float((d * d).sum().item())
        cnt += 3 * n
    return float(np.sqrt(acc / cnt))


@dataclass
class JudgeReport:
    steps: int = 0
    chunks: int = 0
    fallbacks: int = 0
    rmse_per_chunk: List[float] = field(default_factory=list)
    student_seconds: float = 0.0
    teacher_seconds: float = 0.0
    judge_seconds: float = 0.0


def md_with_judge(run_student: Callable, run_teacher: Callable, teacher_forces: Callable,
                  state, n_steps: int, every: int, threshold: float,
                  rmse: Optional[Callable] = None) -> JudgeReport:
    """Production MD with a judge.

    run_student(state, k) / run_teacher(state, k) advance the state by k steps
    in place and return the forces at the final positions; teacher_forces(state)
    evaluates the teacher there; state.save() / state.restore(snapshot) make and
    restore a checkpoint.  Every `every` steps the student's final forces are
    compared with the teacher's (rmse(Fs, Ft), by default numpy on host
    arrays); if the RMSE exceeds `threshold` the chunk is undone and redone
    with the teacher."""
    rep = JudgeReport()
    done = 0
    while done < n_steps:
        k = min(every, n_steps - done)
        ckpt = state.save()
        t0 = time.perf_counter()
        Fs = run_student(state, k)
        t1 = time.perf_counter()
        Ft = teacher_forces(state)
        if rmse is None:
            err = float(np.sqrt(np.mean((np.asarray(Fs) - np.asarray(Ft)) ** 2)))
        else:
            err = float(rmse(Fs, Ft))
        t2 = time.perf_counter()
        rep.rmse_per_chunk.append(err)
        rep.student_seconds += t1 - t0
        rep.judge_seconds += t2 - t1
        if not err <= threshold:
            state.restore(ckpt)
            t3 = time.perf_counter()
            run_teacher(state, k)
            rep.teacher_seconds += time.perf_counter() - t3
            rep.fallbacks += 1
        done += k
        rep.chunks += 1
    rep.steps = done
    return rep


class DeviceState:
    """MD state on the GPU (positions, velocities) with copy checkpoints, for
    md_with_judge driving two contexts."""

    def __init__(self, system, vel, device="cuda:0"):
        import torch
        dev = torch.device(device)
        self.system = system
        self.pos = torch.from_numpy(np.ascontiguousarray(system.pos, dtype=np.float64)).to(dev)
        self.vel = torch.from_numpy(np.ascontiguousarray(vel, dtype=np.float64)).to(dev)
        self.F = torch.empty_like(self.pos)
        self.ep = torch.zeros(1, dtype=torch.float64, device=dev)
        self.ek = torch.zeros(1, dtype=torch.float64, device=dev)

    def save(self):
        return (self.pos.clone(), self.vel.clone())

    def restore(self, ck):
        self.pos.copy_(ck[0])
        self.vel.copy_(ck[1])

    def runner(self, ctx, dt_ps):
        """run(state, k): k MD steps with ctx; returns the final forces (device)."""
        def run(state, k):
            s = state.system
            ctx.md_step_dev(state.pos, state.vel, s.species, s.box, s.pbc, dt_ps, k, state.ep, state.ek, state.F)
            return state.F
        return run

    def forces(self, ctx):
        """f(state): ctx's forces at the state's positions (device)."""
        import torch
        buf = torch.empty_like(self.pos)

        def f(state):
            s = state.system
            ctx.energy_forces_dev(state.pos, s.species, s.box, s.pbc, None, None, buf)
            return buf
        return f

    def rmse(self, ctx):
        """rmse(Fs, Ft) on the device (aenet_rms_diff_dev): one value read back."""
        import torch
        out = torch.zeros(1, dtype=torch.float64, device=self.pos.device)

        def r(a, b):
            ctx.rms_diff_dev(a, b, out)
            return out.item()
        return r
