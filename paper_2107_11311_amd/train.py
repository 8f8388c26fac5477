"""Full-batch training with L-BFGS (Sec. II C): the network parameters that
minimise the training cost over a set of reference structures, with the cost
and its parameter gradient from aenet_loss_grad_dev (double back-propagation
on the GPU).

With lambda_f = 0 the cost is the energy-only objective of Eq. 7, with every
structure's energy error taken per atom and averaged over the structures
(Eq. 7's half sum of squared errors up to that normalisation; for structures
of one size the two differ by a constant factor and have the same minimiser).
lambda_f > 0 adds the force term of the library's energy+force loss.  The
optimiser is SciPy's L-BFGS-B without bounds; only the function and gradient
evaluations run on the GPU.
"""
import time
from dataclasses import dataclass, field
from typing import List

import numpy as np


@dataclass
class LbfgsResult:
    params: np.ndarray
    loss0: float
    loss: float
    grad_norm0: float
    grad_norm: float
    iterations: int
    evaluations: int
    seconds: float
    message: str
    history: List[float] = field(default_factory=list)


def fit_lbfgs(ctx, offsets, pos, species, boxes, pbc, e_ref, f_ref=None, lambda_f: float = 0.0,
              maxiter: int = 100, history: int = 10, gtol: float = 1e-12, log_every: int = 0,
              log=print, target: float = 0.0) -> LbfgsResult:
    """Minimises the cost over the batch (offsets [B+1], pos [N,3] and
    species [N] in structure order, boxes [B,3], e_ref [B], f_ref [N,3] or
    None for an energy-only cost) starting from ctx's current parameters,
    which hold the result on return."""
    import torch
    from scipy.optimize import minimize

    dev = torch.device("cuda", torch.cuda.current_device())
    pos_d = torch.as_tensor(np.ascontiguousarray(pos, dtype=np.float64), device=dev)
    e_d = torch.as_tensor(np.ascontiguousarray(e_ref, dtype=np.float64), device=dev)
    f = np.zeros_like(np.asarray(pos, dtype=np.float64)) if f_ref is None else f_ref
    f_d = torch.as_tensor(np.ascontiguousarray(f, dtype=np.float64), device=dev)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    grad = torch.zeros(ctx.n_params(), dtype=torch.float64, device=dev)
    lam = float(lambda_f) if f_ref is not None else 0.0
    trace = []

    def fun(p):
        ctx.set_params(p)
        ctx.loss_grad_dev(offsets, pos_d, species, boxes, pbc, e_d, f_d, lam, loss, grad)
        torch.cuda.synchronize()
        value = loss.item()
        trace.append(value)
        return value, grad.cpu().numpy()

    p0 = ctx.get_params()
    l0, g0 = fun(p0)
    t0 = time.perf_counter()
    it = [0]

    def progress(intermediate_result):
        it[0] += 1
        if log_every and it[0] % log_every == 0:
            log(f"lbfgs iteration {it[0]}: loss {trace[-1]:.4e} ({time.perf_counter() - t0:.0f} s)")
        if intermediate_result.fun <= target:
            raise StopIteration  # the cost reached the requested value

    res = minimize(fun, p0, jac=True, method="L-BFGS-B", callback=progress,
                   options=dict(maxiter=maxiter, maxcor=history, gtol=gtol, ftol=0.0))
    seconds = time.perf_counter() - t0
    l1, g1 = fun(res.x)  # leaves ctx at the optimiser's result
    return LbfgsResult(params=res.x, loss0=l0, loss=l1, grad_norm0=float(np.linalg.norm(g0)),
                       grad_norm=float(np.linalg.norm(g1)), iterations=int(res.nit),
                       evaluations=int(res.nfev), seconds=seconds, message=str(res.message),
                       history=trace)
