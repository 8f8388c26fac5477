"""The training loss as a torch.autograd.Function (Sec. II C: the network
parameters are fitted by minimising a cost over reference structures, with
gradients from back-propagation).

`energy_force_loss(params, ctx, batch)` (a torch.autograd.Function) returns the scalar cost of the
batch under the parameters `params` (a float64 CUDA tensor in the flat layout
of aenet_n_params); `loss.backward()` leaves dC/dparams in `params.grad`.
Both come from one call of aenet_loss_grad_dev: the energies and forces of
every structure, the cost, and its parameter gradient by the library's
hand-written double back-propagation (a descriptor Jacobian-vector product
along the force adjoint, then a reverse pass through each network and its
tangent).  The forward pass keeps that gradient and the backward pass scales
it by the incoming gradient, so no torch arithmetic is involved beyond that
product.  The parameters reach the library through aenet_set_params_dev
(device to device, repacked on the GPU).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Batch:
    """Reference structures for the cost: structure s owns atoms
    offsets[s]..offsets[s+1] (host int64) of pos (device float64 [n, 3]),
    species (host int32 [n]), box boxes[s] (host [B, 3]); e_ref (device [B])
    and f_ref (device [n, 3]) are the reference energies and forces."""
    offsets: np.ndarray
    pos: "object"
    species: np.ndarray
    boxes: np.ndarray
    pbc: np.ndarray
    e_ref: "object"
    f_ref: "object"
    lambda_f: float = 1.0


def _function():
    import torch

    class _EnergyForceLoss(torch.autograd.Function):
        @staticmethod
        def forward(fctx, params, ctx, batch):
            p = params.detach().contiguous()
            ctx.set_params_dev(p)
            loss = torch.zeros(1, dtype=torch.float64, device=p.device)
            grad = torch.zeros_like(p)
            ctx.loss_grad_dev(batch.offsets, batch.pos, batch.species, batch.boxes, batch.pbc, batch.e_ref,
                              batch.f_ref, batch.lambda_f, loss, grad)
            fctx.save_for_backward(grad)
            return loss[0]

        @staticmethod
        def backward(fctx, g):
            (grad,) = fctx.saved_tensors
            return g * grad, None, None

    return _EnergyForceLoss


_FN = None


def energy_force_loss(params, ctx, batch: Batch):
    """The cost of `batch` under `params` (differentiable w.r.t. params)."""
    global _FN
    if _FN is None:
        _FN = _function()
    return _FN.apply(params, ctx, batch)
