"""torch.autograd.Function for the band energy of a block of vectors.

E(X, V) = sum_i f_i x_i^* Ht(V) x_i  with Ht = M^-1/2 H(V) M^-1/2.
Backward (one library call, band_energy_grad):
  dE/dV_{e,q} = W_{e,q} sum_i f_i |psi_i(x_{e,q})|^2   (the density of the paper's eqnrho times W)
  dE/dX       = 2 Ht X diag(f)                          (PyTorch's convention for complex X)

V is the potential at the quadrature points ([n_cells, nq], float64, host or
device); the forward pass loads it into the operator (oefe_op_set_potential,
which rebuilds the potential-dependent operator data on the device).
"""
from __future__ import annotations

import torch

from . import oefe


class BandEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X: torch.Tensor, V: torch.Tensor, f: torch.Tensor, op: "oefe.Operator"):
        op.set_potential(V.detach())
        need_dV = ctx.needs_input_grad[1]
        need_dX = ctx.needs_input_grad[0]
        E, dV, dX = oefe.band_energy_grad(op, X.detach(), f.detach(), want_dV=need_dV, want_dX=need_dX)
        ctx.save_for_backward(dV if dV is not None else torch.empty(0), dX if dX is not None else torch.empty(0))
        ctx.has = (need_dX, need_dV)
        ctx.vdev = V.device
        return E

    @staticmethod
    def backward(ctx, gE):
        dV, dX = ctx.saved_tensors
        need_dX, need_dV = ctx.has
        gX = gE.to(dX.dtype if dX.numel() else torch.float64) * dX if need_dX else None
        gV = (gE * dV).to(ctx.vdev) if need_dV else None
        return gX, gV, None, None


def band_energy(X: torch.Tensor, V: torch.Tensor, f: torch.Tensor, op: "oefe.Operator") -> torch.Tensor:
    """Differentiable band energy (float64 scalar on the device of X)."""
    return BandEnergy.apply(X, V, f, op)
