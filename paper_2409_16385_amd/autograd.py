"""Differentiable form of the barrier term.

``barrier_energy(q, state)`` is kappa * sum_k b(d_k(W q + x_off)) over a
fixed pair list (Eq. 7, 10-11) as a torch scalar.  Its backward returns the
reduced gradient W^T g (Eq. 17) from the library, and the backward of that
gradient is the Hessian-vector product W^T H W v with the true (not
projected) pair Hessians, recomputed per call: nothing is stored per pair.
Third derivatives are not provided.
"""
from __future__ import annotations

import dataclasses

import torch

from . import binding as B


@dataclasses.dataclass
class BarrierState:
    """Everything but q: context, scene, pair lists and parameters."""
    ctx: B.Context
    scene: B.Scene
    pt: torch.Tensor
    ee: torch.Tensor
    dhat: float
    kappa: float
    mollify: bool = False
    x_off_tangent: torch.Tensor | None = None  # v_off for kinematic directions

    @property
    def flags(self) -> int:
        return B.MOLLIFY if self.mollify else 0


class _BarrierGrad(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, state: BarrierState):
        r = B.barrier_reduce(state.ctx, state.scene, q, state.pt, state.ee, state.dhat, state.kappa,
                             B.GRAD | state.flags, hess=None, count=False)
        ctx.state = state
        ctx.save_for_backward(q)
        return r["grad"]

    @staticmethod
    def backward(ctx, v):
        (q,) = ctx.saved_tensors
        st = ctx.state
        hv = B.barrier_hvp(st.ctx, st.scene, q.detach(), st.pt, st.ee, st.dhat, st.kappa, st.flags,
                           v.contiguous())
        return hv, None


class _BarrierEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, state: BarrierState):
        r = B.barrier_reduce(state.ctx, state.scene, q, state.pt, state.ee, state.dhat, state.kappa,
                             B.ENERGY | state.flags, hess=None, count=False)
        ctx.state = state
        ctx.save_for_backward(q)
        return r["energy"][0].clone()

    @staticmethod
    def backward(ctx, gout):
        (q,) = ctx.saved_tensors
        g = _BarrierGrad.apply(q, ctx.state)
        return gout * g, None


def barrier_energy(q: torch.Tensor, state: BarrierState) -> torch.Tensor:
    """Differentiable barrier energy (scalar tensor) of reduced coordinates q."""
    return _BarrierEnergy.apply(q, state)


def barrier_grad(q: torch.Tensor, state: BarrierState) -> torch.Tensor:
    """Differentiable reduced gradient W^T g (its backward is the HVP)."""
    return _BarrierGrad.apply(q, state)
