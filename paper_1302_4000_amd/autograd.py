"""torch.autograd wrappers: the forward and the hand-written backward both run
in libclusco.so (no autograd tracing through PyTorch ops)."""
from __future__ import annotations

import torch

from . import binding


class CRMSDMatrix(torch.autograd.Function):
    """Packed all-vs-all cRMSD [N(N-1)/2] of x [N, L, 3]."""

    @staticmethod
    def forward(ctx, x, precision="fp32"):
        out = binding.crmsd_matrix(x, precision)
        ctx.save_for_backward(x, out)
        ctx.precision = precision
        return out

    @staticmethod
    def backward(ctx, g):
        x, out = ctx.saved_tensors
        grad = binding.crmsd_backward(x, out, g.contiguous(), ctx.precision)
        return grad, None


class CRMSDCross(torch.autograd.Function):
    """Dense cRMSD [Na, Nb] between a [Na, L, 3] and b [Nb, L, 3]."""

    @staticmethod
    def forward(ctx, a, b, precision="fp32"):
        out = binding.crmsd_cross(a, b, precision)
        ctx.save_for_backward(a, b, out)
        ctx.precision = precision
        return out

    @staticmethod
    def backward(ctx, g):
        a, b, out = ctx.saved_tensors
        ga, gb = binding.crmsd_cross_backward(a, b, out, g.contiguous(), ctx.precision,
                                              need_b=ctx.needs_input_grad[1])
        return ga, gb, None


def crmsd_matrix_ad(x: torch.Tensor, precision="fp32") -> torch.Tensor:
    """Differentiable packed all-vs-all cRMSD."""
    return CRMSDMatrix.apply(x, precision)


def crmsd_cross_ad(a: torch.Tensor, b: torch.Tensor, precision="fp32") -> torch.Tensor:
    """Differentiable dense cRMSD between two sets of models."""
    return CRMSDCross.apply(a, b, precision)
