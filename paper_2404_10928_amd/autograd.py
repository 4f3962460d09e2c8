"""Differentiable wrappers: gradients of losses through A and A^T.

PAForward.apply(x, geom) returns A x and back-propagates through A^T;
PAAdjoint.apply(y, geom) returns A^T y and back-propagates through A.  Both
run the HIP kernels of the C ABI in the dtype of their input (float32:
PA_F32, float64: PA_F64).  Leading batch dimensions are frames.

tv() is the isotropic total variation of the paper's objective (Eq. 8, its
TV term) with a smoothing epsilon, written with ordinary torch operations so
that autograd differentiates it; it is loss code around the operator, not
part of it.
"""
from __future__ import annotations

import torch

from . import ops


class PAForward(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x: torch.Tensor, geom) -> torch.Tensor:
        g = ops.as_device_geometry(geom, x.device)
        ctx.geom = g
        return ops.forward(x.contiguous(), g)

    @staticmethod
    def backward(ctx, grad_y: torch.Tensor):
        return ops.adjoint(grad_y.contiguous(), ctx.geom), None


class PAAdjoint(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y: torch.Tensor, geom) -> torch.Tensor:
        g = ops.as_device_geometry(geom, y.device)
        ctx.geom = g
        return ops.adjoint(y.contiguous(), g)

    @staticmethod
    def backward(ctx, grad_x: torch.Tensor):
        return ops.forward(grad_x.contiguous(), ctx.geom), None


def tv(x: torch.Tensor, eps: float = 1e-8) -> torch.Tensor:
    """Sum over pixels of sqrt(dx^2 + dy^2 + eps^2) for 2D frames (last two dims),
    forward differences, zero difference past the last row/column; summed over
    leading frames in FP64."""
    dx = torch.zeros_like(x)
    dy = torch.zeros_like(x)
    dx[..., :, :-1] = x[..., :, 1:] - x[..., :, :-1]
    dy[..., :-1, :] = x[..., 1:, :] - x[..., :-1, :]
    mag = torch.sqrt(dx.double() ** 2 + dy.double() ** 2 + eps * eps)
    return mag.sum()


def data_term(x: torch.Tensor, y: torch.Tensor, geom) -> torch.Tensor:
    """||A x - y||^2 summed in FP64 over all frames."""
    r = PAForward.apply(x, geom) - y
    return (r.double() ** 2).sum()
