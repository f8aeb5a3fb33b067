"""Differentiable variable-coefficient diffusion: y = A(kappa) u.

A(kappa) is linear in kappa (the coefficient multiplies the geometric
factors at each quadrature point) and symmetric, so for an upstream
gradient gy:

    dL/du     = A(kappa)^T gy = A(kappa) gy          (mfhex_apply_adjoint)
    dL/dkappa = (Dhat gy)^T G0 (Dhat u) per point     (mfhex_kappa_grad)

Both run in the HIP library.
"""
from __future__ import annotations

import torch

from .operator import Operator


class MFHexDiffusion(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u: torch.Tensor, kappa: torch.Tensor, op: Operator):
        op.set_kappa(kappa)
        y = op.apply(u.contiguous())
        ctx.op = op
        ctx.save_for_backward(u, kappa)
        return y

    @staticmethod
    def backward(ctx, gy: torch.Tensor):
        u, kappa = ctx.saved_tensors
        op = ctx.op
        gy = gy.contiguous()
        op.set_kappa(kappa)
        gu = op.apply_adjoint(gy) if ctx.needs_input_grad[0] else None
        gk = op.kappa_grad(u.contiguous(), gy).reshape(kappa.shape) if ctx.needs_input_grad[1] else None
        return gu, gk, None


def diffusion(u: torch.Tensor, kappa: torch.Tensor, op: Operator) -> torch.Tensor:
    return MFHexDiffusion.apply(u, kappa, op)
