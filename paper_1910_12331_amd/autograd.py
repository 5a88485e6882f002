"""The CP objective as a differentiable torch function.

f(A) = 1/2 ||X - [[A(1), ..., A(N)]]||_F^2 (eq. (3)); its gradient with respect to A(n) is
G(n) = A(n) Gamma(n,n) - M(n) (Algorithm 1), with M(n) the MTTKRP of mode n. Both run in the
library's kernels: the forward pass is the direct residual, the backward pass the all-mode
gradient (MTTKRPs, Grams, Gamma). X is data and receives no gradient.
"""
from __future__ import annotations

import torch

from . import api


class CPObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X, *A):
        for a in A:
            if not a.is_contiguous():
                raise ValueError("factor matrices must be contiguous")
        r = api.residual(X, list(A))
        ctx.save_for_backward(X, *A)
        return (0.5 * r[0] * r[0]).to(X.dtype)

    @staticmethod
    def backward(ctx, gout):
        X, *A = ctx.saved_tensors
        if ctx.needs_input_grad[0]:
            raise RuntimeError("cp_objective: no gradient with respect to the tensor X")
        G, _ = api.gn_gradient(X, list(A))
        return (None, *[gout.to(g.dtype) * g for g in G])


def cp_objective(X: torch.Tensor, A) -> torch.Tensor:
    """0-dim tensor f = 1/2 ||X - [[A]]||_F^2, differentiable in every factor matrix."""
    return CPObjective.apply(X, *A)
