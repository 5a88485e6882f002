"""The CP objective as a differentiable torch function.

f(A) = 1/2 ||X - [[A(1), ..., A(N)]]||_F^2 (eq. (3)); its gradient with respect to A(n) is
G(n) = A(n) Gamma(n,n) - M(n) (Algorithm 1), with M(n) the MTTKRP of mode n. Both run in the
library's kernels. X is data and receives no gradient.

Two forms of the forward pass:
  * "direct" (default): f from the direct residual (one reconstruction pass over X, exact to
    rounding at any fit); the backward pass forms the gradient (the all-mode MTTKRP, Grams,
    Gamma).
  * "fused": one call forms the gradient and f together (cp_objective_gradient), f by the
    expansion ||X||^2 - 2 <M(1), A(1)> + sum prod S from the same MTTKRP; the forward keeps G
    and the backward only scales it, so a forward + backward reads X three times (two MTTKRP
    passes and one plain pass for ||X||^2) and does the MTTKRP's matrix work once. The
    expansion's absolute error is about the MTTKRP's relative accuracy times ||X||^2, so f is
    not accurate near an exact fit (the gradient is).
"""
from __future__ import annotations

import torch

from . import api


class CPObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X, method, *A):
        for a in A:
            if not a.is_contiguous():
                raise ValueError("factor matrices must be contiguous")
        if method == "direct":
            r = api.residual(X, list(A))
            ctx.save_for_backward(X, *A)
            ctx.G = None
        elif method == "fused":
            G, r = api.objective_gradient(X, list(A))
            ctx.G = G
        else:
            raise ValueError("method must be 'direct' or 'fused'")
        return (0.5 * r[0] * r[0]).to(A[0].dtype)

    @staticmethod
    def backward(ctx, gout):
        if ctx.needs_input_grad[0]:
            raise RuntimeError("cp_objective: no gradient with respect to the tensor X")
        if ctx.G is not None:
            G = ctx.G
        else:
            X, *A = ctx.saved_tensors
            G, _ = api.gn_gradient(X, list(A))
        return (None, None, *[gout.to(g.dtype) * g for g in G])


def cp_objective(X: torch.Tensor, A, method: str = "direct") -> torch.Tensor:
    """0-dim tensor f = 1/2 ||X - [[A]]||_F^2, differentiable in every factor matrix.
    method: "direct" or "fused" (see the module docstring)."""
    return CPObjective.apply(X, method, *A)
