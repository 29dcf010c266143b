"""torch.autograd wrapper: LAD-LASSO coefficients as a differentiable layer.

forward: the batched solve (HIP kernels) for the plan's layout.
backward: the hand-written gradient kernel through the optimal vertex,
giving dL/dX and dL/dy (lambda gets no gradient: the solution is piecewise
constant in lambda at a fixed vertex, so its derivative is zero almost
everywhere).  Solves without an optimality certificate get zero
gradients; at a certified but non-unique optimum the gradient is that of
the returned vertex.
"""
from __future__ import annotations

import torch

from . import Plan


class LadLassoFunction(torch.autograd.Function):
    """b = LadLassoFunction.apply(X, y, lam, plan)

    X, y, lam: float32 CUDA tensors packed as the plan describes; returns
    the flat coefficient tensor (all solves, all path steps; the gradient
    flows through the last path step)."""

    @staticmethod
    def forward(ctx, X, y, lam, plan: Plan):
        out = plan.solve(X.detach().contiguous(), y.detach().contiguous(), lam.detach().contiguous())
        ctx.plan = plan
        ctx.out = out
        ctx.save_for_backward(X)
        return out["b"]

    @staticmethod
    def backward(ctx, grad_b):
        (X,) = ctx.saved_tensors
        plan: Plan = ctx.plan
        L = plan.path_len
        g = grad_b.contiguous()
        if L > 1:
            # only the last path step carries a gradient through the vertex
            idx = torch.cat([torch.arange(L * int(o) + (L - 1) * int(p), L * int(o) + L * int(p), device=g.device)
                             for o, p in zip(plan.b_off, plan.p_per_solve)])
            g = g[idx].contiguous()
        grad_y, grad_X = plan.backward(X.detach().contiguous(), ctx.out, g, step=L - 1)
        return grad_X, grad_y, None, None


def ladlasso(X, y, lam, plan: Plan):
    return LadLassoFunction.apply(X, y, lam, plan)
