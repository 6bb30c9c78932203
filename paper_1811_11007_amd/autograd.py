"""torch.autograd binding of the batched tree log-likelihood.

Forward returns lnL of every tree of a plan at the given branch lengths;
backward multiplies the incoming gradient by d lnL / d t_e, which the
library's gradient program computes for every edge in the same launch
(post-order and pre-order directional partials, then one edge derivative
per edge).  Torch provides only the device memory and the stream.
"""
from __future__ import annotations

import torch

from ._lib import PT_PLAN_GRAD, Plan


class PTLogLik(torch.autograd.Function):
    """lnL[n_trees] = f(brlen[n_edges]) for a plan created with PT_PLAN_GRAD."""

    @staticmethod
    def forward(ctx, brlen: torch.Tensor, plan: Plan, edge_tree: torch.Tensor):
        if brlen.dtype != torch.float64 or not brlen.is_cuda:
            raise TypeError("brlen must be a float64 CUDA tensor")
        b = brlen.detach().contiguous()
        lnl = torch.empty(plan.trees.n_trees, dtype=torch.float64, device=b.device)
        grad = torch.empty_like(b)
        plan.grad(b, lnl, grad, stream=torch.cuda.current_stream(b.device))
        ctx.save_for_backward(grad, edge_tree)
        return lnl

    @staticmethod
    def backward(ctx, grad_out):
        grad, edge_tree = ctx.saved_tensors
        return grad_out[edge_tree] * grad, None, None


class TreeLogLik(torch.nn.Module):
    """Convenience module: owns a gradient-capable plan for a fixed batch."""

    def __init__(self, ctx, alns, trees, precision):
        super().__init__()
        self.plan = Plan(ctx, alns, trees, PT_PLAN_GRAD, precision)
        counts = torch.tensor(trees.edge_offset[1:] - trees.edge_offset[:-1], dtype=torch.int64)
        self.register_buffer("edge_tree", torch.repeat_interleave(torch.arange(trees.n_trees), counts))

    def forward(self, brlen: torch.Tensor) -> torch.Tensor:
        return PTLogLik.apply(brlen, self.plan, self.edge_tree.to(brlen.device))
