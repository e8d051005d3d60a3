"""torch.autograd.Function wrappers of the forward/backward pairs of the C ABI.

Gradients flow to the cost volume and to the edge weights (so to any torch expression
that produced them, e.g. a scalar pairwise strength times contrast weights).  Labels
are piecewise constant and carry no gradient.  The forward keeps what the backward
needs in its workspace: by default the selection tapes of every half-step
(keep_checkpoints=2, no recompute in the backward); keep_checkpoints=1 keeps only the
dual before every half-step and the backward recomputes (less memory); the refinement
keeps its branch masks.
"""
from __future__ import annotations

import torch

from . import ops

__all__ = ["solve_discrete_ad", "refine_continuous_ad", "DiscreteFn", "RefineFn"]


class DiscreteFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, cost, w_h, w_v, kw):
        kw = dict(kw)
        kw.setdefault("keep_checkpoints", 2)
        res = ops.solve_discrete(cost.detach(), w_h.detach().contiguous(), w_v.detach().contiguous(),
                                 want_bounds=True, **kw)
        ctx.kw = kw
        ctx.res = res
        ctx.save_for_backward(cost, w_h, w_v)
        ctx.mark_non_differentiable(res.labels)
        lb = res.bounds[0:1].to(torch.float32)
        return res.minmarg, lb, res.labels

    @staticmethod
    def backward(ctx, g_mm, g_lb, _g_labels):
        cost, w_h, w_v = ctx.saved_tensors
        res = ctx.res
        kw = {k: v for k, v in ctx.kw.items()
              if k in ("T", "n_iters", "n_half_steps", "minorant", "gammas", "tile", "keep_checkpoints",
                       "recompute_selections")}
        # the bound gradient stays on the device (no host synchronisation in the backward)
        gb = None
        if g_lb is not None:
            gb = torch.zeros(2, dtype=torch.float64, device=cost.device)
            gb[0:1] = g_lb.to(torch.float64).sum(0, keepdim=True)
        gm = None if g_mm is None else g_mm.contiguous().to(torch.float32)
        gc, gwh, gwv = ops.solve_discrete_backward(cost.detach(), w_h.detach().contiguous(), w_v.detach().contiguous(),
                                                   res.dual, res.workspace, grad_minmarg=gm, grad_bounds=gb, **kw)
        return gc.to(cost.dtype), gwh, gwv, None


class RefineFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, cost, labels, w_h, w_v, kw):
        H, W, K = cost.shape
        nbytes = ops.refine_workspace_bytes((H, W, K), keep_tape=True, **kw)
        ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=cost.device)
        u = ops.refine_continuous(cost.detach(), labels, w_h.detach().contiguous(), w_v.detach().contiguous(),
                                  workspace=ws, keep_tape=True, **kw)
        ctx.kw = kw
        ctx.ws = ws
        ctx.save_for_backward(cost, w_h, w_v)
        return u

    @staticmethod
    def backward(ctx, g_u):
        cost, w_h, w_v = ctx.saved_tensors
        gc, gwh, gwv = ops.refine_continuous_backward(g_u.contiguous().to(torch.float32), cost.detach(),
                                                      w_h.detach().contiguous(), w_v.detach().contiguous(), ctx.ws,
                                                      **ctx.kw)
        return gc.to(cost.dtype), None, gwh, gwv, None


def solve_discrete_ad(cost, w_h, w_v, **kw):
    """Differentiable Dual_MM: returns (normalized row min-marginals, lower bound [1], labels).
    keep_checkpoints (2 by default, or 1) selects what the forward keeps for the backward."""
    return DiscreteFn.apply(cost, w_h, w_v, kw)


def refine_continuous_ad(cost, labels, w_h, w_v, **kw):
    """Differentiable refinement: returns u [H][W]."""
    return RefineFn.apply(cost, labels, w_h, w_v, kw)
