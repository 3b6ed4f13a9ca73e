"""Differentiable sDTW: torch.autograd.Function over the library's
checkpointed forward and walk-back backward.

sdtw(queries, query_lens, reference) returns (cost [B], end_pos [B]); cost is
differentiable with respect to the packed queries and the reference, end_pos
is not.  The forward stores DP column checkpoints every ``ckpt_every``
reference columns; the backward recomputes the blocks the optimal path
crosses from them (no N x M matrix is kept).
"""
from __future__ import annotations

import torch

from . import api


class SDTWFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, queries, reference, h_lens, query_lens, cost_kind, ckpt_every):
        h = api._host_lens(h_lens)
        m = reference.numel()
        nck = api.sdtw_checkpoint_floats(h, m, ckpt_every)
        ckpt = torch.empty(max(nck, 1), dtype=torch.float32, device=queries.device)
        cost, end = api.sdtw_forward(queries.detach(), h, query_lens, reference.detach(),
                                     cost_kind, ckpt=ckpt if nck else None,
                                     ckpt_every=ckpt_every, flags=api.SDTW_F_CHECKPOINT)
        ctx.save_for_backward(queries, reference, query_lens, cost, end, ckpt)
        ctx.h_lens = h
        ctx.cost_kind = cost_kind
        ctx.ckpt_every = ckpt_every
        ctx.has_ckpt = nck > 0
        ctx.mark_non_differentiable(end)
        return cost, end

    @staticmethod
    def backward(ctx, grad_cost, grad_end):
        queries, reference, query_lens, cost, end, ckpt = ctx.saved_tensors
        if grad_cost is None:
            return None, None, None, None, None, None
        g = grad_cost.detach().to(torch.float32).contiguous()
        gq, gr = api.sdtw_backward(queries.detach(), ctx.h_lens, query_lens, reference.detach(),
                                   ctx.cost_kind, g, cost, end,
                                   ckpt if ctx.has_ckpt else None,
                                   ctx.ckpt_every)
        return gq, gr, None, None, None, None


def sdtw(queries: torch.Tensor, h_query_lens, reference: torch.Tensor,
         cost_kind: int = api.SDTW_COST_SQUARED, ckpt_every: int = 1024,
         query_lens: torch.Tensor = None):
    """Differentiable batched sDTW -> (cost, end_pos)."""
    h = api._host_lens(h_query_lens)
    if query_lens is None:
        query_lens = torch.from_numpy(h).to(queries.device)
    return SDTWFunction.apply(queries, reference, h, query_lens, cost_kind, ckpt_every)
