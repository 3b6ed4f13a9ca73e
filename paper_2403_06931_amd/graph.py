"""HIP-graph capture of a forward launch sequence.

The persistent batched form is a two-kernel sequence (processing order and
work-counter reset, then the persistent DP kernel) that allocates nothing and
synchronises nothing, so it can be captured once and replayed for new query
values of the same lengths.  Buffers are bound at capture time: refill
``queries`` / ``reference`` in place between replays.
"""
from __future__ import annotations

import torch

from . import api


class ForwardGraph:
    def __init__(self, queries: torch.Tensor, h_query_lens, query_lens: torch.Tensor,
                 reference: torch.Tensor, cost_kind: int = api.SDTW_COST_SQUARED, *,
                 flags: int = api.SDTW_F_PERSISTENT, variant: int = -1):
        dev = queries.device
        self.queries, self.query_lens, self.reference = queries, query_lens, reference
        self.h_lens = api._host_lens(h_query_lens)
        b = self.h_lens.size
        self.cost = torch.empty(b, dtype=torch.float32, device=dev)
        self.end_pos = torch.empty(b, dtype=torch.int64, device=dev)
        self.ws = api.workspace(api.sdtw_forward_workspace_bytes(self.h_lens, reference.numel(),
                                                                 flags, variant), dev)
        self.kw = dict(cost=self.cost, end_pos=self.end_pos, flags=flags, variant=variant,
                       workspace_buf=self.ws)
        self.cost_kind = cost_kind
        # one eager call first (validates the arguments outside the capture)
        self._call()
        torch.cuda.synchronize(dev)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._call()

    def _call(self):
        api.sdtw_forward(self.queries, self.h_lens, self.query_lens, self.reference,
                         self.cost_kind, **self.kw)

    def replay(self):
        self.graph.replay()
        return self.cost, self.end_pos
