"""The normaliser, the binary16, pruned and uint8-code forwards and the path
output enqueue only kernels on the caller's stream and allocate nothing, so a
HIP graph captures them: each replay (with eager work between replays)
matches the eager call."""
import numpy as np
import pytest
import torch

import workloads
from gpu_util import to_dev

pytestmark = pytest.mark.gpu


def _capture(fn):
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()                                    # warm-up outside the graph
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    return g


def _replays(g, outs, want):
    for rep in range(3):
        for o in outs:
            o.fill_(-1)
        g.replay()
        torch.cuda.synchronize()
        for o, w in zip(outs, want):
            assert torch.equal(o, w), f"replay {rep}"
        x = torch.randn(1 << 20, device=outs[0].device).sum()   # eager work between
        torch.cuda.synchronize()
        del x


def test_znorm_graph():
    import paper_2403_06931_amd as P
    lens = [2000] * 16 + [50_000]
    d = torch.device("cuda:0")
    x = torch.from_numpy(workloads.raw_series(lens, seed=3)).to(d)
    h = np.asarray(lens, np.int32)
    lt = torch.from_numpy(h).to(d)
    z = torch.empty_like(x)
    ws = P.workspace(P.sdtw_znorm_workspace_bytes(h), d)
    want = P.sdtw_znorm(x, h, lt, workspace_buf=ws).clone()
    g = _capture(lambda: P.sdtw_znorm(x, h, lt, out=z, workspace_buf=ws))
    _replays(g, [z], [want])


def test_f16_forward_graph():
    import paper_2403_06931_amd as P
    w = workloads.make_random(8, [300] * 8, 4000, seed=4)
    q, l, r = to_dev(w)
    ws = P.workspace(P.sdtw_forward_f16_workspace_bytes(w.lens, w.ref_len), q.device)
    c = torch.empty(w.batch, dtype=torch.float32, device=q.device)
    e = torch.empty(w.batch, dtype=torch.int64, device=q.device)
    wc, we = P.sdtw_forward_f16(q, w.lens, l, r, 0, workspace_buf=ws)
    wc, we = wc.clone(), we.clone()
    g = _capture(lambda: P.sdtw_forward_f16(q, w.lens, l, r, 0, cost=c, end_pos=e,
                                            workspace_buf=ws))
    _replays(g, [c, e], [wc, we])


def test_align_graph():
    import paper_2403_06931_amd as P
    w = workloads.make_random(6, [200] * 6, 3000, seed=6)
    q, l, r = to_dev(w)
    K = 256
    ck = torch.empty(P.sdtw_checkpoint_floats(w.lens, w.ref_len, K), dtype=torch.float32,
                     device=q.device)
    cost, end = P.sdtw_forward(q, w.lens, l, r, 0, ckpt=ck, ckpt_every=K,
                               flags=P.SDTW_F_CHECKPOINT)
    ws = P.workspace(P.sdtw_align_workspace_bytes(w.lens, w.ref_len, K), q.device)
    s0, lo0, hi0 = P.sdtw_align(q, w.lens, l, r, 0, cost, end, ck, K, workspace_buf=ws)
    s0, lo0, hi0 = s0.clone(), lo0.clone(), hi0.clone()
    res = {}

    def run():
        res["out"] = P.sdtw_align(q, w.lens, l, r, 0, cost, end, ck, K, workspace_buf=ws)
    g = _capture(run)
    s, lo, hi = res["out"]
    _replays(g, [s, lo, hi], [s0, lo0, hi0])


def test_pruned_forward_graph():
    """The pruned forward, plain and persistent (work queue reset inside the
    captured sequence)."""
    import paper_2403_06931_amd as P
    w = workloads.make_random(12, [64, 700, 300, 2100] * 3, 3000, seed=6)
    q, l, r = to_dev(w)
    for flags in (0, P.SDTW_F_PERSISTENT):
        ws = P.workspace(P.sdtw_forward_workspace_bytes(w.lens, w.ref_len, flags), q.device)
        c = torch.empty(w.batch, dtype=torch.float32, device=q.device)
        e = torch.empty(w.batch, dtype=torch.int64, device=q.device)
        wc, we = P.sdtw_forward_pruned(q, w.lens, l, r, 1.5, flags=flags, workspace_buf=ws)
        wc, we = wc.clone(), we.clone()
        g = _capture(lambda: P.sdtw_forward_pruned(q, w.lens, l, r, 1.5, cost=c, end_pos=e,
                                                   flags=flags, workspace_buf=ws))
        _replays(g, [c, e], [wc, we])


def test_u8_forward_graph():
    """The uint8-code forward: codebook, codes and DP in one captured call."""
    import paper_2403_06931_amd as P
    w = workloads.make_random(8, [300] * 8, 4000, seed=7)
    q, l, r = to_dev(w)
    ws = P.workspace(P.sdtw_forward_u8_workspace_bytes(w.lens, w.ref_len), q.device)
    c = torch.empty(w.batch, dtype=torch.float32, device=q.device)
    e = torch.empty(w.batch, dtype=torch.int64, device=q.device)
    b = torch.empty(2, dtype=torch.float32, device=q.device)
    wc, we, wb = P.sdtw_forward_u8(q, w.lens, l, r, workspace_buf=ws)
    wc, we, wb = wc.clone(), we.clone(), wb.clone()
    g = _capture(lambda: P.sdtw_forward_u8(q, w.lens, l, r, cost=c, end_pos=e, codebook=b,
                                           workspace_buf=ws))
    _replays(g, [c, e, b], [wc, we, wb])
