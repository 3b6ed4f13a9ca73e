"""GPU tests of the persistent batched form (uneven lengths, one launch with a
device work queue) and of its HIP-graph capture."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_util import assert_bit_exact, gpu_forward, to_dev

pytestmark = pytest.mark.gpu


def _variants():
    import paper_2403_06931_amd as P
    return list(range(P.sdtw_variant_count()))


@pytest.mark.parametrize("kind", [0, 1])
def test_persistent_ragged_all_variants(kind):
    import paper_2403_06931_amd as P
    lens = [1, 5, 64, 65, 700, 2049, 300, 4000, 3, 1500, 513, 2600, 90, 1, 8, 1024]
    w = workloads.make_random(len(lens), lens, 3001, seed=211 + kind)
    want_c, want_e = oracle.sdtw_f32(w.queries, w.lens, w.reference, kind)
    for v in _variants():
        print(f"persistent variant {v} kind {kind}", flush=True)
        c, e = gpu_forward(w, kind, variant=v, flags=P.SDTW_F_PERSISTENT)
        assert_bit_exact(c, e, want_c, want_e, f"persistent variant {v}")


def test_persistent_more_queries_than_slots():
    """More queries than resident workgroups: the queue hands out every query
    exactly once."""
    import paper_2403_06931_amd as P
    rng = np.random.default_rng(5)
    lens = rng.integers(1, 200, 5000)
    w = workloads.make_random(lens.size, list(lens), 600, seed=19)
    want_c, want_e = oracle.sdtw_f32(w.queries, w.lens, w.reference, 0)
    c, e = gpu_forward(w, 0, flags=P.SDTW_F_PERSISTENT)
    assert_bit_exact(c, e, want_c, want_e, "5000 short queries")
    c2, e2 = gpu_forward(w, 0)
    assert_bit_exact(c2, e2, want_c, want_e, "5000 short queries, plain launch")


def test_uneven_batch_subset():
    """4,096 queries of 250..4,000 samples against 200,000: whole batch in one
    persistent launch; a seeded subset (with the shortest and the longest)
    checked against the oracle."""
    import paper_2403_06931_amd as P
    w = workloads.make_config(3)
    c, e = gpu_forward(w, 0, flags=P.SDTW_F_PERSISTENT)
    idx = workloads.subset_indices(w, 24, include_extremes=True)
    sub = w.subset(idx)
    want_c, want_e = oracle.sdtw_f32(sub.queries, sub.lens, sub.reference, 0)
    assert_bit_exact(c[idx], e[idx], want_c, want_e, "uneven batch subset")


def test_graph_replays_match_eager():
    import paper_2403_06931_amd as P
    lens = list(np.random.default_rng(8).integers(100, 3000, 40))
    w = workloads.make_random(len(lens), lens, 20000, seed=23)
    q, l, r = to_dev(w)
    eager_c, eager_e = P.sdtw_forward(q, w.lens, l, r, 0, flags=P.SDTW_F_PERSISTENT)
    eager_c, eager_e = eager_c.cpu().numpy(), eager_e.cpu().numpy()
    g = P.ForwardGraph(q, w.lens, l, r, 0)
    other = workloads.make_random(len(lens), lens, 20000, seed=29)
    oq = torch.from_numpy(other.queries).to(q.device)
    for rep in range(3):
        c, e = g.replay()
        torch.cuda.synchronize()
        assert_bit_exact(c.cpu().numpy(), e.cpu().numpy(), eager_c, eager_e, f"replay {rep}")
        # eager work between replays
        x = torch.randn(1 << 20, device=q.device).sum()
        torch.cuda.synchronize()
        del x
    # new query values in place: the replay follows them
    q.copy_(oq)
    c, e = g.replay()
    torch.cuda.synchronize()
    want_c, want_e = oracle.sdtw_f32(other.queries, other.lens, w.reference, 0)
    assert_bit_exact(c.cpu().numpy(), e.cpu().numpy(), want_c, want_e, "replay after refill")


def test_persistent_grid_sizes():
    """Every persistent grid size (1, 2, 3, 4 and 8 resident wavefronts per
    SIMD) gives the oracle's results bit for bit, on a ragged batch with
    multi-pass queries (one row-buffer slot per workgroup) and on more
    queries than any of the grids has workgroups."""
    import paper_2403_06931_amd as P
    lens = [1, 5, 64, 65, 700, 2049, 300, 4000, 3, 1500, 513, 2600, 90, 1, 8, 1024]
    w = workloads.make_random(len(lens), lens, 3001, seed=613)
    want_c, want_e = oracle.sdtw_f32(w.queries, w.lens, w.reference, 0)
    rng = np.random.default_rng(7)
    many = workloads.make_random(9000, list(rng.integers(1, 120, 9000)), 400, seed=614)
    many_c, many_e = oracle.sdtw_f32(many.queries, many.lens, many.reference, 0)
    for v in (6, 1):     # one-wavefront and four-wavefront tiles
        for wps in (1, 2, 3, 4, 8):
            flags = P.SDTW_F_PERSISTENT | P.SDTW_F_WAVES_PER_SIMD(wps)
            print(f"variant {P.sdtw_variant_info(v)} {wps} waves per SIMD", flush=True)
            c, e = gpu_forward(w, 0, variant=v, flags=flags)
            assert_bit_exact(c, e, want_c, want_e, f"variant {v}, {wps} per SIMD")
            c, e = gpu_forward(many, 0, variant=v, flags=flags)
            assert_bit_exact(c, e, many_c, many_e, f"9000 queries, variant {v}, {wps} per SIMD")
