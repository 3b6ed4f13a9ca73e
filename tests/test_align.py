"""GPU parity of the alignment-path output (sdtw_align): start position and
per-row matched reference ranges, bit-exact against the oracle's walk-back
(ties: diagonal, then up, then left)."""
import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu


def _oracle_rows(query, reference, kind):
    pi, pj = oracle.path_f32(query, reference, kind)
    n = len(query)
    lo = np.full(n, np.iinfo(np.int32).max, np.int64)
    hi = np.full(n, -1, np.int64)
    np.minimum.at(lo, pi, pj)
    np.maximum.at(hi, pi, pj)
    assert (hi >= 0).all()
    return int(lo[0]), lo.astype(np.int32), hi.astype(np.int32)


def _gpu_align(w, kind, K, idx=None):
    import paper_2403_06931_amd as P
    d = torch.device("cuda:0")
    q = torch.from_numpy(w.queries).to(d)
    l = torch.from_numpy(w.lens).to(d)
    r = torch.from_numpy(w.reference).to(d)
    ck = torch.empty(max(1, P.sdtw_checkpoint_floats(w.lens, w.ref_len, K)), dtype=torch.float32,
                     device=d)
    cost, end = P.sdtw_forward(q, w.lens, l, r, kind, ckpt=ck, ckpt_every=K,
                               flags=P.SDTW_F_CHECKPOINT)
    start, lo, hi = P.sdtw_align(q, w.lens, l, r, kind, cost, end, ck, K)
    torch.cuda.synchronize()
    return (cost.cpu().numpy(), end.cpu().numpy(), start.cpu().numpy(), lo.cpu().numpy(),
            hi.cpu().numpy())


def _check(w, kind, K, got, idx):
    cost, end, start, lo, hi = got
    off = np.concatenate([[0], np.cumsum(w.lens)])
    for b in idx:
        qb = w.queries[off[b]:off[b + 1]]
        s, want_lo, want_hi = _oracle_rows(qb, w.reference, kind)
        glo, ghi = lo[off[b]:off[b + 1]], hi[off[b]:off[b + 1]]
        assert start[b] == s, f"query {b}: start {start[b]} oracle {s}"
        assert np.array_equal(glo, want_lo), f"query {b}: row lower bounds differ"
        assert np.array_equal(ghi, want_hi), f"query {b}: row upper bounds differ"
        assert ghi[-1] == end[b]
        # a monotone connected path: consecutive rows touch
        assert np.all((ghi[:-1] == glo[1:]) | (ghi[:-1] == glo[1:] - 1))


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("K", [16, 64, 1024])
def test_align_ragged(kind, K):
    lens = [1, 2, 7, 64, 65, 300, 129, 1000]
    w = workloads.make_random(len(lens), lens, 2500, seed=71 + kind)
    print(f"align ragged kind {kind} K {K}", flush=True)
    got = _gpu_align(w, kind, K)
    _check(w, kind, K, got, range(len(lens)))


def test_align_small_config_both_kinds():
    w = workloads.make_config(0)
    for kind in (0, 1):
        got = _gpu_align(w, kind, 256)
        _check(w, kind, 256, got, range(w.batch))


def test_align_full_size_sampled():
    """256 queries of 1,000 samples against 50,000, checkpoints every 1,024
    columns: start positions of all queries against the oracle's gradient
    walk, full row ranges of a seeded sample of 12."""
    w = workloads.make_config(4)
    print("align full size", flush=True)
    got = _gpu_align(w, 0, 1024)
    _, _, start = oracle.sdtw_grad_f32(w.queries, w.lens, w.reference,
                                       np.ones(w.batch, np.float32), 0)[:3]
    assert np.array_equal(got[2], start)
    idx = workloads.subset_indices(w, 12, seed=5)
    _check(w, 0, 1024, got, idx)


def test_align_degenerate_shapes():
    """One-sample queries, a one-sample reference, queries longer than the
    reference."""
    import paper_2403_06931_amd as P
    for lens, m, seed in (([1, 1, 2], 50, 1), ([3, 1], 1, 2), ([40, 7], 16, 3)):
        rng = np.random.default_rng(seed)
        q = rng.standard_normal(sum(lens)).astype(np.float32)
        r = rng.standard_normal(m).astype(np.float32)
        w = workloads.Workload(name="degenerate", queries=q, lens=np.array(lens, np.int32),
                               reference=r, kinds=(0,), excerpt_start=None, description="")
        for kind in (0, 1):
            got = _gpu_align(w, kind, 16)
            _check(w, kind, 16, got, range(len(lens)))
