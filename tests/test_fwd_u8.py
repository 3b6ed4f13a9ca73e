"""GPU parity of the uint8-code forward (sdtw_forward_u8: codebook from the
reference, codes of both sides, exact integer DP) against the quantisation
oracle (the binary32 DP of the codes): identical codebook, bit-exact cost (in
step^2 units) and end position, every compiled tile variant, ragged and degenerate shapes, values
beyond the codebook's clip, and the full 512 x 2,000 vs 100,000 shape on
sampled queries."""
import numpy as np
import pytest
import torch

import oracle.quant as Q
import workloads
from gpu_util import to_dev

pytestmark = pytest.mark.gpu


def _variants():
    import paper_2403_06931_amd as P
    return list(range(P.sdtw_variant_count()))


def _gpu_u8(w, variant=-1):
    import paper_2403_06931_amd as P
    q, l, r = to_dev(w)
    cost, end, book = P.sdtw_forward_u8(q, w.lens, l, r, variant=variant)
    torch.cuda.synchronize()
    return cost.cpu().numpy(), end.cpu().numpy(), tuple(book.cpu().numpy())


def _check(w, got, what, want=None):
    want_c, want_e, (lo, hi) = Q.sdtw_u8(w.queries, w.lens, w.reference) if want is None else want
    c, e, book = got
    assert book == (lo, hi), (what, book, (lo, hi))
    bad = np.nonzero((c.view(np.uint32) != want_c.view(np.uint32)) | (e != want_e))[0]
    assert bad.size == 0, (f"{what}: {bad.size} mismatches, first {bad[:8].tolist()}: gpu "
                           f"{c[bad[:8]].tolist()} {e[bad[:8]].tolist()} | oracle "
                           f"{want_c[bad[:8]].tolist()} {want_e[bad[:8]].tolist()}")


def test_u8_small_config_all_variants():
    w = workloads.make_config(0)
    for v in _variants():
        print(f"u8 config 0 variant {v}", flush=True)
        _check(w, _gpu_u8(w, v), f"u8 variant {v}")


def test_u8_ragged_all_variants():
    lens = [1, 5, 64, 65, 700, 2049, 4000, 300, 3]
    w = workloads.make_random(len(lens), lens, 6001, seed=919)
    for v in _variants():
        print(f"u8 ragged variant {v}", flush=True)
        _check(w, _gpu_u8(w, v), f"u8 ragged variant {v}")


def test_u8_clipped_and_degenerate():
    """Values scaled past the codebook's clip (end codes), queries longer than
    a short reference, a one-sample reference and a constant one."""
    lens = [50, 400, 1300]
    w = workloads.make_random(len(lens), lens, 2000, seed=920)
    ws = w.__class__(**{**w.__dict__, "queries": (w.queries * 3).astype(np.float32),
                        "reference": (w.reference * 3).astype(np.float32)})
    assert np.abs(ws.reference).max() > 4.0
    for v in (-1, 1, 19):
        print(f"u8 clipped variant {v}", flush=True)
        _check(ws, _gpu_u8(ws, v), f"u8 clipped variant {v}")
    # a query alternating between the end codes: sums pass 2^24, so the
    # binary32 DP of the codes rounds (both sides identically)
    alt = np.tile(np.array([-10.0, 10.0], np.float32), 2000)
    rng = np.random.default_rng(923)
    wa = w.__class__(**{**w.__dict__, "queries": alt, "lens": np.array([4000], np.int32),
                        "reference": workloads.random_walk(rng, 3000).astype(np.float32),
                        "excerpt_start": np.array([-1], np.int64)})
    want = Q.sdtw_u8(wa.queries, wa.lens, wa.reference)
    assert want[0][0] > 2 ** 24
    print("u8 alternating end codes", flush=True)
    _check(wa, _gpu_u8(wa), "u8 sums past 2^24", want=want)
    rng = np.random.default_rng(921)
    for r in (workloads.random_walk(rng, 300), np.zeros(1), np.full(64, 0.25)):
        wr = w.__class__(**{**w.__dict__, "reference": np.asarray(r, np.float32)})
        print(f"u8 reference of {wr.ref_len}", flush=True)
        _check(wr, _gpu_u8(wr), f"u8 reference {wr.ref_len}")


def test_u8_full_size_sampled():
    """512 x 2,000 vs 100,000 in the library's choice and in the tile the
    benchmark's headline uses; 8 sampled queries against the oracle (with the
    codebook of the whole reference)."""
    w = workloads.make_config(1)
    idx = workloads.subset_indices(w, 8, seed=14)
    sub = w.subset(idx)
    want = Q.sdtw_u8(sub.queries, sub.lens, w.reference)
    for v in (-1, 1):
        print(f"u8 full size variant {v}", flush=True)
        c, e, book = _gpu_u8(w, v)
        _check(sub, (c[idx], e[idx], book), f"u8 512x2000 variant {v}", want=want)


def test_u8_uneven_batch_subset():
    """4,096 queries of 250..4,000 samples against 200,000 (offset table
    path); a seeded subset with the shortest and longest against the oracle,
    which codes the subset with the codebook of the whole reference."""
    w = workloads.make_config(3)
    idx = workloads.subset_indices(w, 8, seed=16, include_extremes=True)
    sub = w.subset(idx)
    want = Q.sdtw_u8(sub.queries, sub.lens, w.reference)
    print("u8 uneven batch", flush=True)
    c, e, book = _gpu_u8(w)
    _check(sub, (c[idx], e[idx], book), "u8 uneven batch subset", want=want)
