"""GPU forward parity: the HIP path (through the C ABI) against the CPU
oracle, bit for bit in FP32 (cost bits and end position), and against the
FP64 oracle within 1e-5 relative."""
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
def test_small_config_all_variants(kind):
    w = workloads.make_config(0)
    want_c, want_e = oracle.sdtw_f32(w.queries, w.lens, w.reference, kind)
    for v in _variants():
        print(f"variant {v} kind {kind}", flush=True)
        c, e = gpu_forward(w, kind, variant=v)
        assert_bit_exact(c, e, want_c, want_e, f"variant {v}")


RAGGED_LENS = [1, 2, 63, 64, 65, 300, 511, 512, 513, 1100, 2047, 2048, 2049, 2600]


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("ref_len", [777, 1024 + 3])
def test_ragged_lengths_all_variants(kind, ref_len):
    """Lengths straddling lane, wave and pass boundaries of every variant;
    reference lengths that leave a partial last tile."""
    w = workloads.make_random(len(RAGGED_LENS), RAGGED_LENS, ref_len, seed=101 + ref_len,
                              excerpt_every=0)
    want_c, want_e = oracle.sdtw_f32(w.queries, w.lens, w.reference, kind)
    for v in _variants():
        print(f"variant {v} kind {kind} M {ref_len}", flush=True)
        c, e = gpu_forward(w, kind, variant=v)
        assert_bit_exact(c, e, want_c, want_e, f"variant {v}")


@pytest.mark.parametrize("ref_len", [1, 2, 5, 9, 64])
def test_tiny_references(ref_len):
    w = workloads.make_random(5, [1, 3, 40, 129, 700], 50, seed=7, excerpt_every=0)
    r = np.ascontiguousarray(w.reference[:ref_len])
    w.reference = r
    want_c, want_e = oracle.sdtw_f32(w.queries, w.lens, r, 0)
    for v in _variants():
        c, e = gpu_forward(w, 0, variant=v)
        assert_bit_exact(c, e, want_c, want_e, f"variant {v} M {ref_len}")


def test_exact_excerpts_cost_zero():
    rng = np.random.default_rng(3)
    ref = workloads.random_walk(rng, 20000).astype(np.float32)
    starts = [0, 17, 5000, 19000 - 900]
    lens = [100, 2000, 900, 900]
    qs = np.concatenate([ref[a:a + n] for a, n in zip(starts, lens)])
    w = workloads.Workload("excerpts", qs, np.array(lens, np.int32), ref, (0,),
                           np.array(starts, np.int64))
    c, e = gpu_forward(w, 0)
    assert np.all(c == 0)
    assert e.tolist() == [a + n - 1 for a, n in zip(starts, lens)]


def test_variants_bit_identical_and_permutation_invariant():
    w = workloads.make_random(24, list(np.random.default_rng(5).integers(1, 3000, 24)), 5000,
                              seed=17)
    base_c, base_e = gpu_forward(w, 0, variant=0)
    for v in _variants()[1:]:
        c, e = gpu_forward(w, 0, variant=v)
        assert_bit_exact(c, e, base_c, base_e, f"variant {v} vs 0")
    perm = np.random.default_rng(9).permutation(w.batch)
    wp = w.subset(perm)
    c, e = gpu_forward(wp, 0)
    assert_bit_exact(c, e, base_c[perm], base_e[perm], "permuted batch")


def _fp64_check(c32, c64):
    rel = np.abs(c32.astype(np.float64) - c64) / np.maximum(np.abs(c64), 1e-6)
    assert np.all(rel <= 1e-5), rel.max()


def test_paper_shape_sampled():
    """512 x 2,000 against 100,000 (the paper's Section 6 shape): the whole
    batch on the GPU, in the library's own choice and in the tile the
    benchmark's tuner picks on this shape ((8, 8, 4, 32) with LDS lane
    exchange); eight sampled queries checked against the oracle."""
    import paper_2403_06931_amd as P
    w = workloads.make_config(1)
    idx = workloads.subset_indices(w, 8)
    sub = w.subset(idx)
    want_c, want_e = oracle.sdtw_f32(sub.queries, sub.lens, sub.reference, 0)
    c64, _ = oracle.sdtw_f64(sub.queries, sub.lens, sub.reference, 0)
    headline = [v for v in range(P.sdtw_variant_count())
                if P.sdtw_variant_info(v) == (8, 8, 4, 32, 1)]
    for v in [-1] + headline:
        c, e = gpu_forward(w, 0, variant=v)
        assert_bit_exact(c[idx], e[idx], want_c, want_e, f"512x2000 vs 100k, variant {v}")
        _fp64_check(c[idx], c64)
        # every result is a real last-row value: end inside the reference, finite cost
        assert np.all(np.isfinite(c)) and np.all((e >= 0) & (e < w.ref_len))


@pytest.mark.parametrize("kind", [0, 1])
def test_long_reference_sampled(kind):
    """512 x 2,000 against a 2,000,000-sample reference: streaming the
    reference through the LDS ring; four sampled queries checked."""
    w = workloads.make_config(2)
    c, e = gpu_forward(w, kind)
    idx = workloads.subset_indices(w, 4, seed=11 + kind)
    sub = w.subset(idx)
    want_c, want_e = oracle.sdtw_f32(sub.queries, sub.lens, sub.reference, kind)
    assert_bit_exact(c[idx], e[idx], want_c, want_e, f"2M reference kind {kind}")


def _all_variants_bit_exact(w, kind):
    want_c, want_e = oracle.sdtw_f32(w.queries, w.lens, w.reference, kind)
    for v in _variants():
        c, e = gpu_forward(w, kind, variant=v)
        assert_bit_exact(c, e, want_c, want_e, f"{w.name} kind {kind} variant {v}")
    return want_c, want_e


@pytest.mark.parametrize("kind", [0, 1])
def test_small_integer_ties_all_variants(kind):
    """Small-integer queries and references: exact ties in the cell costs, in
    every three-way minimum and along the last row, so the end position must
    be the first minimiser (the smallest index) on every variant.  A second
    batch uses a periodic reference in which each query occurs many times at
    cost 0."""
    rng = np.random.default_rng(404 + kind)
    lens = [1, 3, 64, 65, 200, 513, 1100, 2049]
    ref = rng.integers(-2, 3, 3001).astype(np.float32)
    qs = rng.integers(-2, 3, sum(lens)).astype(np.float32)
    w = workloads.Workload("small-integers", qs, np.array(lens, np.int32), ref, (kind,),
                           np.full(len(lens), -1, np.int64))
    want_c, want_e = _all_variants_bit_exact(w, kind)
    # the data do tie: some last row attains its minimum more than once
    ties = 0
    for b in range(2):
        row = oracle.last_row_f32(w.query(b), ref, kind)
        ties += int(np.count_nonzero(row == row.min()) > 1)
    assert ties > 0

    period = np.array([0, 1, 2, 1, -1, -2, 0, 2], np.float32)
    ref = np.tile(period, 400)
    lens = [5, 8, 30, 64, 129, 700]
    qs = np.concatenate([np.tile(period, n // 8 + 2)[3:3 + n] for n in lens]).astype(np.float32)
    w = workloads.Workload("periodic", qs, np.array(lens, np.int32), ref, (kind,),
                           np.full(len(lens), -1, np.int64))
    want_c, want_e = _all_variants_bit_exact(w, kind)
    assert np.all(want_c == 0)


@pytest.mark.parametrize("kind,scale", [(0, 1e-20), (0, 3e-19), (1, 2e-39)])
def test_subnormal_values_all_variants(kind, scale):
    """Inputs scaled so that cell costs (squared: (q - r)^2 near 1e-40) or the
    inputs themselves (absolute: values near 1e-39) are subnormal binary32
    numbers; both sides keep subnormals, so results stay bit-exact."""
    w = workloads.make_random(6, [1, 2, 40, 300, 700, 1500], 2500, seed=606, excerpt_every=0)
    w.queries = (w.queries.astype(np.float64) * scale).astype(np.float32)
    w.reference = (w.reference.astype(np.float64) * scale).astype(np.float32)
    tiny = np.finfo(np.float32).tiny
    t = (w.queries[:43, None] - w.reference[None, :]).astype(np.float32)
    c = (t * t).astype(np.float32) if kind == 0 else np.abs(t)
    assert np.any((c > 0) & (c < tiny)), "no subnormal cell cost in the sample"
    want_c, want_e = _all_variants_bit_exact(w, kind)
    assert np.any((want_c > 0) & (want_c < tiny)), "no subnormal result"
