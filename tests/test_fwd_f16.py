"""GPU parity of the binary16 forward (sdtw_forward_f16, two queries per
packed value) against the binary16 oracle: bit-exact cost and end position,
every compiled tile variant, both cost kinds."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_util import assert_bit_exact, to_dev

pytestmark = pytest.mark.gpu


def _variants():
    import paper_2403_06931_amd as P
    return list(range(P.sdtw_variant_count()))


def _gpu_f16(w, kind, variant=-1, reference=None):
    import paper_2403_06931_amd as P
    q, l, r = to_dev(w)
    if reference is not None:
        r = reference
    cost, end = P.sdtw_forward_f16(q, w.lens, l, r, kind, variant=variant)
    torch.cuda.synchronize()
    return cost.cpu().numpy(), end.cpu().numpy()


@pytest.mark.parametrize("kind", [0, 1])
def test_f16_small_config_all_variants(kind):
    w = workloads.make_config(0)
    want_c, want_e = oracle.sdtw_f16(w.queries, w.lens, w.reference, kind)
    for v in _variants():
        print(f"f16 config 0 variant {v} kind {kind}", flush=True)
        c, e = _gpu_f16(w, kind, v)
        assert_bit_exact(c, e, want_c, want_e, f"f16 variant {v}")


@pytest.mark.parametrize("kind", [0, 1])
def test_f16_ragged_pairs_all_variants(kind):
    """Equal-length pairs of many lengths (several row passes for the
    longest), and an odd batch whose last query runs alone."""
    lens = [5, 5, 64, 64, 65, 65, 700, 700, 2049, 2049, 1, 1, 4000, 4000, 300, 300, 3]
    w = workloads.make_random(len(lens), lens, 6001, seed=404 + kind)
    want_c, want_e = oracle.sdtw_f16(w.queries, w.lens, w.reference, kind)
    for v in _variants():
        print(f"f16 ragged variant {v} kind {kind}", flush=True)
        c, e = _gpu_f16(w, kind, v)
        assert_bit_exact(c, e, want_c, want_e, f"f16 ragged variant {v}")


def test_f16_overflow_and_large_values():
    """Inputs scaled so that accumulated costs pass 65504 (binary16's largest
    finite value) for some queries: those costs are +inf on both sides."""
    lens = [40, 40, 200, 200]
    w = workloads.make_random(len(lens), lens, 900, seed=5)
    q = (w.queries * np.float32(100.0)).astype(np.float32)
    r = (w.reference * np.float32(100.0)).astype(np.float32)
    w2 = w.__class__(**{**w.__dict__, "queries": q, "reference": r})
    want_c, want_e = oracle.sdtw_f16(q, w.lens, r, 0)
    assert np.isinf(want_c).any() and np.isfinite(want_c).any()
    c, e = _gpu_f16(w2, 0)
    assert_bit_exact(c, e, want_c, want_e, "f16 overflow")


def test_f16_full_size_sampled():
    """512 x 2,000 vs 100,000 (the evaluation's shape) in the library's own
    variant choice; 8 sampled queries checked against the oracle."""
    w = workloads.make_config(1)
    print("f16 full size", flush=True)
    c, e = _gpu_f16(w, 0)
    idx = workloads.subset_indices(w, 8, seed=9)
    sub = w.subset(idx)
    want_c, want_e = oracle.sdtw_f16(sub.queries, sub.lens, sub.reference, 0)
    assert_bit_exact(c[idx], e[idx], want_c, want_e, "f16 512x2000 sample")


def test_f16_degenerate_shapes():
    """One-sample queries and reference, and queries longer than the reference."""
    for lens, m, seed in (([1, 1], 1, 1), ([1, 1, 5], 50, 2), ([40, 40], 16, 3)):
        rng = np.random.default_rng(seed)
        q = rng.standard_normal(sum(lens)).astype(np.float32)
        r = rng.standard_normal(m).astype(np.float32)
        w = workloads.Workload(name="degenerate", queries=q, lens=np.array(lens, np.int32),
                               reference=r, kinds=(0,), excerpt_start=None, description="")
        for kind in (0, 1):
            want_c, want_e = oracle.sdtw_f16(q, lens, r, kind)
            c, e = _gpu_f16(w, kind)
            assert_bit_exact(c, e, want_c, want_e, f"f16 {lens} vs {m}")


def test_f16_large_batch_offset_table():
    """More queries than the library sums in-kernel (16,384): the offsets come
    from the one-workgroup scan kernel."""
    rng = np.random.default_rng(12)
    pairs = rng.integers(1, 9, 8200)
    lens = np.repeat(pairs, 2)[:16401]           # 16,401 queries, an odd batch
    w = workloads.make_random(len(lens), list(lens), 300, seed=13, excerpt_every=0)
    want_c, want_e = oracle.sdtw_f16(w.queries, w.lens, w.reference, 0)
    c, e = _gpu_f16(w, 0)
    assert_bit_exact(c, e, want_c, want_e, "f16 16,401 queries")
