"""GPU parity of the pruned forward (sdtw_forward_pruned: squared cost, +inf
for a pair with |q - r| > tau, Section 8) against the pruned oracle: bit-exact
cost and end position, every compiled tile variant, plain and persistent
launches, thresholds on both sides of exact |q - r| values, and the full
512 x 2,000 vs 100,000 shape on sampled queries."""
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


def _gpu_pruned(w, tau, variant=-1, flags=0):
    import paper_2403_06931_amd as P
    q, l, r = to_dev(w)
    cost, end = P.sdtw_forward_pruned(q, w.lens, l, r, tau, variant=variant, flags=flags)
    torch.cuda.synchronize()
    return cost.cpu().numpy(), end.cpu().numpy()


@pytest.mark.parametrize("tau", [0.5, 2.0])
def test_pruned_small_config_all_variants(tau):
    import paper_2403_06931_amd as P
    w = workloads.make_config(0)
    want_c, want_e = oracle.sdtw_pruned_f32(w.queries, w.lens, w.reference, tau)
    for v in _variants():
        for flags in (0, P.SDTW_F_PERSISTENT):
            print(f"pruned config 0 variant {v} flags {flags} tau {tau}", flush=True)
            c, e = _gpu_pruned(w, tau, v, flags)
            assert_bit_exact(c, e, want_c, want_e, f"pruned variant {v} flags {flags}")


def test_pruned_ragged_all_variants():
    """Lengths from 1 to several row passes, and a query longer than the
    reference; tau = 1 on z-normalised data prunes about half the pairs."""
    lens = [1, 5, 64, 65, 700, 2049, 4000, 300, 3]
    w = workloads.make_random(len(lens), lens, 6001, seed=909)
    want_c, want_e = oracle.sdtw_pruned_f32(w.queries, w.lens, w.reference, 1.0)
    assert np.isfinite(want_c).any()
    for v in _variants():
        print(f"pruned ragged variant {v}", flush=True)
        c, e = _gpu_pruned(w, 1.0, v)
        assert_bit_exact(c, e, want_c, want_e, f"pruned ragged variant {v}")
    # queries longer than a 300-sample reference, and a 1-sample reference
    rng = np.random.default_rng(910)
    lens = [50, 400, 1300]
    q = np.concatenate([workloads.random_walk(rng, n) for n in lens])
    for m in (300, 1):
        r = workloads.random_walk(rng, m) if m > 1 else np.zeros(1)
        wl = w.__class__(**{**w.__dict__, "queries": q.astype(np.float32),
                            "lens": np.asarray(lens, np.int32),
                            "reference": np.asarray(r, np.float32),
                            "excerpt_start": np.full(len(lens), -1, np.int64)})
        want_c, want_e = oracle.sdtw_pruned_f32(wl.queries, wl.lens, wl.reference, 2.5)
        for v in (-1, 1, 19):
            print(f"pruned short reference {m} variant {v}", flush=True)
            c, e = _gpu_pruned(wl, 2.5, v)
            assert_bit_exact(c, e, want_c, want_e, f"pruned ref {m} variant {v}")


def test_pruned_threshold_edges():
    """Integer-valued inputs put many |q - r| exactly on integer thresholds
    (kept: the comparison is strict); +inf reproduces the squared-cost
    forward; a negative threshold prunes everything (+inf, end 0)."""
    rng = np.random.default_rng(31)
    lens = [7, 30, 130, 257]
    w = workloads.make_random(len(lens), lens, 800, seed=31)
    qi = rng.integers(-3, 4, w.queries.size).astype(np.float32)
    ri = rng.integers(-3, 4, w.reference.size).astype(np.float32)
    wi = w.__class__(**{**w.__dict__, "queries": qi, "reference": ri})
    for tau in (0.0, 1.0, 2.0, np.nextafter(np.float32(1.0), np.float32(0.0))):
        want_c, want_e = oracle.sdtw_pruned_f32(qi, w.lens, ri, tau)
        print(f"pruned edge tau {tau}", flush=True)
        c, e = _gpu_pruned(wi, float(tau))
        assert_bit_exact(c, e, want_c, want_e, f"pruned integer tau {tau}")
    c, e = _gpu_pruned(w, float("inf"))
    sc, se = gpu_forward(w, 0)
    assert_bit_exact(c, e, sc, se, "pruned tau=inf vs squared forward")
    want_c, want_e = oracle.sdtw_f32(w.queries, w.lens, w.reference, 0)
    assert_bit_exact(c, e, want_c, want_e, "pruned tau=inf vs squared oracle")
    c, e = _gpu_pruned(w, -1.0)
    assert np.all(np.isinf(c)) and np.all(e == 0)


def test_pruned_full_size_sampled():
    """512 x 2,000 vs 100,000 with tau = 2, in the library's choice and in the
    tile the benchmark times; 8 sampled queries against the oracle."""
    w = workloads.make_config(1)
    idx = workloads.subset_indices(w, 8, seed=13)
    sub = w.subset(idx)
    want_c, want_e = oracle.sdtw_pruned_f32(sub.queries, sub.lens, sub.reference, 2.0)
    for v in (-1, 1):
        print(f"pruned full size variant {v}", flush=True)
        c, e = _gpu_pruned(w, 2.0, v)
        assert_bit_exact(c[idx], e[idx], want_c, want_e, f"pruned 512x2000 variant {v}")


def test_pruned_uneven_batch_persistent_subset():
    """4,096 queries of 250..4,000 samples against 200,000 in one persistent
    launch with tau = 2; a seeded subset (shortest and longest included)
    checked against the oracle."""
    import paper_2403_06931_amd as P
    w = workloads.make_config(3)
    print("pruned uneven batch, persistent", flush=True)
    c, e = _gpu_pruned(w, 2.0, flags=P.SDTW_F_PERSISTENT)
    idx = workloads.subset_indices(w, 8, seed=15, include_extremes=True)
    sub = w.subset(idx)
    want_c, want_e = oracle.sdtw_pruned_f32(sub.queries, sub.lens, sub.reference, 2.0)
    assert_bit_exact(c[idx], e[idx], want_c, want_e, "pruned uneven batch subset")
