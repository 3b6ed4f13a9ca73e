"""Invariants and closed forms that pin the CPU oracle (Section 2, Eq. (1)).

Every expected value here is computed from a plain definition with NumPy
FP32/FP64 operations, never by the oracle itself.
"""
import numpy as np
import pytest

import oracle
import workloads


def _c32(q, r, kind):
    t = (np.float32(q) - np.asarray(r, np.float32)).astype(np.float32)
    return (t * t).astype(np.float32) if kind == 0 else np.abs(t)


def _fold32(costs):
    """Left-to-right FP32 sum of a path's cell costs."""
    acc = np.float32(costs[0])
    for c in costs[1:]:
        acc = np.float32(acc + np.float32(c))
    return acc


@pytest.mark.parametrize("kind", [0, 1])
def test_single_row_closed_form(kind):
    # N = 1: the free start makes D(1,j) = c(q_1, r_j), so the cost is the
    # smallest local cost and the end position its first index.
    rng = np.random.default_rng(5)
    for m in (1, 2, 7, 300):
        r = rng.standard_normal(m).astype(np.float32)
        q = rng.standard_normal(1).astype(np.float32)
        c = _c32(q[0], r, kind)
        cost, end = oracle.sdtw_f32(q, [1], r, kind)
        assert cost[0].tobytes() == c.min().tobytes()
        assert end[0] == int(np.argmin(c))
    # duplicated minimum: smallest index wins
    r = np.array([2, 0, 2, 5], np.float32)
    cost, end = oracle.sdtw_f32(np.array([2], np.float32), [1], r, kind)
    assert cost[0] == 0 and end[0] == 0


@pytest.mark.parametrize("kind", [0, 1])
def test_exact_excerpt_costs_zero(kind):
    rng = np.random.default_rng(11)
    r = workloads.random_walk(rng, 5000).astype(np.float32)
    for n, a in ((1, 17), (40, 0), (64, 1234), (300, 4700), (500, 4500)):
        q = r[a:a + n].copy()
        cost, end = oracle.sdtw_f32(q, [n], r, kind)
        assert cost[0] == 0.0
        assert end[0] == a + n - 1
        c64, e64 = oracle.sdtw_f64(q, [n], r, kind)
        assert c64[0] == 0.0 and e64[0] == a + n - 1


@pytest.mark.parametrize("kind", [0, 1])
def test_path_upper_bounds(kind):
    """cost <= any particular path's FP32 fold, exactly (the DP is the min over
    all folds): vertical paths, diagonal paths (the sliding-window distance of
    the Euclidean baseline in Section 2) and the global DTW alignment."""
    w = workloads.make_random(6, 24, 400, seed=3)
    cost, _ = oracle.sdtw_f32(w.queries, w.lens, w.reference, kind)
    r = w.reference
    for b in range(w.batch):
        q = w.query(b)
        n = q.size
        vert = min(_fold32([_c32(q[i], r[j:j + 1], kind)[0] for i in range(n)])
                   for j in range(0, r.size, 7))
        diag = min(_fold32([_c32(q[i], r[a + i:a + i + 1], kind)[0] for i in range(n)])
                   for a in range(0, r.size - n, 5))
        glob = oracle.dtw_f32(q, r, kind)
        assert cost[b] <= vert
        assert cost[b] <= diag
        assert cost[b] <= glob


@pytest.mark.parametrize("kind", [0, 1])
def test_reference_extension_is_monotone(kind):
    rng = np.random.default_rng(9)
    w = workloads.make_random(4, 30, 300, seed=4)
    base, _ = oracle.sdtw_f32(w.queries, w.lens, w.reference, kind)
    pre = rng.standard_normal(50).astype(np.float32)
    post = rng.standard_normal(70).astype(np.float32)
    for ext in (np.concatenate([pre, w.reference]), np.concatenate([w.reference, post]),
                np.concatenate([pre, w.reference, post])):
        c, _ = oracle.sdtw_f32(w.queries, w.lens, ext, kind)
        assert np.all(c <= base)


@pytest.mark.parametrize("kind", [0, 1])
def test_end_position_is_first_minimum_of_last_row(kind):
    w = workloads.make_random(5, 16, 200, seed=8)
    cost, end = oracle.sdtw_f32(w.queries, w.lens, w.reference, kind)
    for b in range(w.batch):
        row = oracle.last_row_f32(w.query(b), w.reference, kind)
        assert cost[b].tobytes() == row.min().tobytes()
        assert end[b] == int(np.argmin(row))


def _gamma(k):
    u = 2.0 ** -24
    return k * u / (1 - k * u)


@pytest.mark.parametrize("kind", [0, 1])
def test_f32_f64_within_rounding_bound(kind):
    """|c32 - c64| <= gamma_{L+2} * c64, L the longest possible path (N + M)."""
    w = workloads.make_config(0)
    for k in (0, 1):
        w2 = workloads.make_random(8, 64 * (k + 1), 1024, seed=21 + k)
        for ww in (w, w2):
            c32, e32 = oracle.sdtw_f32(ww.queries, ww.lens, ww.reference, kind)
            c64, e64 = oracle.sdtw_f64(ww.queries, ww.lens, ww.reference, kind)
            bound = _gamma(int(ww.lens.max()) + ww.ref_len + 2) * c64 + 1e-30
            assert np.all(np.abs(c32.astype(np.float64) - c64) <= bound)


def test_batch_equals_one_by_one():
    w = workloads.make_random(7, [5, 33, 1, 70, 12, 64, 2], 150, seed=13)
    cost, end = oracle.sdtw_f32(w.queries, w.lens, w.reference, 0, nthreads=3)
    for b in range(w.batch):
        c1, e1 = oracle.sdtw_f32(w.query(b), [int(w.lens[b])], w.reference, 0, nthreads=1)
        assert c1[0].tobytes() == cost[b].tobytes() and e1[0] == end[b]


def test_query_longer_than_reference():
    rng = np.random.default_rng(2)
    q = rng.standard_normal(40).astype(np.float32)
    r = rng.standard_normal(6).astype(np.float32)
    cost, end = oracle.sdtw_f32(q, [40], r, 0)
    assert np.isfinite(cost[0]) and 0 <= end[0] < 6
    # a vertical path through the single best column bounds it
    assert cost[0] <= min(_fold32([_c32(q[i], r[j:j + 1], 0)[0] for i in range(40)])
                          for j in range(6))


def test_rejects_bad_arguments():
    with pytest.raises(ValueError):
        oracle.sdtw_f32(np.zeros(3, np.float32), [4], np.zeros(5, np.float32))
    with pytest.raises(ValueError):
        oracle.sdtw_f32(np.zeros(3, np.float32), [3], np.zeros(5, np.float32), kind=2)
