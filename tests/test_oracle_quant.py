"""Pins of the uint8 quantisation oracle (Section 8's codebook proposal).

- codebook: the reference's extremes clipped to [-4, 4], checked on arrays
  worked by hand, including the degenerate cases (constant reference, all
  values beyond the clip);
- codes: hand-worked values with a unit step (ties to even, clamping at both
  ends), and the nearest-level bound |lo + code * step - x| <= step / 2 for
  every value inside [lo, hi];
- the exact-integer DP on codes equals a pure-Python enumeration of all warp
  paths, and equals the binary32 DP of the codes (the quantised forward's
  definition, pinned on its own by test_oracle_bruteforce.py) while the sums
  stay below 2^24;
- approximation: along the exact optimal path of the binary32 squared-cost
  DP, the coded costs sum to at least the code DP's minimum, and that sum is
  within the quantisation error of the path's exact cost, so
  cost * step^2 <= exact + sum over the path of step * (2|t| + step).
"""
import numpy as np
import pytest

import oracle
import oracle.quant as Q
import workloads


def test_codebook_by_hand():
    assert Q.codebook(np.array([-5.0, 0.5, 2.0])) == (np.float32(-4.0), np.float32(2.0))
    assert Q.codebook(np.array([-1.25, 3.5, 7.0])) == (np.float32(-1.25), np.float32(4.0))
    assert Q.codebook(np.array([1.0, 1.0])) == (np.float32(1.0), np.float32(1.0))
    lo, hi = Q.codebook(np.array([10.0, 11.0]))            # everything beyond the clip
    assert (lo, hi) == (np.float32(10.0), np.float32(4.0))
    assert np.all(Q.encode(np.array([10.0, 11.0, -3.0]), lo, hi) == 0)
    assert np.all(Q.encode(np.array([1.0, 5.0]), np.float32(1.0), np.float32(1.0)) == 0)


def test_codes_by_hand():
    lo, hi = np.float32(0.0), np.float32(255.0)             # step 1
    x = np.array([0.0, 2.5, 3.5, 254.5, 255.0, -1.0, 300.0, 0.49, 0.51, 127.5])
    want = np.array([0, 2, 4, 254, 255, 0, 255, 0, 1, 128], np.uint8)
    assert np.array_equal(Q.encode(x, lo, hi), want)
    lo, hi = np.float32(-4.0), np.float32(4.0)             # step 8/255
    assert Q.encode(np.array([-4.0]), lo, hi)[0] == 0
    assert Q.encode(np.array([4.0]), lo, hi)[0] == 255
    assert Q.encode(np.array([0.0]), lo, hi)[0] == 128     # 127.5 rounds to even


def test_nearest_level_bound():
    rng = np.random.default_rng(5)
    r = rng.standard_normal(5000).astype(np.float32) * 1.7
    lo, hi = Q.codebook(r)
    step = (np.float64(hi) - np.float64(lo)) / 255.0
    x = rng.uniform(lo, hi, 20000).astype(np.float32)
    c = Q.encode(x, lo, hi).astype(np.float64)
    err = np.abs(np.float64(lo) + c * step - x.astype(np.float64))
    assert err.max() <= step / 2 * (1 + 1e-9)


def _brute_codes(q, r):
    n, m = len(q), len(r)
    c = [[(int(q[i]) - int(r[j])) ** 2 for j in range(m)] for i in range(n)]
    best = [None] * m

    def walk(i, j, acc):
        if i == n - 1 and (best[j] is None or acc < best[j]):
            best[j] = acc
        for di, dj in ((1, 0), (0, 1), (1, 1)):
            ni, nj = i + di, j + dj
            if ni < n and nj < m:
                walk(ni, nj, acc + c[ni][nj])

    for a in range(m):
        walk(0, a, c[0][a])
    k = min(range(m), key=lambda j: (best[j], j))
    return best[k], k


def test_code_dp_equals_brute_force():
    rng = np.random.default_rng(17)
    for t in range(80):
        n, m = int(rng.integers(1, 5)), int(rng.integers(1, 8))
        hi = 4 if t % 2 == 0 else 256                       # many ties, or the full range
        q = rng.integers(0, hi, n).astype(np.uint8)
        r = rng.integers(0, hi, m).astype(np.uint8)
        cost, end = oracle.sdtw_codes(q, [n], r)
        assert (cost[0], end[0]) == _brute_codes(q, r), (q, r)


def test_code_dp_equals_binary32_dp_on_codes():
    w = workloads.make_random(6, [40, 90, 130, 7, 64, 200], 900, seed=3)
    lo, hi = Q.codebook(w.reference)
    qc, rc = Q.encode(w.queries, lo, hi), Q.encode(w.reference, lo, hi)
    cost, end = oracle.sdtw_codes(qc, w.lens, rc)
    assert cost.max() < 2 ** 24                             # binary32 sums are exact
    fc, fe = oracle.sdtw_f32(qc.astype(np.float32), w.lens, rc.astype(np.float32),
                             oracle.SQUARED)
    assert np.array_equal(fc.astype(np.int64), cost)
    assert np.array_equal(fe, end)


def test_quantised_cost_within_error_of_exact_path():
    w = workloads.make_random(8, 120, 1500, seed=21)
    cost, end, (lo, hi) = Q.sdtw_u8(w.queries, w.lens, w.reference)
    step = (np.float64(hi) - np.float64(lo)) / 255.0
    qc, rc = Q.encode(w.queries, lo, hi), Q.encode(w.reference, lo, hi)
    exact, _ = oracle.sdtw_f64(w.queries, w.lens, w.reference, oracle.SQUARED)
    off = np.concatenate([[0], np.cumsum(w.lens)])
    inside = (w.reference >= lo).all() and (w.reference <= hi).all()
    for b in range(w.batch):
        qb = w.queries[off[b]:off[b + 1]]
        pi, pj = oracle.path_f32(qb, w.reference, oracle.SQUARED)
        coded = np.sum((qc[off[b] + pi].astype(np.int64) - rc[pj].astype(np.int64)) ** 2)
        assert cost[b] <= coded                             # the DP is a minimum over paths
        if inside and (qb >= lo).all() and (qb <= hi).all():
            t = np.abs(qb[pi].astype(np.float64) - w.reference[pj].astype(np.float64))
            assert cost[b] * step * step <= exact[b] + np.sum(step * (2 * t + step)) + 1e-9


def test_degenerate_reference_codes_everything_zero():
    q = np.array([0.3, -0.2, 1.0], np.float32)
    cost, end, (lo, hi) = Q.sdtw_u8(q, [3], np.full(5, 0.7, np.float32))
    assert lo == hi and cost[0] == 0 and end[0] == 0


@pytest.mark.parametrize("bad", [[0], [2, 0]])
def test_code_dp_rejects_bad_lengths(bad):
    with pytest.raises(ValueError):
        oracle.sdtw_codes(np.zeros(sum(bad), np.uint8), bad, np.zeros(3, np.uint8))
