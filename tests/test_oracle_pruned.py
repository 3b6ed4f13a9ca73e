"""Pins of the pruned-cost oracle (Section 8's early pruning: after the
subtraction t = q - r, a pair with |t| > tau costs +inf; otherwise t*t).

- brute force: every warp path enumerated in pure Python with the pruned cost,
  folded left to right in FP32, equals the oracle bit for bit (cost and end
  position), including thresholds equal to a pair's |t| (not pruned: the
  comparison is strict), zero, negative and infinite thresholds;
- tau = +inf, and any tau >= max |q - r|, is the squared-cost oracle exactly;
- the walk-back path of the squared-cost DP survives any tau at or above the
  largest |t| on it, so there the pruned cost and end position equal the
  exact ones; below it the pruned cost can only be larger, and the cost is
  non-increasing in tau;
- tau < 0 prunes every pair: cost +inf, end position 0.

Nothing here takes an expected value from the oracle under test: the brute
force is independent, and the other pins compare against the squared-cost
oracle, which test_oracle_bruteforce.py pins on its own.
"""
import numpy as np
import pytest

import oracle
import workloads


def _c32_pruned(q, r, tau):
    t = np.float32(q) - np.float32(r)
    if abs(t) > np.float32(tau):
        return np.float32(np.inf)
    return np.float32(t * t)


def brute_force_pruned(q, r, tau):
    """Best FP32 left-to-right fold over all warp paths from row 1 to row N,
    per end column; returns (cost, first argmin)."""
    n, m = len(q), len(r)
    c = [[_c32_pruned(q[i], r[j], tau) for j in range(m)] for i in range(n)]
    best = [np.float32(np.inf)] * m

    def walk(i, j, acc):
        if i == n - 1 and acc < best[j]:
            best[j] = acc
        for di, dj in ((1, 0), (0, 1), (1, 1)):
            ni, nj = i + di, j + dj
            if ni < n and nj < m:
                walk(ni, nj, np.float32(acc + c[ni][nj]))

    for a in range(m):
        walk(0, a, c[0][a])
    best = np.array(best, dtype=np.float32)
    return best.min(), int(np.argmin(best))


def _cases():
    rng = np.random.default_rng(8_2024)
    out = []
    for t in range(48):
        n = int(rng.integers(1, 5))
        m = int(rng.integers(1, 8))
        if t % 2 == 0:
            # small integers: |t| lands exactly on integer thresholds
            q = rng.integers(-3, 4, n).astype(np.float32)
            r = rng.integers(-3, 4, m).astype(np.float32)
        else:
            q = rng.standard_normal(n).astype(np.float32)
            r = rng.standard_normal(m).astype(np.float32)
        out.append((q, r))
    return out


@pytest.mark.parametrize("tau", [0.0, 0.5, 1.0, 1.5, 2.0, 3.0, -1.0, np.inf])
def test_pruned_equals_brute_force_bit_exact(tau):
    for q, r in _cases():
        want, arg = brute_force_pruned(q, r, tau)
        cost, end = oracle.sdtw_pruned_f32(q, [q.size], r, tau)
        assert cost[0].tobytes() == np.float32(want).tobytes(), (q, r, tau, cost, want)
        assert end[0] == arg, (q, r, tau, end, arg)


def test_threshold_is_strict():
    # |q - r| = 1 everywhere: tau = 1 keeps every pair, the next float below prunes all
    q = np.array([0.0, 0.0, 0.0], np.float32)
    r = np.array([1.0, -1.0, 1.0, -1.0], np.float32)
    cost, end = oracle.sdtw_pruned_f32(q, [3], r, 1.0)
    exact, eend = oracle.sdtw_f32(q, [3], r, oracle.SQUARED)
    assert cost[0] == exact[0] == np.float32(3.0) and end[0] == eend[0]
    below = np.nextafter(np.float32(1.0), np.float32(0.0))
    cost, end = oracle.sdtw_pruned_f32(q, [3], r, below)
    assert np.isinf(cost[0]) and end[0] == 0


def _medium():
    w = workloads.make_random(6, 96, 700, seed=77)
    return w.queries, w.lens, w.reference


def test_infinite_or_wide_threshold_is_the_squared_cost():
    q, lens, r = _medium()
    exact_c, exact_e = oracle.sdtw_f32(q, lens, r, oracle.SQUARED)
    wide = float(max(abs(q.max() - r.min()), abs(r.max() - q.min()))) + 1.0
    for tau in (np.inf, wide):
        c, e = oracle.sdtw_pruned_f32(q, lens, r, tau)
        assert c.tobytes() == exact_c.tobytes()
        assert np.array_equal(e, exact_e)


def test_optimal_path_survives_its_largest_difference():
    q, lens, r = _medium()
    off = np.concatenate([[0], np.cumsum(lens)])
    for b in range(lens.size):
        qb = q[off[b]:off[b + 1]]
        exact_c, exact_e = oracle.sdtw_f32(qb, [qb.size], r, oracle.SQUARED)
        pi, pj = oracle.path_f32(qb, r, oracle.SQUARED)
        delta = np.abs(qb[pi] - r[pj]).astype(np.float32).max()      # largest |t| on the path
        c, e = oracle.sdtw_pruned_f32(qb, [qb.size], r, delta)
        assert c[0].tobytes() == exact_c[0].tobytes() and e[0] == exact_e[0]
        # below delta: never cheaper than the exact cost, and monotone in tau
        prev = np.float32(np.inf)
        for tau in (0.05, 0.25, 0.5, 1.0, float(delta)):
            c_tau, _ = oracle.sdtw_pruned_f32(qb, [qb.size], r, tau)
            assert c_tau[0] >= exact_c[0]
            assert c_tau[0] <= prev
            prev = c_tau[0]


def test_negative_threshold_prunes_everything():
    q, lens, r = _medium()
    c, e = oracle.sdtw_pruned_f32(q, lens, r, -0.5)
    assert np.all(np.isinf(c)) and np.all(e == 0)


def test_nan_threshold_is_rejected():
    with pytest.raises(ValueError):
        oracle.sdtw_pruned_f32(np.zeros(2, np.float32), [2], np.zeros(3, np.float32), np.nan)
