"""Pins of the CPU oracle against brute force and a hand-worked example.

The DP of Section 2, Eq. (1) (subsequence form) must equal the minimum, over
every warp path that starts anywhere in row 1 and ends in row N, of the path's
summed local cost.  In FP32 the DP equals that minimum *bit for bit* when each
path's costs are summed left to right from its start cell: rounding to
nearest is monotone (x <= y implies fl(x + c) <= fl(y + c)), so taking the
minimum before or after each rounded addition gives the same value.

Nothing here calls the oracle to produce an expected value: the brute force
below is an independent enumeration in pure Python, and the hand example is
a text fixture computed by hand.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _c32(q, r, kind):
    t = np.float32(q) - np.float32(r)
    return np.float32(t * t) if kind == 0 else np.float32(abs(t))


def brute_force_f32(q, r, kind):
    """Enumerate every warp path (steps down, right, diagonal) from any cell of
    row 1 to any cell of row N; fold each path's FP32 costs left to right.
    Returns (best per end column [M], argmin end column)."""
    n, m = len(q), len(r)
    c = [[_c32(q[i], r[j], kind) for j in range(m)] for i in range(n)]
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
    return best, int(np.argmin(best))


def brute_force_all_cells_f32(q, r, kind):
    """Brute-force minimum fold over all paths ending at every cell (i, j)."""
    n, m = len(q), len(r)
    c = [[_c32(q[i], r[j], kind) for j in range(m)] for i in range(n)]
    best = np.full((n, m), np.inf, dtype=np.float32)

    def walk(i, j, acc):
        if acc < best[i, j]:
            best[i, j] = acc
        for di, dj in ((1, 0), (0, 1), (1, 1)):
            ni, nj = i + di, j + dj
            if ni < n and nj < m:
                walk(ni, nj, np.float32(acc + c[ni][nj]))

    for a in range(m):
        walk(0, a, c[0][a])
    return best


def brute_force_exact(q, r, kind):
    """Same enumeration in exact rational arithmetic (for the FP64 oracle)."""
    n, m = len(q), len(r)

    def cost(i, j):
        t = Fraction(float(np.float32(q[i]))) - Fraction(float(np.float32(r[j])))
        return t * t if kind == 0 else abs(t)

    c = [[cost(i, j) for j in range(m)] for i in range(n)]
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
    return best


def _cases():
    rng = np.random.default_rng(20240306)
    cases = []
    for t in range(60):
        n = int(rng.integers(1, 5))
        m = int(rng.integers(1, 8))
        if t % 3 == 0:
            # small integers: many exact ties in costs, sums and the end position
            q = rng.integers(-2, 3, n).astype(np.float32)
            r = rng.integers(-2, 3, m).astype(np.float32)
        else:
            q = rng.standard_normal(n).astype(np.float32)
            r = rng.standard_normal(m).astype(np.float32)
        cases.append((q, r))
    # a few at the largest brute-force size
    for _ in range(4):
        cases.append((rng.standard_normal(5).astype(np.float32),
                      rng.standard_normal(8).astype(np.float32)))
    cases.append((np.array([1, 1, 1, 1, 1], np.float32), np.array([1] * 8, np.float32)))
    return cases


@pytest.mark.parametrize("kind", [0, 1])
def test_dp_equals_brute_force_bit_exact(kind):
    for q, r in _cases():
        best, arg = brute_force_f32(q, r, kind)
        row = oracle.last_row_f32(q, r, kind)
        assert row.tobytes() == best.tobytes(), (q, r, row, best)
        cost, end = oracle.sdtw_f32(q, [q.size], r, kind)
        assert cost[0].tobytes() == best[arg].tobytes()
        assert end[0] == arg


@pytest.mark.parametrize("kind", [0, 1])
def test_f64_oracle_against_exact_paths(kind):
    for q, r in _cases()[:30]:
        exact = brute_force_exact(q, r, kind)
        bmin = min(exact)
        arg = exact.index(bmin)
        cost, end = oracle.sdtw_f64(q, [q.size], r, kind)
        # binary64 sums of at most 12 terms: relative error far below 1e-14
        assert abs(Fraction(float(cost[0])) - bmin) <= Fraction(1, 10**14) * (bmin + 1)
        # the exact argmin may differ from the FP64 one only on a near-tie
        if end[0] != arg:
            assert abs(exact[end[0]] - bmin) <= Fraction(1, 10**12) * (bmin + 1)


def _read_golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split("=")
            vals[k.strip()] = [float(x) for x in v.split()]
    return vals


def test_hand_worked_example():
    g = _read_golden("hand_sdtw_3x6.txt")
    q = np.array(g["q"], np.float32)
    r = np.array(g["r"], np.float32)
    row = oracle.last_row_f32(q, r, 0)
    np.testing.assert_array_equal(row, np.array(g["squared.D3"], np.float32))
    # rows 1 and 2 are the last rows of the one- and two-row prefixes
    np.testing.assert_array_equal(oracle.last_row_f32(q[:1], r, 0), np.array(g["squared.D1"], np.float32))
    np.testing.assert_array_equal(oracle.last_row_f32(q[:2], r, 0), np.array(g["squared.D2"], np.float32))
    cost, end = oracle.sdtw_f32(q, [3], r, 0)
    assert cost[0] == g["squared.cost"][0] and end[0] == int(g["squared.end"][0])
    pi, pj = oracle.path_f32(q, r, 0)
    assert pi.tolist() == [int(x) for x in g["squared.path_rows"]]
    assert pj.tolist() == [int(x) for x in g["squared.path_refs"]]
    c, e, s, gq, gr = oracle.sdtw_grad_f32(q, [3], r, [1.0], 0)
    np.testing.assert_array_equal(gq, np.array(g["squared.grad_q"], np.float32))
    np.testing.assert_array_equal(gr, np.array(g["squared.grad_r"], np.float32))
    assert s[0] == int(g["squared.path_refs"][-1])
    np.testing.assert_array_equal(oracle.last_row_f32(q, r, 1), np.array(g["absolute.D3"], np.float32))
    cost, end = oracle.sdtw_f32(q, [3], r, 1)
    assert cost[0] == g["absolute.cost"][0] and end[0] == int(g["absolute.end"][0])


@pytest.mark.parametrize("kind", [0, 1])
def test_walk_back_tie_break(kind):
    """The walk-back (Section 2) from the first minimum of the last row follows
    the cheapest of (i-1,j-1), (i-1,j), (i,j-1); ties go to the diagonal, then
    up, then left.  The cell values come from the brute force above."""
    rng = np.random.default_rng(77)
    for t in range(80):
        n = int(rng.integers(1, 5))
        m = int(rng.integers(1, 7))
        q = rng.integers(-1, 2, n).astype(np.float32)
        r = rng.integers(-1, 2, m).astype(np.float32)
        D = brute_force_all_cells_f32(q, r, kind)
        i, j = n - 1, int(np.argmin(D[n - 1]))
        want = [(i, j)]
        while i > 0:
            cand = [(i - 1, j - 1), (i - 1, j), (i, j - 1)]
            vals = [D[a, b] if b >= 0 else np.float32(np.inf) for a, b in cand]
            k = int(np.argmin(vals))              # first of equal minima
            i, j = cand[k]
            want.append((i, j))
        pi, pj = oracle.path_f32(q, r, kind)
        assert list(zip(pi.tolist(), pj.tolist())) == want, (q, r)


def brute_force_dtw_f32(q, r, kind):
    """Global (corner-to-corner) DTW of Section 2 by enumeration: every warp
    path from cell (1, 1) to cell (N, M) with steps down, right and diagonal,
    its FP32 costs folded left to right from (1, 1); the minimum fold."""
    n, m = len(q), len(r)
    c = [[_c32(q[i], r[j], kind) for j in range(m)] for i in range(n)]
    best = [np.float32(np.inf)]

    def walk(i, j, acc):
        if i == n - 1 and j == m - 1:
            if acc < best[0]:
                best[0] = acc
            return
        for di, dj in ((1, 0), (0, 1), (1, 1)):
            ni, nj = i + di, j + dj
            if ni < n and nj < m:
                walk(ni, nj, np.float32(acc + c[ni][nj]))

    walk(0, 0, c[0][0])
    return best[0]


@pytest.mark.parametrize("kind", [0, 1])
def test_global_dtw_equals_brute_force_bit_exact(kind):
    """oracle.dtw_f32 (the corner-to-corner DTW the subsequence cost is bounded
    by) against the enumeration above, bit for bit, including small-integer
    inputs with many ties and single-row / single-column shapes."""
    for q, r in _cases():
        want = brute_force_dtw_f32(q, r, kind)
        got = oracle.dtw_f32(q, r, kind)
        assert np.float32(got).tobytes() == want.tobytes(), (q, r, got, want)
        # the free start can only lower the cost, and the corner path is one
        # of the subsequence paths
        cost, _ = oracle.sdtw_f32(q, [q.size], r, kind)
        assert cost[0] <= got


def test_global_dtw_hand_worked_example():
    """Every entry G(i, j) of the hand-worked global DTW table is the DTW of
    the prefixes q[:i] and r[:j]."""
    g = _read_golden("hand_sdtw_3x6.txt")
    q = np.array(g["q"], np.float32)
    r = np.array(g["r"], np.float32)
    for kind, name in ((0, "squared"), (1, "absolute")):
        rows = np.array(g[f"{name}.dtw_rows"], np.float32).reshape(3, 6)
        for i in range(1, 4):
            for j in range(1, 7):
                assert oracle.dtw_f32(q[:i], r[:j], kind) == rows[i - 1, j - 1], (name, i, j)
        assert oracle.dtw_f32(q, r, kind) == g[f"{name}.dtw"][0]
