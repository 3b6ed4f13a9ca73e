"""Pins of the binary16 oracle (sDTW in the paper's own precision).

* its rounding helper against NumPy's float64 -> float16 conversion, a
  library routine that rounds to nearest, ties to even, with subnormals and
  overflow to infinity;
* the DP against a brute-force enumeration of every warp path whose costs
  are folded left to right in NumPy float16 arithmetic (each NumPy float16
  operation is correctly rounded: it computes in binary32, which has more
  than 2 x 11 + 2 significand bits, so the double rounding is innocuous);
  rounding to nearest is monotone, so the DP equals that minimum bit for bit;
* small-integer inputs, where binary16 is exact, against the FP32 oracle;
* overflow past 65504 to infinity.
"""
import numpy as np
import pytest

import oracle


def test_rounding_matches_numpy_float16():
    rng = np.random.default_rng(1)
    xs = np.concatenate([
        rng.standard_normal(4000) * 10.0 ** rng.uniform(-9, 5, 4000),
        np.arange(-3000, 3000) * 2.0 ** -25,           # subnormal grid and ties
        np.arange(2040, 2060, 0.5),                    # ties at spacing 1 and 2
        np.array([65504.0, 65519.999, 65520.0, 70000.0, -65520.0, 0.0, -0.0, 2.0 ** -24]),
    ])
    with np.errstate(over="ignore"):
        want = xs.astype(np.float16).astype(np.float64)
    got = np.array([oracle.round_f16(x) for x in xs])
    np.testing.assert_array_equal(got, want)


def _c16(q, r, kind):
    t = np.float16(q) - np.float16(r)
    return np.float16(t * t) if kind == 0 else np.float16(abs(t))


def _brute_f16(q, r, kind):
    n, m = len(q), len(r)
    c = [[_c16(q[i], r[j], kind) for j in range(m)] for i in range(n)]
    best = [np.float16(np.inf)] * m

    def walk(i, j, acc):
        if i == n - 1 and acc < best[j]:
            best[j] = acc
        for di, dj in ((1, 0), (0, 1), (1, 1)):
            ni, nj = i + di, j + dj
            if ni < n and nj < m:
                walk(ni, nj, np.float16(acc + c[ni][nj]))

    for a in range(m):
        walk(0, a, c[0][a])
    best = np.array(best, dtype=np.float16)
    return best.min(), int(np.argmin(best))


@pytest.mark.parametrize("kind", [0, 1])
def test_dp_equals_brute_force_f16(kind):
    rng = np.random.default_rng(20 + kind)
    with np.errstate(over="ignore"):
        for t in range(60):
            n = int(rng.integers(1, 5))
            m = int(rng.integers(1, 7))
            scale = [0.3, 3.0, 40.0][t % 3]
            q = (rng.standard_normal(n) * scale).astype(np.float32)
            r = (rng.standard_normal(m) * scale).astype(np.float32)
            bc, be = _brute_f16(q, r, kind)
            c, e = oracle.sdtw_f16(q, [n], r, kind)
            assert np.float32(bc) == c[0] or (np.isinf(bc) and np.isinf(c[0])), (q, r)
            assert e[0] == be, (q, r)


@pytest.mark.parametrize("kind", [0, 1])
def test_small_integers_match_fp32(kind):
    rng = np.random.default_rng(30 + kind)
    lens = [1, 3, 7, 12]
    q = rng.integers(-3, 4, sum(lens)).astype(np.float32)
    r = rng.integers(-3, 4, 40).astype(np.float32)
    c16, e16 = oracle.sdtw_f16(q, lens, r, kind)
    c32, e32 = oracle.sdtw_f32(q, lens, r, kind)
    np.testing.assert_array_equal(c16, c32)
    np.testing.assert_array_equal(e16, e32)


def test_overflow_to_infinity():
    # every cell costs 200^2 = 40000; two rows sum past 65504
    c, e = oracle.sdtw_f16(np.array([200, 200], np.float32), [2], np.zeros(3, np.float32), 0)
    assert np.isinf(c[0]) and e[0] == 0
    c, e = oracle.sdtw_f16(np.array([200], np.float32), [1], np.zeros(3, np.float32), 0)
    assert c[0] == 40000.0 and e[0] == 0
