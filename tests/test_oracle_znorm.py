"""Pins of the z-normalisation oracle against closed forms and invariants
(the paper's normaliser section prints no worked example)."""
import numpy as np
import pytest

from oracle import znorm as Z


def test_closed_form_four_values():
    # mean 2.5, deviations -1.5 -0.5 0.5 1.5, population variance 1.25 = 5/4
    z = Z.znorm_f32(np.array([1, 2, 3, 4], np.float32), [4])
    s5 = np.sqrt(5.0)
    np.testing.assert_array_equal(z, np.array([-3 / s5, -1 / s5, 1 / s5, 3 / s5], np.float32))


def test_two_values_map_to_minus_one_plus_one():
    rng = np.random.default_rng(3)
    for _ in range(50):
        a, b = np.sort(rng.standard_normal(2).astype(np.float32))
        if a == b:
            continue
        np.testing.assert_array_equal(Z.znorm_f32(np.array([a, b], np.float32), [2]),
                                      np.array([-1, 1], np.float32))


def test_constant_and_single_series_are_zero():
    x = np.array([7.5] * 9 + [-2.0] + [3.25] * 5, np.float32)
    z = Z.znorm_f32(x, [9, 1, 5])
    assert np.all(z == 0.0)


def test_population_moments():
    rng = np.random.default_rng(4)
    lens = [1000, 17, 4097, 3]
    x = (rng.standard_normal(sum(lens)) * 3.7 + 11.0).astype(np.float32)
    z = Z.znorm_f32(x, lens).astype(np.float64)
    off = 0
    for n in lens:
        v = z[off:off + n]
        assert abs(v.mean()) < 1e-6
        assert abs(v.std() - 1.0) < 1e-6       # numpy's std divides by n
        off += n


def test_affine_invariance():
    rng = np.random.default_rng(5)
    x = rng.standard_normal(513).astype(np.float32)
    z = Z.znorm_f32(x, [513]).astype(np.float64)
    for a, b in ((4.0, -3.0), (0.25, 100.0), (-2.0, 1.0)):
        y = (x.astype(np.float64) * a + b).astype(np.float32)
        zy = Z.znorm_f32(y, [513]).astype(np.float64)
        # y is x rescaled up to one binary32 rounding per element
        np.testing.assert_allclose(zy, np.sign(a) * z, atol=2e-5)


def test_sum_of_squares_form_agrees():
    """The section's form, variance = sum(x^2)/n - mean^2, is the same
    quantity; in binary64 on well-scaled data the two agree to rounding."""
    rng = np.random.default_rng(6)
    lens = [2000, 250, 4000]
    x = np.cumsum(rng.standard_normal(sum(lens))).astype(np.float32)
    mean, std = Z.znorm_stats_f64(x, lens)
    off = 0
    for b, n in enumerate(lens):
        v = x[off:off + n].astype(np.float64)
        m = v.sum() / n
        var = (v * v).sum() / n - m * m
        assert mean[b] == pytest.approx(m, rel=1e-14, abs=1e-12)
        assert std[b] == pytest.approx(np.sqrt(var), rel=1e-9)
        off += n


def test_rejects_bad_lengths():
    with pytest.raises(ValueError):
        Z.znorm_f32(np.zeros(5, np.float32), [2, 2])
    with pytest.raises(ValueError):
        Z.znorm_f32(np.zeros(2, np.float32), [2, 0])
