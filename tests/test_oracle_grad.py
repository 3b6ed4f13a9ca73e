"""Pins of the oracle's walk-back gradient (the differentiable form of the path).

The cost is the summed local cost along the optimal warp path (Section 2,
Eq. (1)); away from ties the path is locally constant, so the gradient with
respect to a query or reference value is the sum, over that value's path
cells, of the local-cost derivative.  Pins:

* central finite differences of the FP64 oracle cost (exact for a piecewise
  quadratic whose path does not change, up to FP64 rounding);
* the path itself: connected, monotone, from row N to row 1, and its FP32
  fold equals the cost bit for bit;
* the identities sum(dq) + sum(dref) = 0 (each cell contributes +term and
  -term) and Euler's q.dq + r.dref = 2 cost (squared) or cost (absolute).
"""
import numpy as np
import pytest

import oracle
import workloads


def _c32(q, r, kind):
    t = np.float32(np.float32(q) - np.float32(r))
    return np.float32(t * t) if kind == 0 else np.float32(abs(t))


@pytest.mark.parametrize("kind", [0, 1])
def test_path_is_valid_and_folds_to_cost(kind):
    w = workloads.make_random(6, [20, 1, 35, 8, 50, 3], 180, seed=31)
    cost, end = oracle.sdtw_f32(w.queries, w.lens, w.reference, kind)
    for b in range(w.batch):
        q = w.query(b)
        pi, pj = oracle.path_f32(q, w.reference, kind)
        n = q.size
        assert pi[0] == n - 1 and pj[0] == end[b] and pi[-1] == 0
        steps = set(zip(-np.diff(pi), -np.diff(pj)))
        assert steps <= {(1, 0), (0, 1), (1, 1)}
        fold = np.float32(0)
        for i, j in zip(pi[::-1], pj[::-1]):
            fold = np.float32(fold + _c32(q[i], w.reference[j], kind))
        assert fold.tobytes() == cost[b].tobytes()


def _fd_check(w, kind, h=1e-3, rtol=1e-3):
    g = np.ones(w.batch, np.float32)
    _, _, _, gq, gr = oracle.sdtw_grad_f32(w.queries, w.lens, w.reference, g, kind)
    base_paths = [oracle.path_f32(w.query(b), w.reference, kind) for b in range(w.batch)]

    def total(q, r):
        c, _ = oracle.sdtw_f64(q, w.lens, r, kind)
        return c.sum()

    def same_paths(q, r):
        off = np.concatenate([[0], np.cumsum(w.lens)])
        for b in range(w.batch):
            pi, pj = oracle.path_f32(q[off[b]:off[b + 1]], r, kind)
            if not (np.array_equal(pi, base_paths[b][0]) and np.array_equal(pj, base_paths[b][1])):
                return False
        return True

    checked = skipped = 0
    q0 = w.queries.astype(np.float32)
    r0 = w.reference.astype(np.float32)
    for which, base, grad in (("q", q0, gq), ("r", r0, gr)):
        for k in range(base.size):
            hp, hm = base.copy(), base.copy()
            hp[k] += np.float32(h)
            hm[k] -= np.float32(h)
            step = float(hp[k]) - float(hm[k])         # the FP32 step actually taken
            if which == "q":
                fp, fm = total(hp, r0), total(hm, r0)
                stable = same_paths(hp, r0) and same_paths(hm, r0)
            else:
                fp, fm = total(q0, hp), total(q0, hm)
                stable = same_paths(q0, hp) and same_paths(q0, hm)
            if not stable:
                skipped += 1
                continue
            fd = (fp - fm) / step
            assert abs(fd - grad[k]) <= rtol * abs(fd) + 1e-4, (which, k, fd, grad[k])
            checked += 1
    assert checked > 0.9 * (checked + skipped)
    return checked


def test_gradient_matches_central_differences_squared():
    w = workloads.make_random(3, [12, 7, 15], 60, seed=41, excerpt_every=0)
    assert _fd_check(w, 0) > 50


def test_gradient_matches_central_differences_absolute():
    # |t| has a kink at t = 0; continuous data never lands on it
    w = workloads.make_random(2, [9, 11], 40, seed=43, excerpt_every=0)
    assert _fd_check(w, 1) > 30


@pytest.mark.parametrize("kind", [0, 1])
def test_gradient_identities(kind):
    w = workloads.make_random(5, 40, 500, seed=47)
    g = np.linspace(0.5, 2.0, w.batch).astype(np.float32)
    cost, _, _, gq, gr = oracle.sdtw_grad_f32(w.queries, w.lens, w.reference, g, kind)
    q = w.queries.astype(np.float64)
    r = w.reference.astype(np.float64)
    scale = np.abs(gq).sum() + np.abs(gr).sum()
    assert abs(gq.astype(np.float64).sum() + gr.astype(np.float64).sum()) <= 1e-5 * scale
    euler = (q * gq).sum() + (r * gr).sum()
    expect = (2.0 if kind == 0 else 1.0) * (g.astype(np.float64) * cost).sum()
    assert abs(euler - expect) <= 1e-4 * abs(expect) + 1e-5


def test_untouched_reference_entries_have_zero_gradient():
    w = workloads.make_random(3, 20, 400, seed=53)
    _, end, start, gq, gr = oracle.sdtw_grad_f32(w.queries, w.lens, w.reference,
                                                 np.ones(3, np.float32), 0)
    touched = np.zeros(w.ref_len, bool)
    for b in range(3):
        touched[start[b]:end[b] + 1] = True
    assert np.all(gr[~touched] == 0)


def test_batch_gradient_is_sum_of_single_gradients():
    w = workloads.make_random(4, [10, 25, 17, 30], 120, seed=59)
    g = np.array([1.0, -0.5, 2.0, 0.25], np.float32)
    _, _, _, gq, gr = oracle.sdtw_grad_f32(w.queries, w.lens, w.reference, g, 0)
    off = w.offsets
    acc = np.zeros(w.ref_len, np.float32)
    for b in range(4):
        _, _, s, gq1, gr1 = oracle.sdtw_grad_f32(w.query(b), [int(w.lens[b])], w.reference,
                                                 g[b:b + 1], 0)
        np.testing.assert_array_equal(gq[off[b]:off[b + 1]], gq1)
        acc = (acc + gr1).astype(np.float32)
    np.testing.assert_allclose(gr, acc, rtol=1e-6, atol=1e-7)
