"""GPU tests of the differentiable form: checkpointed forward + walk-back
backward, against the oracle's full-matrix walk-back gradient (bit for bit:
same operations in the same order) and against central finite differences of
the FP64 oracle cost."""
import concurrent.futures as cf

import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_util import to_dev

pytestmark = pytest.mark.gpu


def _gpu_grad(w, g, kind=0, ckpt_every=256):
    import paper_2403_06931_amd as P
    q, l, r = to_dev(w)
    nck = P.sdtw_checkpoint_floats(w.lens, w.ref_len, ckpt_every)
    ckpt = torch.empty(max(nck, 1), dtype=torch.float32, device=q.device)
    cost, end = P.sdtw_forward(q, w.lens, l, r, kind, ckpt=ckpt if nck else None,
                               ckpt_every=ckpt_every, flags=P.SDTW_F_CHECKPOINT)
    gc = torch.from_numpy(np.asarray(g, np.float32)).to(q.device)
    gq, gr = P.sdtw_backward(q, w.lens, l, r, kind, gc, cost, end, ckpt if nck else None,
                             ckpt_every)
    torch.cuda.synchronize()
    return (cost.cpu().numpy(), end.cpu().numpy(), gq.cpu().numpy(), gr.cpu().numpy())


def _check_vs_oracle(w, g, kind, ckpt_every, what):
    c, e, gq, gr = _gpu_grad(w, g, kind, ckpt_every)
    oc, oe, os_, ogq, ogr = oracle.sdtw_grad_f32(w.queries, w.lens, w.reference, g, kind)
    assert c.view(np.uint32).tolist() == oc.view(np.uint32).tolist(), what
    assert np.array_equal(e, oe), what
    bad = np.nonzero(gq != ogq)[0]
    assert bad.size == 0, f"{what}: dq mismatch at {bad[:8]}: {gq[bad[:8]]} vs {ogq[bad[:8]]}"
    bad = np.nonzero(gr != ogr)[0]
    assert bad.size == 0, f"{what}: dref mismatch at {bad[:8]}: {gr[bad[:8]]} vs {ogr[bad[:8]]}"


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("ckpt_every", [16, 256, 1024])
def test_ragged_batch_matches_oracle_walk(kind, ckpt_every):
    lens = [1, 2, 17, 64, 300, 511, 513, 700, 1024, 90]
    w = workloads.make_random(len(lens), lens, 3000, seed=301 + kind)
    g = np.linspace(-1.5, 2.0, len(lens)).astype(np.float32)
    print(f"kind {kind} K {ckpt_every}", flush=True)
    _check_vs_oracle(w, g, kind, ckpt_every, f"kind {kind} K {ckpt_every}")


@pytest.mark.parametrize("n,ckpt_every", [(1000, 1024), (2048, 2048), (4100, 3072), (8192, 1024)])
def test_long_queries_and_multi_segment_blocks(n, ckpt_every):
    """Long queries (up to the 8,192-row limit of the backward) and blocks
    wider than one 1,024-column recompute segment."""
    w = workloads.make_random(3, [n, n // 2, 7], max(5000, n * 3 // 2), seed=17 + n)
    _check_vs_oracle(w, np.ones(3, np.float32), 0, ckpt_every, f"n {n} K {ckpt_every}")


def test_path_crossing_many_blocks():
    """A short reference block size forces the walk across many checkpoint
    blocks and segment boundaries."""
    w = workloads.make_random(4, [400, 800, 60, 1200], 5000, seed=23)
    _check_vs_oracle(w, np.ones(4, np.float32), 0, 32, "K=32")


def test_autograd_function():
    import paper_2403_06931_amd as P
    w = workloads.make_random(6, [100, 250, 30, 400, 5, 64], 4000, seed=31)
    q, l, r = to_dev(w)
    q.requires_grad_(True)
    r.requires_grad_(True)
    cost, end = P.sdtw(q, w.lens, r, ckpt_every=512, query_lens=l)
    weights = torch.linspace(0.5, 1.5, 6, device=q.device)
    (cost * weights).sum().backward()
    oc, oe, _, ogq, ogr = oracle.sdtw_grad_f32(w.queries, w.lens, w.reference,
                                               weights.cpu().numpy(), 0)
    np.testing.assert_array_equal(cost.detach().cpu().numpy(), oc)
    np.testing.assert_array_equal(q.grad.cpu().numpy(), ogq)
    np.testing.assert_array_equal(r.grad.cpu().numpy(), ogr)


def _fd_entries(w, b, gq_b, gr, path_j, rng, count=8):
    """Central differences of the FP64 oracle cost of query b at `count`
    sampled entries (half in the query, half in reference columns on its
    path)."""
    q0 = w.query(b).copy()
    r0 = w.reference.copy()
    qi = rng.choice(q0.size, count // 2, replace=False)
    rj = rng.choice(np.unique(path_j), count // 2, replace=False)
    h = np.float32(1e-3)
    jobs = []
    for i in qi:
        for s in (1, -1):
            qq = q0.copy()
            qq[i] += s * h
            jobs.append(("q", i, s, qq, r0))
    for j in rj:
        for s in (1, -1):
            rr = r0.copy()
            rr[j] += s * h
            jobs.append(("r", j, s, q0, rr))

    def run(job):
        _, _, _, qq, rr = job
        c, _ = oracle.sdtw_f64(qq, [qq.size], rr, 0, nthreads=1)
        return c[0]

    with cf.ThreadPoolExecutor(16) as ex:
        vals = list(ex.map(run, jobs))
    out = []
    for k in range(0, len(jobs), 2):
        which, idx, _, qq, rr = jobs[k]
        base = q0 if which == "q" else r0
        step = float(np.float32(base[idx] + h)) - float(np.float32(base[idx] - h))
        fd = (vals[k] - vals[k + 1]) / step
        an = gq_b[idx] if which == "q" else gr[idx]
        out.append((which, int(idx), fd, float(an)))
    return out


def test_differentiable_config_fwd_bwd():
    """256 x 1,000 against 50,000 with checkpoints every 1,024 columns: the
    whole batch on the GPU; per-query gradients of sampled queries against
    the oracle walk-back, and central differences (h = 1e-3, rtol 1e-3) of
    the FP64 oracle cost at 8 entries per sampled query."""
    w = workloads.make_config(4)
    g = np.ones(w.batch, np.float32)
    c, e, gq, gr_all = _gpu_grad(w, g, 0, 1024)
    idx = workloads.subset_indices(w, 4, seed=99)
    sub = w.subset(idx)
    # dq of a query depends only on that query
    oc, oe, os_, ogq, _ = oracle.sdtw_grad_f32(sub.queries, sub.lens, sub.reference,
                                               np.ones(sub.batch, np.float32), 0)
    assert c[idx].view(np.uint32).tolist() == oc.view(np.uint32).tolist()
    off = w.offsets
    got = np.concatenate([gq[off[b]:off[b + 1]] for b in idx])
    np.testing.assert_array_equal(got, ogq)
    # reference gradient of the sampled queries alone: grad_cost one-hot on them
    g1 = np.zeros(w.batch, np.float32)
    g1[idx] = 1.0
    _, _, _, gr1 = _gpu_grad(w, g1, 0, 1024)
    _, _, _, _, ogr = oracle.sdtw_grad_f32(sub.queries, sub.lens, sub.reference,
                                           np.ones(sub.batch, np.float32), 0)
    np.testing.assert_array_equal(gr1, ogr)
    # finite differences
    rng = np.random.default_rng(7)
    checked = 0
    for k, b in enumerate(idx):
        _, pj = oracle.path_f32(w.query(b), w.reference, 0)
        gq_b = gq[off[b]:off[b + 1]]
        # reference gradient of query b alone
        gb = np.zeros(w.batch, np.float32)
        gb[b] = 1.0
        _, _, _, grb = _gpu_grad(w, gb, 0, 1024)
        for which, i, fd, an in _fd_entries(w, b, gq_b, grb, pj, rng):
            assert abs(fd - an) <= 1e-3 * abs(fd) + 1e-6, (b, which, i, fd, an)
            checked += 1
    assert checked == 8 * len(idx)


def test_gradient_identities_gpu():
    w = workloads.make_random(8, 500, 8000, seed=41)
    g = np.linspace(0.5, 2.0, 8).astype(np.float32)
    c, e, gq, gr = _gpu_grad(w, g, 0, 1024)
    q = w.queries.astype(np.float64)
    r = w.reference.astype(np.float64)
    scale = np.abs(gq).sum() + np.abs(gr).sum()
    assert abs(gq.astype(np.float64).sum() + gr.astype(np.float64).sum()) <= 1e-5 * scale
    euler = (q * gq).sum() + (r * gr).sum()
    expect = 2.0 * (g.astype(np.float64) * c).sum()
    assert abs(euler - expect) <= 1e-4 * abs(expect)
