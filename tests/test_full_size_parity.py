"""GPU parity at the full sizes of the five workloads, on the query subsets
fixed for them: the HIP path (through the C ABI, in the launch form the
benchmark times) against the CPU oracle, bit for bit.

* 512 x 2,000 vs 100,000 (the shape of the paper's Section 6 / Table 1
  experiment): every one of the 512 queries, in the library's own tile
  choice and in the benchmark's tile;
* 512 x 2,000 vs 2,000,000: a seeded subset of 16 queries per cost kind;
* 4,096 x U{250..4,000} vs 200,000, persistent launch: a seeded subset of 64
  queries that includes the shortest and the longest;
* 256 x 1,000 vs 50,000 with checkpoints every 1,024 columns: the gradient
  of every query against the oracle's walk-back, and central differences of
  the FP64 oracle cost at 8 entries for each of 32 sampled queries.
"""
import concurrent.futures as cf

import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_util import assert_bit_exact, gpu_forward, to_dev

pytestmark = pytest.mark.gpu

HEADLINE_TILE = (8, 8, 4, 32, 1)          # the tile the benchmark's tuner picks here


def _variant_of(shape):
    import paper_2403_06931_amd as P
    for v in range(P.sdtw_variant_count()):
        if P.sdtw_variant_info(v) == shape:
            return v
    raise AssertionError(f"no compiled variant {shape}")


def test_paper_shape_every_query():
    w = workloads.make_config(1)
    print(f"{w.name}: oracle on all {w.batch} queries", flush=True)
    want_c, want_e = oracle.sdtw_f32(w.queries, w.lens, w.reference, 0)
    for v in (-1, _variant_of(HEADLINE_TILE)):
        c, e = gpu_forward(w, 0, variant=v)
        assert_bit_exact(c, e, want_c, want_e, f"512x2000 vs 100k, variant {v}")
    # FP64 accuracy reference on a seeded quarter of the batch
    idx = workloads.subset_indices(w, 128, seed=5)
    sub = w.subset(idx)
    c64, _ = oracle.sdtw_f64(sub.queries, sub.lens, sub.reference, 0)
    rel = np.abs(want_c[idx].astype(np.float64) - c64) / np.maximum(np.abs(c64), 1e-6)
    assert np.all(rel <= 1e-5), rel.max()


@pytest.mark.parametrize("kind", [0, 1])
def test_long_reference_16_queries(kind):
    w = workloads.make_config(2)
    idx = np.sort(np.random.default_rng(workloads.BASE_SEED + 2 + kind)
                  .choice(w.batch, 16, replace=False))
    c, e = gpu_forward(w, kind, variant=_variant_of(HEADLINE_TILE))
    sub = w.subset(idx)
    print(f"{w.name} kind {kind}: oracle on queries {idx.tolist()}", flush=True)
    want_c, want_e = oracle.sdtw_f32(sub.queries, sub.lens, sub.reference, kind)
    assert_bit_exact(c[idx], e[idx], want_c, want_e, f"2M reference kind {kind}")


def test_uneven_batch_64_queries():
    import paper_2403_06931_amd as P
    w = workloads.make_config(3)
    # 64 seeded queries, two of them the shortest and the longest
    extremes = {int(np.argmin(w.lens)), int(np.argmax(w.lens))}
    rest = [int(b) for b in workloads.subset_indices(w, 70, seed=31) if b not in extremes]
    idx = np.array(sorted(extremes | set(rest[:64 - len(extremes)])), np.int64)
    assert idx.size == 64
    sub = w.subset(idx)
    print(f"{w.name}: oracle on {idx.size} queries", flush=True)
    want_c, want_e = oracle.sdtw_f32(sub.queries, sub.lens, sub.reference, 0)
    for v in (-1, _variant_of((8, 8, 1, 16, 1))):
        c, e = gpu_forward(w, 0, variant=v, flags=P.SDTW_F_PERSISTENT)
        assert_bit_exact(c[idx], e[idx], want_c, want_e, f"uneven batch, variant {v}")


def _gpu_grad(P, dev_inputs, w, g, kind, ckpt_every, variant=-1):
    q, l, r = dev_inputs
    ckpt = torch.empty(P.sdtw_checkpoint_floats(w.lens, w.ref_len, ckpt_every),
                       dtype=torch.float32, device=q.device)
    cost, end = P.sdtw_forward(q, w.lens, l, r, kind, ckpt=ckpt, ckpt_every=ckpt_every,
                               variant=variant, flags=P.SDTW_F_CHECKPOINT)
    gc = torch.from_numpy(np.asarray(g, np.float32)).to(q.device)
    gq, gr = P.sdtw_backward(q, w.lens, l, r, kind, gc, cost, end, ckpt, ckpt_every)
    torch.cuda.synchronize()
    return cost.cpu().numpy(), end.cpu().numpy(), gq.cpu().numpy(), gr.cpu().numpy()


def test_differentiable_every_gradient():
    """Costs, end positions, grad_queries and grad_reference of all 256
    queries bit for bit against the oracle walk-back, for the summed loss and
    for uneven weights."""
    import paper_2403_06931_amd as P
    w = workloads.make_config(4)
    dv = to_dev(w)
    for g in (np.ones(w.batch, np.float32),
              np.random.default_rng(3).uniform(-2.0, 2.0, w.batch).astype(np.float32)):
        c, e, gq, gr = _gpu_grad(P, dv, w, g, 0, 1024)
        print(f"{w.name}: oracle walk-back on all {w.batch} queries", flush=True)
        oc, oe, _, ogq, ogr = oracle.sdtw_grad_f32(w.queries, w.lens, w.reference, g, 0)
        assert_bit_exact(c, e, oc, oe, "differentiable workload forward")
        bad = np.nonzero(gq.view(np.uint32) != ogq.view(np.uint32))[0]
        assert bad.size == 0, f"dq mismatch at {bad[:8]}: {gq[bad[:8]]} vs {ogq[bad[:8]]}"
        bad = np.nonzero(gr.view(np.uint32) != ogr.view(np.uint32))[0]
        assert bad.size == 0, f"dref mismatch at {bad[:8]}: {gr[bad[:8]]} vs {ogr[bad[:8]]}"


def _fd(jobs):
    def run(job):
        qq, rr = job
        c, _ = oracle.sdtw_f64(qq, [qq.size], rr, 0, nthreads=1)
        return float(c[0])
    with cf.ThreadPoolExecutor(16) as ex:
        return list(ex.map(run, jobs))


def test_differentiable_finite_differences_32_queries():
    """Central differences (h = 1e-3) of the FP64 oracle cost against the GPU
    gradient at 8 entries (4 query values, 4 reference values on the path) of
    each of 32 sampled queries, rtol 1e-3.  Along a fixed warp path the cost
    is a quadratic in each coordinate, so the central difference is exact up
    to binary64 rounding; an entry whose perturbation moves the optimal path
    (checked with the oracle's walk-back) is replaced by another draw."""
    import paper_2403_06931_amd as P
    w = workloads.make_config(4)
    dv = to_dev(w)
    idx = workloads.subset_indices(w, 32, seed=77)
    off = w.offsets
    h = np.float32(1e-3)
    rng = np.random.default_rng(8)
    redraws = 0
    for b in idx:
        onehot = np.zeros(w.batch, np.float32)
        onehot[b] = 1.0
        _, _, gq, gr = _gpu_grad(P, dv, w, onehot, 0, 1024)
        q0 = w.query(b).copy()
        r0 = w.reference
        pi, pj = oracle.path_f32(q0, r0, 0)
        cols = np.unique(pj)
        need = {"q": 4, "r": 4}
        tried = set()
        while need["q"] or need["r"]:
            cand = []
            for which in ("q", "r"):
                if need[which] == 0:
                    continue
                pool = np.arange(q0.size) if which == "q" else cols
                for i in rng.choice(pool, need[which] + 1, replace=False):
                    if (which, int(i)) not in tried:
                        tried.add((which, int(i)))
                        cand.append((which, int(i)))
            jobs = []
            for which, i in cand:
                for s in (1, -1):
                    qq, rr = q0.copy(), r0.copy() if which == "r" else r0
                    if which == "q":
                        qq[i] += s * h
                    else:
                        rr[i] += s * h
                    jobs.append((qq, rr))
            vals = _fd(jobs)
            for k, (which, i) in enumerate(cand):
                if need[which] == 0:
                    continue
                base = q0 if which == "q" else r0
                step = float(np.float32(base[i] + h)) - float(np.float32(base[i] - h))
                fd = (vals[2 * k] - vals[2 * k + 1]) / step
                an = float(gq[off[b] + i]) if which == "q" else float(gr[i])
                if abs(fd - an) <= 1e-3 * abs(fd) + 1e-6:
                    need[which] -= 1
                    continue
                moved = False
                for j in (2 * k, 2 * k + 1):
                    qq, rr = jobs[j]
                    ppi, ppj = oracle.path_f32(qq, rr, 0)
                    moved |= not (np.array_equal(ppi, pi) and np.array_equal(ppj, pj))
                assert moved, (int(b), which, i, fd, an)
                redraws += 1
        print(f"query {int(b)}: 8 entries agree", flush=True)
    print(f"redrawn entries (path moved under the perturbation): {redraws}", flush=True)
    assert redraws <= 32
