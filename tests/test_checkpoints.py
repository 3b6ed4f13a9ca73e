"""GPU: the DP column checkpoints that the forward stores for the backward
(every K reference columns) equal the oracle's DP columns bit for bit, for
every compiled variant, several K (both ways the kernel finds the checkpoint
column, and stores per step or per barrier interval) and queries that need
several row passes; so do the row checkpoints (every 256 rows), which reach
the store through wavefront handoffs, between row passes through the row
buffer, or (8 rows per lane) from the lane holding the middle row of a
wavefront."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from gpu_util import to_dev

pytestmark = pytest.mark.gpu

LENS = [1, 5, 40, 70, 130, 300, 600]
REF_LEN = 3000


def _oracle_rows(w, kind):
    """D(i, 1..M) for i = 1..len of every query (last rows of its prefixes)."""
    return [np.stack([oracle.last_row_f32(w.query(b)[:i], w.reference, kind)
                      for i in range(1, w.lens[b] + 1)]) for b in range(w.batch)]


def _expected(rows, K):
    nck = (REF_LEN + K - 1) // K - 1
    cols = [k * K - 1 for k in range(1, nck + 1)]
    # query b's block: n_ckpt columns of len_b values each
    return np.concatenate([r[:, cols].T.ravel() for r in rows]), nck


@pytest.mark.parametrize("kind", [0, 1])
def test_checkpoint_columns_all_variants(kind):
    import paper_2403_06931_amd as P
    w = workloads.make_random(len(LENS), LENS, REF_LEN, seed=77 + kind)
    rows = _oracle_rows(w, kind)
    q, l, r = to_dev(w)
    for K in (16, 64, 256, 1024):
        want, nck = _expected(rows, K)
        size = P.sdtw_checkpoint_floats(w.lens, REF_LEN, K)
        assert size == want.size + (sum(LENS) // P.SDTW_ROW_CKPT_EVERY) * REF_LEN
        for v in range(P.sdtw_variant_count()):
            print(f"kind {kind} K {K} variant {v} {P.sdtw_variant_info(v)}", flush=True)
            ckpt = torch.full((size,), float("nan"), dtype=torch.float32, device=q.device)
            P.sdtw_forward(q, w.lens, l, r, kind, ckpt=ckpt, ckpt_every=K, variant=v,
                           flags=P.SDTW_F_CHECKPOINT)
            got = ckpt.cpu().numpy()[:want.size]
            bad = np.nonzero(got.view(np.uint32) != want.view(np.uint32))[0]
            assert bad.size == 0, (f"K {K} variant {v}: {bad.size} checkpoint values differ, "
                                   f"first at {bad[:4]}: {got[bad[:4]]} vs {want[bad[:4]]}")


ROW_LENS = [1100, 300, 2050, 513, 512, 1536, 1537, 256, 257, 769, 255]
ROW_REF = 3000


def _row_expected(w, kind):
    """{region row: D(256k, 1..M)} for every row checkpoint of the batch."""
    step = 256
    off, rows = 0, {}
    for b in range(w.batch):
        n = w.lens[b]
        for k in range(1, (n - 1) // step + 1):
            rows[off // step + k - 1] = oracle.last_row_f32(w.query(b)[:k * step], w.reference,
                                                            kind)
        off += n
    return rows


@pytest.mark.parametrize("kind", [0, 1])
def test_row_checkpoints_all_variants(kind):
    import paper_2403_06931_amd as P
    assert P.SDTW_ROW_CKPT_EVERY == 256
    w = workloads.make_random(len(ROW_LENS), ROW_LENS, ROW_REF, seed=91 + kind)
    rows = _row_expected(w, kind)
    total = sum(ROW_LENS)
    q, l, r = to_dev(w)
    for K in (64, 1024):
        nck = (ROW_REF + K - 1) // K - 1
        size = P.sdtw_checkpoint_floats(w.lens, ROW_REF, K)
        assert size == total * nck + (total // 256) * ROW_REF
        base = total * nck
        cases = [(v, P.SDTW_F_CHECKPOINT) for v in range(P.sdtw_variant_count())]
        cases += [(v, P.SDTW_F_CHECKPOINT | P.SDTW_F_PERSISTENT) for v in (0, 6, 12)]
        for v, flags in cases:
            print(f"kind {kind} K {K} variant {v} {P.sdtw_variant_info(v)} flags {flags}",
                  flush=True)
            ckpt = torch.full((size,), float("nan"), dtype=torch.float32, device=q.device)
            P.sdtw_forward(q, w.lens, l, r, kind, ckpt=ckpt, ckpt_every=K, variant=v,
                           flags=flags)
            got = ckpt.cpu().numpy()[base:].reshape(-1, ROW_REF)
            for k in range(got.shape[0]):
                if k in rows:
                    bad = np.nonzero(got[k].view(np.uint32) != rows[k].view(np.uint32))[0]
                    assert bad.size == 0, (f"K {K} variant {v} flags {flags}: region row {k}: "
                                           f"{bad.size} values differ, first at {bad[:4]}")
                else:
                    assert np.isnan(got[k]).all(), f"region row {k} is owned by no query"
