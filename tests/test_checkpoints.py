"""GPU: the DP column checkpoints that the forward stores for the backward
(every K reference columns) equal the oracle's DP columns bit for bit, for
every compiled variant, several K (both ways the kernel finds the checkpoint
column, and stores per step or per barrier interval) and queries that need
several row passes."""
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
        assert P.sdtw_checkpoint_floats(w.lens, REF_LEN, K) == want.size
        for v in range(P.sdtw_variant_count()):
            print(f"kind {kind} K {K} variant {v} {P.sdtw_variant_info(v)}", flush=True)
            ckpt = torch.full((want.size,), float("nan"), dtype=torch.float32, device=q.device)
            P.sdtw_forward(q, w.lens, l, r, kind, ckpt=ckpt, ckpt_every=K, variant=v,
                           flags=P.SDTW_F_CHECKPOINT)
            got = ckpt.cpu().numpy()
            bad = np.nonzero(got.view(np.uint32) != want.view(np.uint32))[0]
            assert bad.size == 0, (f"K {K} variant {v}: {bad.size} checkpoint values differ, "
                                   f"first at {bad[:4]}: {got[bad[:4]]} vs {want[bad[:4]]}")
