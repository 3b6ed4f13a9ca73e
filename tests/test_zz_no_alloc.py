"""The allocation-free forward (sdtw_forward_noalloc, through the C ABI)
against sdtw_forward on the same inputs, bit for bit: cost, end position and
checkpoint columns, for plain, persistent and checkpointed launches, each
followed by a second call on a smaller batch (the library's array keeps the
previous call's contents); and a batch too large for the array is refused
before anything is launched."""
import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu


def _ragged(batch, lo, hi, ref_len, seed):
    rng = np.random.default_rng(seed)
    lens = [int(x) for x in rng.integers(lo, hi + 1, batch)]
    return workloads.make_random(batch, lens, ref_len, seed=seed)


def _run_pair(P, w, kind, flags=0, variant=-1, ckpt_every=0):
    dev = torch.device("cuda:0")
    q = torch.from_numpy(w.queries).to(dev)
    l = torch.from_numpy(w.lens).to(dev)
    r = torch.from_numpy(w.reference).to(dev)
    ck_a = ck_b = None
    if flags & P.SDTW_F_CHECKPOINT:
        n = max(1, P.sdtw_checkpoint_floats(w.lens, w.ref_len, ckpt_every))
        ck_a = torch.full((n,), -1.0, dtype=torch.float32, device=dev)
        ck_b = torch.full((n,), -2.0, dtype=torch.float32, device=dev)
    ca, ea = P.sdtw_forward(q, w.lens, l, r, kind, ckpt=ck_a, ckpt_every=ckpt_every,
                            variant=variant, flags=flags)
    cb = torch.full((w.batch,), -1.0, dtype=torch.float32, device=dev)
    eb = torch.full((w.batch,), -1, dtype=torch.int64, device=dev)
    P.sdtw_forward_noalloc(q, w.lens, l, r, kind, cost=cb, end_pos=eb, ckpt=ck_b,
                           ckpt_every=ckpt_every, variant=variant, flags=flags)
    torch.cuda.synchronize()
    assert np.array_equal(ca.cpu().numpy().view(np.uint32), cb.cpu().numpy().view(np.uint32))
    assert np.array_equal(ea.cpu().numpy(), eb.cpu().numpy())
    if ck_a is not None:
        # every checkpoint column, then the row checkpoints of each query
        # (rows of the row region that no query owns are never written)
        a = ck_a.cpu().numpy().view(np.uint32)
        b = ck_b.cpu().numpy().view(np.uint32)
        total = int(w.lens.sum())
        cols = total * ((w.ref_len + ckpt_every - 1) // ckpt_every - 1)
        assert np.array_equal(a[:cols], b[:cols])
        step, off = P.SDTW_ROW_CKPT_EVERY, 0
        for n in w.lens:
            for k in range(1, (int(n) - 1) // step + 1):
                at = cols + (off // step + k - 1) * w.ref_len
                assert np.array_equal(a[at:at + w.ref_len], b[at:at + w.ref_len])
            off += int(n)


def _variant_of(P, shape):
    for v in range(P.sdtw_variant_count()):
        if P.sdtw_variant_info(v) == shape:
            return v
    raise AssertionError(f"no compiled variant {shape}")


@pytest.mark.parametrize("kind", [0, 1])
def test_plain_then_smaller(kind):
    import paper_2403_06931_amd as P
    # several tiles, ragged lengths, queries longer than one row pass of the
    # (8, 8, 4, 32) tile (2,048 rows) so the row buffer is used
    big = _ragged(37, 1, 2600, 30_000, seed=11)
    small = _ragged(5, 1, 300, 3_000, seed=12)
    v = _variant_of(P, (8, 8, 4, 32, 1))
    print(f"noalloc plain kind {kind}: 37 queries vs 30,000, then 5 vs 3,000", flush=True)
    _run_pair(P, big, kind, variant=v)
    _run_pair(P, small, kind, variant=v)
    _run_pair(P, small, kind)                    # the library's own tile choice


def test_persistent_then_smaller():
    import paper_2403_06931_amd as P
    big = _ragged(40, 200, 3000, 20_000, seed=13)
    small = _ragged(3, 1, 700, 1_500, seed=14)
    v = _variant_of(P, (8, 8, 1, 16, 1))            # 512-row passes: tail passes too
    print("noalloc persistent: 40 queries vs 20,000, then 3 vs 1,500", flush=True)
    _run_pair(P, big, 0, flags=P.SDTW_F_PERSISTENT, variant=v)
    _run_pair(P, small, 0, flags=P.SDTW_F_PERSISTENT, variant=v)


def test_checkpointed_then_smaller():
    import paper_2403_06931_amd as P
    big = _ragged(9, 100, 1200, 10_000, seed=15)
    small = _ragged(2, 1, 64, 600, seed=16)
    print("noalloc checkpoints: 9 queries vs 10,000, then 2 vs 600", flush=True)
    _run_pair(P, big, 0, flags=P.SDTW_F_CHECKPOINT, ckpt_every=256)
    _run_pair(P, small, 1, flags=P.SDTW_F_CHECKPOINT, ckpt_every=64)


def test_too_large_is_refused():
    import paper_2403_06931_amd as P
    # 40 queries longer than one pass of the (8, 8, 4, 32) tile against
    # 200,000 columns: 40 row-buffer slots of 800 KB, more than the array
    lens = np.full(40, 5000, np.int32)
    v = _variant_of(P, (8, 8, 4, 32, 1))
    assert P.sdtw_forward_workspace_bytes(lens, 200_000, 0, v) > P._lib.SDTW_NOALLOC_SCRATCH_BYTES
    dev = torch.device("cuda:0")
    q = torch.zeros(int(lens.sum()), dtype=torch.float32, device=dev)
    l = torch.from_numpy(lens).to(dev)
    r = torch.zeros(200_000, dtype=torch.float32, device=dev)
    c = torch.full((40,), 7.0, dtype=torch.float32, device=dev)
    e = torch.full((40,), 7, dtype=torch.int64, device=dev)
    with pytest.raises(P.SdtwError) as ex:
        P.sdtw_forward_noalloc(q, lens, l, r, 0, cost=c, end_pos=e, variant=v)
    assert ex.value.status == P._lib.SDTW_ERR_WORKSPACE
    torch.cuda.synchronize()
    assert (c.cpu().numpy() == 7.0).all() and (e.cpu().numpy() == 7).all()
