"""The C-ABI library loads, exports every function include/sdtw.h declares,
and rejects invalid arguments on the host before any HIP call (so these run
without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sdtw.h")


@pytest.fixture(scope="module")
def L():
    from paper_2403_06931_amd import _lib
    return _lib


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sdtw_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol(L):
    names = _declared_functions()
    assert len(names) >= 9
    for n in names:
        assert hasattr(L.lib, n), n
    # and the shared object really exports them (not just resolvable by ctypes)
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True,
                         text=True).stdout
    for n in names:
        assert re.search(rf"\bT {n}\b", out), n


def test_status_strings(L):
    for s in (0, -1, -2, -3, -4, 7):
        assert isinstance(L.status_string(s), str) and L.status_string(s)


def test_variants_describe(L):
    import paper_2403_06931_amd as P
    n = P.sdtw_variant_count()
    assert n >= 1
    for v in range(n):
        r, t, w, ks, xl = P.sdtw_variant_info(v)
        assert r >= 1 and t in (4, 8, 16) and 1 <= w <= 16 and ks in (8, 16, 32, 64)
        assert xl in (0, 1)
        assert 16 % t == 0   # checkpoint intervals are multiples of 16
    with pytest.raises(P.SdtwError):
        P.sdtw_variant_info(n)


def _vp(x):
    return ctypes.c_void_p(x)


FAKE = 0x100000   # never dereferenced: validation fails first


def _fwd(L, lens, batch=None, ref_len=100, kind=0, flags=0, ws_bytes=1 << 40, q=FAKE, r=FAKE,
         c=FAKE, e=FAKE, ws=FAKE, ckpt=0, every=0, variant=-1, dlens=FAKE):
    h = np.ascontiguousarray(lens, dtype=np.int32)
    b = h.size if batch is None else batch
    return L.lib.sdtw_forward(_vp(q), _vp(h.ctypes.data if h.size else 0), _vp(dlens), b,
                              _vp(r), ref_len, kind, _vp(c), _vp(e), _vp(ckpt), every,
                              variant, flags, _vp(ws), ws_bytes, _vp(0))


def test_forward_rejects_invalid_arguments(L):
    E = L.SDTW_ERR_INVALID_ARG
    assert _fwd(L, [3, 4], q=0) == E
    assert _fwd(L, [3, 4], r=0) == E
    assert _fwd(L, [3, 4], c=0) == E
    assert _fwd(L, [3, 4], e=0) == E
    assert _fwd(L, [3, 4], ws=0) == E
    assert _fwd(L, [3, 4], dlens=0) == E
    assert _fwd(L, [3, 0]) == E                  # empty query
    assert _fwd(L, [3, -2]) == E
    assert _fwd(L, [3, 4], batch=0) == E
    assert _fwd(L, [3, 4], ref_len=0) == E
    assert _fwd(L, [3, 4], ref_len=(1 << 30) + 1) == E
    assert _fwd(L, [3, 4], kind=2) == E
    assert _fwd(L, [3, 4], flags=64) == E
    assert _fwd(L, [3, 4], ws=FAKE + 4) == E     # misaligned workspace
    # checkpointing: interval must be a positive multiple of 16 and the buffer present
    assert _fwd(L, [3, 4], flags=L.SDTW_F_CHECKPOINT, every=0, ckpt=FAKE) == E
    assert _fwd(L, [3, 4], flags=L.SDTW_F_CHECKPOINT, every=24, ckpt=FAKE) == E
    assert _fwd(L, [3, 4], flags=L.SDTW_F_CHECKPOINT, every=32, ckpt=0) == E
    assert _fwd(L, [3, 4], variant=10**6) == L.SDTW_ERR_UNSUPPORTED
    assert _fwd(L, [3, 4], ws_bytes=16) == L.SDTW_ERR_WORKSPACE


def _variant_of(shape):
    import paper_2403_06931_amd as P
    for v in range(P.sdtw_variant_count()):
        if P.sdtw_variant_info(v) == shape:
            return v
    raise AssertionError(shape)


def test_workspace_sizes(L):
    import paper_2403_06931_amd as P
    row = lambda m: -(-m // 64) * 64 * 4            # one row-buffer slot, bytes
    small = _variant_of((8, 8, 1, 16, 1))           # 512 rows per pass
    big = _variant_of((8, 8, 4, 32, 1))             # 2,048 rows per pass
    lens = np.array([5, 7, 300, 2000, 600], np.int32)
    # plain launch: one slot per query longer than one pass of the tile
    a = P.sdtw_forward_workspace_bytes(lens, 100000, 0, small)
    assert 2 * row(100000) <= a < 2 * row(100000) + 4096
    b = P.sdtw_forward_workspace_bytes(lens, 100000, 0, big)
    assert 0 < b < 4096                              # every query fits in one pass
    assert P.sdtw_forward_workspace_bytes(lens, 1000, 0, small) < a
    # library choice: the size of the variant the library would pick
    d = P.sdtw_default_variant(lens, 100000, 0)
    assert P.sdtw_forward_workspace_bytes(lens, 100000, 0) == \
        P.sdtw_forward_workspace_bytes(lens, 100000, 0, d)
    assert P.sdtw_forward_workspace_bytes(np.array([0], np.int32), 10) == 0
    assert P.sdtw_forward_workspace_bytes(lens, 0) == 0
    assert P.sdtw_forward_workspace_bytes(lens, 1000, 0, 10**6) == 0
    assert P.sdtw_forward_workspace_bytes(lens, 1000, 0, -2) == 0
    # persistent launch: one slot per workgroup of its grid (at most 8 waves
    # per CU), and none when no query needs a second pass
    many = np.full(10000, 300, np.int32)
    assert P.sdtw_forward_workspace_bytes(many, 1000, P.SDTW_F_PERSISTENT, small) < 10000 * 16 + 4096
    many[7] = 3000
    pers = P.sdtw_forward_workspace_bytes(many, 1000, P.SDTW_F_PERSISTENT, small)
    assert pers >= 256 * 8 * row(1000) and pers < 256 * 8 * row(1000) + 2 * 10000 * 8 + 4096
    plain = P.sdtw_forward_workspace_bytes(many, 1000, 0, small)
    assert row(1000) <= plain < row(1000) + 10000 * 16
    # one workspace for the whole differentiable path
    ck = P.SDTW_F_CHECKPOINT
    all_ = P.sdtw_workspace_bytes(lens, 50000, ck, 1024)
    assert all_ >= P.sdtw_forward_workspace_bytes(lens, 50000, ck)
    assert all_ >= P.sdtw_backward_workspace_bytes(lens, 50000, 1024)
    assert all_ >= P.sdtw_align_workspace_bytes(lens, 50000, 1024)
    assert P.sdtw_workspace_bytes(lens, 50000, 0, 0) == P.sdtw_forward_workspace_bytes(lens, 50000)
    assert P.sdtw_workspace_bytes(lens, 50000, ck, 24) == 0
    # checkpoint columns: ceil(M/K) - 1 per query row; then floor(sum/256)
    # rows of M values (row checkpoints every 256 rows)
    rows = int(lens.sum()) // P.SDTW_ROW_CKPT_EVERY
    assert P.sdtw_checkpoint_floats(lens, 1000, 256) == lens.sum() * 3 + rows * 1000
    assert P.sdtw_checkpoint_floats(lens, 1024, 256) == lens.sum() * 3 + rows * 1024
    assert P.sdtw_checkpoint_floats(lens, 1025, 256) == lens.sum() * 4 + rows * 1025
    assert P.sdtw_checkpoint_floats(lens, 256, 256) == 0
    # (the row region is sized by the batch total: two rows here, one for
    # D(256, .) of the 511-row query and one that no query owns)
    short = np.array([511, 1], np.int32)
    assert P.sdtw_checkpoint_floats(short, 1000, 256) == 512 * 3 + 2 * 1000


def _bwd(L, lens, ref_len=100, kind=0, every=64, ckpt=FAKE, ws_bytes=1 << 40, **ptrs):
    h = np.ascontiguousarray(lens, dtype=np.int32)
    a = dict(q=FAKE, dlens=FAKE, r=FAKE, g=FAKE, c=FAKE, e=FAKE, gq=FAKE, gr=FAKE, ws=FAKE)
    a.update(ptrs)
    return L.lib.sdtw_backward(_vp(a["q"]), _vp(h.ctypes.data), _vp(a["dlens"]), h.size,
                               _vp(a["r"]), ref_len, kind, _vp(a["g"]), _vp(a["c"]), _vp(a["e"]),
                               _vp(ckpt), every, _vp(a["gq"]), _vp(a["gr"]), _vp(a["ws"]),
                               ws_bytes, _vp(0))


def test_backward_rejects_invalid_arguments(L):
    E = L.SDTW_ERR_INVALID_ARG
    for name in ("q", "dlens", "r", "g", "c", "e", "gq", "gr", "ws"):
        assert _bwd(L, [3, 4], **{name: 0}) == E, name
    assert _bwd(L, [3, 0]) == E
    assert _bwd(L, [3, 4], kind=5) == E
    assert _bwd(L, [3, 4], every=0) == E
    assert _bwd(L, [3, 4], every=24) == E
    assert _bwd(L, [3, 4], ref_len=1000, every=64, ckpt=0) == E   # checkpoints needed
    assert _bwd(L, [3, 4], ws_bytes=8) == L.SDTW_ERR_WORKSPACE
    assert _bwd(L, [8193], ref_len=100) == L.SDTW_ERR_UNSUPPORTED   # longer than 8,192 rows
    assert _bwd(L, [3, 4], ws=FAKE + 8) == E


def test_backward_workspace_sizes(L):
    import paper_2403_06931_amd as P
    lens = np.array([100, 1000, 2048], np.int32)
    ws = P.sdtw_backward_workspace_bytes(lens, 50000, 1024)
    # reference partials, plus the direction codes of at least one block
    # (2 bits per cell, rows padded by 63) per query
    assert ws >= 3 * 50000 * 4 + (lens.sum() + 63 * 3) * 1024 // 4
    assert ws < 2 << 30
    assert P.sdtw_backward_workspace_bytes(np.array([8192], np.int32), 100, 64) > 0
    assert P.sdtw_backward_workspace_bytes(np.array([8193], np.int32), 100, 64) == 0
    assert P.sdtw_backward_workspace_bytes(lens, 50000, 0) == 0
    assert P.sdtw_backward_workspace_bytes(lens, 50000, 24) == 0


def _zn(L, lens, batch=None, x=FAKE, dlens=FAKE, z=FAKE, ws=FAKE, ws_bytes=1 << 40):
    h = np.ascontiguousarray(lens, dtype=np.int32)
    b = h.size if batch is None else batch
    return L.lib.sdtw_znorm(_vp(x), _vp(h.ctypes.data if h.size else 0), _vp(dlens), b, _vp(z),
                            _vp(ws), ws_bytes, _vp(0))


def test_znorm_rejects_invalid_arguments(L):
    E = L.SDTW_ERR_INVALID_ARG
    for name in ("x", "dlens", "z", "ws"):
        assert _zn(L, [3, 4], **{name: 0}) == E, name
    assert _zn(L, [3, 0]) == E
    assert _zn(L, [3, -1]) == E
    assert _zn(L, [3, 4], batch=0) == E
    assert _zn(L, [3, 4], ws=FAKE + 8) == E
    assert _zn(L, [3, 4], ws_bytes=16) == L.SDTW_ERR_WORKSPACE


def test_znorm_workspace_sizes(L):
    import paper_2403_06931_amd as P
    a = P.sdtw_znorm_workspace_bytes(np.array([10, 20], np.int32))
    b = P.sdtw_znorm_workspace_bytes(np.array([10, 2_000_000], np.int32))
    assert 0 < a < b
    # 16 bytes of binary64 partials per 4,096-element chunk at least
    assert b >= 16 * (2_000_000 // 4096)
    assert P.sdtw_znorm_workspace_bytes(np.array([10, 0], np.int32)) == 0


def _al(L, lens, ref_len=100, kind=0, every=64, ckpt=FAKE, ws_bytes=1 << 40, **ptrs):
    h = np.ascontiguousarray(lens, dtype=np.int32)
    a = dict(q=FAKE, dlens=FAKE, r=FAKE, c=FAKE, e=FAKE, s=FAKE, lo=FAKE, hi=FAKE, ws=FAKE)
    a.update(ptrs)
    return L.lib.sdtw_align(_vp(a["q"]), _vp(h.ctypes.data), _vp(a["dlens"]), h.size,
                            _vp(a["r"]), ref_len, kind, _vp(a["c"]), _vp(a["e"]), _vp(ckpt),
                            every, _vp(a["s"]), _vp(a["lo"]), _vp(a["hi"]), _vp(a["ws"]),
                            ws_bytes, _vp(0))


def test_align_rejects_invalid_arguments(L):
    E = L.SDTW_ERR_INVALID_ARG
    for name in ("q", "dlens", "r", "c", "e", "s", "lo", "hi", "ws"):
        assert _al(L, [3, 4], **{name: 0}) == E, name
    assert _al(L, [3, 0]) == E
    assert _al(L, [3, 4], kind=2) == E
    assert _al(L, [3, 4], every=40) == E
    assert _al(L, [3, 4], ref_len=1000, ckpt=0) == E
    assert _al(L, [3, 4], ws=FAKE + 64) == E
    assert _al(L, [3, 4], ws_bytes=100) == L.SDTW_ERR_WORKSPACE
    assert _al(L, [8193]) == L.SDTW_ERR_UNSUPPORTED


def test_align_workspace_smaller_than_backward(L):
    import paper_2403_06931_amd as P
    lens = np.array([1000] * 256, np.int32)
    a = P.sdtw_align_workspace_bytes(lens, 50000, 1024)
    b = P.sdtw_backward_workspace_bytes(lens, 50000, 1024)
    # no per-query reference partials (256 x 50,000 floats)
    assert 0 < a and a + 256 * 50000 * 4 <= b
    assert P.sdtw_align_workspace_bytes(np.array([8193], np.int32), 100, 64) == 0


def test_forward_f16_validation(L):
    import paper_2403_06931_amd as P
    h = np.array([10, 10, 7], np.int32)
    assert P.sdtw_forward_f16_workspace_bytes(h, 1000) > 0
    assert P.sdtw_forward_f16_workspace_bytes(np.array([10, 11], np.int32), 1000) == 0
    hh = np.ascontiguousarray([10, 11], dtype=np.int32)
    call = lambda lens, **k: L.lib.sdtw_forward_f16(
        _vp(k.get("q", FAKE)), _vp(lens.ctypes.data), _vp(FAKE), lens.size, _vp(FAKE), 100,
        k.get("kind", 0), _vp(k.get("c", FAKE)), _vp(FAKE), -1, _vp(k.get("ws", FAKE)),
        1 << 40, _vp(0))
    assert call(hh) == L.SDTW_ERR_UNSUPPORTED            # a pair of unequal lengths
    h2 = np.ascontiguousarray([10, 10], dtype=np.int32)
    assert call(h2, q=0) == L.SDTW_ERR_INVALID_ARG
    assert call(h2, c=0) == L.SDTW_ERR_INVALID_ARG
    assert call(h2, kind=3) == L.SDTW_ERR_INVALID_ARG
    assert call(h2, ws=FAKE + 4) == L.SDTW_ERR_INVALID_ARG


def test_forward_pruned_validation(L):
    FAKE = 1 << 20
    h = np.ascontiguousarray([10, 12], dtype=np.int32)
    call = lambda **k: L.lib.sdtw_forward_pruned(
        _vp(k.get("q", FAKE)), _vp(h.ctypes.data), _vp(FAKE), h.size, _vp(FAKE), 100,
        k.get("tau", 1.0), _vp(k.get("c", FAKE)), _vp(FAKE), k.get("v", -1), k.get("flags", 0),
        _vp(k.get("ws", FAKE)), k.get("wsb", 1 << 40), _vp(0))
    assert call(tau=float("nan")) == L.SDTW_ERR_INVALID_ARG
    assert call(flags=L.SDTW_F_CHECKPOINT) == L.SDTW_ERR_INVALID_ARG
    assert call(flags=8) == L.SDTW_ERR_INVALID_ARG
    assert call(q=0) == L.SDTW_ERR_INVALID_ARG
    assert call(c=0) == L.SDTW_ERR_INVALID_ARG
    assert call(ws=FAKE + 4) == L.SDTW_ERR_INVALID_ARG
    assert call(wsb=16) == L.SDTW_ERR_WORKSPACE
    assert call(v=10_000) == L.SDTW_ERR_UNSUPPORTED


def test_forward_u8_validation(L):
    import paper_2403_06931_amd as P
    FAKE = 1 << 20
    h = np.ascontiguousarray([10, 12], dtype=np.int32)
    assert P.sdtw_forward_u8_workspace_bytes(h, 1000) > P.sdtw_forward_workspace_bytes(h, 1000, 0, 0)
    assert P.sdtw_forward_u8_workspace_bytes(np.array([40000], np.int32), 1000) > 0
    call = lambda hh=h, **k: L.lib.sdtw_forward_u8(
        _vp(k.get("q", FAKE)), _vp(hh.ctypes.data), _vp(FAKE), hh.size, _vp(FAKE), 100,
        _vp(k.get("c", FAKE)), _vp(FAKE), _vp(k.get("book", FAKE)), k.get("v", -1),
        _vp(k.get("ws", FAKE)), k.get("wsb", 1 << 40), _vp(0))
    assert call(q=0) == L.SDTW_ERR_INVALID_ARG
    assert call(c=0) == L.SDTW_ERR_INVALID_ARG
    assert call(book=0) == L.SDTW_ERR_INVALID_ARG
    assert call(ws=FAKE + 4) == L.SDTW_ERR_INVALID_ARG
    assert call(wsb=16) == L.SDTW_ERR_WORKSPACE
    assert call(v=10_000) == L.SDTW_ERR_UNSUPPORTED
    assert call(np.ascontiguousarray([5, 0], dtype=np.int32)) == L.SDTW_ERR_INVALID_ARG


def test_binding_checks_sizes_before_any_call():
    """The Python binding compares every tensor's dtype and size with what the
    host lengths imply before calling the library (a short buffer would be
    written out of bounds on the GPU), and reports it the same way with or
    without a GPU."""
    import torch

    import paper_2403_06931_amd as P
    h = np.array([3, 5], np.int32)
    q = torch.zeros(8)
    l = torch.from_numpy(h)
    r = torch.zeros(100)

    def raises(fn, what):
        with pytest.raises(ValueError, match=what):
            fn()
    raises(lambda: P.sdtw_forward(torch.zeros(7), h, l, r), "queries must hold exactly 8")
    raises(lambda: P.sdtw_forward(q, h, torch.from_numpy(h[:1].copy()), r),
           "query_lens must hold exactly 2")
    raises(lambda: P.sdtw_forward(q, h, l.to(torch.int64), r), "query_lens must be torch.int32")
    raises(lambda: P.sdtw_forward(q.double(), h, l, r), "queries must be torch.float64|queries must be torch.float32")
    raises(lambda: P.sdtw_forward(q, h, l, torch.zeros(0)), "reference must hold at least one")
    raises(lambda: P.sdtw_forward(q, h, l, r, cost=torch.zeros(1)), "cost must hold at least 2")
    raises(lambda: P.sdtw_forward(q, h, l, r, end_pos=torch.zeros(2)), "end_pos must be torch.int64")
    raises(lambda: P.sdtw_forward(q, h, l, r, ckpt=None, ckpt_every=32,
                                  flags=P.SDTW_F_CHECKPOINT), "ckpt is required")
    raises(lambda: P.sdtw_forward(q, h, l, r, ckpt=torch.zeros(5), ckpt_every=32,
                                  flags=P.SDTW_F_CHECKPOINT), "ckpt must hold at least 24")
    raises(lambda: P.sdtw_backward(q, h, l, r, 0, torch.zeros(3), torch.zeros(2),
                                   torch.zeros(2, dtype=torch.int64), torch.zeros(24), 32),
           "grad_cost must hold exactly 2")
    raises(lambda: P.sdtw_backward(q, h, l, r, 0, torch.zeros(2), torch.zeros(2),
                                   torch.zeros(2, dtype=torch.int64), torch.zeros(20), 32),
           "ckpt must hold at least 24")
    raises(lambda: P.sdtw_backward(q, h, l, r, 0, torch.zeros(2), torch.zeros(2),
                                   torch.zeros(2, dtype=torch.int64), torch.zeros(24), 32,
                                   grad_reference=torch.zeros(99)),
           "grad_reference must hold at least 100")
    raises(lambda: P.sdtw_align(q, h, l, r, 0, torch.zeros(1),
                                torch.zeros(2, dtype=torch.int64), torch.zeros(24), 32),
           "cost must hold at least 2")
    raises(lambda: P.sdtw_forward_u8(q, h, l, r, codebook=torch.zeros(1)),
           "codebook must hold at least 2")
    raises(lambda: P.sdtw_znorm(torch.zeros(9), h, l), "x must hold exactly 8")
    raises(lambda: P.sdtw_znorm(q, h, l, out=torch.zeros(9)), "out must hold exactly 8")
    # right sizes: the remaining complaint is the device
    raises(lambda: P.sdtw_forward(q, h, l, r), "must be a CUDA tensor")


def test_hip_failure_reported_without_a_device(L):
    """With valid arguments but no usable GPU, the launch fails and the call
    returns SDTW_ERR_HIP (every pointer is a placeholder that only a kernel
    would dereference, so this runs only where no GPU is visible)."""
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is visible: the placeholder pointers must not reach a kernel")
    rc = _fwd(L, [3, 4], ref_len=100, ws_bytes=1 << 20)
    assert rc == L.SDTW_ERR_HIP, L.status_string(rc)


def _fwd_noalloc(L, lens, ref_len=100, kind=0, flags=0, q=FAKE, r=FAKE, c=FAKE, e=FAKE,
                 ckpt=0, every=0, variant=-1, dlens=FAKE):
    h = np.ascontiguousarray(lens, dtype=np.int32)
    return L.lib.sdtw_forward_noalloc(_vp(q), _vp(h.ctypes.data if h.size else 0), _vp(dlens),
                                      h.size, _vp(r), ref_len, kind, _vp(c), _vp(e), _vp(ckpt),
                                      every, variant, flags, _vp(0))


def test_forward_noalloc_validation(L):
    """The allocation-free forward validates like sdtw_forward and refuses,
    before any HIP call, a batch whose workspace exceeds its fixed array."""
    E = L.SDTW_ERR_INVALID_ARG
    assert _fwd_noalloc(L, [3, 4], q=0) == E
    assert _fwd_noalloc(L, [3, 4], c=0) == E
    assert _fwd_noalloc(L, [3, 0]) == E
    assert _fwd_noalloc(L, [3, 4], kind=2) == E
    assert _fwd_noalloc(L, [3, 4], flags=4) == E
    assert _fwd_noalloc(L, [3, 4], flags=1, every=24) == E       # not a multiple of 16
    assert _fwd_noalloc(L, [3, 4], variant=10**6) == L.SDTW_ERR_UNSUPPORTED
    import paper_2403_06931_amd as P
    big = _variant_of((8, 8, 4, 32, 1))
    lens = np.full(40, 5000, np.int32)       # 40 row-buffer slots of 800 KB
    assert P.sdtw_forward_workspace_bytes(lens, 200_000, 0, big) > L.SDTW_NOALLOC_SCRATCH_BYTES
    assert _fwd_noalloc(L, lens, ref_len=200_000, variant=big) == L.SDTW_ERR_WORKSPACE


def test_forward_noalloc_without_a_device(L):
    """Valid arguments but no GPU: the array's address cannot be looked up
    and the call returns SDTW_ERR_HIP."""
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is visible: the placeholder pointers must not reach a kernel")
    rc = _fwd_noalloc(L, [3, 4], ref_len=100)
    assert rc == L.SDTW_ERR_HIP, L.status_string(rc)


def test_persistent_grid_flag(L):
    """The grid-size field of the flags: accepted for 0..8 wavefronts per
    SIMD, refused above; the persistent workspace holds one row-buffer slot
    per workgroup of the grid it asks for."""
    import paper_2403_06931_amd as P
    small = _variant_of((8, 8, 1, 16, 1))           # 512 rows per pass, one wavefront
    lens = np.full(10000, 300, np.int32)
    lens[7] = 3000                                   # one query needs several passes
    row = -(-1000 // 64) * 64 * 4
    sizes = {}
    for wps in (1, 2, 3, 4, 8):
        f = P.SDTW_F_PERSISTENT | P.SDTW_F_WAVES_PER_SIMD(wps)
        sizes[wps] = P.sdtw_forward_workspace_bytes(lens, 1000, f, small)
        assert 256 * 4 * wps * row <= sizes[wps] < 256 * 4 * wps * row + 2 * 10000 * 8 + 4096
    assert sizes[2] == P.sdtw_forward_workspace_bytes(lens, 1000, P.SDTW_F_PERSISTENT, small)
    assert P.sdtw_forward_workspace_bytes(
        lens, 1000, P.SDTW_F_PERSISTENT | P.SDTW_F_WAVES_PER_SIMD(9), small) == 0
    assert _fwd(L, [3, 4], flags=P.SDTW_F_PERSISTENT | P.SDTW_F_WAVES_PER_SIMD(9)) == \
        L.SDTW_ERR_INVALID_ARG
    assert _fwd(L, [3, 4], flags=P.SDTW_F_PERSISTENT | (1 << 12)) == L.SDTW_ERR_INVALID_ARG
