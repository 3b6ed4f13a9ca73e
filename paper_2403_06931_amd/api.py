"""Python binding of the C ABI with the same names (argument marshalling only).

PyTorch supplies device memory and the current stream; every arithmetic step
runs in the library's HIP kernels.  Functions take torch tensors that live on
the GPU, plus a host (NumPy) copy of the query lengths, which the library uses
for validation, workspace sizing and scheduling.

Before each library call the binding checks what the library cannot see
from its pointers: that every tensor has the dtype, layout and size the host
lengths imply (a short buffer would otherwise be written out of bounds on
the GPU), then that every tensor is on the GPU, and, once per lengths tensor
and version, that the device lengths hold the host lengths.  A mismatch
raises ValueError and nothing is launched.
"""
from __future__ import annotations

import collections
import ctypes
from typing import Optional, Tuple

import numpy as np
import torch

from . import _lib
from ._lib import (SDTW_COST_ABSOLUTE, SDTW_COST_SQUARED, SDTW_F_CHECKPOINT,  # noqa: F401
                   SDTW_F_PERSISTENT, SDTW_F_WAVES_PER_SIMD, SDTW_ROW_CKPT_EVERY, SdtwError,
                   check)

_ALIGN = 256


def _host_lens(lens) -> np.ndarray:
    if isinstance(lens, torch.Tensor):
        lens = lens.detach().to("cpu").numpy()
    a = np.ascontiguousarray(np.asarray(lens), dtype=np.int32)
    if a.ndim != 1:
        raise ValueError("query lengths must be one-dimensional")
    return a


def _hp(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _dp(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr() if t is not None else 0)


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check(name: str, t, dtype, numel: Optional[int] = None,
           at_least: Optional[int] = None, optional: bool = False) -> None:
    """Type, dtype, layout and size (the device is checked afterwards, for
    every argument at once, so a wrong size is reported the same way with or
    without a GPU)."""
    if t is None and optional:
        return
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must hold exactly {numel} values, it holds {t.numel()}")
    if at_least is not None and t.numel() < at_least:
        raise ValueError(f"{name} must hold at least {at_least} values, it holds {t.numel()}")


def _on_gpu(**tensors) -> None:
    for name, t in tensors.items():
        if t is not None and not t.is_cuda:
            raise ValueError(f"{name} must be a CUDA tensor")


def _new(t: Optional[torch.Tensor], dtype, n: int, device) -> torch.Tensor:
    return t if t is not None else torch.empty(n, dtype=dtype, device=device)


# (pointer, device, numel) of device length tensors already compared with the
# host lengths -> (tensor version, host lengths bytes)
_VERIFIED: "collections.OrderedDict[tuple, tuple]" = collections.OrderedDict()


def _check_lens_match(h: np.ndarray, lens: torch.Tensor, name: str) -> None:
    """The device lengths must hold the host lengths: the kernels take loop
    bounds and offsets from them.  Compared once per tensor version (one
    device-to-host copy), not inside a graph capture."""
    key = (lens.data_ptr(), lens.device.index, lens.numel())
    tag = (lens._version, h.tobytes())
    if _VERIFIED.get(key) == tag:
        return
    if torch.cuda.is_current_stream_capturing():
        raise ValueError(f"{name} has not been checked against the host lengths; make one "
                         "call outside the graph capture first")
    if not np.array_equal(lens.detach().cpu().numpy(), h):
        raise ValueError(f"{name} (device) does not hold the host lengths")
    _VERIFIED[key] = tag
    _VERIFIED.move_to_end(key)
    while len(_VERIFIED) > 64:
        _VERIFIED.popitem(last=False)


def _check_batch(h: np.ndarray, queries, query_lens, reference=None,
                 qname: str = "queries", lname: str = "query_lens") -> None:
    if h.size < 1:
        raise ValueError("the batch must hold at least one query")
    _check(qname, queries, torch.float32, numel=int(h.astype(np.int64).sum()))
    _check(lname, query_lens, torch.int32, numel=h.size)
    if reference is not None:
        _check("reference", reference, torch.float32)
        if reference.numel() < 1:
            raise ValueError("reference must hold at least one value")


def workspace(nbytes: int, device) -> torch.Tensor:
    """A device byte buffer of at least nbytes, 256-byte aligned (torch's
    caching allocator returns 512-byte aligned blocks)."""
    t = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
    if t.data_ptr() % _ALIGN:
        raise RuntimeError("allocator returned a misaligned workspace")
    return t


def _workspace_arg(buf: Optional[torch.Tensor], need: int, device) -> torch.Tensor:
    if buf is None:
        return workspace(need, device)
    _check("workspace_buf", buf, torch.uint8)
    _on_gpu(workspace_buf=buf)
    return buf


def sdtw_variant_count() -> int:
    return int(_lib.lib.sdtw_variant_count())


def sdtw_variant_info(v: int) -> Tuple[int, int, int, int, int]:
    """(rows per lane, columns per step, wavefronts per query, steps per barrier,
    lane exchange: 1 through LDS, 0 DPP lane shift)."""
    r, t, w, k, x = (ctypes.c_int32() for _ in range(5))
    check(_lib.lib.sdtw_variant_info(int(v), ctypes.byref(r), ctypes.byref(t), ctypes.byref(w),
                                     ctypes.byref(k), ctypes.byref(x)), "sdtw_variant_info")
    return r.value, t.value, w.value, k.value, x.value


def sdtw_default_variant(h_query_lens, ref_len: int, flags: int = 0) -> int:
    h = _host_lens(h_query_lens)
    return int(_lib.lib.sdtw_default_variant(_hp(h), h.size, int(ref_len), int(flags)))


def sdtw_forward_workspace_bytes(h_query_lens, ref_len: int, flags: int = 0,
                                 variant: int = -1) -> int:
    h = _host_lens(h_query_lens)
    return int(_lib.lib.sdtw_forward_workspace_bytes(_hp(h), h.size, int(ref_len), int(flags),
                                                     int(variant)))


def sdtw_workspace_bytes(h_query_lens, ref_len: int, flags: int = 0,
                         ckpt_every: int = 0) -> int:
    h = _host_lens(h_query_lens)
    return int(_lib.lib.sdtw_workspace_bytes(_hp(h), h.size, int(ref_len), int(flags),
                                             int(ckpt_every)))


def sdtw_checkpoint_floats(h_query_lens, ref_len: int, ckpt_every: int) -> int:
    h = _host_lens(h_query_lens)
    return int(_lib.lib.sdtw_checkpoint_floats(_hp(h), h.size, int(ref_len), int(ckpt_every)))


def sdtw_backward_workspace_bytes(h_query_lens, ref_len: int, ckpt_every: int) -> int:
    h = _host_lens(h_query_lens)
    return int(_lib.lib.sdtw_backward_workspace_bytes(_hp(h), h.size, int(ref_len),
                                                      int(ckpt_every)))


def _ckpt_arg(h, ref_len: int, ckpt: Optional[torch.Tensor], ckpt_every: int,
              required: bool) -> None:
    """A checkpoint buffer, when one is used, must hold the forward's columns."""
    if not required:
        return
    need = sdtw_checkpoint_floats(h, ref_len, ckpt_every)
    if need == 0:
        if ckpt is not None:
            _check("ckpt", ckpt, torch.float32)
        return
    if ckpt is None:
        raise ValueError(f"ckpt is required: {need} checkpoint values for this batch")
    _check("ckpt", ckpt, torch.float32, at_least=need)


def sdtw_forward(queries: torch.Tensor, h_query_lens, query_lens: torch.Tensor,
                 reference: torch.Tensor, cost_kind: int = SDTW_COST_SQUARED, *,
                 cost: Optional[torch.Tensor] = None, end_pos: Optional[torch.Tensor] = None,
                 ckpt: Optional[torch.Tensor] = None, ckpt_every: int = 0,
                 variant: int = -1, flags: int = 0,
                 workspace_buf: Optional[torch.Tensor] = None,
                 stream=None) -> Tuple[torch.Tensor, torch.Tensor]:
    """Per-query (cost float32 [B], end_pos int64 [B]) on the GPU."""
    h = _host_lens(h_query_lens)
    _check_batch(h, queries, query_lens, reference)
    b = h.size
    _check("cost", cost, torch.float32, at_least=b, optional=True)
    _check("end_pos", end_pos, torch.int64, at_least=b, optional=True)
    _ckpt_arg(h, reference.numel(), ckpt, ckpt_every, bool(flags & SDTW_F_CHECKPOINT))
    _on_gpu(queries=queries, query_lens=query_lens, reference=reference, cost=cost,
            end_pos=end_pos, ckpt=ckpt)
    _check_lens_match(h, query_lens, "query_lens")
    dev = queries.device
    cost = _new(cost, torch.float32, b, dev)
    end_pos = _new(end_pos, torch.int64, b, dev)
    need = sdtw_forward_workspace_bytes(h, reference.numel(), flags, variant)
    if need == 0:
        raise SdtwError(_lib.SDTW_ERR_INVALID_ARG, "sdtw_forward_workspace_bytes")
    workspace_buf = _workspace_arg(workspace_buf, need, dev)
    st = _lib.lib.sdtw_forward(
        _dp(queries), _hp(h), _dp(query_lens), b, _dp(reference), reference.numel(),
        int(cost_kind), _dp(cost), _dp(end_pos), _dp(ckpt), int(ckpt_every), int(variant),
        int(flags), _dp(workspace_buf), workspace_buf.numel(), _stream(stream))
    check(st, "sdtw_forward")
    return cost, end_pos


def sdtw_forward_noalloc(queries: torch.Tensor, h_query_lens, query_lens: torch.Tensor,
                         reference: torch.Tensor, cost_kind: int = SDTW_COST_SQUARED, *,
                         cost: torch.Tensor, end_pos: torch.Tensor,
                         ckpt: Optional[torch.Tensor] = None, ckpt_every: int = 0,
                         variant: int = -1, flags: int = 0,
                         stream=None) -> Tuple[torch.Tensor, torch.Tensor]:
    """sdtw_forward without a workspace (the library's fixed per-GPU array
    serves instead) and without allocations: the caller passes the outputs.
    A batch whose workspace would exceed SDTW_NOALLOC_SCRATCH_BYTES raises
    SdtwError (SDTW_ERR_WORKSPACE).  Calls that overlap on one GPU race."""
    h = _host_lens(h_query_lens)
    _check_batch(h, queries, query_lens, reference)
    b = h.size
    _check("cost", cost, torch.float32, at_least=b)
    _check("end_pos", end_pos, torch.int64, at_least=b)
    _ckpt_arg(h, reference.numel(), ckpt, ckpt_every, bool(flags & SDTW_F_CHECKPOINT))
    _on_gpu(queries=queries, query_lens=query_lens, reference=reference, cost=cost,
            end_pos=end_pos, ckpt=ckpt)
    _check_lens_match(h, query_lens, "query_lens")
    st = _lib.lib.sdtw_forward_noalloc(
        _dp(queries), _hp(h), _dp(query_lens), b, _dp(reference), reference.numel(),
        int(cost_kind), _dp(cost), _dp(end_pos), _dp(ckpt), int(ckpt_every), int(variant),
        int(flags), _stream(stream))
    check(st, "sdtw_forward_noalloc")
    return cost, end_pos


def sdtw_forward_pruned(queries: torch.Tensor, h_query_lens, query_lens: torch.Tensor,
                        reference: torch.Tensor, prune_tau: float, *,
                        cost: Optional[torch.Tensor] = None,
                        end_pos: Optional[torch.Tensor] = None,
                        variant: int = -1, flags: int = 0,
                        workspace_buf: Optional[torch.Tensor] = None,
                        stream=None) -> Tuple[torch.Tensor, torch.Tensor]:
    """Squared-cost forward with early pruning: a pair with |q - r| > prune_tau
    costs +inf.  Same outputs and workspace as sdtw_forward (flags 0 or
    SDTW_F_PERSISTENT)."""
    h = _host_lens(h_query_lens)
    _check_batch(h, queries, query_lens, reference)
    b = h.size
    _check("cost", cost, torch.float32, at_least=b, optional=True)
    _check("end_pos", end_pos, torch.int64, at_least=b, optional=True)
    _on_gpu(queries=queries, query_lens=query_lens, reference=reference, cost=cost,
            end_pos=end_pos)
    _check_lens_match(h, query_lens, "query_lens")
    dev = queries.device
    cost = _new(cost, torch.float32, b, dev)
    end_pos = _new(end_pos, torch.int64, b, dev)
    need = sdtw_forward_workspace_bytes(h, reference.numel(), flags, variant)
    if need == 0:
        raise SdtwError(_lib.SDTW_ERR_INVALID_ARG, "sdtw_forward_workspace_bytes")
    workspace_buf = _workspace_arg(workspace_buf, need, dev)
    st = _lib.lib.sdtw_forward_pruned(
        _dp(queries), _hp(h), _dp(query_lens), b, _dp(reference), reference.numel(),
        float(prune_tau), _dp(cost), _dp(end_pos), int(variant), int(flags),
        _dp(workspace_buf), workspace_buf.numel(), _stream(stream))
    check(st, "sdtw_forward_pruned")
    return cost, end_pos


def sdtw_forward_u8_workspace_bytes(h_query_lens, ref_len: int) -> int:
    h = _host_lens(h_query_lens)
    return int(_lib.lib.sdtw_forward_u8_workspace_bytes(_hp(h), h.size, int(ref_len)))


def sdtw_forward_u8(queries: torch.Tensor, h_query_lens, query_lens: torch.Tensor,
                    reference: torch.Tensor, *,
                    cost: Optional[torch.Tensor] = None,
                    end_pos: Optional[torch.Tensor] = None,
                    codebook: Optional[torch.Tensor] = None,
                    variant: int = -1,
                    workspace_buf: Optional[torch.Tensor] = None,
                    stream=None) -> Tuple[torch.Tensor, torch.Tensor, torch.Tensor]:
    """Forward on uint8 codes (codebook from the reference, binary32 DP of the
    codes) -> (cost float32 [B] in step^2 units, end_pos int64 [B],
    codebook float32 [2] = lo, hi)."""
    h = _host_lens(h_query_lens)
    _check_batch(h, queries, query_lens, reference)
    b = h.size
    _check("cost", cost, torch.float32, at_least=b, optional=True)
    _check("end_pos", end_pos, torch.int64, at_least=b, optional=True)
    _check("codebook", codebook, torch.float32, at_least=2, optional=True)
    _on_gpu(queries=queries, query_lens=query_lens, reference=reference, cost=cost,
            end_pos=end_pos, codebook=codebook)
    _check_lens_match(h, query_lens, "query_lens")
    dev = queries.device
    cost = _new(cost, torch.float32, b, dev)
    end_pos = _new(end_pos, torch.int64, b, dev)
    codebook = _new(codebook, torch.float32, 2, dev)
    need = sdtw_forward_u8_workspace_bytes(h, reference.numel())
    if need == 0:
        raise SdtwError(_lib.SDTW_ERR_INVALID_ARG, "sdtw_forward_u8_workspace_bytes")
    workspace_buf = _workspace_arg(workspace_buf, need, dev)
    st = _lib.lib.sdtw_forward_u8(
        _dp(queries), _hp(h), _dp(query_lens), b, _dp(reference), reference.numel(),
        _dp(cost), _dp(end_pos), _dp(codebook), int(variant), _dp(workspace_buf),
        workspace_buf.numel(), _stream(stream))
    check(st, "sdtw_forward_u8")
    return cost, end_pos, codebook


def sdtw_backward(queries: torch.Tensor, h_query_lens, query_lens: torch.Tensor,
                  reference: torch.Tensor, cost_kind: int, grad_cost: torch.Tensor,
                  cost: torch.Tensor, end_pos: torch.Tensor, ckpt: Optional[torch.Tensor],
                  ckpt_every: int, *,
                  grad_queries: Optional[torch.Tensor] = None,
                  grad_reference: Optional[torch.Tensor] = None,
                  workspace_buf: Optional[torch.Tensor] = None,
                  stream=None) -> Tuple[torch.Tensor, torch.Tensor]:
    """Walk-back gradient (grad_queries packed like queries, grad_reference [M]);
    cost and end_pos are the forward's outputs."""
    h = _host_lens(h_query_lens)
    _check_batch(h, queries, query_lens, reference)
    b = h.size
    _check("grad_cost", grad_cost, torch.float32, numel=b)
    _check("cost", cost, torch.float32, at_least=b)
    _check("end_pos", end_pos, torch.int64, at_least=b)
    _ckpt_arg(h, reference.numel(), ckpt, ckpt_every, True)
    _check("grad_queries", grad_queries, torch.float32, at_least=queries.numel(), optional=True)
    _check("grad_reference", grad_reference, torch.float32, at_least=reference.numel(),
           optional=True)
    _on_gpu(queries=queries, query_lens=query_lens, reference=reference, grad_cost=grad_cost,
            cost=cost, end_pos=end_pos, ckpt=ckpt, grad_queries=grad_queries,
            grad_reference=grad_reference)
    _check_lens_match(h, query_lens, "query_lens")
    dev = queries.device
    grad_queries = _new(grad_queries, torch.float32, queries.numel(), dev)
    grad_reference = _new(grad_reference, torch.float32, reference.numel(), dev)
    need = sdtw_backward_workspace_bytes(h, reference.numel(), ckpt_every)
    if need == 0:
        raise SdtwError(_lib.SDTW_ERR_INVALID_ARG, "sdtw_backward_workspace_bytes")
    workspace_buf = _workspace_arg(workspace_buf, need, dev)
    st = _lib.lib.sdtw_backward(
        _dp(queries), _hp(h), _dp(query_lens), b, _dp(reference), reference.numel(),
        int(cost_kind), _dp(grad_cost), _dp(cost), _dp(end_pos), _dp(ckpt), int(ckpt_every),
        _dp(grad_queries), _dp(grad_reference), _dp(workspace_buf), workspace_buf.numel(),
        _stream(stream))
    check(st, "sdtw_backward")
    return grad_queries, grad_reference


def sdtw_forward_f16_workspace_bytes(h_query_lens, ref_len: int) -> int:
    h = _host_lens(h_query_lens)
    return int(_lib.lib.sdtw_forward_f16_workspace_bytes(_hp(h), h.size, int(ref_len)))


def sdtw_forward_f16(queries: torch.Tensor, h_query_lens, query_lens: torch.Tensor,
                     reference: torch.Tensor, cost_kind: int = SDTW_COST_SQUARED, *,
                     cost: Optional[torch.Tensor] = None,
                     end_pos: Optional[torch.Tensor] = None, variant: int = -1,
                     workspace_buf: Optional[torch.Tensor] = None,
                     stream=None) -> Tuple[torch.Tensor, torch.Tensor]:
    """sDTW in binary16 arithmetic on float32 inputs: (cost float32 [B] holding
    binary16 values, end_pos int64 [B]).  Queries 2i and 2i+1 must have equal
    lengths."""
    h = _host_lens(h_query_lens)
    _check_batch(h, queries, query_lens, reference)
    b = h.size
    _check("cost", cost, torch.float32, at_least=b, optional=True)
    _check("end_pos", end_pos, torch.int64, at_least=b, optional=True)
    _on_gpu(queries=queries, query_lens=query_lens, reference=reference, cost=cost,
            end_pos=end_pos)
    _check_lens_match(h, query_lens, "query_lens")
    dev = queries.device
    cost = _new(cost, torch.float32, b, dev)
    end_pos = _new(end_pos, torch.int64, b, dev)
    need = sdtw_forward_f16_workspace_bytes(h, reference.numel())
    if need == 0:
        raise SdtwError(_lib.SDTW_ERR_UNSUPPORTED, "sdtw_forward_f16_workspace_bytes")
    workspace_buf = _workspace_arg(workspace_buf, need, dev)
    st = _lib.lib.sdtw_forward_f16(
        _dp(queries), _hp(h), _dp(query_lens), b, _dp(reference), reference.numel(),
        int(cost_kind), _dp(cost), _dp(end_pos), int(variant), _dp(workspace_buf),
        workspace_buf.numel(), _stream(stream))
    check(st, "sdtw_forward_f16")
    return cost, end_pos


def sdtw_align_workspace_bytes(h_query_lens, ref_len: int, ckpt_every: int) -> int:
    h = _host_lens(h_query_lens)
    return int(_lib.lib.sdtw_align_workspace_bytes(_hp(h), h.size, int(ref_len),
                                                   int(ckpt_every)))


def sdtw_align(queries: torch.Tensor, h_query_lens, query_lens: torch.Tensor,
               reference: torch.Tensor, cost_kind: int, cost: torch.Tensor,
               end_pos: torch.Tensor, ckpt: Optional[torch.Tensor], ckpt_every: int, *,
               workspace_buf: Optional[torch.Tensor] = None,
               stream=None) -> Tuple[torch.Tensor, torch.Tensor, torch.Tensor]:
    """Optimal alignment path of every query: (start_pos int64 [B], path_lo,
    path_hi int32 packed like queries), the reference columns matched to each
    query element; cost, end_pos and ckpt come from a checkpointed forward."""
    h = _host_lens(h_query_lens)
    _check_batch(h, queries, query_lens, reference)
    b = h.size
    _check("cost", cost, torch.float32, at_least=b)
    _check("end_pos", end_pos, torch.int64, at_least=b)
    _ckpt_arg(h, reference.numel(), ckpt, ckpt_every, True)
    _on_gpu(queries=queries, query_lens=query_lens, reference=reference, cost=cost,
            end_pos=end_pos, ckpt=ckpt)
    _check_lens_match(h, query_lens, "query_lens")
    dev = queries.device
    start = torch.empty(b, dtype=torch.int64, device=dev)
    lo = torch.empty(queries.numel(), dtype=torch.int32, device=dev)
    hi = torch.empty(queries.numel(), dtype=torch.int32, device=dev)
    need = sdtw_align_workspace_bytes(h, reference.numel(), ckpt_every)
    if need == 0:
        raise SdtwError(_lib.SDTW_ERR_INVALID_ARG, "sdtw_align_workspace_bytes")
    workspace_buf = _workspace_arg(workspace_buf, need, dev)
    st = _lib.lib.sdtw_align(
        _dp(queries), _hp(h), _dp(query_lens), b, _dp(reference), reference.numel(),
        int(cost_kind), _dp(cost), _dp(end_pos), _dp(ckpt), int(ckpt_every), _dp(start),
        _dp(lo), _dp(hi), _dp(workspace_buf), workspace_buf.numel(), _stream(stream))
    check(st, "sdtw_align")
    return start, lo, hi


def sdtw_znorm_workspace_bytes(h_lens) -> int:
    h = _host_lens(h_lens)
    return int(_lib.lib.sdtw_znorm_workspace_bytes(_hp(h), h.size))


def sdtw_znorm(x: torch.Tensor, h_lens, lens: torch.Tensor, *,
               out: Optional[torch.Tensor] = None,
               workspace_buf: Optional[torch.Tensor] = None,
               stream=None) -> torch.Tensor:
    """Z-normalise every series of the packed batch x (float32, lengths h_lens);
    out may be x itself."""
    h = _host_lens(h_lens)
    _check_batch(h, x, lens, qname="x", lname="lens")
    _check("out", out, torch.float32, numel=x.numel(), optional=True)
    _on_gpu(x=x, lens=lens, out=out)
    _check_lens_match(h, lens, "lens")
    if out is None:
        out = torch.empty_like(x)
    need = sdtw_znorm_workspace_bytes(h)
    if need == 0:
        raise SdtwError(_lib.SDTW_ERR_INVALID_ARG, "sdtw_znorm_workspace_bytes")
    workspace_buf = _workspace_arg(workspace_buf, need, x.device)
    st = _lib.lib.sdtw_znorm(_dp(x), _hp(h), _dp(lens), h.size, _dp(out), _dp(workspace_buf),
                             workspace_buf.numel(), _stream(stream))
    check(st, "sdtw_znorm")
    return out
