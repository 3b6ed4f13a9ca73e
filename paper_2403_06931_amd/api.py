"""Python binding of the C ABI with the same names (argument marshalling only).

PyTorch supplies device memory and the current stream; every arithmetic step
runs in the library's HIP kernels.  Functions take torch tensors that live on
the GPU, plus a host (NumPy) copy of the query lengths, which the library uses
for validation, workspace sizing and scheduling.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Tuple

import numpy as np
import torch

from . import _lib
from ._lib import (SDTW_COST_ABSOLUTE, SDTW_COST_SQUARED, SDTW_F_CHECKPOINT,  # noqa: F401
                   SDTW_F_PERSISTENT, SdtwError, check)

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


def _require_cuda(name: str, t: torch.Tensor, dtype) -> None:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def workspace(nbytes: int, device) -> torch.Tensor:
    """A device byte buffer of at least nbytes, 256-byte aligned (torch's
    caching allocator returns 512-byte aligned blocks)."""
    t = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
    if t.data_ptr() % _ALIGN:
        raise RuntimeError("allocator returned a misaligned workspace")
    return t


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


def sdtw_forward_workspace_bytes(h_query_lens, ref_len: int, flags: int = 0) -> int:
    h = _host_lens(h_query_lens)
    return int(_lib.lib.sdtw_forward_workspace_bytes(_hp(h), h.size, int(ref_len), int(flags)))


def sdtw_checkpoint_floats(h_query_lens, ref_len: int, ckpt_every: int) -> int:
    h = _host_lens(h_query_lens)
    return int(_lib.lib.sdtw_checkpoint_floats(_hp(h), h.size, int(ref_len), int(ckpt_every)))


def sdtw_backward_workspace_bytes(h_query_lens, ref_len: int, ckpt_every: int) -> int:
    h = _host_lens(h_query_lens)
    return int(_lib.lib.sdtw_backward_workspace_bytes(_hp(h), h.size, int(ref_len),
                                                      int(ckpt_every)))


def sdtw_forward(queries: torch.Tensor, h_query_lens, query_lens: torch.Tensor,
                 reference: torch.Tensor, cost_kind: int = SDTW_COST_SQUARED, *,
                 cost: Optional[torch.Tensor] = None, end_pos: Optional[torch.Tensor] = None,
                 ckpt: Optional[torch.Tensor] = None, ckpt_every: int = 0,
                 variant: int = -1, flags: int = 0,
                 workspace_buf: Optional[torch.Tensor] = None,
                 stream=None) -> Tuple[torch.Tensor, torch.Tensor]:
    """Per-query (cost float32 [B], end_pos int64 [B]) on the GPU."""
    h = _host_lens(h_query_lens)
    _require_cuda("queries", queries, torch.float32)
    _require_cuda("query_lens", query_lens, torch.int32)
    _require_cuda("reference", reference, torch.float32)
    dev = queries.device
    b = h.size
    if cost is None:
        cost = torch.empty(b, dtype=torch.float32, device=dev)
    if end_pos is None:
        end_pos = torch.empty(b, dtype=torch.int64, device=dev)
    need = sdtw_forward_workspace_bytes(h, reference.numel(), flags)
    if need == 0:
        raise SdtwError(_lib.SDTW_ERR_INVALID_ARG, "sdtw_forward_workspace_bytes")
    if workspace_buf is None:
        workspace_buf = workspace(need, dev)
    st = _lib.lib.sdtw_forward(
        _dp(queries), _hp(h), _dp(query_lens), b, _dp(reference), reference.numel(),
        int(cost_kind), _dp(cost), _dp(end_pos), _dp(ckpt), int(ckpt_every), int(variant),
        int(flags), _dp(workspace_buf), workspace_buf.numel(), _stream(stream))
    check(st, "sdtw_forward")
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
    _require_cuda("queries", queries, torch.float32)
    _require_cuda("query_lens", query_lens, torch.int32)
    _require_cuda("reference", reference, torch.float32)
    dev = queries.device
    b = h.size
    if cost is None:
        cost = torch.empty(b, dtype=torch.float32, device=dev)
    if end_pos is None:
        end_pos = torch.empty(b, dtype=torch.int64, device=dev)
    need = sdtw_forward_workspace_bytes(h, reference.numel(), flags)
    if need == 0:
        raise SdtwError(_lib.SDTW_ERR_INVALID_ARG, "sdtw_forward_workspace_bytes")
    if workspace_buf is None:
        workspace_buf = workspace(need, dev)
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
    _require_cuda("queries", queries, torch.float32)
    _require_cuda("query_lens", query_lens, torch.int32)
    _require_cuda("reference", reference, torch.float32)
    dev = queries.device
    b = h.size
    if cost is None:
        cost = torch.empty(b, dtype=torch.float32, device=dev)
    if end_pos is None:
        end_pos = torch.empty(b, dtype=torch.int64, device=dev)
    if codebook is None:
        codebook = torch.empty(2, dtype=torch.float32, device=dev)
    need = sdtw_forward_u8_workspace_bytes(h, reference.numel())
    if need == 0:
        raise SdtwError(_lib.SDTW_ERR_INVALID_ARG, "sdtw_forward_u8_workspace_bytes")
    if workspace_buf is None:
        workspace_buf = workspace(need, dev)
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
    _require_cuda("queries", queries, torch.float32)
    _require_cuda("query_lens", query_lens, torch.int32)
    _require_cuda("reference", reference, torch.float32)
    _require_cuda("grad_cost", grad_cost, torch.float32)
    _require_cuda("cost", cost, torch.float32)
    _require_cuda("end_pos", end_pos, torch.int64)
    dev = queries.device
    if grad_queries is None:
        grad_queries = torch.empty_like(queries)
    if grad_reference is None:
        grad_reference = torch.empty_like(reference)
    need = sdtw_backward_workspace_bytes(h, reference.numel(), ckpt_every)
    if need == 0:
        raise SdtwError(_lib.SDTW_ERR_INVALID_ARG, "sdtw_backward_workspace_bytes")
    if workspace_buf is None:
        workspace_buf = workspace(need, dev)
    st = _lib.lib.sdtw_backward(
        _dp(queries), _hp(h), _dp(query_lens), h.size, _dp(reference), reference.numel(),
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
    _require_cuda("queries", queries, torch.float32)
    _require_cuda("query_lens", query_lens, torch.int32)
    _require_cuda("reference", reference, torch.float32)
    dev = queries.device
    b = h.size
    if cost is None:
        cost = torch.empty(b, dtype=torch.float32, device=dev)
    if end_pos is None:
        end_pos = torch.empty(b, dtype=torch.int64, device=dev)
    need = sdtw_forward_f16_workspace_bytes(h, reference.numel())
    if need == 0:
        raise SdtwError(_lib.SDTW_ERR_UNSUPPORTED, "sdtw_forward_f16_workspace_bytes")
    if workspace_buf is None:
        workspace_buf = workspace(need, dev)
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
    _require_cuda("queries", queries, torch.float32)
    _require_cuda("query_lens", query_lens, torch.int32)
    _require_cuda("reference", reference, torch.float32)
    _require_cuda("cost", cost, torch.float32)
    _require_cuda("end_pos", end_pos, torch.int64)
    dev = queries.device
    start = torch.empty(h.size, dtype=torch.int64, device=dev)
    lo = torch.empty(queries.numel(), dtype=torch.int32, device=dev)
    hi = torch.empty(queries.numel(), dtype=torch.int32, device=dev)
    need = sdtw_align_workspace_bytes(h, reference.numel(), ckpt_every)
    if need == 0:
        raise SdtwError(_lib.SDTW_ERR_INVALID_ARG, "sdtw_align_workspace_bytes")
    if workspace_buf is None:
        workspace_buf = workspace(need, dev)
    st = _lib.lib.sdtw_align(
        _dp(queries), _hp(h), _dp(query_lens), h.size, _dp(reference), reference.numel(),
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
    _require_cuda("x", x, torch.float32)
    _require_cuda("lens", lens, torch.int32)
    if out is None:
        out = torch.empty_like(x)
    else:
        _require_cuda("out", out, torch.float32)
    if out.numel() != x.numel():
        raise ValueError("out must have the size of x")
    need = sdtw_znorm_workspace_bytes(h)
    if need == 0:
        raise SdtwError(_lib.SDTW_ERR_INVALID_ARG, "sdtw_znorm_workspace_bytes")
    if workspace_buf is None:
        workspace_buf = workspace(need, x.device)
    st = _lib.lib.sdtw_znorm(_dp(x), _hp(h), _dp(lens), h.size, _dp(out), _dp(workspace_buf),
                             workspace_buf.numel(), _stream(stream))
    check(st, "sdtw_znorm")
    return out
