"""Autotuner for the forward tile variant (rows per lane, columns per step,
wavefronts per query).

The paper tuned its per-thread reference segment width by sweeping it on the
target shape (Section 6: ten timed runs after two warm-ups).  Here every
compiled variant of the library is timed on the caller's actual batch with
HIP events on the current stream (two warm-ups, then the median of the timed
runs) and the fastest is cached in a JSON file keyed by the device and a
coarse description of the shape.  All variants compute bit-identical results,
so tuning only ever changes speed.

Environment:
  SDTW_TUNE        "1" (default): use the cache, tune on a miss;
                   "0": never tune, use the library's built-in choice;
                   "force": retune even on a cache hit.
  SDTW_TUNE_CACHE  cache file (default ~/.cache/sdtw_tune.json).
"""
from __future__ import annotations

import json
import os
import statistics
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import api


def cache_path() -> str:
    return os.environ.get("SDTW_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "sdtw_tune.json"))


def _bucket(x: int) -> int:
    """Round up to a power of two (shapes in one bucket share a tuning)."""
    return 1 << max(0, int(x - 1).bit_length())


def shape_key(h_lens, ref_len: int, cost_kind: int, flags: int, device=None) -> str:
    h = api._host_lens(h_lens)
    props = torch.cuda.get_device_properties(device or torch.cuda.current_device())
    arch = getattr(props, "gcnArchName", props.name).split(":")[0]
    lens_sorted = np.sort(h)
    p50 = int(lens_sorted[len(lens_sorted) // 2])
    return "|".join(str(v) for v in (
        arch, props.multi_processor_count, "B", _bucket(h.size), "Nmax", _bucket(int(h.max())),
        "N50", _bucket(p50), "M", _bucket(int(ref_len)), "k", int(cost_kind), "f", int(flags)))


def _load_cache() -> Dict[str, dict]:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(cache: Dict[str, dict]) -> None:
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + f".tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_variant(variant: int, queries, h_lens, query_lens, reference, cost_kind: int,
                 flags: int, reps: int = 5, warmup: int = 2, workspace_buf=None,
                 ckpt=None, ckpt_every: int = 0) -> float:
    """Median milliseconds of one sdtw_forward call with this variant (with
    checkpoints when flags has SDTW_F_CHECKPOINT: pass ckpt and ckpt_every)."""
    h = api._host_lens(h_lens)
    dev = queries.device
    if workspace_buf is None:
        workspace_buf = api.workspace(api.sdtw_forward_workspace_bytes(h, reference.numel(),
                                                                       flags, variant), dev)
    cost = torch.empty(h.size, dtype=torch.float32, device=dev)
    end = torch.empty(h.size, dtype=torch.int64, device=dev)
    kw = dict(cost=cost, end_pos=end, variant=variant, flags=flags, workspace_buf=workspace_buf,
              ckpt=ckpt, ckpt_every=ckpt_every)
    for _ in range(warmup):
        api.sdtw_forward(queries, h, query_lens, reference, cost_kind, **kw)
    times: List[float] = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        api.sdtw_forward(queries, h, query_lens, reference, cost_kind, **kw)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    return statistics.median(times)


def tune(queries, h_lens, query_lens, reference, cost_kind: int = 0, flags: int = 0,
         candidates: Optional[Sequence[int]] = None, reps: int = 5,
         record: Optional[dict] = None, ckpt=None, ckpt_every: int = 0) -> int:
    """Time every candidate variant on this batch; return the fastest."""
    h = api._host_lens(h_lens)
    if candidates is None:
        candidates = range(api.sdtw_variant_count())
    candidates = [int(v) for v in candidates]
    # one workspace large enough for every candidate tile
    ws = api.workspace(max(api.sdtw_forward_workspace_bytes(h, reference.numel(), flags, v)
                           for v in candidates), queries.device)
    results = {}
    for v in candidates:
        results[int(v)] = time_variant(int(v), queries, h, query_lens, reference, cost_kind,
                                       flags, reps=reps, workspace_buf=ws, ckpt=ckpt,
                                       ckpt_every=ckpt_every)
    best = min(results, key=results.get)
    if record is not None:
        record.update({"times_ms": results, "best": best})
    return best


def tune_persistent(queries, h_lens, query_lens, reference, cost_kind: int = 0,
                    flags: int = api.SDTW_F_PERSISTENT,
                    candidates: Optional[Sequence[int]] = None,
                    waves_per_simd: Sequence[int] = (2, 3, 4), reps: int = 3,
                    record: Optional[dict] = None) -> Tuple[int, int]:
    """Time every (variant, grid size) pair of the persistent launch on this
    batch: the grid holds waves_per_simd resident wavefronts per SIMD
    (SDTW_F_WAVES_PER_SIMD).  Returns the fastest (variant, flags)."""
    h = api._host_lens(h_lens)
    if candidates is None:
        candidates = range(api.sdtw_variant_count())
    base = (int(flags) | api.SDTW_F_PERSISTENT) & ~(0xf << 8)
    pairs = [(int(v), base | api.SDTW_F_WAVES_PER_SIMD(w)) for v in candidates
             for w in waves_per_simd]
    ws = api.workspace(max(api.sdtw_forward_workspace_bytes(h, reference.numel(), f, v)
                           for v, f in pairs), queries.device)
    results = {}
    for v, f in pairs:
        results[(v, f)] = time_variant(v, queries, h, query_lens, reference, cost_kind, f,
                                       reps=reps, workspace_buf=ws)
    best = min(results, key=results.get)
    if record is not None:
        record.update({"times_ms": {f"{v}/{f >> 8}": t for (v, f), t in results.items()},
                       "best": best})
    return best


def tuned_variant(queries, h_lens, query_lens, reference, cost_kind: int = 0,
                  flags: int = 0) -> int:
    """Variant for this batch: from the cache, by tuning, or the library default."""
    mode = os.environ.get("SDTW_TUNE", "1")
    h = api._host_lens(h_lens)
    if mode == "0":
        return api.sdtw_default_variant(h, reference.numel(), flags)
    key = shape_key(h, reference.numel(), cost_kind, flags, queries.device)
    cache = _load_cache()
    if mode != "force" and key in cache:
        v = int(cache[key]["best"])
        # a cached index is used only if it still names the same tile (the
        # library's variant table may have changed since it was tuned)
        shape = cache[key].get("variants", {}).get(str(v))
        if 0 <= v < api.sdtw_variant_count() and shape is not None and \
                tuple(shape) == tuple(api.sdtw_variant_info(v)):
            return v
    rec: dict = {}
    best = tune(queries, h, query_lens, reference, cost_kind, flags, record=rec)
    rec["variants"] = {str(v): api.sdtw_variant_info(v) for v in rec["times_ms"]}
    rec["times_ms"] = {str(k): v for k, v in rec["times_ms"].items()}
    cache = _load_cache()
    cache[key] = rec
    _store_cache(cache)
    return best
