"""CPU oracle for subsequence DTW -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports, links or calls it, and shares no code with
it.

The arithmetic lives in ``sdtw_oracle.c`` (plain C, gcc ``-O2
-ffp-contract=off``); this module only marshals NumPy arrays through ctypes.
Every function follows Section 2, Eq. (1) of the paper with the subsequence
initialisation (row 0 = 0, column 0 = +inf); see the header of
``sdtw_oracle.c`` for the readings taken where the paper is silent.  The
z-normalisation oracle is ``oracle/znorm.py`` (NumPy, binary64).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# SDTW_ORACLE_LIBRARY may name another build of the same source (for
# example one built with sanitizers)
_LIB_PATH = os.environ.get("SDTW_ORACLE_LIBRARY") or os.path.join(_HERE, "liboracle.so")
_lib = None

SQUARED = 0
ABSOLUTE = 1

_f32p = ctypes.POINTER(ctypes.c_float)
_f64p = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build
        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_sdtw_f32.argtypes = [_f32p, _i32p, ctypes.c_int32, _f32p, ctypes.c_int64,
                                    ctypes.c_int, _f32p, _i64p, ctypes.c_int]
    lib.oracle_sdtw_pruned_f32.argtypes = [_f32p, _i32p, ctypes.c_int32, _f32p, ctypes.c_int64,
                                           ctypes.c_float, _f32p, _i64p, ctypes.c_int]
    lib.oracle_sdtw_codes.argtypes = [ctypes.POINTER(ctypes.c_uint8), _i32p, ctypes.c_int32,
                                      ctypes.POINTER(ctypes.c_uint8), ctypes.c_int64, _i64p,
                                      _i64p, ctypes.c_int]
    lib.oracle_sdtw_f64.argtypes = [_f32p, _i32p, ctypes.c_int32, _f32p, ctypes.c_int64,
                                    ctypes.c_int, _f64p, _i64p, ctypes.c_int]
    lib.oracle_sdtw_f16.argtypes = [_f32p, _i32p, ctypes.c_int32, _f32p, ctypes.c_int64,
                                    ctypes.c_int, _f32p, _i64p, ctypes.c_int]
    lib.oracle_round_f16.argtypes = [ctypes.c_double]
    lib.oracle_round_f16.restype = ctypes.c_double
    lib.oracle_sdtw_last_row_f32.argtypes = [_f32p, ctypes.c_int32, _f32p, ctypes.c_int64,
                                             ctypes.c_int, _f32p]
    lib.oracle_dtw_f32.argtypes = [_f32p, ctypes.c_int32, _f32p, ctypes.c_int64,
                                   ctypes.c_int, _f32p]
    lib.oracle_sdtw_grad_f32.argtypes = [_f32p, _i32p, ctypes.c_int32, _f32p, ctypes.c_int64,
                                         ctypes.c_int, _f32p, _f32p, _i64p, _i64p,
                                         _f32p, _f32p, ctypes.c_int]
    lib.oracle_sdtw_path_f32.argtypes = [_f32p, ctypes.c_int32, _f32p, ctypes.c_int64,
                                         ctypes.c_int, _i64p, _i64p]
    lib.oracle_sdtw_path_f32.restype = ctypes.c_int64
    lib.oracle_max_threads.restype = ctypes.c_int
    for name in ("oracle_sdtw_f32", "oracle_sdtw_pruned_f32", "oracle_sdtw_codes", "oracle_sdtw_f64", "oracle_sdtw_f16", "oracle_sdtw_last_row_f32",
                 "oracle_dtw_f32", "oracle_sdtw_grad_f32"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _p(a, t):
    return a.ctypes.data_as(t)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _lens(queries, lens):
    lens = np.ascontiguousarray(lens, dtype=np.int32)
    if lens.ndim != 1 or lens.size < 1 or int(lens.sum()) != queries.size:
        raise ValueError("query_lens must sum to the number of packed query values")
    return lens


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def sdtw_f32(queries, lens, reference, kind=SQUARED, nthreads=0):
    """Batched FP32 sDTW -> (cost float32 [B], end_pos int64 [B])."""
    lib = _load()
    q = _f32(queries).ravel()
    lens = _lens(q, lens)
    r = _f32(reference).ravel()
    cost = np.empty(lens.size, np.float32)
    end = np.empty(lens.size, np.int64)
    rc = lib.oracle_sdtw_f32(_p(q, _f32p), _p(lens, _i32p), lens.size, _p(r, _f32p), r.size,
                             int(kind), _p(cost, _f32p), _p(end, _i64p), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_sdtw_f32 rejected its arguments")
    return cost, end


def sdtw_pruned_f32(queries, lens, reference, tau, nthreads=0):
    """Batched FP32 sDTW with Section 8's early pruning: squared cost, +inf for
    a pair with |q - r| > tau -> (cost float32 [B], end_pos int64 [B])."""
    lib = _load()
    q = _f32(queries).ravel()
    lens = _lens(q, lens)
    r = _f32(reference).ravel()
    cost = np.empty(lens.size, np.float32)
    end = np.empty(lens.size, np.int64)
    rc = lib.oracle_sdtw_pruned_f32(_p(q, _f32p), _p(lens, _i32p), lens.size, _p(r, _f32p),
                                    r.size, float(tau), _p(cost, _f32p), _p(end, _i64p),
                                    int(nthreads))
    if rc != 0:
        raise ValueError("oracle_sdtw_pruned_f32 rejected its arguments")
    return cost, end


def sdtw_codes(qcodes, lens, rcodes, nthreads=0):
    """Batched sDTW on uint8 codes, local cost (a - b)^2, exact integers ->
    (cost int64 [B], end_pos int64 [B])."""
    lib = _load()
    q = np.ascontiguousarray(qcodes, dtype=np.uint8).ravel()
    lens = _lens(q, lens)
    r = np.ascontiguousarray(rcodes, dtype=np.uint8).ravel()
    cost = np.empty(lens.size, np.int64)
    end = np.empty(lens.size, np.int64)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    rc = lib.oracle_sdtw_codes(_p(q, u8p), _p(lens, _i32p), lens.size, _p(r, u8p), r.size,
                               _p(cost, _i64p), _p(end, _i64p), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_sdtw_codes rejected its arguments")
    return cost, end


def sdtw_f64(queries, lens, reference, kind=SQUARED, nthreads=0):
    """Batched FP64 sDTW of the FP32 inputs -> (cost float64 [B], end_pos int64 [B])."""
    lib = _load()
    q = _f32(queries).ravel()
    lens = _lens(q, lens)
    r = _f32(reference).ravel()
    cost = np.empty(lens.size, np.float64)
    end = np.empty(lens.size, np.int64)
    rc = lib.oracle_sdtw_f64(_p(q, _f32p), _p(lens, _i32p), lens.size, _p(r, _f32p), r.size,
                             int(kind), _p(cost, _f64p), _p(end, _i64p), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_sdtw_f64 rejected its arguments")
    return cost, end


def sdtw_f16(queries, lens, reference, kind=SQUARED, nthreads=0):
    """Batched sDTW in binary16 arithmetic (inputs and every operation rounded
    to binary16) -> (cost float32 [B] holding binary16 values, end_pos int64 [B])."""
    lib = _load()
    q = _f32(queries).ravel()
    lens = _lens(q, lens)
    r = _f32(reference).ravel()
    cost = np.empty(lens.size, np.float32)
    end = np.empty(lens.size, np.int64)
    rc = lib.oracle_sdtw_f16(_p(q, _f32p), _p(lens, _i32p), lens.size, _p(r, _f32p), r.size,
                             int(kind), _p(cost, _f32p), _p(end, _i64p), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_sdtw_f16 rejected its arguments")
    return cost, end


def round_f16(x: float) -> float:
    """The oracle's own rounding to the nearest binary16 value (ties to even)."""
    return float(_load().oracle_round_f16(float(x)))


def last_row_f32(query, reference, kind=SQUARED):
    """FP32 last DP row D(N, 1..M) of one query."""
    lib = _load()
    q = _f32(query).ravel()
    r = _f32(reference).ravel()
    out = np.empty(r.size, np.float32)
    if lib.oracle_sdtw_last_row_f32(_p(q, _f32p), q.size, _p(r, _f32p), r.size, int(kind),
                                    _p(out, _f32p)) != 0:
        raise ValueError("bad arguments")
    return out


def dtw_f32(query, reference, kind=SQUARED):
    """FP32 global (corner-to-corner) DTW of one query against the reference."""
    lib = _load()
    q = _f32(query).ravel()
    r = _f32(reference).ravel()
    out = np.empty(1, np.float32)
    if lib.oracle_dtw_f32(_p(q, _f32p), q.size, _p(r, _f32p), r.size, int(kind),
                          _p(out, _f32p)) != 0:
        raise ValueError("bad arguments")
    return out[0]


def sdtw_grad_f32(queries, lens, reference, grad_cost, kind=SQUARED, nthreads=0):
    """FP32 cost, end, path start and walk-back gradient of sum_b grad_cost[b]*cost_b.

    Returns (cost [B], end_pos [B], path_start [B], grad_queries (packed), grad_ref [M]).
    """
    lib = _load()
    q = _f32(queries).ravel()
    lens = _lens(q, lens)
    r = _f32(reference).ravel()
    g = _f32(grad_cost).ravel()
    if g.size != lens.size:
        raise ValueError("grad_cost must have one entry per query")
    cost = np.empty(lens.size, np.float32)
    end = np.empty(lens.size, np.int64)
    start = np.empty(lens.size, np.int64)
    gq = np.empty(q.size, np.float32)
    gr = np.empty(r.size, np.float32)
    rc = lib.oracle_sdtw_grad_f32(_p(q, _f32p), _p(lens, _i32p), lens.size, _p(r, _f32p),
                                  r.size, int(kind), _p(g, _f32p), _p(cost, _f32p),
                                  _p(end, _i64p), _p(start, _i64p), _p(gq, _f32p),
                                  _p(gr, _f32p), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_sdtw_grad_f32 rejected its arguments")
    return cost, end, start, gq, gr


def path_f32(query, reference, kind=SQUARED):
    """Walk-back path of one query: (rows, reference indices), 0-based, in walk order."""
    lib = _load()
    q = _f32(query).ravel()
    r = _f32(reference).ravel()
    cap = q.size + r.size
    pi = np.empty(cap, np.int64)
    pj = np.empty(cap, np.int64)
    n = lib.oracle_sdtw_path_f32(_p(q, _f32p), q.size, _p(r, _f32p), r.size, int(kind),
                                 _p(pi, _i64p), _p(pj, _i64p))
    if n < 0:
        raise ValueError("bad arguments")
    return pi[:n].copy(), pj[:n].copy()
