"""uint8 codebook quantisation oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline``
leg may import this module; the product path never does.

Section 8 proposes quantising the values to uint8 through a codebook built
from the reference: take the distribution of its values, divide the bulk of
it evenly over the 256 codes, clamp outliers to the end codes.  Readings
(listed in the design notes): the inputs are z-normalised, so the bulk is the
values within ``CLIP`` = 4 standard deviations of the mean; the codebook is
256 evenly spaced levels from lo = max(min(reference), -4) to
hi = min(max(reference), 4); a value's code is the nearest level, computed as
clamp(rint((x - lo) * 255 / (hi - lo)), 0, 255) in binary64 with ties to
even, and every code is 0 when hi <= lo.  The DP on the codes is the
binary32 DP of ``oracle.sdtw_f32`` applied to the codes as numbers 0..255 with
the squared cost (each cost (a - b)^2 <= 65025 is exact; the sums are exact
integers below 2^24); ``oracle.sdtw_codes`` is its exact-integer twin.
"""
import numpy as np

from . import SQUARED, sdtw_f32

CLIP = np.float32(4.0)


def codebook(reference):
    """(lo, hi) as float32: the reference's extremes clipped to [-CLIP, CLIP]."""
    r = np.asarray(reference, dtype=np.float32)
    lo = max(np.float32(r.min()), -CLIP)
    hi = min(np.float32(r.max()), CLIP)
    return np.float32(lo), np.float32(hi)


def encode(x, lo, hi):
    """uint8 codes of x (the nearest of the 256 levels, ends clamped)."""
    lo64, hi64 = np.float64(lo), np.float64(hi)
    scale = 255.0 / (hi64 - lo64) if hi64 > lo64 else 0.0
    v = np.rint((np.asarray(x, dtype=np.float32).astype(np.float64) - lo64) * scale)
    return np.clip(v, 0.0, 255.0).astype(np.uint8)


def sdtw_u8(queries, lens, reference, nthreads=0):
    """Codebook from the reference, codes of both sides, binary32 sDTW of the
    codes -> (cost float32 [B] in step^2 units, end_pos int64 [B], (lo, hi))."""
    lo, hi = codebook(reference)
    qc = encode(queries, lo, hi).astype(np.float32)
    rc = encode(reference, lo, hi).astype(np.float32)
    cost, end = sdtw_f32(qc, lens, rc, SQUARED, nthreads)
    return cost, end, (lo, hi)
