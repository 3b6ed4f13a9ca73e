"""Z-normalisation oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline``
leg may import this module; the HIP library shares no code with it.

The paper's normaliser (Section 5.1, "Normalizer implementation", and its
standardisation equation) rescales every series of a packed batch to mean 0
and standard deviation 1: z = (x - mean) / S.  Readings where the paper is
silent or loose:

* S is the population standard deviation (divide by n): the formula the
  section gives for the variance divides the sum of squares by n.
* Arithmetic is binary64 on the binary32 inputs, and each z is rounded once
  to binary32.  The variance is written as its definition, the mean of the
  squared deviations from the mean (the section's sum-of-squares form is the
  same quantity; it is checked against this one in the tests).
* A constant series (S = 0) has no standardised form; it maps to all zeros.

Series are packed back to back with no gaps (lengths ``lens``), as the
section describes for the query batch.
"""
import numpy as np


def znorm_stats_f64(series: np.ndarray, lens) -> tuple:
    """Per-series (mean, S) in binary64, S the population standard deviation."""
    x = np.asarray(series, dtype=np.float32)
    lens = np.asarray(lens, dtype=np.int64)
    if lens.sum() != x.size:
        raise ValueError("lengths do not add up to the packed size")
    mean = np.empty(lens.size)
    std = np.empty(lens.size)
    off = 0
    for b, n in enumerate(lens):
        if n < 1:
            raise ValueError("empty series")
        v = x[off:off + n].astype(np.float64)
        m = v.sum() / n
        d = v - m
        mean[b] = m
        std[b] = np.sqrt((d * d).sum() / n)
        off += n
    return mean, std


def znorm_f32(series: np.ndarray, lens) -> np.ndarray:
    """Standardised series, packed like the input, binary32."""
    x = np.asarray(series, dtype=np.float32)
    lens = np.asarray(lens, dtype=np.int64)
    mean, std = znorm_stats_f64(x, lens)
    out = np.empty(x.size, dtype=np.float32)
    off = 0
    for b, n in enumerate(lens):
        v = x[off:off + n].astype(np.float64)
        if std[b] > 0.0:
            out[off:off + n] = ((v - mean[b]) / std[b]).astype(np.float32)
        else:
            out[off:off + n] = 0.0
        off += n
    return out
