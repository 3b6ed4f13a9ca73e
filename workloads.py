"""Seeded synthetic sDTW workloads.

This module only draws input arrays; it holds none of the sDTW arithmetic.
It is the one piece of code that both the CPU oracle's tests and the HIP
path's tests and benchmark use, so that both sides see identical inputs.

The paper evaluates on cylinder-bell-funnel series from an external package
(Section 4) at 512 queries of 2,000 samples against a 100,000-sample
reference (Section 6).  That generator is not available here; z-normalised
Gaussian random walks of the same shapes stand in for it:

* reference: cumulative sum of N(0,1) steps in float64, optionally plus white
  noise, z-normalised (population standard deviation), cast to float32;
* "excerpt" queries: a random window of the reference, time-warped piecewise
  over 8 segments with stretch factors drawn uniformly from [0.8, 1.25]
  (linear interpolation), plus N(0, 0.1^2) noise, then z-normalised;
* "walk" queries: independent random walks, z-normalised.

Even-indexed queries are excerpts and odd-indexed ones are walks (where a
config mixes them), so every prefix or subset holds both kinds.

Arrays are reproducible for a given NumPy version; ``digest()`` gives a
SHA-256 of a workload so logs can record exactly what was run.
"""
from __future__ import annotations

import dataclasses
import hashlib
from typing import List, Optional, Tuple

import numpy as np

BASE_SEED = 240306931


@dataclasses.dataclass
class Workload:
    name: str
    queries: np.ndarray          # float32, packed (query b starts at sum(lens[:b]))
    lens: np.ndarray             # int32 [B]
    reference: np.ndarray        # float32 [M]
    kinds: Tuple[int, ...]       # cost kinds exercised: 0 squared, 1 absolute
    excerpt_start: np.ndarray    # int64 [B]; -1 for walk queries
    description: str = ""

    @property
    def batch(self) -> int:
        return int(self.lens.size)

    @property
    def ref_len(self) -> int:
        return int(self.reference.size)

    @property
    def cells(self) -> int:
        return int(self.lens.astype(np.int64).sum()) * self.ref_len

    @property
    def offsets(self) -> np.ndarray:
        off = np.zeros(self.batch + 1, np.int64)
        np.cumsum(self.lens, out=off[1:])
        return off

    def query(self, b: int) -> np.ndarray:
        off = self.offsets
        return self.queries[off[b]:off[b + 1]]

    def subset(self, idx) -> "Workload":
        idx = np.asarray(idx, dtype=np.int64)
        qs = [self.query(int(b)) for b in idx]
        return Workload(
            name=f"{self.name}[subset {idx.size}]",
            queries=np.concatenate(qs).astype(np.float32),
            lens=self.lens[idx].astype(np.int32),
            reference=self.reference,
            kinds=self.kinds,
            excerpt_start=self.excerpt_start[idx],
            description=self.description,
        )


def znorm(x: np.ndarray) -> np.ndarray:
    """z-normalise with the population standard deviation (float64)."""
    x = np.asarray(x, dtype=np.float64)
    mu = x.mean()
    sd = x.std()
    if sd == 0.0:
        return x - mu
    return (x - mu) / sd


def random_walk(rng: np.random.Generator, n: int, white_noise: float = 0.0) -> np.ndarray:
    """z-normalised Gaussian random walk (float64)."""
    w = np.cumsum(rng.standard_normal(n))
    if white_noise > 0.0:
        w = w + rng.normal(0.0, white_noise, n)
    return znorm(w)


def warped_excerpt(rng: np.random.Generator, ref64: np.ndarray, n: int,
                   segments: int = 8, lo: float = 0.8, hi: float = 1.25,
                   noise: float = 0.1) -> Tuple[np.ndarray, int]:
    """Time-warped noisy excerpt of ``ref64`` of length ``n`` -> (float64 values, source start)."""
    m = ref64.size
    s = max(1, min(segments, n))
    sizes = np.full(s, n // s, dtype=np.int64)
    sizes[: n % s] += 1
    stretch = rng.uniform(lo, hi, size=s)
    consumed = sizes / stretch                 # source samples per segment
    span = int(np.ceil(consumed.sum())) + 1
    if span >= m:
        raise ValueError("reference too short for a warped excerpt of this length")
    a = int(rng.integers(0, m - span))
    pos = []
    base = float(a)
    for k in range(s):
        pos.append(base + np.arange(sizes[k]) / stretch[k])
        base += consumed[k]
    pos = np.concatenate(pos)
    vals = np.interp(pos, np.arange(m, dtype=np.float64), ref64)
    vals = vals + rng.normal(0.0, noise, n)
    return znorm(vals), a


def make_batch(name: str, rng: np.random.Generator, ref64: np.ndarray, lens,
               excerpt_every: int = 2, kinds=(0,), description: str = "") -> Workload:
    """Queries of the given lengths: every ``excerpt_every``-th query (from 0) is an excerpt."""
    lens = np.asarray(lens, dtype=np.int32)
    out: List[np.ndarray] = []
    starts = np.full(lens.size, -1, dtype=np.int64)
    for b, n in enumerate(lens):
        if excerpt_every and b % excerpt_every == 0:
            v, a = warped_excerpt(rng, ref64, int(n))
            starts[b] = a
        else:
            v = random_walk(rng, int(n))
        out.append(v.astype(np.float32))
    return Workload(name=name, queries=np.concatenate(out).astype(np.float32), lens=lens,
                    reference=ref64.astype(np.float32), kinds=tuple(kinds),
                    excerpt_start=starts, description=description)


CONFIG_DESCRIPTIONS = {
    0: "4 warped excerpts x 64 vs 1,024 random walk; squared",
    1: "512 x 2,000 (half warped excerpts, half walks) vs 100,000 random walk; squared",
    2: "512 x 2,000 vs 2,000,000 random walk + N(0,0.3^2) noise; squared and absolute",
    3: "4,096 queries, lengths uniform-int [250, 4,000], vs 200,000 random walk; squared",
    4: "256 x 1,000 vs 50,000 random walk (continuous, tie-free); squared; fwd+bwd",
}


def make_config(k: int, seed: Optional[int] = None) -> Workload:
    """The five workload shapes: plain small, paper-shaped, long reference,
    uneven batch and differentiable."""
    rng = np.random.default_rng(BASE_SEED + k if seed is None else seed)
    if k == 0:
        ref = random_walk(rng, 1024)
        return make_batch("sdtw-4x64-vs-1k", rng, ref, [64] * 4, excerpt_every=1,
                          description=CONFIG_DESCRIPTIONS[0])
    if k == 1:
        ref = random_walk(rng, 100_000)
        return make_batch("sdtw-512x2000-vs-100k", rng, ref, [2000] * 512,
                          description=CONFIG_DESCRIPTIONS[1])
    if k == 2:
        ref = random_walk(rng, 2_000_000, white_noise=0.3)
        return make_batch("sdtw-512x2000-vs-2M", rng, ref, [2000] * 512, kinds=(0, 1),
                          description=CONFIG_DESCRIPTIONS[2])
    if k == 3:
        ref = random_walk(rng, 200_000)
        lens = rng.integers(250, 4001, size=4096)
        return make_batch("sdtw-4096xU[250,4000]-vs-200k", rng, ref, lens,
                          description=CONFIG_DESCRIPTIONS[3])
    if k == 4:
        ref = random_walk(rng, 50_000)
        return make_batch("sdtw-256x1000-vs-50k-fwdbwd", rng, ref, [1000] * 256,
                          description=CONFIG_DESCRIPTIONS[4])
    raise ValueError(f"unknown config {k}")


def subset_indices(w: Workload, count: int, seed: Optional[int] = None,
                   include_extremes: bool = False) -> np.ndarray:
    """Seeded sorted subset of query indices (optionally with the shortest and longest)."""
    rng = np.random.default_rng((BASE_SEED + 7919) if seed is None else seed)
    count = min(count, w.batch)
    idx = set(int(i) for i in rng.choice(w.batch, size=count, replace=False))
    if include_extremes:
        idx.add(int(np.argmin(w.lens)))
        idx.add(int(np.argmax(w.lens)))
    return np.array(sorted(idx), dtype=np.int64)


def make_random(batch: int, qlen, ref_len: int, seed: int, excerpt_every: int = 2,
                kinds=(0,)) -> Workload:
    """Generic seeded workload (lengths may be an int or a list)."""
    rng = np.random.default_rng(seed)
    ref = random_walk(rng, ref_len)
    lens = [qlen] * batch if np.isscalar(qlen) else list(qlen)
    return make_batch(f"random-{batch}x{qlen}-vs-{ref_len}", rng, ref, lens,
                      excerpt_every=excerpt_every, kinds=kinds)


def digest(w: Workload) -> str:
    h = hashlib.sha256()
    for a in (w.queries, w.lens, w.reference):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def raw_series(lens, seed: int) -> np.ndarray:
    """Packed float32 series before any normalisation, as captured in
    different units: per series a Gaussian random walk (or, for every fourth
    series, white noise) times a scale drawn log-uniformly from [1e-3, 1e3],
    plus an offset of up to 50 scales."""
    rng = np.random.default_rng(seed)
    out = []
    for k, n in enumerate(lens):
        n = int(n)
        base = rng.standard_normal(n) if k % 4 == 3 else np.cumsum(rng.standard_normal(n))
        scale = 10.0 ** rng.uniform(-3.0, 3.0)
        offset = rng.uniform(-50.0, 50.0) * scale
        out.append((base * scale + offset).astype(np.float32))
    return np.concatenate(out) if out else np.zeros(0, np.float32)
