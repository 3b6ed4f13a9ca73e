"""GPU parity of the batch z-normaliser (sdtw_znorm) against the binary64
oracle: every element within one binary32 ulp, constant series exactly zero,
results independent of the call (fixed-order reductions)."""
import numpy as np
import pytest
import torch

import workloads
from oracle import znorm as Z

pytestmark = pytest.mark.gpu


def _run(x, lens, inplace=False):
    import paper_2403_06931_amd as P
    d = torch.device("cuda:0")
    xt = torch.from_numpy(x).to(d)
    lt = torch.from_numpy(np.asarray(lens, np.int32)).to(d)
    out = P.sdtw_znorm(xt, lens, lt, out=xt if inplace else None)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _check(got, want, what):
    got = np.asarray(got, np.float32)
    want = np.asarray(want, np.float32)
    assert got.shape == want.shape
    ulp = np.spacing(np.abs(want)).astype(np.float64)
    err = np.abs(got.astype(np.float64) - want.astype(np.float64))
    bad = np.nonzero(err > ulp)[0]
    if bad.size:
        i = bad[:8]
        raise AssertionError(f"{what}: {bad.size} elements beyond 1 ulp, first {i.tolist()}: "
                             f"gpu {got[i].tolist()} oracle {want[i].tolist()}")
    return int(np.count_nonzero(got != want))


@pytest.mark.parametrize("lens", [
    [1], [2], [3, 1, 7], [255, 256, 257],
    [4095, 4096, 4097],                       # one chunk, exactly one, two chunks
    [8191, 8192, 8193, 12289],
    [100_000],                                # a reference: 25 chunks
    [5, 70_001, 2, 4096 * 3 + 1, 31],
])
def test_znorm_matches_oracle(lens):
    x = workloads.raw_series(lens, seed=sum(lens) % 1000 + 7)
    print(f"znorm lens {lens}", flush=True)
    want = Z.znorm_f32(x, lens)
    got = _run(x, lens)
    _check(got, want, f"lens {lens}")


def test_znorm_constant_series_are_zero():
    lens = [1, 9, 5000, 4096, 3]
    x = np.concatenate([np.full(n, v, np.float32) for n, v in zip(lens, [3.5, -2.0, 1e3, 0.0, 7.0])])
    got = _run(x, lens)
    assert np.all(got == 0.0)


def test_znorm_in_place_and_repeatable():
    lens = [2000] * 64 + [30_000]
    x = workloads.raw_series(lens, seed=77)
    want = Z.znorm_f32(x, lens)
    a = _run(x, lens)
    b = _run(x, lens, inplace=True)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    _check(a, want, "in place")


def test_znorm_full_size_batches():
    """The shapes of the evaluation: 512 queries of 2,000 samples plus the
    100,000-sample reference; 4,096 queries of U[250, 4000] samples; a
    2,000,000-sample reference."""
    rng = np.random.default_rng(11)
    for lens in ([2000] * 512 + [100_000], list(rng.integers(250, 4001, 4096)), [2_000_000]):
        x = workloads.raw_series(lens, seed=len(lens))
        print(f"znorm full size: {len(lens)} series, {x.size} samples", flush=True)
        want = Z.znorm_f32(x, lens)
        got = _run(x, lens)
        n = _check(got, want, f"{len(lens)} series")
        print(f"  {n} of {x.size} elements differ by one ulp", flush=True)
        # and the outputs are standardised
        off = np.concatenate([[0], np.cumsum(lens)])
        for k in range(0, len(lens), max(1, len(lens) // 16)):
            v = got[off[k]:off[k + 1]].astype(np.float64)
            assert abs(v.mean()) < 1e-5 and abs(v.std() - 1.0) < 1e-5


def test_znorm_many_long_series():
    """More multi-chunk series than the index kernel lists for its
    workgroup-wide chunk-map fill (the rest are mapped by their own thread)."""
    lens = [4096 * 9 + 5] * 300 + [17, 4096 * 8, 4096 * 8 + 1]
    x = workloads.raw_series(lens, seed=123)
    want = Z.znorm_f32(x, lens)
    got = _run(x, lens)
    _check(got, want, "300 long series")


@pytest.mark.parametrize("nlong", [32, 33])
def test_znorm_long_series_listed_in_arguments(nlong):
    """Up to 32 series longer than one wavefront's 4,096 samples are listed in
    the kernel arguments (two launches, no offset table); a 33rd sends the
    batch to the offset-table form.  Both must agree with the oracle."""
    rng = np.random.default_rng(nlong)
    lens = list(rng.integers(1, 4097, 200))
    for k in range(nlong):
        lens.insert(int(rng.integers(0, len(lens) + 1)), int(rng.integers(4097, 20000)))
    x = workloads.raw_series(lens, seed=nlong + 1)
    _check(_run(x, lens), Z.znorm_f32(x, lens), f"{nlong} long series")


def test_znorm_batch_beyond_direct_form():
    """More than 16,384 series: the offset-table form."""
    lens = list(np.random.default_rng(5).integers(1, 300, 17000))
    x = workloads.raw_series(lens, seed=17)
    _check(_run(x, lens), Z.znorm_f32(x, lens), "17,000 series")
