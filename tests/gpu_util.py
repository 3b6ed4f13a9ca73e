"""Helpers for the GPU tests: move a workload to the device and run the
library through its C ABI (via the ctypes binding)."""
import numpy as np
import torch


def device():
    return torch.device("cuda:0")


def to_dev(w):
    d = device()
    return (torch.from_numpy(np.ascontiguousarray(w.queries)).to(d),
            torch.from_numpy(np.ascontiguousarray(w.lens)).to(d),
            torch.from_numpy(np.ascontiguousarray(w.reference)).to(d))


def gpu_forward(w, kind=0, variant=-1, flags=0, reference=None):
    import paper_2403_06931_amd as P
    q, l, r = to_dev(w)
    if reference is not None:
        r = reference
    cost, end = P.sdtw_forward(q, w.lens, l, r, kind, variant=variant, flags=flags)
    torch.cuda.synchronize()
    return cost.cpu().numpy(), end.cpu().numpy()


def assert_bit_exact(got_c, got_e, want_c, want_e, what=""):
    got_c = np.asarray(got_c, np.float32)
    want_c = np.asarray(want_c, np.float32)
    bad = np.nonzero((got_c.view(np.uint32) != want_c.view(np.uint32)) |
                     (np.asarray(got_e) != np.asarray(want_e)))[0]
    if bad.size:
        i = bad[:8]
        raise AssertionError(f"{what}: {bad.size} mismatches, first {i.tolist()}: "
                             f"gpu cost {got_c[i].tolist()} end {np.asarray(got_e)[i].tolist()} | "
                             f"oracle cost {want_c[i].tolist()} end {np.asarray(want_e)[i].tolist()}")
