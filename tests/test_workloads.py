"""The seeded input generator is deterministic: the same seed gives the same
arrays (SHA-256 of queries, lengths and reference), within a process and
against the digests recorded in tests/golden/workload_digests.txt."""
import os

import numpy as np
import pytest

import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "workload_digests.txt")


def _recorded():
    out = {}
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split("=")
                out[k.strip()] = v.strip()
    return out


@pytest.mark.parametrize("k", [0, 1, 2, 3, 4])
def test_config_digests(k):
    rec = _recorded()
    a = workloads.digest(workloads.make_config(k))
    assert a == workloads.digest(workloads.make_config(k))      # repeatable in-process
    if np.__version__ != "2.2.6":
        pytest.skip(f"digests recorded with NumPy 2.2.6, this is {np.__version__}")
    assert a == rec[f"config{k}"]


def test_random_workload_digest_and_seed_sensitivity():
    rec = _recorded()
    w = workloads.make_random(3, [5, 17, 40], 300, seed=12345)
    other = workloads.make_random(3, [5, 17, 40], 300, seed=12346)
    assert workloads.digest(w) != workloads.digest(other)
    if np.__version__ == "2.2.6":
        assert workloads.digest(w) == rec["random_3x[5,17,40]_vs_300_seed12345"]
