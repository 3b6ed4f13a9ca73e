"""Autotuner: every variant gives bit-identical results, the tuner returns one
of them and caches it by shape."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads
from gpu_util import assert_bit_exact, gpu_forward, to_dev


def test_shape_key_buckets(monkeypatch):
    torch = pytest.importorskip("torch")
    import paper_2403_06931_amd.autotune as A
    assert A._bucket(1) == 1 and A._bucket(1000) == 1024 and A._bucket(1024) == 1024
    assert A._bucket(1025) == 2048


@pytest.mark.gpu
def test_tuner_picks_a_variant_and_caches(tmp_path, monkeypatch):
    import paper_2403_06931_amd as P
    monkeypatch.setenv("SDTW_TUNE_CACHE", str(tmp_path / "tune.json"))
    monkeypatch.setenv("SDTW_TUNE", "1")
    w = workloads.make_random(64, 700, 20000, seed=5)
    q, l, r = to_dev(w)
    v = P.autotune.tuned_variant(q, w.lens, l, r, 0, 0)
    assert 0 <= v < P.sdtw_variant_count()
    data = json.load(open(tmp_path / "tune.json"))
    (key, rec), = data.items()
    assert rec["best"] == v and len(rec["times_ms"]) == P.sdtw_variant_count()
    assert min(rec["times_ms"].values()) == rec["times_ms"][str(v)]
    # cache hit
    assert P.autotune.tuned_variant(q, w.lens, l, r, 0, 0) == v
    # an entry whose recorded tile no longer matches the library's table is
    # not trusted: the batch is tuned again and the entry rewritten
    rec["variants"][str(v)] = [99, 99, 99, 99, 99]
    json.dump({key: rec}, open(tmp_path / "tune.json", "w"))
    v2 = P.autotune.tuned_variant(q, w.lens, l, r, 0, 0)
    assert 0 <= v2 < P.sdtw_variant_count()
    rec2 = json.load(open(tmp_path / "tune.json"))[key]
    assert tuple(rec2["variants"][str(v2)]) == tuple(P.sdtw_variant_info(v2))
    # every variant computes the same bits as the oracle
    want_c, want_e = oracle.sdtw_f32(w.queries, w.lens, w.reference, 0)
    for k in range(P.sdtw_variant_count()):
        c, e = gpu_forward(w, 0, variant=k)
        assert_bit_exact(c, e, want_c, want_e, f"variant {k}")
