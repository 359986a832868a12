"""The stored oracle order of the d = 1024, n = 8192 workload (seed 0), which
the GPU's free-running order is tested against, checked on the CPU: the file
is a finished ordering (a permutation), every step's record is consistent
with it (the choice is the first maximum of M, ties to the smaller id, and the
four best are in descending order), and the oracle recomputed from the
seeded input along the stored prefix reproduces the stored measures at the
late steps 1000 and 1022 (every active variable)."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2403_03772_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "gene_d1024_n8192_seed0.json")
D, N = 1024, 8192


@pytest.fixture(scope="module")
def golden():
    g = json.load(open(GOLDEN))
    assert g["finished"] and g["d"] == D and g["n"] == N and g["seed"] == 0
    return g


def test_stored_order_is_consistent(golden):
    order = np.asarray(golden["order"])
    assert sorted(order.tolist()) == list(range(D))
    steps = golden["steps"]
    assert [r["t"] for r in steps] == list(range(D - 1))
    for r in steps:
        t = r["t"]
        assert r["choice"] == order[t]
        assert r["top_ids"][0] == r["choice"]
        top = np.asarray(r["top_M"])
        assert np.all(np.diff(top) <= 0) and np.all(top <= 0.0)
        ids = np.asarray(r["top_ids"] + r["sample_ids"] + r.get("all_ids", []))
        assert not np.isin(ids, order[:t]).any()           # only active variables
        assert r["max_abs"] >= np.max(np.abs(top))
        if "all_ids" in r:
            assert len(r["all_ids"]) == D - t
            allm = np.asarray(r["all_M"])
            best = np.flatnonzero(allm == allm.max())
            assert r["all_ids"][best[0]] == r["choice"]   # first maximum by id


@pytest.mark.parametrize("t", [1000, 1022])
def test_late_steps_reproduce(golden, t):
    X = np.ascontiguousarray(synth.workload_gene_scale(seed=0, d=D, n=N).X, dtype=np.float32)
    order = np.asarray(golden["order"], dtype=np.int32)
    ref = oracle.step_measures_all(X, order[:t])
    rec = golden["steps"][t]
    ids = np.asarray(rec["all_ids"])
    got = np.asarray(rec["all_M"])
    assert np.array_equal(np.flatnonzero(np.isfinite(ref)), np.sort(ids))
    err = np.abs(ref[ids] - got) / np.maximum(np.abs(got), 1e-12)
    assert err.max() <= 1e-9, err.max()
    assert ids[np.argmax(got)] == order[t]
