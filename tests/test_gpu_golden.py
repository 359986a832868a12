"""The library against the stored oracle values of tests/golden/ (written by
tests/golden/make_golden.py from the oracle only)."""
import json
import os

import numpy as np
import pytest

from paper_2403_03772_amd import synth
from gpu_helpers import check_step

pytestmark = pytest.mark.gpu


def test_golden_small_sem(lib):
    import torch
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                    "small_sem_d10_n1000.json")))
    s = synth.workload_small(seed=0)
    X = torch.as_tensor(s.X.astype(np.float32)).cuda()
    out = lib.causal_order(X, with_measures=True)
    order = out["order"].cpu().numpy()
    assert [int(v) for v in order] == g["order"]
    ref = np.array([[np.nan if x is None else x for x in row] for row in g["measures"]])
    meas = out["measures"].cpu().numpy()
    for t in range(ref.shape[0]):
        bad, ok = check_step(meas[t], ref[t], order[t])
        assert bad == 0 and ok, t
    B = lib.adjacency(X, order).cpu().numpy()
    A = np.array(g["adjacency"])
    assert np.max(np.abs(B - A)) <= 1e-8 * max(1.0, np.max(np.abs(A)))
