"""Writes the stored expected values under tests/golden/ (run from the repo root:
``python tests/golden/make_golden.py``).  It calls only the oracle and the
seeded input generators.

small_sem_d10_n1000.json: the plain DirectLiNGAM order (Section 2.2,
Algorithm 1, literal mode) of the d = 10, n = 1000 SEM (seed 0, uniform noise),
every step's measures M_t (-k by original id) and the least-squares adjacency
along that order.  A later oracle must reproduce them; the GPU parity tests
compare the library with the same values.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2403_03772_amd import synth  # noqa: E402


def main() -> None:
    s = synth.workload_small(seed=0)
    X32 = s.X.astype(np.float32)
    order, meas, gaps = oracle.causal_order(X32, mode="literal", with_measures=True)
    B = oracle.ols_adjacency(X32.astype(np.float64), order)
    out = {
        "source": "oracle (literal Algorithm 1, FP64) on synth.workload_small(seed=0) cast to FP32",
        "order": [int(v) for v in order],
        "measures": [[None if not np.isfinite(x) else float(x) for x in row] for row in meas],
        "gaps": [float(g) for g in gaps],
        "adjacency": [[float(x) for x in row] for row in B],
    }
    with open(os.path.join(HERE, "small_sem_d10_n1000.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
