"""The arithmetic behind bench.py's reported figures, on the CPU:

* the evaluation count of one ordering, n (d^3 - d) / 3, against the sum over
  the steps of m (m - 1) n (both residual directions of every unordered pair
  at every sample, m = d, d - 1, ..., 2 active variables);
* the roofline record: 12 flops per evaluation against the published FP32
  peak, and the issue model 1 / (7 / R_fma + 2 / R_exp) from measured rates;
* Kendall's tau against a brute-force count of concordant and discordant
  pairs, and the reversed-edge count against a direct walk over the edges.
"""
import itertools

import numpy as np
import pytest

import bench


@pytest.mark.parametrize("d", [2, 3, 10, 64, 1024, 4096])
def test_evals_per_ordering_is_the_sum_over_steps(d):
    n = 8192
    want = sum(m * (m - 1) * n for m in range(2, d + 1))
    assert bench.evals_per_ordering(n, d) == float(want)


def test_roofline_record():
    e = 3.3e12
    rec = bench.pair_roofline(e, None)
    assert rec["bound"] == "alu" and rec["unit"] == "TFLOP/s" and rec["peak"] == 157.3
    assert rec["achieved"] == pytest.approx(e * 12 / 1e12, rel=1e-12)
    assert rec["frac"] == pytest.approx(e * 12 / 157.3e12, rel=1e-12)
    rates = {"fma_lane_ops_per_s": 3.8e13, "exp_lane_ops_per_s": 1.9e13,
             "eval_mix_per_s": 3.5e12}
    rec = bench.pair_roofline(e, rates)
    model = 1.0 / (7 / 3.8e13 + 2 / 1.9e13)
    assert rec["issue_model"]["evals_per_s"] == pytest.approx(model, rel=1e-12)
    assert rec["issue_model_frac"] == pytest.approx(e / model, rel=1e-12)
    assert rec["eval_mix_frac"] == pytest.approx(e / 3.5e12, rel=1e-12)


def _tau_brute(a, b):
    pa = {v: i for i, v in enumerate(a)}
    pb = {v: i for i, v in enumerate(b)}
    s = 0
    for u, v in itertools.combinations(a, 2):
        s += np.sign(pa[u] - pa[v]) * np.sign(pb[u] - pb[v])
    n = len(a)
    return s / (n * (n - 1) / 2)


def test_kendall_tau_against_pair_count():
    rng = np.random.default_rng(0)
    for n in (2, 3, 7, 40):
        for _ in range(5):
            a, b = rng.permutation(n), rng.permutation(n)
            assert bench.kendall_tau(a, b) == pytest.approx(_tau_brute(a, b), abs=1e-12)
    a = np.arange(10)
    assert bench.kendall_tau(a, a) == pytest.approx(1.0)
    assert bench.kendall_tau(a, a[::-1]) == pytest.approx(-1.0)


def test_reversed_edges_against_edge_walk():
    rng = np.random.default_rng(1)
    d = 30
    B = np.zeros((d, d))
    for child in range(d):
        for parent in range(child):
            if rng.random() < 0.2:
                B[child, parent] = rng.uniform(0.5, 2.0)
    topo = np.arange(d)
    assert bench.reversed_edges(topo, B) == 0
    assert bench.reversed_edges(topo[::-1], B) == int(np.count_nonzero(B))
    order = rng.permutation(d)
    pos = {v: i for i, v in enumerate(order)}
    want = sum(1 for c in range(d) for p in range(d) if B[c, p] != 0 and pos[c] < pos[p])
    assert bench.reversed_edges(order, B) == want
