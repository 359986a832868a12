"""The seeded input generators against the workload recipes they implement
(the shapes, graphs, weights and noise distributions of the paper's
workloads), on the CPU:

* every noise family has mean 0 and variance 1, and the skewness / excess
  kurtosis of its distribution (uniform: 0 / -1.2, Laplace: 0 / 3,
  Exp(1) - 1: 2 / 6, t4 / sqrt 2: 0 / heavy);
* an ER SEM is acyclic in its generating order, has the requested expected
  in-degree, |w| in [lo, hi] (before rescaling), unit-variance columns with
  rescaling, and each variable minus its parents' contribution is exactly
  its own (rescaled) noise draw: uncorrelated with its parents;
* the two-level protocol has edges only from level 0 to level 1;
* the VAR series has the stated reduced-form spectral radius and an acyclic
  instantaneous graph;
* the bootstrap batch has the stated counts and size ranges, and is
  reproducible from its seed.
"""
import numpy as np
import pytest

from paper_2403_03772_amd import synth

MOMENTS = {  # skewness, excess kurtosis
    "uniform": (0.0, -1.2),
    "laplace": (0.0, 3.0),
    "exp": (2.0, 6.0),
    "gauss": (0.0, 0.0),
}


@pytest.mark.parametrize("fam", list(MOMENTS) + ["t4"])
def test_noise_families_are_standardised(fam):
    rng = np.random.default_rng(3)
    n = 2_000_000
    e = synth.noise(rng, fam, n)
    assert abs(e.mean()) < 5e-3
    assert abs(e.var() - 1.0) < (2e-2 if fam == "t4" else 5e-3)
    if fam in MOMENTS:
        z = (e - e.mean()) / e.std()
        skew, kurt = np.mean(z ** 3), np.mean(z ** 4) - 3.0
        s_want, k_want = MOMENTS[fam]
        assert abs(skew - s_want) < 0.05, (fam, skew)
        assert abs(kurt - k_want) < (0.3 if fam == "exp" else 0.1), (fam, kurt)
    else:  # Student t with 4 degrees of freedom: heavy tails (kurtosis unbounded)
        z = e / e.std()
        assert np.mean(z ** 4) - 3.0 > 2.0


def test_er_sem_recipe():
    d, n, indeg = 400, 4000, 4.0
    s = synth.er_sem(d, n, indeg=indeg, wlo=0.5, whi=2.0,
                     noise_family=("uniform", "laplace", "exp"), seed=5, rescale=False)
    assert s.X.shape == (n, d) and sorted(s.order.tolist()) == list(range(d))
    assert synth.is_topological(s.order, s.B)
    w = np.abs(s.B[s.B != 0])
    assert w.min() >= 0.5 and w.max() <= 2.0
    # expected in-degree: each position draws its parents with p = 2 indeg / (d - 1)
    mean_indeg = np.count_nonzero(s.B) / d
    assert abs(mean_indeg - indeg) < 0.4, mean_indeg
    assert set(s.families) <= {"uniform", "laplace", "exp"}


def test_er_sem_rescaled_columns_and_noise():
    s = synth.er_sem(120, 20000, indeg=3.0, noise_family=("uniform", "laplace", "exp"),
                     seed=8, rescale=True)
    assert np.allclose(s.X.std(axis=0), 1.0, atol=1e-12)
    assert synth.is_topological(s.order, s.B)
    # each variable minus its parents' contribution is its own noise (scaled):
    # uncorrelated with every parent, of the family's shape
    for v in s.order[1:40]:
        parents = np.flatnonzero(s.B[v])
        e = s.X[:, v] - s.X @ s.B[v]
        if parents.size:
            c = np.corrcoef(np.column_stack([e, s.X[:, parents]]).T)[0, 1:]
            assert np.max(np.abs(c)) < 0.05, (v, c)
        z = (e - e.mean()) / e.std()
        skew, kurt = np.mean(z ** 3), np.mean(z ** 4) - 3.0
        want_s, want_k = MOMENTS[s.families[v]]
        assert abs(skew - want_s) < 0.25 and abs(kurt - want_k) < 1.0, (v, s.families[v])


def test_complete_dag_has_every_edge():
    s = synth.er_sem(12, 500, complete=True, seed=2)
    pos = np.empty(12, dtype=int)
    pos[s.order] = np.arange(12)
    for c in range(12):
        for p in range(12):
            assert (s.B[c, p] != 0) == (pos[p] < pos[c])


def test_two_level_protocol():
    s = synth.two_level_sem(n=2000, seed=4)
    lvl0, lvl1 = set(s.order[:5].tolist()), set(s.order[5:].tolist())
    child, parent = np.nonzero(s.B)
    assert all(c in lvl1 and p in lvl0 for c, p in zip(child, parent))
    assert np.all(s.X[:, list(lvl0)] >= 0.0) and np.all(s.X[:, list(lvl0)] <= 1.0)


def test_var_series_recipe():
    v = synth.var_series(d=60, T=500, seed=1)
    assert v.X.shape == (500, 60)
    radius = np.max(np.abs(np.linalg.eigvals(v.A1)))
    assert radius == pytest.approx(0.6, rel=1e-9)
    assert synth.is_topological(v.order, v.B0)
    w = np.abs(v.B0[v.B0 != 0])
    assert w.min() >= 0.3 and w.max() <= 1.0
    inv = np.linalg.inv(np.eye(60) - v.B0)
    assert np.allclose(v.A1, inv @ v.B1)


def test_bootstrap_batch_recipe():
    wl = synth.workload_bootstrap_batch(seed=0, n_resamples=20, n_sems=6)
    assert wl.base.X.shape == (5000, 200)
    assert len(wl.rows) == 20 and len(wl.sems) == 6
    assert all(500 <= r.size <= 5000 and r.min() >= 0 and r.max() < 5000 for r in wl.rows)
    assert all(50 <= s.X.shape[1] <= 400 and 500 <= s.X.shape[0] <= 5000 for s in wl.sems)
    again = synth.workload_bootstrap_batch(seed=0, n_resamples=20, n_sems=6)
    assert all(np.array_equal(a, b) for a, b in zip(wl.rows, again.rows))
    assert np.array_equal(wl.base.X, again.base.X)
