"""Pins of the FP64 oracle against what the mathematics and the paper fix.

None of these re-types the oracle's arithmetic and compares it with itself:

* the entropy constants are pinned to the maximum-entropy theory they come
  from (orthonormalised contrast functions under the standard Gaussian,
  evaluated by numerical quadrature);
* E[log cosh u] and E[u exp(-u^2/2)] are pinned to quadrature of five
  densities on quantile-grid samples; H of a Gaussian to the Gaussian entropy;
* the pairwise measure is pinned by antisymmetry, by invariance under affine
  maps of either column, and by the direction of a textbook two-variable
  LiNGAM pair;
* the full search is pinned by exact recovery of the generating order on
  complete DAGs at large n, by valid topological orders on ER DAGs and on the
  paper's two-level protocol (Section 3.1, 50 seeds), and by the literal and
  memoised forms agreeing;
* residualisation by orthogonality, the VAR fit by a library least-squares
  solve.
"""
import numpy as np
import pytest
from scipy import integrate, special, stats

import oracle
from paper_2403_03772_amd import synth

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _gauss_expect(f):
    phi = lambda x: np.exp(-0.5 * x * x) / np.sqrt(2 * np.pi)
    return integrate.quad(lambda x: f(x) * phi(x), -40, 40, epsabs=1e-15, epsrel=1e-13,
                          limit=400)[0]


def _logcosh(x):
    a = np.abs(x)
    return a + np.log1p(np.exp(-2 * a)) - np.log(2.0)


# ---------------------------------------------------------------------------
# entropy approximation
# ---------------------------------------------------------------------------

def test_constants_match_maximum_entropy_theory():
    """k1, k2, gamma come from contrast functions orthonormalised under N(0,1):
    gamma = E[log cosh nu]; k = 1 / (2 ||G - proj_{poly<=2} G||^2)."""
    c = oracle.constants()
    gamma = _gauss_expect(_logcosh)
    assert abs(c["gamma"] - gamma) < 1e-4
    # even contrast: project out 1 and x^2 (E 1 = 1, E x^2 = 1, E x^4 = 3)
    rhs = np.array([gamma, _gauss_expect(lambda x: _logcosh(x) * x * x)])
    a, b = np.linalg.solve(np.array([[1.0, 1.0], [1.0, 3.0]]), rhs)
    norm2 = _gauss_expect(lambda x: (_logcosh(x) - a - b * x * x) ** 2)
    assert abs(c["k1"] - 1 / (2 * norm2)) / c["k1"] < 1e-3
    # odd contrast x exp(-x^2/2): project out x; closed form 36 / (8 sqrt 3 - 9)
    g = lambda x: x * np.exp(-0.5 * x * x)
    cx = _gauss_expect(lambda x: g(x) * x)
    norm2 = _gauss_expect(lambda x: (g(x) - cx * x) ** 2)
    assert abs(c["k2"] - 1 / (2 * norm2)) / c["k2"] < 1e-4
    assert abs(c["k2"] - 36.0 / (8.0 * np.sqrt(3.0) - 9.0)) < 1e-4
    # H(nu) is the differential entropy of N(0, 1)
    assert abs(c["hnu"] - stats.norm.entropy()) < 1e-14


_DISTS = {
    "gauss": stats.norm(),
    "uniform": stats.uniform(loc=-np.sqrt(3), scale=2 * np.sqrt(3)),
    "laplace": stats.laplace(scale=1 / np.sqrt(2)),
    "exp": stats.expon(loc=-1.0),
    "t4": stats.t(4, scale=1 / np.sqrt(2)),
}


def _density_expect(dist, f):
    lo, hi = dist.support()
    lo, hi = max(lo, -60.0), min(hi, 60.0)
    pts = [p for p in (-1.0, 0.0) if lo < p < hi]
    return integrate.quad(lambda x: f(x) * dist.pdf(x), lo, hi, points=pts or None,
                          epsabs=1e-14, epsrel=1e-12, limit=500)[0]


@pytest.mark.parametrize("name", sorted(_DISTS))
def test_entropy_moments_match_quadrature(name):
    dist = _DISTS[name]
    assert abs(dist.var() - 1.0) < 1e-12
    n = 1_000_000
    u = dist.ppf((np.arange(n) + 0.5) / n)
    e_lc, e_g = oracle.entropy_moments(u)
    assert abs(e_lc - _density_expect(dist, _logcosh)) < 2e-6
    assert abs(e_g - _density_expect(dist, lambda x: x * np.exp(-0.5 * x * x))) < 2e-6


def test_entropy_gaussian_is_maximal():
    n = 1_000_000
    q = (np.arange(n) + 0.5) / n
    h_gauss = oracle.entropy(stats.norm.ppf(q))
    # the Gaussian reaches H(nu) up to the rounding of gamma
    assert abs(h_gauss - oracle.constants()["hnu"]) < 1e-8
    for name in ("uniform", "laplace", "exp", "t4"):
        u = _DISTS[name].ppf(q)
        assert oracle.entropy(u) < h_gauss - 1e-3, name


def test_entropy_skew_term_matters():
    """Exp(1)-1 has E[u exp(-u^2/2)] != 0: H must drop by k2 * E[g]^2 beyond the
    log cosh term (a dropped skew term fails here)."""
    n = 1_000_000
    u = _DISTS["exp"].ppf((np.arange(n) + 0.5) / n)
    e_lc, e_g = oracle.entropy_moments(u)
    assert abs(e_g) > 0.1
    c = oracle.constants()
    only_even = c["hnu"] - c["k1"] * (e_lc - c["gamma"]) ** 2
    assert oracle.entropy(u) < only_even - 0.1


# ---------------------------------------------------------------------------
# pairwise measure
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("fam", ["uniform", "laplace", "exp", "t4"])
def test_pair_antisymmetry(fam):
    rng = np.random.default_rng(7)
    n = 2000
    x = synth.noise(rng, fam, n)
    y = 0.8 * x + synth.noise(rng, fam, n)
    r_xy = oracle.pair_measure(x, y)
    r_yx = oracle.pair_measure(y, x)
    assert abs(r_xy + r_yx) <= 1e-12 * max(1.0, abs(r_xy))
    assert abs(r_xy) > 1e-4


def test_pair_affine_invariance():
    rng = np.random.default_rng(11)
    n = 3000
    x = synth.noise(rng, "laplace", n)
    y = -1.3 * x + synth.noise(rng, "uniform", n)
    base = oracle.pair_measure(x, y)
    for a, b in [(2.5, 0.0), (-1.0, 3.0), (1e-3, -7.0)]:
        assert abs(oracle.pair_measure(a * x + b, y) - base) < 1e-10
        assert abs(oracle.pair_measure(x, a * y + b) - base) < 1e-10


@pytest.mark.parametrize("fam", ["uniform", "laplace", "exp"])
def test_pair_textbook_direction(fam):
    """x0 -> x1 with non-Gaussian noise: the measure must say 0 precedes 1."""
    rng = np.random.default_rng(3)
    n = 1_000_000
    x0 = synth.noise(rng, fam, n)
    x1 = 1.5 * x0 + synth.noise(rng, fam, n)
    assert oracle.pair_measure(x0, x1) > 0
    X = np.stack([x1, x0], axis=1)           # cause in column 1
    assert list(oracle.causal_order(X, mode="table")) == [1, 0]


def test_pair_gaussian_is_undecided():
    """With Gaussian data both directions fit equally well: R ~ 0."""
    rng = np.random.default_rng(5)
    n = 200_000
    x0 = rng.standard_normal(n)
    x1 = 0.7 * x0 + rng.standard_normal(n)
    assert abs(oracle.pair_measure(x0, x1)) < 2e-4


def test_pair_brute_force_tiny():
    """n = 4, written out with Python's math module in a different arrangement
    (residual by projection, population moments by explicit sums)."""
    import math

    xi = [0.3, -1.2, 2.0, 0.7]
    xj = [1.1, 0.4, -0.9, 2.2]

    def std(v):
        mu = sum(v) / len(v)
        sd = math.sqrt(sum((a - mu) ** 2 for a in v) / len(v))
        return [(a - mu) / sd for a in v]

    def H(u):
        lc = sum(math.log(math.cosh(a)) for a in u) / len(u)
        g = sum(a * math.exp(-a * a / 2) for a in u) / len(u)
        return (1 + math.log(2 * math.pi)) / 2 - 79.047 * (lc - 0.37457) ** 2 - 7.4129 * g * g

    zi, zj = std(xi), std(xj)
    rho = sum(a * b for a, b in zip(zi, zj)) / 4
    ri = std([a - rho * b for a, b in zip(zi, zj)])
    rj = std([b - rho * a for a, b in zip(zi, zj)])
    want = (H(zj) + H(ri)) - (H(zi) + H(rj))
    assert abs(oracle.pair_measure(np.array(xi), np.array(xj)) - want) < 1e-11


# ---------------------------------------------------------------------------
# full search
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("fam", ["uniform", "laplace", "exp"])
@pytest.mark.parametrize("d,seed", [(3, 0), (5, 1), (8, 2), (8, 3)])
def test_exact_recovery_complete_dag(fam, d, seed):
    s = synth.er_sem(d, 200_000, wlo=0.5, whi=2.0, noise_family=fam, seed=seed, complete=True)
    assert list(oracle.causal_order(s.X, mode="table")) == list(s.order)


@pytest.mark.parametrize("seed", range(4))
def test_er_dag_topological_at_large_n(seed):
    s = synth.er_sem(10, 100_000, indeg=1.5, noise_family="uniform", seed=seed)
    assert synth.is_topological(oracle.causal_order(s.X, mode="table"), s.B)


def test_paper_two_level_protocol_50_seeds():
    """Sequential-vs-parallel protocol of Section 3.1: d = 10, n = 10000,
    theta ~ N(0,1), e ~ U(0,1); the order must be a valid topological order."""
    for seed in range(50):
        s = synth.two_level_sem(seed=seed)
        assert synth.is_topological(oracle.causal_order(s.X, mode="table"), s.B), seed


def test_literal_equals_table():
    s = synth.er_sem(12, 600, indeg=2.0, noise_family=("uniform", "laplace", "exp"), seed=9)
    o1, m1, g1 = oracle.causal_order(s.X, mode="literal", with_measures=True)
    o2, m2, g2 = oracle.causal_order(s.X, mode="table", with_measures=True)
    assert list(o1) == list(o2)
    fin = np.isfinite(m1)
    assert np.array_equal(fin, np.isfinite(m2))
    assert np.max(np.abs(m1[fin] - m2[fin])) <= 1e-12
    assert np.max(np.abs(g1 - g2)) <= 1e-12


def test_measures_nonpositive_and_choice_is_argmax():
    s = synth.workload_small(3)
    order, meas, gaps = oracle.causal_order(s.X, with_measures=True)
    for t in range(9):
        row = meas[t]
        fin = np.isfinite(row)
        assert fin.sum() == 10 - t
        assert np.all(row[fin] <= 0)
        best = np.flatnonzero(fin)[np.argmax(row[fin])]
        assert best == order[t]
        assert gaps[t] >= 0


def test_permutation_and_scale_equivariance():
    s = synth.er_sem(9, 5000, indeg=2.0, noise_family="laplace", seed=21)
    base = oracle.causal_order(s.X, mode="table")
    rng = np.random.default_rng(0)
    perm = rng.permutation(9)
    scale = rng.uniform(0.2, 5.0, 9) * rng.choice([-1, 1], 9)
    Xp = (s.X * scale)[:, perm]
    got = oracle.causal_order(Xp, mode="table")
    assert list(perm[got]) == list(base)


def test_teacher_forcing_and_row_measures_agree():
    s = synth.er_sem(11, 800, indeg=2.0, noise_family="exp", seed=4)
    forced = np.array([3, 7, 0], dtype=np.int32)
    order, meas, _ = oracle.causal_order(s.X, forced=forced, with_measures=True)
    assert list(order[:3]) == list(forced)
    rows = np.array([v for v in range(11) if v not in forced], dtype=np.int32)
    got = oracle.step_measures_rows(s.X, forced, rows)
    assert np.max(np.abs(got - meas[3, rows])) <= 1e-12


def test_step_measures_all_equals_literal_rows():
    """Table-mode step after a forced prefix equals literal Algorithm 1 on every
    active row (1e-12), with NaN exactly on the prefix."""
    s = synth.er_sem(13, 900, indeg=2.0, noise_family=("uniform", "laplace", "exp"), seed=6)
    prefix = np.array([5, 0, 11, 2], dtype=np.int32)
    got = oracle.step_measures_all(s.X, prefix)
    assert np.array_equal(np.isnan(got), np.isin(np.arange(13), prefix))
    rows = np.array([v for v in range(13) if v not in prefix], dtype=np.int32)
    lit = oracle.step_measures_rows(s.X, prefix, rows)
    assert np.max(np.abs(got[rows] - lit)) <= 1e-12 * max(1.0, np.max(np.abs(lit)))
    # FP64 input that is exactly the FP32 data gives the same numbers bit for bit
    got64 = oracle.step_measures_all(s.X.astype(np.float32).astype(np.float64), prefix,
                                     fp64=True)
    assert np.array_equal(got64[rows], got[rows])


def test_step_measures_all_prefix_is_a_projection():
    """The outer loop's sequential regressions (R6) leave, up to centring, each
    remaining column minus its least-squares projection on the prefix columns,
    and the measures depend on the centred residuals only.  So the forced step
    equals a plain step 0 on numpy's projection residuals (lstsq on the
    centred prefix columns) of the remaining columns."""
    s = synth.er_sem(12, 3000, indeg=2.0, noise_family=("uniform", "laplace"), seed=8)
    X = s.X.astype(np.float32).astype(np.float64)
    prefix = np.array([7, 3, 10], dtype=np.int32)
    rest = np.array([v for v in range(12) if v not in prefix])
    Xc = X - X.mean(axis=0)
    A = Xc[:, prefix]
    coef, *_ = np.linalg.lstsq(A, Xc[:, rest], rcond=None)
    R = Xc[:, rest] - A @ coef
    ref = oracle.step_measures_all(R, [], fp64=True)
    got = oracle.step_measures_all(s.X, prefix)[rest]
    assert np.max(np.abs(got - ref)) <= 1e-9 * np.max(np.abs(ref))


def test_degenerate_inputs_are_reported():
    rng = np.random.default_rng(1)
    X = rng.uniform(size=(100, 4))
    Xc = X.copy()
    Xc[:, 2] = 1.5
    with pytest.raises(oracle.OracleError) as e:
        oracle.causal_order(Xc)
    assert e.value.code == oracle.DEGENERATE
    Xd = X.copy()
    Xd[:, 3] = -2.0 * Xd[:, 1]
    with pytest.raises(oracle.OracleError) as e:
        oracle.causal_order(Xd)
    assert e.value.code == oracle.DEGENERATE
    with pytest.raises(oracle.OracleError):
        oracle.causal_order(X[:1])


def test_single_variable():
    X = np.random.default_rng(0).uniform(size=(50, 1))
    assert list(oracle.causal_order(X)) == [0]


# ---------------------------------------------------------------------------
# residualisation and VAR least squares
# ---------------------------------------------------------------------------

def test_residualize_orthogonal():
    s = synth.er_sem(6, 4000, indeg=2.0, seed=2)
    active = np.arange(6, dtype=np.int32)
    R = oracle.residualize(s.X, active, 4)
    assert np.array_equal(R[:, 4], s.X[:, 4])
    for v in range(6):
        if v == 4:
            continue
        c = np.mean((R[:, v] - R[:, v].mean()) * (R[:, 4] - R[:, 4].mean()))
        assert abs(c) < 1e-12 * np.std(s.X[:, v]) * np.std(s.X[:, 4]) * 10
    # only active columns move
    R2 = oracle.residualize(s.X, np.array([0, 4], dtype=np.int32), 4)
    assert np.array_equal(R2[:, 1:4], s.X[:, 1:4])


def test_var_fit_matches_lstsq_and_is_orthogonal():
    v = synth.var_series(d=12, T=400, seed=3)
    coef, resid = oracle.var_fit(v.X, lags=1)
    Z = np.hstack([np.ones((399, 1)), v.X[:-1]])
    ref, *_ = np.linalg.lstsq(Z, v.X[1:], rcond=None)
    assert np.max(np.abs(coef - ref)) < 1e-10
    assert np.max(np.abs(Z.T @ resid)) / (np.linalg.norm(Z) * np.linalg.norm(resid)) < 1e-12
    assert np.allclose(resid, v.X[1:] - Z @ coef, atol=1e-12)


def test_var_fit_lag2_matches_lstsq():
    v = synth.var_series(d=5, T=300, seed=8)
    coef, resid = oracle.var_fit(v.X, lags=2)
    Z = np.hstack([np.ones((298, 1)), v.X[1:-1], v.X[:-2]])
    ref, *_ = np.linalg.lstsq(Z, v.X[2:], rcond=None)
    assert np.max(np.abs(coef - ref)) < 1e-10


def test_var_fit_consistency():
    """The LS estimate of the reduced-form matrix approaches the truth ~ 1/sqrt(T)."""
    errs = []
    for T in (500, 8000):
        v = synth.var_series(d=6, T=T, seed=1)
        coef, _ = oracle.var_fit(v.X, lags=1)
        errs.append(np.linalg.norm(coef[1:].T - v.A1))
    assert errs[1] < errs[0] / 2.0


# ---------------------------------------------------------------------------
# VarLiNGAM pieces (Section 3.2)
# ---------------------------------------------------------------------------

def test_ols_adjacency_matches_lstsq():
    s = synth.er_sem(7, 3000, indeg=2.0, noise_family="laplace", seed=12)
    order = s.order
    B = oracle.ols_adjacency(s.X, order)
    for k in range(7):
        c = order[k]
        P = list(order[:k])
        row = np.zeros(7)
        if P:
            Z = np.hstack([np.ones((3000, 1)), s.X[:, P]])
            coef, *_ = np.linalg.lstsq(Z, s.X[:, c], rcond=None)
            row[P] = coef[1:]
        assert np.max(np.abs(B[c] - row)) < 1e-9, c


def test_ols_adjacency_recovers_true_weights():
    s = synth.er_sem(6, 200_000, indeg=2.5, noise_family="uniform", seed=4, rescale=False)
    B = oracle.ols_adjacency(s.X, s.order)
    assert np.max(np.abs(B - s.B)) < 0.02


def _orthogonal_sem(n, d, seed):
    """Data of an exact linear SEM whose noise columns are exactly orthogonal
    and centred: x = B x + e, so X = E (I - B)^-T, plus column offsets."""
    rng = np.random.default_rng(seed)
    order = rng.permutation(d)
    B = np.zeros((d, d))
    for k in range(1, d):
        for q in range(k):
            if rng.random() < 0.5:
                B[order[k], order[q]] = rng.uniform(0.5, 2.0) * rng.choice([-1.0, 1.0])
    E = rng.laplace(size=(n, d))
    E -= E.mean(axis=0)
    Q, _ = np.linalg.qr(E)
    E = Q * rng.uniform(0.5, 3.0, size=d)  # orthogonal, centred, unequal scales
    X = E @ np.linalg.inv(np.eye(d) - B).T + rng.normal(size=d) * 10.0
    return X, B, order


def test_ols_adjacency_exact_on_orthogonal_noise():
    """With noise columns exactly orthogonal to each other and to the constant,
    each variable's noise is orthogonal to its predecessors (which are
    combinations of earlier noises), so least squares on the order
    predecessors returns the generating weights exactly (up to rounding);
    a transposed or mis-permuted matrix fails this."""
    X, B, order = _orthogonal_sem(500, 9, seed=21)
    Bh = oracle.ols_adjacency(X, order)
    assert np.max(np.abs(Bh - B)) < 1e-9
    assert np.all(Bh[order[0]] == 0.0) and np.all(np.diag(Bh) == 0.0)


def test_ols_adjacency_simple_regression_slope():
    """d = 2: the coefficient is the textbook simple-regression slope
    cov(x0, x1) / var(x_parent), whichever variable comes first."""
    rng = np.random.default_rng(5)
    X = rng.exponential(size=(300, 2))
    X[:, 1] += 0.7 * X[:, 0]
    c = X - X.mean(axis=0)
    for order, child, parent in (([0, 1], 1, 0), ([1, 0], 0, 1)):
        Bh = oracle.ols_adjacency(X, np.array(order, dtype=np.int32))
        slope = np.sum(c[:, 0] * c[:, 1]) / np.sum(c[:, parent] ** 2)
        assert abs(Bh[child, parent] - slope) < 1e-12
        assert Bh[parent, child] == 0.0


def test_var_lagged_effects_inverts_the_reduced_form():
    """theta_tau from M_tau = (I - B0)^-1 theta_tau (the reduced form of the
    structural model) comes back exactly; B0 = 0 leaves M unchanged."""
    rng = np.random.default_rng(2)
    d, lags = 6, 2
    perm = rng.permutation(d)
    B0 = np.zeros((d, d))
    for k in range(1, d):
        for q in range(k):
            B0[perm[k], perm[q]] = rng.normal() * (rng.random() < 0.6)
    theta = rng.normal(size=(lags, d, d)) * 0.3
    M = np.stack([np.linalg.solve(np.eye(d) - B0, theta[t]) for t in range(lags)])
    assert np.max(np.abs(oracle.var_lagged_effects(M, B0) - theta)) < 1e-12
    assert np.array_equal(oracle.var_lagged_effects(M, np.zeros((d, d))), M)


def test_bootstrap_counts_invariants():
    """Every unordered pair is ordered one way in each resample; an edge needs
    its parent to precede; duplicating every row leaves least squares (and so
    the counts) unchanged; one identity resample gives the plain adjacency."""
    s = synth.er_sem(6, 400, indeg=2.0, noise_family="laplace", seed=3)
    rng = np.random.default_rng(0)
    res = [rng.integers(0, 400, size=400) for _ in range(5)]
    ords = [rng.permutation(6) for _ in range(5)]
    oc, ec, cs = oracle.bootstrap_counts(s.X, res, ords, threshold=0.05)
    assert np.array_equal(oc + oc.T, 5 * (1 - np.eye(6, dtype=np.int64)))
    assert np.all(ec <= oc)
    twice = [np.repeat(r, 2) for r in res]
    oc2, ec2, cs2 = oracle.bootstrap_counts(s.X, twice, ords, threshold=0.05)
    assert np.array_equal(oc2, oc) and np.array_equal(ec2, ec)
    assert np.max(np.abs(cs2 - cs)) < 1e-9
    ident = np.arange(400)
    _, ec1, cs1 = oracle.bootstrap_counts(s.X, [ident], [s.order], threshold=0.0)
    B = oracle.ols_adjacency(s.X, s.order)
    assert np.array_equal(ec1, (B != 0).astype(np.int64))
    assert np.array_equal(cs1, B)


def test_total_effects_paths():
    """T = (I - B)^-1 equals the sum over directed paths (the Neumann series
    of the nilpotent B of a DAG), a chain multiplies its weights, and the
    diagonal is 1."""
    rng = np.random.default_rng(4)
    d = 8
    perm = rng.permutation(d)
    B = np.zeros((d, d))
    for k in range(1, d):
        for q in range(k):
            if rng.random() < 0.4:
                B[perm[k], perm[q]] = rng.uniform(-1.5, 1.5)
    T = oracle.total_effects(B)
    S, P = np.eye(d), np.eye(d)
    for _ in range(d):
        P = P @ B
        S += P
    assert np.max(np.abs(T - S)) < 1e-12
    assert np.allclose(np.diag(T), 1.0)
    C = np.zeros((3, 3))
    C[1, 0], C[2, 1] = 0.7, -2.0
    Tc = oracle.total_effects(C)
    assert abs(Tc[2, 0] - (-1.4)) < 1e-15 and Tc[0, 2] == 0.0


def test_fp64_and_fp32_entries_agree():
    s = synth.er_sem(9, 800, indeg=2.0, seed=6)
    X32 = s.X.astype(np.float32)
    o32, m32, _ = oracle.causal_order(X32, mode="table", with_measures=True)
    o64, m64, _ = oracle._order_fp64(X32.astype(np.float64), None, True)
    assert list(o32) == list(o64)
    fin = np.isfinite(m32)
    assert np.max(np.abs(m32[fin] - m64[fin])) == 0.0


def test_varlingam_recovers_structure():
    v = synth.var_series(d=8, T=20000, indeg=1.5, seed=2)
    out = oracle.varlingam(v.X, lags=1)
    assert np.max(np.abs(out["M"][0] - v.A1)) < 0.05
    assert synth.is_topological(out["order"], v.B0)
    assert np.max(np.abs(out["B0"] - v.B0)) < 0.08


def test_golden_small_sem_reproduced():
    """The stored oracle values (tests/golden/make_golden.py) are reproduced:
    a drift of the oracle's arithmetic shows here."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                    "small_sem_d10_n1000.json")))
    s = synth.workload_small(seed=0)
    X32 = s.X.astype(np.float32)
    order, meas, gaps = oracle.causal_order(X32, mode="literal", with_measures=True)
    assert [int(v) for v in order] == g["order"]
    ref = np.array([[np.nan if x is None else x for x in row] for row in g["measures"]])
    assert np.array_equal(np.isfinite(ref), np.isfinite(meas))
    fin = np.isfinite(ref)
    assert np.max(np.abs(meas[fin] - ref[fin])) <= 1e-13 * np.max(np.abs(ref[fin]))
    B = oracle.ols_adjacency(X32.astype(np.float64), order)
    assert np.max(np.abs(B - np.array(g["adjacency"]))) <= 1e-12
