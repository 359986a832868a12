"""Pins of the adaptive-lasso pruning oracle (no GPU)."""
import warnings

import numpy as np

from oracle import lasso as LA
from paper_2403_03772_amd import synth


def test_lars_path_matches_library():
    """Breakpoints of the lasso path against scikit-learn's lars_path."""
    from sklearn.linear_model import lars_path
    rng = np.random.default_rng(0)
    for trial in range(4):
        n, p = 300, 12
        Z = rng.normal(size=(n, p)) @ rng.normal(size=(p, p)) * 0.3 + rng.normal(size=(n, p))
        y = Z[:, :3] @ np.array([1.5, -2.0, 0.7]) + rng.laplace(size=n)
        Z -= Z.mean(axis=0)
        y -= y.mean()
        with warnings.catch_warnings():
            warnings.simplefilter("ignore")
            _, _, coefs = lars_path(Z, y, method="lasso", alpha_min=0.0)
        path = LA.lars_lasso_path(Z.T @ Z, Z.T @ y)
        ours = np.array(path).T
        assert ours.shape == coefs.shape, (ours.shape, coefs.shape)
        assert np.max(np.abs(ours - coefs)) <= 1e-8 * max(1.0, np.max(np.abs(coefs)))


def test_path_ends_at_least_squares_and_respects_cap():
    rng = np.random.default_rng(1)
    Z = rng.normal(size=(200, 6))
    Z -= Z.mean(axis=0)
    y = Z @ rng.normal(size=6) + rng.normal(size=200)
    y -= y.mean()
    path = LA.lars_lasso_path(Z.T @ Z, Z.T @ y)
    ls = np.linalg.solve(Z.T @ Z, Z.T @ y)
    assert np.max(np.abs(path[-1] - ls)) < 1e-10
    capped = LA.lars_lasso_path(Z.T @ Z, Z.T @ y, max_active=3)
    assert max(np.count_nonzero(b) for b in capped) <= 3
    k = len(capped)
    assert np.allclose(np.array(capped), np.array(path[:k]), atol=1e-12)


def test_adaptive_lasso_matches_library_pipeline():
    """The whole pruning against scikit-learn's LassoLarsIC (BIC) on weighted
    standardized predictors, refitted by least squares."""
    from sklearn.linear_model import LassoLarsIC, LinearRegression
    s = synth.er_sem(9, 800, indeg=2.0, noise_family=("uniform", "laplace"), seed=5)
    X = s.X
    order = s.order
    B = LA.adaptive_lasso_adjacency(X, order)
    Z = (X - X.mean(axis=0)) / X.std(axis=0)
    ref = np.zeros_like(B)
    for pos in range(1, 9):
        y, P = order[pos], order[:pos]
        w = np.abs(LinearRegression().fit(Z[:, P], Z[:, y]).coef_)
        with warnings.catch_warnings():
            warnings.simplefilter("ignore")
            reg = LassoLarsIC(criterion="bic").fit(Z[:, P] * w, Z[:, y])
        keep = np.abs(reg.coef_ * w) > 0.0
        if keep.any():
            ref[y, P[keep]] = LinearRegression().fit(X[:, P[keep]], X[:, y]).coef_
    assert np.array_equal(B != 0, ref != 0)
    assert np.max(np.abs(B - ref)) <= 1e-8 * max(1.0, np.max(np.abs(ref)))


def test_adaptive_lasso_keeps_true_edges_at_large_n():
    s = synth.er_sem(8, 20000, indeg=2.0, noise_family="uniform", seed=2, rescale=False)
    B = LA.adaptive_lasso_adjacency(s.X, s.order)
    assert np.array_equal(B != 0, s.B != 0)
    assert np.max(np.abs(B - s.B)) < 0.05
