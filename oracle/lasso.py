"""Adaptive-lasso pruning of the adjacency matrix (test infrastructure only).

The paper regresses every variable on its predecessors in the causal order
(the second phase of DirectLiNGAM, Section 1) and says no more; these
functions define the pruning that commonly follows, as a reading of our own:

* every variable is standardized (population moments);
* for target y with predictors P (its order predecessors), the least-squares
  coefficients b on standardized data give adaptive weights w = |b|;
* the lasso path of y on the weighted predictors z_P w is followed by least
  angle regression with the lasso modification (Efron, Hastie, Johnstone and
  Tibshirani, "Least angle regression", Ann. Statist. 2004, Section 3.1), in
  covariance form, up to ``max_active`` active predictors;
* among the path's breakpoints the one with the least Bayesian information
  criterion n log(2 pi s2) + RSS / s2 + log(n) df is kept, s2 being the
  least-squares residual variance RSS_ols / (n - p - 1) and df the number of
  nonzero coefficients;
* the kept predictors S are refitted by least squares with an intercept on
  the original data; their coefficients are row y of the pruned matrix.

Only the test-suite may import this module.  It shares no code with the GPU
library.
"""
from __future__ import annotations

import numpy as np


def lars_lasso_path(G, c, max_active: int | None = None) -> list:
    """Breakpoints of the lasso path (first: all zero) by least angle
    regression with the lasso modification, from G = Z'Z and c = Z'y of
    centred data.  Each step moves the active coefficients along the
    equiangular direction until an inactive predictor's correlation reaches
    the active ones' (it joins) or an active coefficient reaches zero (it
    leaves).  Stops at the least-squares fit of all predictors, when no
    correlation is left, or before a join that would exceed max_active."""
    G = np.asarray(G, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    p = c.size
    beta = np.zeros(p)
    path = [beta.copy()]
    if p == 0:
        return path
    cap = p if max_active is None else min(p, max_active)
    corr = c.copy()
    active: list = []
    tiny = 1e-14 * max(1.0, float(np.max(np.abs(c))))
    joined = True
    while True:
        inactive = [q for q in range(p) if q not in active]
        if joined:
            if not inactive:
                break
            j = max(inactive, key=lambda q: (abs(corr[q]), -q))
            if abs(corr[j]) <= tiny:
                break
            active.append(j)
            inactive.remove(j)
        A = np.array(active, dtype=np.int64)
        s = np.sign(corr[A])
        x = np.linalg.solve(G[np.ix_(A, A)], s)
        AA = 1.0 / np.sqrt(s @ x)
        w = AA * x
        a = G[:, A] @ w
        C = float(np.max(np.abs(corr[A])))
        gam, event, who = C / AA, "end", -1
        for q in inactive:
            for num, den in ((C - corr[q], AA - a[q]), (C + corr[q], AA + a[q])):
                if den > 0.0:
                    g = num / den
                    if 0.0 < g < gam:
                        gam, event, who = g, "join", q
        for i, q in enumerate(A):
            if w[i] != 0.0:
                g = -beta[q] / w[i]
                if 0.0 < g < gam:
                    gam, event, who = g, "leave", int(q)
        beta[A] += gam * w
        corr -= gam * a
        if event == "leave":
            beta[who] = 0.0
            active.remove(who)
        path.append(beta.copy())
        if event == "end":
            break
        if event == "join" and len(active) >= cap:
            break
        joined = event == "join"
    return path


def bic_select(G, c, n: int, rss_ols: float, path) -> int:
    """Index of the breakpoint with the least BIC (first on ties); y'y = n
    (standardized target), RSS(beta) = n - 2 beta'c + beta'G beta in sums
    over the samples when G, c are correlations times n."""
    p = c.size
    s2 = rss_ols / (n - p - 1)
    best, arg = np.inf, 0
    for i, b in enumerate(path):
        rss = n - 2.0 * b @ c + b @ G @ b
        crit = n * np.log(2.0 * np.pi * s2) + rss / s2 + np.log(n) * np.count_nonzero(b)
        if crit < best:
            best, arg = crit, i
    return arg


def adaptive_lasso_adjacency(X, order, max_active: int = 64, positions=None) -> np.ndarray:
    """Pruned weighted adjacency matrix: B[y, j] is the refitted coefficient
    of x_j for every predictor j the adaptive lasso keeps in the regression
    of x_y on its order predecessors; 0 elsewhere (see the module header).
    ``positions``: only the rows of the variables at these order positions
    (the others stay 0)."""
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    order = np.asarray(order, dtype=np.int64)
    Xc = X - X.mean(axis=0)
    sd = np.sqrt(np.mean(Xc * Xc, axis=0))
    Z = Xc / sd
    R = (Z.T @ Z) / n                      # correlation matrix
    B = np.zeros((d, d))
    for pos in (range(1, d) if positions is None else positions):
        if pos < 1:
            continue
        y, P = order[pos], order[:pos]
        p = P.size
        Rpp, rpy = R[np.ix_(P, P)], R[P, y]
        b = np.linalg.solve(Rpp, rpy)      # least squares on standardized data
        rss_ols = n * (1.0 - b @ rpy)
        w = np.abs(b)
        G = n * (w[:, None] * Rpp * w[None, :])
        cc = n * (w * rpy)
        path = lars_lasso_path(G, cc, max_active)
        beta = path[bic_select(G, cc, n, rss_ols, path)]
        S = P[beta != 0.0]
        if S.size:
            Zs = np.column_stack([np.ones(n), X[:, S]])
            coef, *_ = np.linalg.lstsq(Zs, X[:, y], rcond=None)
            B[y, S] = coef[1:]
    return B
