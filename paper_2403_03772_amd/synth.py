"""Seeded synthetic inputs: linear non-Gaussian acyclic SEMs and VAR series.

This module draws data only.  It contains none of the ordering method's
arithmetic, so the GPU path and the FP64 oracle can both be fed from it.
Everything is generated in FP64 with ``numpy.random.default_rng(seed)``
(PCG64); callers cast to FP32 where the library needs it.

Model (LiNGAM, Section 2.2): x_i = sum_{k(j) < k(i)} theta_ij x_j + e_i with
mutually independent, continuous, non-Gaussian e_i and an acyclic graph.

Workload recipes (sizes and distributions of the paper's workloads):

* :func:`er_sem` -- random causal order, Erdos-Renyi DAG on it with a given
  expected in-degree, |w| ~ U[lo, hi] with a random sign, noise from a unit
  variance family.  With ``rescale=True`` every variable is scaled to unit
  sample variance as soon as it is generated (before its children use it);
  this keeps the same order and graph but stops variances from growing down
  the DAG, which at d >= 1000 would otherwise push the noise share of deep
  variables below FP32 resolution.
* :func:`two_level_sem` -- the paper's parity protocol (Section 3.1): nodes on
  two levels, edges only from level 0 to level 1, theta ~ N(0, 1),
  e ~ U(0, 1).
* :func:`var_series` -- VAR(1) with an instantaneous DAG (VarLiNGAM model,
  Section 3.2), reduced-form spectral radius fixed, Student-t(4) noise.
* :func:`bootstrap_indices` -- row resampling with replacement.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

NOISE_FAMILIES = ("uniform", "laplace", "exp", "t4")


def noise(rng: np.random.Generator, family: str, n: int) -> np.ndarray:
    """n draws of a zero-mean, unit-variance noise of the given family."""
    if family == "uniform":
        return rng.uniform(-np.sqrt(3.0), np.sqrt(3.0), n)
    if family == "laplace":
        return rng.laplace(0.0, 1.0 / np.sqrt(2.0), n)
    if family == "exp":
        return rng.exponential(1.0, n) - 1.0
    if family == "t4":
        return rng.standard_t(4.0, n) / np.sqrt(2.0)
    if family == "gauss":
        return rng.standard_normal(n)
    raise ValueError(f"unknown noise family {family!r}")


@dataclass
class SEM:
    X: np.ndarray            # n x d, FP64, row-major
    order: np.ndarray        # int32[d]: generating causal order (first = exogenous)
    B: np.ndarray            # d x d, B[child, parent] = weight used (after rescaling)
    families: list           # noise family per variable


def er_sem(d: int, n: int, indeg: float = 1.5, wlo: float = 0.5, whi: float = 2.0,
           noise_family="uniform", seed: int = 0, rescale: bool = True,
           complete: bool = False) -> SEM:
    """Random linear SEM on an Erdos-Renyi DAG.

    ``noise_family`` is one family name, or a sequence of names to draw a family
    per variable uniformly from.  ``complete=True`` puts an edge on every
    ordered pair (the causal order is then the only valid one).
    """
    rng = np.random.default_rng(seed)
    perm = rng.permutation(d).astype(np.int32)
    p_edge = 1.0 if complete else (min(1.0, 2.0 * indeg / (d - 1)) if d > 1 else 0.0)
    if isinstance(noise_family, str):
        fams = [noise_family] * d
    else:
        choices = list(noise_family)
        fams = [choices[k] for k in rng.integers(0, len(choices), d)]
    X = np.zeros((n, d), dtype=np.float64)
    B = np.zeros((d, d), dtype=np.float64)
    for pos in range(d):
        v = int(perm[pos])
        x = noise(rng, fams[v], n)
        if pos > 0:
            mask = rng.random(pos) < p_edge
            parents = perm[:pos][mask]
            if parents.size:
                w = rng.uniform(wlo, whi, parents.size) * rng.choice([-1.0, 1.0], parents.size)
                B[v, parents] = w
                x = x + X[:, parents] @ w
        if rescale:
            s = x.std()
            x = x / s
            B[v, :] /= s
        X[:, v] = x
    return SEM(X=X, order=perm, B=B, families=fams)


def two_level_sem(n: int = 10000, n0: int = 5, n1: int = 5, p_edge: float = 0.5,
                  seed: int = 0) -> SEM:
    """Two-level DAG of the paper's sequential-vs-parallel comparison."""
    rng = np.random.default_rng(seed)
    d = n0 + n1
    perm = rng.permutation(d).astype(np.int32)
    lvl0, lvl1 = perm[:n0], perm[n0:]
    X = np.zeros((n, d), dtype=np.float64)
    B = np.zeros((d, d), dtype=np.float64)
    for v in lvl0:
        X[:, v] = rng.uniform(0.0, 1.0, n)
    for v in lvl1:
        mask = rng.random(n0) < p_edge
        parents = lvl0[mask]
        w = rng.standard_normal(parents.size)
        B[v, parents] = w
        X[:, v] = X[:, parents] @ w + rng.uniform(0.0, 1.0, n)
    return SEM(X=X, order=perm, B=B, families=["uniform01"] * d)


@dataclass
class VARSeries:
    X: np.ndarray     # T x d
    B0: np.ndarray    # instantaneous effects, B0[child, parent]
    B1: np.ndarray    # lag-1 structural effects
    A1: np.ndarray    # reduced-form lag-1 matrix (I - B0)^-1 B1
    order: np.ndarray


def var_series(d: int = 487, T: int = 1258, indeg: float = 2.0, wlo: float = 0.3,
               whi: float = 1.0, radius: float = 0.6, noise_family: str = "t4",
               burn_in: int = 200, seed: int = 0) -> VARSeries:
    """x(t) = B0 x(t) + B1 x(t-1) + e(t), i.e. x(t) = (I-B0)^-1 (B1 x(t-1) + e(t))."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(d).astype(np.int32)
    p_edge = min(1.0, 2.0 * indeg / (d - 1)) if d > 1 else 0.0
    B0 = np.zeros((d, d))
    for pos in range(1, d):
        v = perm[pos]
        mask = rng.random(pos) < p_edge
        parents = perm[:pos][mask]
        if parents.size:
            B0[v, parents] = rng.uniform(wlo, whi, parents.size) * rng.choice([-1.0, 1.0],
                                                                                parents.size)
    inv = np.linalg.inv(np.eye(d) - B0)
    B1 = rng.standard_normal((d, d))
    A1 = inv @ B1
    rho = np.max(np.abs(np.linalg.eigvals(A1)))
    B1 *= radius / rho
    A1 = inv @ B1
    X = np.zeros((T + burn_in, d))
    x = np.zeros(d)
    for t in range(T + burn_in):
        e = noise(rng, noise_family, d)
        x = A1 @ x + inv @ e
        X[t] = x
    return VARSeries(X=X[burn_in:].copy(), B0=B0, B1=B1, A1=A1, order=perm)


def bootstrap_indices(n_base: int, n_draw: int, seed: int) -> np.ndarray:
    """Row indices drawn uniformly with replacement (int32)."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, n_base, n_draw).astype(np.int32)


def is_topological(order, B) -> bool:
    """True when no edge of B (B[child, parent] != 0) points backwards in ``order``."""
    pos = np.empty(len(order), dtype=np.int64)
    pos[np.asarray(order)] = np.arange(len(order))
    child, parent = np.nonzero(B)
    return bool(np.all(pos[parent] < pos[child]))


# ---------------------------------------------------------------------------
# the named workloads
# ---------------------------------------------------------------------------

def workload_small(seed: int = 0) -> SEM:
    """d = 10, n = 1000, in-degree 1.5, |w| in [0.5, 2], uniform noise."""
    return er_sem(10, 1000, indeg=1.5, wlo=0.5, whi=2.0, noise_family="uniform", seed=seed)


def workload_gene_scale(seed: int = 0, d: int = 1024, n: int = 8192,
                        rescale: bool = True) -> SEM:
    """Gene-expression-scale SEM: d = 1024, n = 8192, in-degree 4, |w| in [0.5, 2],
    per-variable noise family from {uniform, Laplace, exponential - 1}."""
    return er_sem(d, n, indeg=4.0, wlo=0.5, whi=2.0,
                  noise_family=("uniform", "laplace", "exp"), seed=seed, rescale=rescale)


@dataclass
class BootstrapBatch:
    base: SEM                 # the shared base sample (n_base x d_base)
    rows: list                # int32 row-index arrays, one per bootstrap resample
    sems: list                # independent SEMs of uneven size


def workload_bootstrap_batch(seed: int = 0, n_resamples: int = 256, d_base: int = 200,
                             n_base: int = 5000, n_sems: int = 64, n_lo: int = 500,
                             n_hi: int = 5000, d_lo: int = 50, d_hi: int = 400
                             ) -> BootstrapBatch:
    """Many independent orderings in one batch: bootstrap resamples of one base
    sample (d_base variables, n_base rows; each resample draws n ~ U[n_lo, n_hi]
    rows with replacement) plus independent SEMs with d ~ U[d_lo, d_hi] and
    n ~ U[n_lo, n_hi].  All SEMs use the gene-expression-scale family."""
    rng = np.random.default_rng(seed)
    fam = ("uniform", "laplace", "exp")
    base = er_sem(d_base, n_base, indeg=4.0, wlo=0.5, whi=2.0, noise_family=fam,
                  seed=int(rng.integers(1 << 31)))
    rows = [bootstrap_indices(n_base, int(rng.integers(n_lo, n_hi + 1)),
                              seed=int(rng.integers(1 << 31))) for _ in range(n_resamples)]
    sems = []
    for _ in range(n_sems):
        d = int(rng.integers(d_lo, d_hi + 1))
        n = int(rng.integers(n_lo, n_hi + 1))
        sems.append(er_sem(d, n, indeg=4.0, wlo=0.5, whi=2.0, noise_family=fam,
                           seed=int(rng.integers(1 << 31))))
    return BootstrapBatch(base=base, rows=rows, sems=sems)
