"""FP64 CPU oracle for the DirectLiNGAM causal-ordering search.

TEST INFRASTRUCTURE ONLY.  The oracle is the yardstick the GPU library is
checked against.  Only the test-suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  The GPU library neither
imports nor links it, and shares no code with it.

The arithmetic lives in ``lingam_oracle.c`` (plain C, FP64, OpenMP over
candidate variables only); this module compiles it with gcc and wraps it with
ctypes and numpy.  Each wrapper names the part of the paper it follows:

* :func:`entropy` -- maximum-entropy approximation H(u) used by the pairwise
  likelihood-ratio measure (the measure DirectLiNGAM's ``_diff_mutual_info``
  stands for, Section 2.2 and the Hyvarinen-Smith measure cited in Section 1).
* :func:`pair_measure` -- one ordered pair of Algorithm 1: standardize both
  columns, the two least-squares residuals, the difference of mutual
  informations.
* :func:`causal_order` -- the DirectLiNGAM outer loop (Section 2.2) around
  Algorithm 1, in literal or memoised ("table") mode, with optional teacher
  forcing.
* :class:`OrderRun` -- the same search advanced in resumable pieces.
* :func:`step_measures_rows` -- k_list entries of chosen rows at one step.
* :func:`step_measures_all` -- every k_list entry of one teacher-forced step
  (table mode).
* :func:`pair_matrix` -- the whole measure matrix between active columns.
* :func:`residualize` -- least-squares removal of one variable's effect.
* :func:`var_fit` -- least-squares VAR fit with intercept (Section 3.2, the
  first stage of VarLiNGAM).
* :func:`ols_adjacency` -- least-squares regression of every variable on its
  order predecessors (the instantaneous matrix B0 of VarLiNGAM).
* :func:`varlingam` -- the three stages of VarLiNGAM together.
* :func:`var_lagged_effects` -- the lagged effects of VarLiNGAM's structural
  model, theta_tau = (I - B0) M_tau.
* :func:`bootstrap_counts` -- order / edge counts over row resamples, each
  regressed along a given order.
* :func:`total_effects` -- total causal effects (I - B)^-1 of a weighted
  adjacency matrix (Section 4.2 ranks variables by them).

The learned-proposal form of the search (features, the scoring network with
its gradients and optimiser, the certified / margin / audit decisions) is in
:mod:`oracle.proposer`.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lingam_oracle.c")
_LIB = os.path.join(_HERE, "liblingam_oracle.so")

OK, INVALID, DEGENERATE, NOMEM = 0, -1, -2, -3
_lock = threading.Lock()
_lib = None


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O3, OpenMP, no fast-math). Returns the path."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O3", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        lib.lo_entropy.argtypes = [P, i64]
        lib.lo_entropy.restype = dbl
        lib.lo_entropy_moments.argtypes = [P, i64, P, P]
        lib.lo_entropy_moments.restype = None
        lib.lo_entropy_constants.argtypes = [P, P, P, P]
        lib.lo_entropy_constants.restype = None
        lib.lo_pair_matrix.argtypes = [P, i64, P, i32, P]
        lib.lo_pair_matrix.restype = ctypes.c_int
        lib.lo_pair_measure.argtypes = [P, P, i64, P]
        lib.lo_pair_measure.restype = ctypes.c_int
        lib.lo_causal_order.argtypes = [P, i64, i64, i64, P, i32, i32, P, P, P]
        lib.lo_causal_order.restype = ctypes.c_int
        lib.lo_causal_order_f64.argtypes = [P, i64, i64, i64, P, i32, i32, P, P, P]
        lib.lo_causal_order_f64.restype = ctypes.c_int
        lib.lo_step_measures_rows.argtypes = [P, i64, i64, i64, P, i32, P, i32, P]
        lib.lo_step_measures_rows.restype = ctypes.c_int
        lib.lo_step_measures_all.argtypes = [P, i64, i64, i64, P, i32, P]
        lib.lo_step_measures_all.restype = ctypes.c_int
        lib.lo_step_measures_all_f64.argtypes = [P, i64, i64, i64, P, i32, P]
        lib.lo_step_measures_all_f64.restype = ctypes.c_int
        lib.lo_residualize.argtypes = [P, i64, i64, i64, P, i32, i32]
        lib.lo_residualize.restype = ctypes.c_int
        lib.lo_var_fit.argtypes = [P, i64, i64, i64, i32, P, P]
        lib.lo_var_fit.restype = ctypes.c_int
        lib.lo_ols_adjacency.argtypes = [P, i64, i64, i64, P, P]
        lib.lo_ols_adjacency.restype = ctypes.c_int
        lib.lo_causal_order_resume.argtypes = [P, i64, i64, P, P, i32, i32, P, P, P]
        lib.lo_causal_order_resume.restype = ctypes.c_int
        lib.lo_num_threads.argtypes = []
        lib.lo_num_threads.restype = ctypes.c_int
        _lib = lib
        return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(code: int, what: str):
    if code != OK:
        raise OracleError(code, what)


def num_threads() -> int:
    return int(_load().lo_num_threads())


def constants() -> dict:
    """k1, k2, gamma and H(nu) as the oracle uses them."""
    vals = [ctypes.c_double() for _ in range(4)]
    _load().lo_entropy_constants(*[ctypes.byref(v) for v in vals])
    return dict(zip(("k1", "k2", "gamma", "hnu"), (v.value for v in vals)))


def entropy(u) -> float:
    """H(u) of a sample assumed to have unit variance."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    return float(_load().lo_entropy(_ptr(u), u.size))


def entropy_moments(u) -> tuple[float, float]:
    """(E log cosh u, E u exp(-u^2/2))."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    a, b = ctypes.c_double(), ctypes.c_double()
    _load().lo_entropy_moments(_ptr(u), u.size, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def pair_measure(xi, xj) -> float:
    """diff(i, j) of Algorithm 1 for raw columns xi, xj (positive: i precedes j)."""
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    xj = np.ascontiguousarray(xj, dtype=np.float64)
    assert xi.shape == xj.shape and xi.ndim == 1
    out = ctypes.c_double()
    _check(_load().lo_pair_measure(_ptr(xi), _ptr(xj), xi.size, ctypes.byref(out)),
           "pair_measure")
    return out.value


def pair_matrix(X, active) -> np.ndarray:
    """D[p, q] = diff(active[p], active[q]) (Algorithm 1's measure, R1) between
    the columns ``active`` of the FP64 matrix X (n x d); D[p, p] = 0."""
    Xc = np.ascontiguousarray(np.asarray(X, dtype=np.float64).T)
    n = Xc.shape[1]
    U = np.ascontiguousarray(active, dtype=np.int32)
    D = np.empty((U.size, U.size), dtype=np.float64)
    _check(_load().lo_pair_matrix(_ptr(Xc), n, _ptr(U), U.size, _ptr(D)), "pair_matrix")
    return D


def causal_order(X, forced=None, mode: str = "literal", with_measures: bool = False):
    """Causal order of the columns of X (n x d).

    X is cast to float32 first (the GPU receives FP32 data), then to FP64.
    Returns ``order`` (int32[d]) or ``(order, measures[(d-1), d], gaps[d-1])``.
    """
    X = np.ascontiguousarray(X, dtype=np.float32)
    n, d = X.shape
    order = np.empty(d, dtype=np.int32)
    meas = np.empty((max(d - 1, 1), d), dtype=np.float64) if with_measures else None
    gaps = np.empty(max(d - 1, 1), dtype=np.float64) if with_measures else None
    f = None if forced is None else np.ascontiguousarray(forced, dtype=np.int32)
    flen = 0 if f is None else f.size
    code = _load().lo_causal_order(
        _ptr(X), n, d, d, None if f is None else _ptr(f), flen,
        {"literal": 0, "table": 1}[mode], _ptr(order),
        None if meas is None else _ptr(meas), None if gaps is None else _ptr(gaps))
    _check(code, "causal_order")
    if with_measures:
        return order, meas[: d - 1], gaps[: d - 1]
    return order


class OrderRun:
    """The free-running search (DirectLiNGAM outer loop, Section 2.2, around
    Algorithm 1) advanced in pieces, so that a long ordering can be
    checkpointed between pieces and resumed.  Same arithmetic as
    :func:`causal_order`: X is cast to FP32 (what the GPU receives), then to
    FP64.  State: ``Xc`` (the residual columns, FP64, variable-major), ``U``
    (active original ids, ascending), ``m`` (their count); results so far:
    ``order``, ``measures`` (row t = k_list of step t by original id, NaN for
    ordered columns) and ``gaps``."""

    FIELDS = ("Xc", "U", "m", "order", "measures", "gaps", "mode")

    def __init__(self, X=None, mode: str = "table"):
        if X is None:
            return
        X = np.asarray(X, dtype=np.float32)
        n, d = X.shape
        self.Xc = np.ascontiguousarray(X.T, dtype=np.float64)
        self.U = np.arange(d, dtype=np.int32)
        self.m = np.array([d], dtype=np.int32)
        self.order = np.full(d, -1, dtype=np.int32)
        self.measures = np.full((max(d - 1, 1), d), np.nan)
        self.gaps = np.full(max(d - 1, 1), np.nan)
        self.mode = np.array([{"literal": 0, "table": 1}[mode]], dtype=np.int32)

    @property
    def d(self) -> int:
        return self.Xc.shape[0]

    @property
    def steps_done(self) -> int:
        return self.d - int(self.m[0])

    @property
    def finished(self) -> bool:
        return int(self.m[0]) <= 1

    def run(self, nsteps: int) -> int:
        """Run up to ``nsteps`` more steps; returns the number run."""
        before = self.steps_done
        d, n = self.Xc.shape
        code = _load().lo_causal_order_resume(
            _ptr(self.Xc), n, d, _ptr(self.U), _ptr(self.m), int(nsteps), int(self.mode[0]),
            _ptr(self.order), _ptr(self.measures), _ptr(self.gaps))
        _check(code, "causal_order_resume")
        return self.steps_done - before

    def save(self, path: str) -> None:
        np.savez(path, **{k: getattr(self, k) for k in self.FIELDS})

    @classmethod
    def load(cls, path: str) -> "OrderRun":
        run = cls()
        with np.load(path, allow_pickle=False) as z:
            for k in cls.FIELDS:
                setattr(run, k, np.ascontiguousarray(z[k]))
        return run


def step_measures_rows(X, prefix, rows) -> np.ndarray:
    """k_list entries for original columns ``rows`` after regressing out ``prefix``."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    n, d = X.shape
    p = np.ascontiguousarray(prefix, dtype=np.int32)
    r = np.ascontiguousarray(rows, dtype=np.int32)
    out = np.empty(r.size, dtype=np.float64)
    code = _load().lo_step_measures_rows(_ptr(X), n, d, d, _ptr(p) if p.size else None,
                                         p.size, _ptr(r) if r.size else None, r.size, _ptr(out))
    _check(code, "step_measures_rows")
    return out


def step_measures_all(X, prefix, fp64: bool = False) -> np.ndarray:
    """Every k_list entry of step t = len(prefix) after regressing out
    ``prefix`` in order (table mode), by original column id; NaN for the
    prefix.  X is cast to FP32 first (what the GPU receives) unless ``fp64``
    (VAR residuals are FP64 data)."""
    p = np.ascontiguousarray(prefix, dtype=np.int32)
    if fp64:
        X = np.ascontiguousarray(X, dtype=np.float64)
        fn = _load().lo_step_measures_all_f64
    else:
        X = np.ascontiguousarray(X, dtype=np.float32)
        fn = _load().lo_step_measures_all
    n, d = X.shape
    out = np.empty(d, dtype=np.float64)
    _check(fn(_ptr(X), n, d, d, _ptr(p) if p.size else None, p.size, _ptr(out)),
           "step_measures_all")
    return out


def residualize(X, active, exo) -> np.ndarray:
    """Copy of X (FP64) with ``exo`` regressed out of every other ``active`` column."""
    X = np.array(X, dtype=np.float64, order="C", copy=True)
    n, d = X.shape
    a = np.ascontiguousarray(active, dtype=np.int32)
    _check(_load().lo_residualize(_ptr(X), n, d, d, _ptr(a), a.size, int(exo)), "residualize")
    return X


def var_fit(X, lags: int = 1):
    """Least-squares VAR(lags) with intercept. Returns (coef[(1+d*lags), d], resid)."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    T, d = X.shape
    coef = np.empty((1 + d * lags, d), dtype=np.float64)
    resid = np.empty((T - lags, d), dtype=np.float64)
    _check(_load().lo_var_fit(_ptr(X), T, d, d, int(lags), _ptr(coef), _ptr(resid)), "var_fit")
    return coef, resid


def ols_adjacency(E, order) -> np.ndarray:
    """B[c, p]: coefficient of column p when column c is regressed (with
    intercept) on every column preceding it in ``order``."""
    E = np.ascontiguousarray(E, dtype=np.float64)
    n, d = E.shape
    o = np.ascontiguousarray(order, dtype=np.int32)
    B = np.empty((d, d), dtype=np.float64)
    _check(_load().lo_ols_adjacency(_ptr(E), n, d, d, _ptr(o), _ptr(B)), "ols_adjacency")
    return B


def varlingam(X, lags: int = 1, forced=None, with_measures: bool = False):
    """VarLiNGAM (Section 3.2): least-squares VAR(lags) with intercept, the
    DirectLiNGAM order of its residuals, B0 by least squares on the order.

    Returns a dict with ``coef`` ((1 + d*lags) x d), ``M`` (lags x d x d,
    M[tau-1][i, j] = coefficient of x_j(t - tau) in the equation of x_i),
    ``resid``, ``order``, ``B0`` (and ``measures`` / ``gaps``).  The residuals
    are ordered as FP64 data (reading R9): no FP32 rounding between the VAR
    fit and the search.
    """
    X = np.ascontiguousarray(X, dtype=np.float64)
    T, d = X.shape
    coef, resid = var_fit(X, lags)
    M = np.stack([coef[1 + (tau - 1) * d: 1 + tau * d].T for tau in range(1, lags + 1)])
    out = {"coef": coef, "M": M, "resid": resid}
    if with_measures:
        order, meas, gaps = _order_fp64(resid, forced, True)
        out.update(measures=meas, gaps=gaps)
    else:
        order = _order_fp64(resid, forced, False)
    out["order"] = order
    out["B0"] = ols_adjacency(resid, order)
    return out


def var_lagged_effects(M, B0) -> np.ndarray:
    """Lagged effects theta_tau (tau = 1 .. lags) of VarLiNGAM's structural model.

    Section 3.2 writes the model as x(t) = sum over tau = 0 .. k of
    theta_tau x(t - tau) + eps(t), with theta_0 = B0 the instantaneous effects.
    Moving theta_0 x(t) to the left gives (I - B0) x(t) = sum over tau >= 1 of
    theta_tau x(t - tau) + eps(t), so the VAR (reduced-form) matrices are
    M_tau = (I - B0)^-1 theta_tau and, inverted, theta_tau = (I - B0) M_tau.
    ``M`` is lags x d x d (M[tau-1][i, j]: coefficient of x_j(t - tau) in the
    equation of x_i); the result has the same layout.
    """
    M = np.asarray(M, dtype=np.float64)
    B0 = np.asarray(B0, dtype=np.float64)
    d = B0.shape[0]
    A = np.eye(d) - B0
    return np.stack([A @ M[t] for t in range(M.shape[0])])


def total_effects(B) -> np.ndarray:
    """Total causal effects of the linear acyclic model x = B x + e (Section
    2.2): x = (I - B)^-1 e, so T = (I - B)^-1 and T[i, j] is the effect on
    x_i of a unit change of x_j along all directed paths (T[i, i] = 1).
    Section 4.2 ranks the variables that exert and receive the largest total
    effects."""
    B = np.asarray(B, dtype=np.float64)
    return np.linalg.inv(np.eye(B.shape[0]) - B)


def bootstrap_counts(X, resamples, orders, threshold: float = 0.0):
    """Bootstrap statistics by definition: for every resample (row indices into
    X, with replacement) and its causal order, B = least squares of each
    variable on its order predecessors (:func:`ols_adjacency` on X[rows]);
    order_count[i, j] counts resamples in which x_j precedes x_i,
    edge_count[i, j] those with |B[i, j]| > threshold; coef_sum adds B."""
    X = np.asarray(X, dtype=np.float64)
    d = X.shape[1]
    order_count = np.zeros((d, d), dtype=np.int64)
    edge_count = np.zeros((d, d), dtype=np.int64)
    coef_sum = np.zeros((d, d))
    for rows, order in zip(resamples, orders):
        order = np.asarray(order)
        B = ols_adjacency(X[np.asarray(rows)], order)
        pos = np.empty(d, dtype=np.int64)
        pos[order] = np.arange(d)
        order_count += pos[None, :] < pos[:, None]
        edge_count += np.abs(B) > threshold
        coef_sum += B
    return order_count, edge_count, coef_sum


def _order_fp64(E, forced, with_measures):
    """Causal order of FP64 data (no FP32 rounding of the input)."""
    E = np.ascontiguousarray(E, dtype=np.float64)
    n, d = E.shape
    # the oracle's C entry takes FP32 input (what the library receives);
    # VAR residuals are FP64, so order them through a float64 wrapper
    order = np.empty(d, dtype=np.int32)
    meas = np.empty((max(d - 1, 1), d), dtype=np.float64) if with_measures else None
    gaps = np.empty(max(d - 1, 1), dtype=np.float64) if with_measures else None
    f = None if forced is None else np.ascontiguousarray(forced, dtype=np.int32)
    code = _load().lo_causal_order_f64(
        _ptr(E), n, d, d, None if f is None else _ptr(f), 0 if f is None else f.size, 1,
        _ptr(order), None if meas is None else _ptr(meas), None if gaps is None else _ptr(gaps))
    _check(code, "causal_order_f64")
    if with_measures:
        return order, meas[: d - 1], gaps[: d - 1]
    return order
