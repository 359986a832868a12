"""FP64 oracle of the learned-proposal form of the ordering search.

TEST INFRASTRUCTURE ONLY: the yardstick for the library's proposer kernels.
Only the test-suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import it; the library never calls it and shares no code
with it.

The paper accelerates the exact DirectLiNGAM search (Section 2.2, Algorithm 1)
and does not itself propose candidates; this module defines the proposal form
built on top of that search, in plain numpy (FP64) plus the pairwise measure
matrix of the C oracle:

* 16 per-variable features of the current (standardized) residuals: entropy
  moments, higher moments, correlation statistics, rank and progress;
* a 16 -> 128 -> 128 -> 1 ReLU perceptron scoring every active variable
  (forward, backward, listwise softmax cross-entropy against the plain
  search's choice or against a soft target distribution, Adam);
* one learned step: the K best-scored variables are the candidates, their
  exact k_i = sum_j min(0, R(i, j))^2 is taken from the measure.  For an
  excluded variable l the candidates' rows already give R(l, c) = -R(c, l),
  so k_l >= LB_l = sum_{c in C} max(0, R(c, l))^2, and its witnesses (its
  most correlated excluded variables w) add min(0, R(l, w))^2 each.  The
  suspects are the excluded variables with LB_l <= k_best (1 + tie_rel) +
  tie_abs (the library decides near-ties of that width in FP64, so every
  variable whose k could come within it needs its exact row; tie_rel =
  tie_abs = 0 is the FP32-ties form).  No suspect: the best candidate is
  the plain choice (certified).  At most cap(m) = min(1024, m/2 - K) (rounded
  down to a multiple of 8) suspects: their exact k is evaluated and the best
  of candidates and suspects is the plain choice.  More: the best candidate
  is taken when its score beats every excluded variable's by at least a
  margin delta, else (and at every audit step) the full plain step decides.

Where the library rounds to BF16 (network inputs, weights, first hidden
layer) ``emulate_bf16=True`` applies the same rounding (round to nearest
even from FP32), so both sides take their top-K decisions at the same
precision; accumulation stays FP64 here.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import constants, pair_matrix

N_FEAT = 16
HIDDEN = 128
# flat parameter layout (FP32 on the device): W1[h][f], b1, W2[h][g], b2, w3, b3
SHAPES = (("W1", (HIDDEN, N_FEAT)), ("b1", (HIDDEN,)), ("W2", (HIDDEN, HIDDEN)),
          ("b2", (HIDDEN,)), ("w3", (HIDDEN,)), ("b3", (1,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)  # 18817
N_NORM = 2 * N_FEAT  # feature mean and scale, stored ahead of the weights


def unpack(flat) -> dict:
    flat = np.asarray(flat, dtype=np.float64)
    assert flat.size == N_PARAMS
    out, o = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = flat[o:o + k].reshape(shp).copy()
        o += k
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def init_params(seed: int = 0) -> np.ndarray:
    """He-uniform weights, zero biases (flat FP64)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in SHAPES:
        if name.startswith("b"):
            p[name] = np.zeros(shp)
        else:
            fan_in = shp[-1] if len(shp) == 2 else HIDDEN
            lim = np.sqrt(6.0 / fan_in)
            p[name] = rng.uniform(-lim, lim, shp)
    return pack(p)


def bf16(x) -> np.ndarray:
    """Round to BF16 (nearest, ties to even) via FP32; returned as FP64."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    b = a.view(np.uint32).astype(np.uint64)
    b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------------------
# features
# ---------------------------------------------------------------------------

def standardize(x) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    c = x - x.mean()
    return c / np.sqrt(np.mean(c * c))


def features(Xc, active, t: int, d: int) -> np.ndarray:
    """F[p] (16 values) of the active columns ``active`` (ascending original
    ids) of the current residual matrix Xc (n x d, FP64) at step t.

    1 E log cosh z   2 E z exp(-z^2/2)   3 H(z)   4 E z^3   5 E z^4 - 3
    6 E |z|   7 (E z^3)^2   8 max_j |rho_ij|   9 sum_j rho_ij^2 / m
    10 mean_j |rho_ij|   11 fraction of j with |rho_ij| > 0.5
    12 #{j : H_j < H_i, or H_j = H_i and j < i} / m   13 t / d   14 m / d
    15 ln n   16 sum_j rho_ij^2 H_j / sum_j rho_ij^2 (0 when all rho_ij = 0)
    with z the standardized column (population moments), j over the other
    active variables, H the maximum-entropy approximation of the entropy.
    """
    c = constants()
    U = np.asarray(active)
    m = U.size
    n = Xc.shape[0]
    Z = np.stack([standardize(Xc[:, v]) for v in U])          # m x n
    e_lc = np.array([np.mean(np.log(np.cosh(z))) for z in Z])
    e_g = np.array([np.mean(z * np.exp(-0.5 * z * z)) for z in Z])
    H = c["hnu"] - c["k1"] * (e_lc - c["gamma"]) ** 2 - c["k2"] * e_g ** 2
    rho = (Z @ Z.T) / n
    F = np.zeros((m, N_FEAT))
    for p in range(m):
        z = Z[p]
        others = np.array([q for q in range(m) if q != p], dtype=np.int64)
        r = rho[p, others]
        F[p, 0], F[p, 1], F[p, 2] = e_lc[p], e_g[p], H[p]
        F[p, 3] = np.mean(z ** 3)
        F[p, 4] = np.mean(z ** 4) - 3.0
        F[p, 5] = np.mean(np.abs(z))
        F[p, 6] = F[p, 3] ** 2
        if others.size:
            F[p, 7] = np.max(np.abs(r))
            F[p, 8] = np.sum(r * r) / m
            F[p, 9] = np.mean(np.abs(r))
            F[p, 10] = np.mean(np.abs(r) > 0.5)
            w = r * r
            F[p, 15] = np.sum(w * H[others]) / np.sum(w) if np.sum(w) > 0 else 0.0
        F[p, 11] = sum(1 for q in range(m)
                       if H[q] < H[p] or (H[q] == H[p] and U[q] < U[p])) / m
        F[p, 12] = t / d
        F[p, 13] = m / d
        F[p, 14] = np.log(n)
    return F


# ---------------------------------------------------------------------------
# the network
# ---------------------------------------------------------------------------

def normalize(F, norm) -> np.ndarray:
    """(F - mean) / scale with norm = [mean(16), scale(16)]."""
    norm = np.asarray(norm, dtype=np.float64)
    return (np.asarray(F, dtype=np.float64) - norm[:N_FEAT]) / norm[N_FEAT:]


def forward(flat, Xn, emulate_bf16: bool = False):
    """Scores of the rows of Xn (already normalized).  Returns (s, cache)."""
    p = unpack(flat)
    W1, W2, w3 = p["W1"], p["W2"], p["w3"]
    x = np.asarray(Xn, dtype=np.float64)
    if emulate_bf16:
        W1, W2, w3, x = bf16(W1), bf16(W2), bf16(w3), bf16(x)
    a1 = x @ W1.T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    if emulate_bf16:
        h1 = bf16(h1)
    a2 = h1 @ W2.T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    s = h2 @ w3 + p["b3"][0]
    return s, dict(x=x, a1=a1, h1=h1, a2=a2, h2=h2, W2=W2, w3=w3)


def backward(flat, cache, ds) -> np.ndarray:
    """Gradient of sum_r ds[r] * s[r] with respect to the flat parameters
    (at the weights the forward pass used)."""
    ds = np.asarray(ds, dtype=np.float64)
    x, a1, h1, a2, h2 = (cache[k] for k in ("x", "a1", "h1", "a2", "h2"))
    g = {}
    g["w3"] = h2.T @ ds
    g["b3"] = np.array([ds.sum()])
    dh2 = np.outer(ds, cache["w3"]) * (a2 > 0)
    g["W2"] = dh2.T @ h1
    g["b2"] = dh2.sum(axis=0)
    dh1 = (dh2 @ cache["W2"]) * (a1 > 0)
    g["W1"] = dh1.T @ x
    g["b1"] = dh1.sum(axis=0)
    return pack(g)


def listwise_ce(s, offsets, targets):
    """Mean over lists of -log softmax(s_list)[target].  List L is rows
    offsets[L] .. offsets[L+1]-1, ``targets[L]`` a row index inside it.
    Returns (loss, ds)."""
    s = np.asarray(s, dtype=np.float64)
    ds = np.zeros_like(s)
    nl = len(offsets) - 1
    loss = 0.0
    for L in range(nl):
        a, b = offsets[L], offsets[L + 1]
        z = s[a:b]
        mx = z.max()
        e = np.exp(z - mx)
        lse = mx + np.log(e.sum())
        loss += lse - s[targets[L]]
        ds[a:b] = e / e.sum()
        ds[targets[L]] -= 1.0
    return loss / nl, ds / nl


def listwise_ce_soft(s, offsets, weights):
    """Mean over lists of the cross-entropy between the target distribution
    q = weights / sum(weights) (per list, weights >= 0, positive sum) and
    softmax(s_list): sum_r -q_r log softmax(s)_r.  With one-hot weights this
    is :func:`listwise_ce`.  Returns (loss, ds)."""
    s = np.asarray(s, dtype=np.float64)
    w = np.asarray(weights, dtype=np.float64)
    ds = np.zeros_like(s)
    nl = len(offsets) - 1
    loss = 0.0
    for L in range(nl):
        a, b = offsets[L], offsets[L + 1]
        z = s[a:b]
        q = w[a:b] / w[a:b].sum()
        mx = z.max()
        e = np.exp(z - mx)
        lse = mx + np.log(e.sum())
        loss += np.sum(q * (lse - z))
        ds[a:b] = e / e.sum() - q
    return loss / nl, ds / nl


@dataclass
class Adam:
    """Adam (Kingma & Ba, 2015) with bias correction."""
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    t: int = 0
    m: np.ndarray = field(default=None)
    v: np.ndarray = field(default=None)

    def step(self, params, grad) -> np.ndarray:
        if self.m is None:
            self.m = np.zeros_like(params)
            self.v = np.zeros_like(params)
        self.t += 1
        self.m = self.beta1 * self.m + (1 - self.beta1) * grad
        self.v = self.beta2 * self.v + (1 - self.beta2) * grad * grad
        mh = self.m / (1 - self.beta1 ** self.t)
        vh = self.v / (1 - self.beta2 ** self.t)
        return params - self.lr * mh / (np.sqrt(vh) + self.eps)


# ---------------------------------------------------------------------------
# the learned step and ordering
# ---------------------------------------------------------------------------

def topk(scores, slots, K: int) -> np.ndarray:
    """Positions of the K best scores (higher first, ties to the smaller slot)."""
    idx = sorted(range(len(scores)), key=lambda p: (-scores[p], slots[p]))
    return np.array(idx[:K], dtype=np.int64)


def step_topk(m: int, K: int) -> int:
    """Candidates of a learned step with m variables and at most K: about m/16
    rounded up to a multiple of 8, at least min(32, K), at most K."""
    k = -(-(m // 16) // 8) * 8
    return min(max(k, min(32, K)), K)


def suspect_cap(m: int, K: int, cap: int = 1024) -> int:
    """Most suspects the second pass evaluates at a step with m variables."""
    c = min(m // 2 - K, cap)
    return c // 8 * 8 if c > 0 else 0


@dataclass
class StepInfo:
    t: int
    kind: str            # "plain" (small m), "learned", "expanded", "fallback", "audit"
    chosen: int
    plain_choice: int
    learned_choice: int = -1
    certified: bool = False
    margin: float = float("nan")
    candidates: np.ndarray = None
    suspects: int = 0
    rows: int = 0        # suspects whose full rows were measured (after the extension)
    extension: np.ndarray = None  # extension positions (ranked after the candidates)


def _plain_choice(k, U):
    # argmax of -k with ties to the smallest original id (U ascending)
    best = 0
    for p in range(1, len(U)):
        if k[p] < k[best]:
            best = p
    return best


def witnesses(Xc, active, W: int = 4) -> np.ndarray:
    """For every active column (position p into ``active``), the positions of
    the W other active columns with the largest |correlation| with it (ties to
    the smaller position; -1 past the last when fewer exist).  Their pair
    measures are the extra columns of the learned form's lower bound on k: a
    variable with parents is strongly correlated with them, and R against a
    parent is strongly negative."""
    U = np.asarray(active)
    m = U.size
    n = Xc.shape[0]
    Z = np.stack([standardize(Xc[:, v]) for v in U])
    a = np.abs((Z @ Z.T) / n)
    out = np.full((m, W), -1, dtype=np.int64)
    for p in range(m):
        others = sorted((q for q in range(m) if q != p), key=lambda q: (-a[p, q], q))
        out[p, :min(W, len(others))] = others[:W]
    return out


def lower_bounds(D, C, wit=None) -> np.ndarray:
    """Lower bound on k_l = sum_j min(0, R(l, j))^2 for every position l from
    the columns measured in a learned step: the candidate rows give R(c, l) =
    -R(l, c) for every c in C, and each non-candidate's witnesses w (not in C)
    give R(l, w).  Every column is counted once, so the bound never exceeds
    k_l.  D[a, b] = R(U[a], U[b])."""
    D = np.asarray(D, dtype=np.float64)
    m = D.shape[0]
    inC = np.zeros(m, dtype=bool)
    inC[np.asarray(C, dtype=np.int64)] = True
    pos = np.maximum(D[np.asarray(C, dtype=np.int64)], 0.0)
    lb = np.sum(pos * pos, axis=0)
    if wit is not None:
        for l in range(m):
            if inC[l]:
                continue
            for w in wit[l]:
                if w >= 0 and not inC[w]:
                    lb[l] += min(0.0, D[l, w]) ** 2
    return lb


def extension_bounds(D, lb, S, E, wit=None) -> np.ndarray:
    """The suspects' bounds after the extension columns: for every suspect l
    in S, add min(0, R(l, j))^2 for each extension column j in E (variables
    ranked right after the candidates) that is not l itself and not one of
    l's witnesses (already counted).  E holds no candidate, so every column
    still enters a bound at most once and the bound stays <= k_l.  Returns a
    new array; D[a, b] = R(U[a], U[b])."""
    D = np.asarray(D, dtype=np.float64)
    out = np.array(lb, dtype=np.float64, copy=True)
    for l in np.asarray(S, dtype=np.int64):
        seen = set() if wit is None else {int(w) for w in wit[l] if w >= 0}
        for j in np.asarray(E, dtype=np.int64):
            if j != l and int(j) not in seen:
                out[l] += min(0.0, D[l, j]) ** 2
    return out


TIE_REL, TIE_ABS = 4e-3, 1e-12


def learned_order(X, proposer, K: int = 64, delta: float = np.inf, audit_every: int = 32,
                  min_m: int | None = None, emulate_bf16: bool = True,
                  max_suspects: int = 1024, n_witness: int = 8, n_ext: int = 0,
                  tie_rel: float = TIE_REL, tie_abs: float = TIE_ABS):
    """Causal order by the learned-proposal form.

    X: n x d samples (cast to FP32 first, like the library's input).
    proposer: flat [norm(32), params(18817)].
    delta: score margin that accepts the best candidate when the suspects
    are too many for the second pass (+inf: never, so the order is the plain
    order).  audit_every: full step at t % audit_every == 0 (0: no audits).
    Steps with m <= min_m (default 2 min(K, 64)) are plain steps.  K is the
    most candidates; a step with m variables takes step_topk(m, K).  The
    lower bound on the non-candidates' k adds ``n_witness`` witness columns
    per variable (:func:`witnesses`, :func:`lower_bounds`).  Before the
    second pass the suspects' bounds also take the ``n_ext`` variables ranked
    right after the candidates (:func:`extension_bounds`); only suspects whose
    bound still does not exceed the best candidate's k have their rows
    measured.  A suspect is an excluded variable whose bound does not exceed
    k_best (1 + tie_rel) + tie_abs.  Returns (order, [StepInfo]).
    """
    X = np.asarray(np.asarray(X, dtype=np.float32), dtype=np.float64).copy()
    n, d = X.shape
    prop = np.asarray(proposer, dtype=np.float64)
    norm, flat = prop[:N_NORM], prop[N_NORM:]
    if min_m is None:
        min_m = 2 * min(K, 64)
    U = list(range(d))
    order, info = [], []
    t = 0
    while len(U) > 1:
        m = len(U)
        D = pair_matrix(X, U)
        neg = np.minimum(D, 0.0)
        k = np.sum(neg * neg, axis=1)
        pc = _plain_choice(k, U)
        if m <= min_m:
            p = pc
            info.append(StepInfo(t, "plain", U[p], U[pc]))
        else:
            F = features(X, U, t, d)
            s, _ = forward(flat, normalize(F, norm), emulate_bf16)
            if emulate_bf16:
                s = s.astype(np.float32).astype(np.float64)
            Kt = step_topk(m, K)
            ranked = topk(s, U, min(m, Kt + n_ext))
            C, E = ranked[:Kt], ranked[Kt:]
            inC = np.zeros(m, dtype=bool)
            inC[C] = True
            best = C[0]
            for c in C[1:]:
                if k[c] < k[best] or (k[c] == k[best] and U[c] < U[best]):
                    best = c
            wit = witnesses(X, U, n_witness) if n_witness > 0 else None
            lb = lower_bounds(D, C, wit)
            excl = ~inC
            lim = k[best] * (1.0 + tie_rel) + tie_abs
            sus = np.flatnonzero(excl & ~(lb > lim))
            certified = sus.size == 0
            s_out = np.max(s[excl]) if excl.any() else -np.inf
            margin = s[best] - s_out
            audit = audit_every > 0 and t % audit_every == 0
            expand = (not audit) and (not certified) and \
                sus.size <= suspect_cap(m, Kt, max_suspects)
            rows = 0
            if expand:
                # extension columns first; the rest of the suspects' rows
                # only where the bound still allows them to win
                lb2 = extension_bounds(D, lb, sus, E, wit)
                rest = sus[~(lb2[sus] > lim)]
                rows = int(rest.size)
            if audit:
                p, kind = pc, "audit"
            elif certified:
                p, kind = best, "learned"
            elif expand:
                # exact k of the remaining suspects; the best of candidates and them
                p = best
                for c in rest:
                    if k[c] < k[p] or (k[c] == k[p] and U[c] < U[p]):
                        p = c
                kind = "expanded"
            elif margin >= delta:
                p, kind = best, "learned"
            else:
                p, kind = pc, "fallback"
            info.append(StepInfo(t, kind, U[p], U[pc], U[best], certified, float(margin), C,
                                 int(sus.size), rows, E))
        e = U[p]
        order.append(e)
        xe = X[:, e]
        ve = np.mean((xe - xe.mean()) ** 2)
        for v in U:
            if v != e:
                b = np.mean((X[:, v] - X[:, v].mean()) * (xe - xe.mean())) / ve
                X[:, v] = X[:, v] - b * xe
        U.remove(e)
        t += 1
    order.append(U[0])
    return np.array(order, dtype=np.int32), info


def kendall_tau(a, b) -> float:
    """Kendall rank correlation between two orders of the same items."""
    a = np.asarray(a)
    b = np.asarray(b)
    n = a.size
    pa = np.empty(n, dtype=np.int64)
    pb = np.empty(n, dtype=np.int64)
    pa[a] = np.arange(n)
    pb[b] = np.arange(n)
    x = pa[np.argsort(pb)]  # positions in a, listed in b's order
    # count inversions of x (merge sort)
    def inv(v):
        if v.size <= 1:
            return v, 0
        h = v.size // 2
        l, il = inv(v[:h])
        r, ir = inv(v[h:])
        out = np.empty(v.size, dtype=v.dtype)
        i = j = k = 0
        c = il + ir
        while i < l.size and j < r.size:
            if l[i] <= r[j]:
                out[k] = l[i]
                i += 1
            else:
                out[k] = r[j]
                c += l.size - i
                j += 1
            k += 1
        out[k:] = np.concatenate([l[i:], r[j:]])
        return out, c
    _, d = inv(x)
    pairs = n * (n - 1) // 2
    return 1.0 - 2.0 * d / pairs
