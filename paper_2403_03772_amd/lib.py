"""ctypes binding of ``liblingam_mi355x.so``.

Only argument marshalling lives here.  Tensors must already be on the GPU;
the binding hands the library their device pointers and the current HIP
stream of PyTorch, allocates the workspace the library asks for, and turns
non-OK status codes into :class:`LingamError`.
"""
from __future__ import annotations

import ctypes
import math
import os
import threading
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblingam_mi355x.so")

OK, E_INVALID, E_DEGENERATE, E_HIP, E_WORKSPACE, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
FLAG_NO_SYNC, FLAG_GRAPH, FLAG_AUTOTUNE, FLAG_FP32_TIES = 1, 2, 4, 8

# proposer network (include/lingam.h)
N_FEATURES = 16
HIDDEN = 128
N_PARAMS = 18817
N_NORM = 32
PROPOSER_SIZE = N_NORM + N_PARAMS

_lock = threading.Lock()
_lib = None


class LingamError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lingam status {code}: {msg}")
        self.code = code


class _Profile(ctypes.Structure):
    _fields_ = [
        ("total_ms", ctypes.c_double),
        ("pair_ms", ctypes.c_double),
        ("pair_launches", ctypes.c_int64),
        ("pair_evals", ctypes.c_double),
        ("gram_ms", ctypes.c_double),
        ("gram_flops", ctypes.c_double),
        ("resid_ms", ctypes.c_double),
        ("resid_bytes", ctypes.c_double),
        ("cand_ms", ctypes.c_double),
        ("cand_launches", ctypes.c_int64),
        ("cand_evals", ctypes.c_double),
        ("tie_steps", ctypes.c_int32),
        ("tie_rows", ctypes.c_int32),
        ("tie_overflow", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class _LearnedStats(ctypes.Structure):
    _fields_ = [
        ("learned_steps", ctypes.c_int32),
        ("certified", ctypes.c_int32),
        ("fallbacks", ctypes.c_int32),
        ("audits", ctypes.c_int32),
        ("audit_agree", ctypes.c_int32),
        ("suspects_max", ctypes.c_int32),
        ("suspects_sum", ctypes.c_int64),
        ("expanded", ctypes.c_int32),
        ("cleared", ctypes.c_int32),
        ("rows_sum", ctypes.c_int64),
    ]


class _Opts(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
        ("forced_order", ctypes.c_void_p),
        ("forced_len", ctypes.c_int32),
        ("reserved0", ctypes.c_int32),
        ("step_measures", ctypes.c_void_p),
        ("step_gap", ctypes.c_void_p),
        ("dev_status", ctypes.c_void_p),
        ("profile", ctypes.POINTER(_Profile)),
        ("proposer", ctypes.c_void_p),
        ("topk", ctypes.c_int32),
        ("audit_every", ctypes.c_int32),
        ("margin", ctypes.c_float),
        ("learned_min_m", ctypes.c_int32),
        ("learned_stats", ctypes.POINTER(_LearnedStats)),
        ("record_features", ctypes.c_void_p),
        ("max_suspects", ctypes.c_int32),
        ("extension", ctypes.c_int32),
        ("step_log", ctypes.c_void_p),
        ("waves_all", ctypes.c_int32),
        ("waves_rows", ctypes.c_int32),
    ]


class _Job(ctypes.Structure):
    _fields_ = [
        ("X", ctypes.c_void_p),
        ("n_rows", ctypes.c_int64),
        ("ldx", ctypes.c_int64),
        ("rows", ctypes.c_void_p),
        ("n", ctypes.c_int64),
        ("d", ctypes.c_int64),
        ("order", ctypes.c_void_p),
        ("step_measures", ctypes.c_void_p),
        ("step_gap", ctypes.c_void_p),
        ("record_features", ctypes.c_void_p),
    ]


@dataclass
class Profile:
    total_ms: float
    pair_ms: float
    pair_launches: int
    pair_evals: float
    gram_ms: float
    gram_flops: float
    resid_ms: float
    resid_bytes: float
    cand_ms: float
    cand_launches: int
    cand_evals: float
    tie_steps: int
    tie_rows: int
    tie_overflow: int
    reserved: int


@dataclass
class LearnedStats:
    learned_steps: int
    certified: int
    fallbacks: int
    audits: int
    audit_agree: int
    suspects_max: int
    suspects_sum: int
    expanded: int
    cleared: int        # expanded steps whose suspects the extension columns all cleared
    rows_sum: int       # suspects whose full rows were measured


@dataclass
class Learned:
    """Learned-proposal configuration: ``proposer`` is a CUDA float32 tensor
    of PROPOSER_SIZE values (feature mean, feature scale, network weights).

    ``topk``: most candidates per step (a step with m variables takes about
    m/16, at least min(32, topk)); ``audit_every``: full-step audit period
    (0 = none); ``margin``: score lead that accepts the best candidate when
    the suspects are too many (+inf = never, the exact mode); ``min_m``:
    steps with at most this many variables are plain (default 2 min(topk,
    64)); ``max_suspects``: most suspects whose rows the second pass
    measures; ``extension``: extension columns measured against the suspects
    first (0 = none).  Mirrors the learned fields of ``lingam_opts``."""
    proposer: object
    topk: int = 64
    audit_every: int = 0
    margin: float = math.inf
    min_m: int | None = None
    max_suspects: int = 1024
    extension: int = 0


def load():
    """Load the shared library (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2403_03772_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        P, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
        f32 = ctypes.c_float
        O = ctypes.POINTER(_Opts)
        lib.lingam_opts_init.argtypes = [O]
        lib.lingam_opts_init.restype = None
        lib.lingam_workspace_size.argtypes = [i64, i64, O]
        lib.lingam_workspace_size.restype = sz
        lib.lingam_causal_order.argtypes = [P, i64, i64, i64, P, O, P, sz, P]
        lib.lingam_causal_order.restype = ctypes.c_int
        lib.lingam_causal_order_noalloc.argtypes = [P, i64, i64, i64, P, O, P]
        lib.lingam_causal_order_noalloc.restype = ctypes.c_int
        lib.lingam_residualize_workspace_size.argtypes = [i64, i64]
        lib.lingam_residualize_workspace_size.restype = sz
        lib.lingam_residualize.argtypes = [P, i64, i64, i64, P, i32, i32, P, sz, P]
        lib.lingam_residualize.restype = ctypes.c_int
        lib.varlingam_workspace_size.argtypes = [i64, i64, i32, O]
        lib.varlingam_workspace_size.restype = sz
        lib.varlingam_fit.argtypes = [P, i64, i64, i64, i32, P, P, P, P, O, P, sz, P]
        lib.varlingam_fit.restype = ctypes.c_int
        lib.lingam_batch_workspace_size.argtypes = [ctypes.POINTER(_Job), i32, O]
        lib.lingam_batch_workspace_size.restype = sz
        lib.lingam_batch_causal_order.argtypes = [ctypes.POINTER(_Job), i32, P, O, P, sz, P]
        lib.lingam_batch_causal_order.restype = ctypes.c_int
        lib.lingam_proposer_scores_workspace_size.argtypes = []
        lib.lingam_proposer_scores_workspace_size.restype = sz
        lib.lingam_proposer_scores.argtypes = [P, P, i64, P, P, sz, P]
        lib.lingam_proposer_scores.restype = ctypes.c_int
        lib.lingam_proposer_grad_workspace_size.argtypes = [i64, i32]
        lib.lingam_proposer_grad_workspace_size.restype = sz
        lib.lingam_proposer_grad.argtypes = [P, P, i64, P, P, i32, P, P, P, P, sz, P]
        lib.lingam_proposer_grad.restype = ctypes.c_int
        lib.lingam_proposer_grad_soft.argtypes = [P, P, i64, P, P, i32, P, P, P, P, sz, P]
        lib.lingam_proposer_grad_soft.restype = ctypes.c_int
        lib.lingam_proposer_adam.argtypes = [P, P, P, P, i32, f32, f32, f32, f32, P]
        lib.lingam_proposer_adam.restype = ctypes.c_int
        lib.lingam_adjacency_workspace_size.argtypes = [i64, i64]
        lib.lingam_adjacency_workspace_size.restype = sz
        lib.lingam_adjacency.argtypes = [P, i64, i64, P, i64, i64, P, P, P, sz, P]
        lib.lingam_adjacency_pruned_workspace_size.argtypes = [i64, i64]
        lib.lingam_adjacency_pruned_workspace_size.restype = sz
        lib.lingam_adjacency_pruned.argtypes = [P, i64, i64, P, i64, i64, P, i32, P, P, sz, P]
        lib.lingam_adjacency_pruned.restype = ctypes.c_int
        lib.lingam_bootstrap_accumulate.argtypes = [P, P, i64, ctypes.c_double, P, P, P, P]
        lib.lingam_bootstrap_accumulate.restype = ctypes.c_int
        lib.lingam_bootstrap_finalize.argtypes = [P, P, P, i64, i32, P, P, P, P]
        lib.lingam_bootstrap_finalize.restype = ctypes.c_int
        lib.lingam_adjacency.restype = ctypes.c_int
        lib.lingam_total_effects_workspace_size.argtypes = [i64]
        lib.lingam_total_effects_workspace_size.restype = sz
        lib.lingam_total_effects.argtypes = [P, i64, P, P, P, sz, P]
        lib.lingam_total_effects.restype = ctypes.c_int
        lib.varlingam_lagged_effects.argtypes = [P, P, i64, i32, P, P]
        lib.varlingam_lagged_effects.restype = ctypes.c_int
        lib.lingam_last_error.argtypes = []
        lib.lingam_last_error.restype = ctypes.c_char_p
        lib.lingam_version.argtypes = []
        lib.lingam_version.restype = ctypes.c_char_p
        _lib = lib
        return lib


def last_error() -> str:
    return load().lingam_last_error().decode()


def version() -> str:
    return load().lingam_version().decode()


def _check(code: int):
    if code != OK:
        raise LingamError(code, last_error())


def _stream_ptr(torch, device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _cuda_f32_matrix(torch, X, name="X"):
    if not (isinstance(X, torch.Tensor) and X.is_cuda and X.dtype == torch.float32):
        raise TypeError(f"{name} must be a CUDA float32 tensor")
    if X.dim() != 2 or X.stride(1) != 1:
        raise ValueError(f"{name} must be 2-D with unit column stride")


def _new_opts(lib, *, sync=True, graph=False, autotune=False, learned=None, profile=False,
              keep=None, waves=None, fp32_ties=False):
    """lingam_opts with flags, the learned configuration, the profile and the
    launch shape (``waves`` = (all-pairs, row kernels) waves per workgroup)."""
    opts = _Opts()
    lib.lingam_opts_init(ctypes.byref(opts))
    if waves is not None:
        opts.waves_all, opts.waves_rows = int(waves[0]), int(waves[1])
    if not sync:
        opts.flags |= FLAG_NO_SYNC
    if graph:
        opts.flags |= FLAG_GRAPH
    if autotune:
        opts.flags |= FLAG_AUTOTUNE
    if fp32_ties:
        opts.flags |= FLAG_FP32_TIES
    stats = None
    if learned is not None:
        import torch
        p = learned.proposer
        if not (isinstance(p, torch.Tensor) and p.is_cuda and p.dtype == torch.float32
                and p.is_contiguous() and p.numel() == PROPOSER_SIZE):
            raise TypeError(f"proposer must be a contiguous CUDA float32 tensor of "
                            f"{PROPOSER_SIZE} values")
        opts.proposer = p.data_ptr()
        opts.topk = int(learned.topk)
        opts.audit_every = int(learned.audit_every)
        opts.margin = float(learned.margin)
        opts.learned_min_m = int(learned.min_m if learned.min_m is not None
                                 else max(2 * min(learned.topk, 64), 64))
        opts.max_suspects = int(learned.max_suspects)
        opts.extension = int(learned.extension)
        stats = _LearnedStats()
        opts.learned_stats = ctypes.pointer(stats)
        if keep is not None:
            keep.append(stats)
    prof = _Profile() if profile else None
    if prof is not None:
        opts.profile = ctypes.pointer(prof)
    return opts, prof, stats


def _profile_of(prof):
    return Profile(**{k: getattr(prof, k) for k, _ in _Profile._fields_})


def _stats_of(stats):
    return LearnedStats(**{k: getattr(stats, k) for k, _ in _LearnedStats._fields_})


def workspace_size(n: int, d: int, learned: Learned | None = None) -> int:
    lib = load()
    keep = []
    opts, _, _ = _new_opts(lib, learned=learned, keep=keep)
    return int(lib.lingam_workspace_size(int(n), int(d), ctypes.byref(opts)))


def residualize_workspace_size(n: int, d: int) -> int:
    return int(load().lingam_residualize_workspace_size(int(n), int(d)))


def causal_order(X, *, forced=None, with_measures: bool = False, profile: bool = False,
                 workspace=None, sync: bool = True, graph: bool = False,
                 autotune: bool = False, learned: Learned | None = None,
                 record_features: bool = False, step_log: bool = False, out=None,
                 waves=None, fp32_ties: bool = False, _noalloc: bool = False):
    """DirectLiNGAM causal order of the columns of ``X`` (a CUDA float32 tensor, n x d).

    Returns ``order`` (int32 CUDA tensor, original column ids, exogenous first),
    or a dict with ``order``, ``measures`` ((d-1) x d FP64, NaN for columns
    already ordered), ``gaps``, ``profile``, ``features`` ((d-1) x d x 16
    FP32, NaN where not recorded) and ``learned_stats`` when any of those is
    asked for.  ``forced`` (sequence or tensor of column ids) fixes the first
    ``len(forced)`` choices (teacher forcing).  ``learned`` switches on the
    learned-proposal form; ``step_log`` returns its per-step decisions (see
    ``lingam_opts.step_log``).  ``out``: an int32 CUDA tensor of d entries to
    receive the order (a graph-mode call replays its graph only for the same
    buffers).  ``waves``: (all-pairs, row kernels) waves per workgroup, each
    1, 2 or 4 (``lingam_opts.waves_all`` / ``waves_rows``; None = default or
    autotuned); the results do not depend on it.  ``fp32_ties``: decide
    near-ties from the FP32 measures (``LINGAM_FLAG_FP32_TIES``).
    """
    import torch

    lib = load()
    _cuda_f32_matrix(torch, X)
    n, d = X.shape
    ldx = X.stride(0) if n > 1 else d
    dev = X.device
    if out is not None:
        if not (isinstance(out, torch.Tensor) and out.is_cuda and out.dtype == torch.int32
                and out.numel() == d and out.is_contiguous()):
            raise TypeError("out must be a contiguous CUDA int32 tensor of d entries")
        order = out
    else:
        order = torch.empty(d, dtype=torch.int32, device=dev)
    keep = []
    opts, prof, stats = _new_opts(lib, sync=sync, graph=graph, autotune=autotune,
                                  learned=learned, profile=profile, keep=keep, waves=waves,
                                  fp32_ties=fp32_ties)
    if forced is not None:
        f = torch.as_tensor(forced, dtype=torch.int32).to(dev).contiguous()
        keep.append(f)
        opts.forced_order = f.data_ptr()
        opts.forced_len = f.numel()
    meas = gaps = feats = None
    if with_measures and d > 1:
        meas = torch.empty((d - 1, d), dtype=torch.float64, device=dev)
        gaps = torch.empty(d - 1, dtype=torch.float64, device=dev)
        opts.step_measures = meas.data_ptr()
        opts.step_gap = gaps.data_ptr()
    if record_features and d > 1:
        feats = torch.full((d - 1, d, N_FEATURES), math.nan, dtype=torch.float32, device=dev)
        opts.record_features = feats.data_ptr()
    slog = None
    if step_log:
        slog = torch.zeros(d, dtype=torch.int32, device=dev)
        opts.step_log = slog.data_ptr()
    if _noalloc:
        code = lib.lingam_causal_order_noalloc(_ptr(X), n, d, ldx, _ptr(order),
                                               ctypes.byref(opts), _stream_ptr(torch, dev))
    else:
        need = int(lib.lingam_workspace_size(n, d, ctypes.byref(opts)))
        if need == 0:
            raise LingamError(E_UNSUPPORTED, last_error() or f"unsupported size n={n} d={d}")
        if workspace is None or workspace.numel() < need:
            workspace = torch.empty(need, dtype=torch.uint8, device=dev)
        code = lib.lingam_causal_order(_ptr(X), n, d, ldx, _ptr(order), ctypes.byref(opts),
                                       _ptr(workspace), workspace.numel(),
                                       _stream_ptr(torch, dev))
    _check(code)
    if not (with_measures or profile or record_features or step_log or learned is not None):
        return order
    out = {"order": order, "measures": meas, "gaps": gaps, "workspace": workspace}
    if slog is not None:
        out["step_log"] = slog
    if feats is not None:
        out["features"] = feats
    if prof is not None:
        out["profile"] = _profile_of(prof)
    if stats is not None and sync:
        out["learned_stats"] = _stats_of(stats)
    return out


def causal_order_noalloc(X, *, forced=None, with_measures: bool = False, sync: bool = True,
                         learned: Learned | None = None, step_log: bool = False, out=None):
    """:func:`causal_order` through ``lingam_causal_order_noalloc``: the library
    keeps the workspace in its per-GPU scratch array (sizes up to
    ``LINGAM_NOALLOC_SCRATCH_BYTES`` of workspace), so the call itself
    allocates no device memory (outputs still come from the caller; here the
    binding makes the order and measure tensors unless ``out`` is given).
    Graph capture, autotuning and profiles are not available through it."""
    return causal_order(X, forced=forced, with_measures=with_measures, sync=sync,
                        learned=learned, step_log=step_log, out=out, _noalloc=True)


def residualize(X, active, exo: int):
    """In place: regress column ``exo`` out of every other ``active`` column of X."""
    import torch

    lib = load()
    _cuda_f32_matrix(torch, X)
    n, d = X.shape
    a = torch.as_tensor(active, dtype=torch.int32).to(X.device).contiguous()
    need = int(lib.lingam_residualize_workspace_size(n, d))
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=X.device)
    code = lib.lingam_residualize(_ptr(X), n, d, X.stride(0), _ptr(a), a.numel(), int(exo),
                                  _ptr(ws), ws.numel(), _stream_ptr(torch, X.device))
    _check(code)
    return X


def adjacency(X, order, *, rows=None, workspace=None):
    """Least-squares adjacency of a CUDA float32 ``X`` (n_rows x d) given a
    causal ``order``: B[i, j] = coefficient of x_j when x_i is regressed (with
    intercept) on its order predecessors.  ``rows`` (int32 row indices, e.g. a
    bootstrap resample) selects the samples; default all rows.  Returns a
    d x d float64 tensor."""
    import torch

    lib = load()
    _cuda_f32_matrix(torch, X)
    n_rows, d = X.shape
    o = torch.as_tensor(order, dtype=torch.int32).to(X.device).contiguous()
    if o.numel() != d:
        raise ValueError(f"order has {o.numel()} entries, X has {d} columns")
    r = None
    n = n_rows
    if rows is not None:
        r = torch.as_tensor(rows, dtype=torch.int32).to(X.device).contiguous()
        n = r.numel()
    need = int(lib.lingam_adjacency_workspace_size(n, d))
    if need == 0:
        raise LingamError(E_INVALID, f"unsupported size n={n} d={d}")
    ws = workspace
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=X.device)
    B = torch.empty((d, d), dtype=torch.float64, device=X.device)
    code = lib.lingam_adjacency(_ptr(X), n_rows, X.stride(0), _ptr(r), n, d, _ptr(o), _ptr(B),
                                _ptr(ws), ws.numel(), _stream_ptr(torch, X.device))
    _check(code)
    return B


def adjacency_pruned(X, order, *, rows=None, max_active: int = 64, workspace=None):
    """Adjacency of a CUDA float32 ``X`` along ``order`` pruned by the adaptive
    lasso (BIC over the least-angle lasso path, least-squares refit of the
    kept predictors; ``lingam_adjacency_pruned``).  Returns d x d float64."""
    import torch

    lib = load()
    _cuda_f32_matrix(torch, X)
    n_rows, d = X.shape
    o = torch.as_tensor(order, dtype=torch.int32).to(X.device).contiguous()
    if o.numel() != d:
        raise ValueError(f"order has {o.numel()} entries, X has {d} columns")
    r = None
    n = n_rows
    if rows is not None:
        r = torch.as_tensor(rows, dtype=torch.int32).to(X.device).contiguous()
        n = r.numel()
    need = int(lib.lingam_adjacency_pruned_workspace_size(n, d))
    if need == 0:
        raise LingamError(E_INVALID, f"unsupported size n={n} d={d}")
    ws = workspace
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=X.device)
    B = torch.empty((d, d), dtype=torch.float64, device=X.device)
    code = lib.lingam_adjacency_pruned(_ptr(X), n_rows, X.stride(0), _ptr(r), n, d, _ptr(o),
                                       int(max_active), _ptr(B), _ptr(ws), ws.numel(),
                                       _stream_ptr(torch, X.device))
    _check(code)
    return B


def total_effects(B, order, *, workspace=None):
    """Total causal effects T = (I - B)^-1 of a CUDA float64 adjacency ``B``
    (d x d) along ``order`` (``lingam_total_effects``): T[i, j] is the effect
    on x_i of a unit change of x_j over all directed paths.  Entries of ``B``
    not below the order's diagonal are ignored.  Returns d x d float64."""
    import torch

    lib = load()
    if not (isinstance(B, torch.Tensor) and B.is_cuda and B.dtype == torch.float64
            and B.dim() == 2 and B.shape[0] == B.shape[1]):
        raise ValueError("B must be a square CUDA float64 tensor")
    B = B.contiguous()
    d = B.shape[0]
    o = torch.as_tensor(order, dtype=torch.int32).to(B.device).contiguous()
    if o.numel() != d:
        raise ValueError(f"order has {o.numel()} entries, B is {d} x {d}")
    need = int(lib.lingam_total_effects_workspace_size(d))
    if need == 0:
        raise LingamError(E_UNSUPPORTED, f"unsupported size d={d}")
    ws = workspace
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=B.device)
    T = torch.empty((d, d), dtype=torch.float64, device=B.device)
    _check(lib.lingam_total_effects(_ptr(B), d, _ptr(o), _ptr(T), _ptr(ws), ws.numel(),
                                    _stream_ptr(torch, B.device)))
    return T


def bootstrap_accumulate(order, B, threshold, order_count, edge_count, coef_sum=None):
    """Add one resample's order and adjacency to the running counts (in place)."""
    import torch

    lib = load()
    d = B.shape[0]
    _check(lib.lingam_bootstrap_accumulate(_ptr(order), _ptr(B), d, float(threshold),
                                           _ptr(order_count), _ptr(edge_count), _ptr(coef_sum),
                                           _stream_ptr(torch, B.device)))


def bootstrap(X, resamples, *, threshold: float = 0.0, graph: bool = False,
              autotune: bool = False, learned: Learned | None = None, prune: bool = False):
    """Bootstrap statistics of DirectLiNGAM on a CUDA float32 ``X`` (n x d).

    ``resamples``: sequence of int32 row-index arrays (drawn by the caller,
    with replacement).  All resamples are ordered in one batched run, then
    regressed along their orders; returns a dict with ``orders`` (list),
    ``order_prob`` (d x d: P(x_j precedes x_i) at [i, j]), ``edge_prob``
    (P(|B[i, j]| > threshold)), ``coef_mean`` (mean of B) and ``n`` (the
    number of resamples).  ``prune``: B from :func:`adjacency_pruned`.
    """
    import torch

    lib = load()
    _cuda_f32_matrix(torch, X)
    d = X.shape[1]
    dev = X.device
    rows = [torch.as_tensor(r, dtype=torch.int32).to(dev).contiguous() for r in resamples]
    if not rows:
        raise ValueError("no resamples")
    out = batch_causal_order([{"X": X, "rows": r} for r in rows], graph=graph,
                             autotune=autotune, learned=learned)
    order_count = torch.zeros((d, d), dtype=torch.int32, device=dev)
    edge_count = torch.zeros((d, d), dtype=torch.int32, device=dev)
    coef_sum = torch.zeros((d, d), dtype=torch.float64, device=dev)
    size_of = (lib.lingam_adjacency_pruned_workspace_size if prune
               else lib.lingam_adjacency_workspace_size)
    need = max(int(size_of(r.numel(), d)) for r in rows)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    fit = adjacency_pruned if prune else adjacency
    for r, o in zip(rows, out["orders"]):
        B = fit(X, o, rows=r, workspace=ws)
        bootstrap_accumulate(o, B, threshold, order_count, edge_count, coef_sum)
    probs = bootstrap_finalize(order_count, edge_count, coef_sum, len(rows))
    return {"orders": out["orders"], **probs, "n": len(rows),
            "order_count": order_count, "edge_count": edge_count}


def bootstrap_finalize(order_count, edge_count, coef_sum, n_resamples: int) -> dict:
    """Order / edge probabilities and mean coefficients from the running
    counts of :func:`bootstrap_accumulate` (the library divides)."""
    import torch

    lib = load()
    d = order_count.shape[0]
    dev = order_count.device
    order_prob = torch.empty((d, d), dtype=torch.float64, device=dev)
    edge_prob = torch.empty_like(order_prob)
    coef_mean = torch.empty_like(order_prob) if coef_sum is not None else None
    _check(lib.lingam_bootstrap_finalize(_ptr(order_count), _ptr(edge_count), _ptr(coef_sum), d,
                                         int(n_resamples), _ptr(order_prob), _ptr(edge_prob),
                                         _ptr(coef_mean), _stream_ptr(torch, dev)))
    return {"order_prob": order_prob, "edge_prob": edge_prob, "coef_mean": coef_mean}


def varlingam_lagged_effects(M, B0):
    """theta_tau = (I - B0) M_tau for CUDA float64 ``M`` (lags x d x d) and ``B0``."""
    import torch

    lib = load()
    if not (isinstance(M, torch.Tensor) and M.is_cuda and M.dtype == torch.float64
            and M.dim() == 3 and M.shape[1] == M.shape[2] and M.is_contiguous()):
        raise TypeError("M must be a contiguous CUDA float64 tensor of shape (lags, d, d)")
    lags, d, _ = M.shape
    if not (isinstance(B0, torch.Tensor) and B0.is_cuda and B0.dtype == torch.float64
            and tuple(B0.shape) == (d, d) and B0.is_contiguous()):
        raise TypeError("B0 must be a contiguous CUDA float64 tensor of shape (d, d)")
    theta = torch.empty_like(M)
    _check(lib.varlingam_lagged_effects(_ptr(M), _ptr(B0), d, int(lags), _ptr(theta),
                                        _stream_ptr(torch, M.device)))
    return theta


def varlingam_fit(X, lags: int = 1, *, forced=None, with_measures: bool = False,
                  profile: bool = False, learned: Learned | None = None,
                  lagged_effects: bool = True):
    """VarLiNGAM on a CUDA float32 series ``X`` (T x d, time in rows).

    Returns a dict: ``M`` (lags x d x d float64), ``resid`` ((T-lags) x d
    float32), ``order`` (int32), ``B0`` (d x d float64), ``theta``
    (lags x d x d float64, the lagged effects (I - B0) M_tau, unless
    ``lagged_effects`` is False), plus ``measures`` / ``gaps`` / ``profile``
    / ``learned_stats`` when asked.
    """
    import torch

    lib = load()
    _cuda_f32_matrix(torch, X)
    T, d = X.shape
    dev = X.device
    keep = []
    opts, prof, stats = _new_opts(lib, learned=learned, profile=profile, keep=keep)
    if forced is not None:
        f = torch.as_tensor(forced, dtype=torch.int32).to(dev).contiguous()
        keep.append(f)
        opts.forced_order = f.data_ptr()
        opts.forced_len = f.numel()
    out = {
        "M": torch.empty((lags, d, d), dtype=torch.float64, device=dev),
        "resid": torch.empty((T - lags, d), dtype=torch.float32, device=dev),
        "order": torch.empty(d, dtype=torch.int32, device=dev),
        "B0": torch.empty((d, d), dtype=torch.float64, device=dev),
    }
    if with_measures and d > 1:
        out["measures"] = torch.empty((d - 1, d), dtype=torch.float64, device=dev)
        out["gaps"] = torch.empty(d - 1, dtype=torch.float64, device=dev)
        opts.step_measures = out["measures"].data_ptr()
        opts.step_gap = out["gaps"].data_ptr()
    need = int(lib.varlingam_workspace_size(T, d, int(lags), ctypes.byref(opts)))
    if need == 0:
        raise LingamError(E_INVALID, f"unsupported size T={T} d={d} lags={lags}")
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    code = lib.varlingam_fit(_ptr(X), T, d, X.stride(0), int(lags), _ptr(out["M"]),
                             _ptr(out["resid"]), _ptr(out["order"]), _ptr(out["B0"]),
                             ctypes.byref(opts), _ptr(ws), ws.numel(), _stream_ptr(torch, dev))
    _check(code)
    if lagged_effects:
        out["theta"] = varlingam_lagged_effects(out["M"], out["B0"])
    if prof is not None:
        out["profile"] = _profile_of(prof)
    if stats is not None:
        out["learned_stats"] = _stats_of(stats)
    return out


def batch_causal_order(jobs, *, graph: bool = False, autotune: bool = False,
                       profile: bool = False, workspace=None, with_measures: bool = False,
                       raise_on_error: bool = True, learned: Learned | None = None,
                       record_features: bool = False, waves=None):
    """Causal orders of many jobs in one batched run.

    ``jobs``: sequence of dicts with ``X`` (CUDA float32, rows x d; jobs may
    share one tensor) and optionally ``rows`` (int32 CUDA tensor of row
    indices, bootstrap resampling) or ``n`` (use the first n rows).  Returns a
    dict with ``orders`` (list of int32 tensors), ``status`` (int32 tensor per
    job), ``measures`` / ``features`` (lists, when asked), ``profile`` and
    ``learned_stats``.
    """
    import torch

    lib = load()
    njobs = len(jobs)
    arr = (_Job * njobs)()
    orders, meas, feats, keep = [], [], [], []
    dev = None
    for k, j in enumerate(jobs):
        X = j["X"]
        _cuda_f32_matrix(torch, X)
        dev = X.device
        rows = j.get("rows")
        if rows is not None:
            rows = torch.as_tensor(rows, dtype=torch.int32).to(dev).contiguous()
            keep.append(rows)
            n = rows.numel()
        else:
            n = int(j.get("n", X.shape[0]))
        d = X.shape[1]
        o = torch.empty(d, dtype=torch.int32, device=dev)
        orders.append(o)
        a = arr[k]
        a.X, a.n_rows, a.ldx = X.data_ptr(), X.shape[0], X.stride(0)
        a.rows = rows.data_ptr() if rows is not None else None
        a.n, a.d, a.order = n, d, o.data_ptr()
        m = f = None
        if with_measures and d > 1:
            m = torch.empty((d - 1, d), dtype=torch.float64, device=dev)
            a.step_measures = m.data_ptr()
        if record_features and d > 1:
            f = torch.full((d - 1, d, N_FEATURES), math.nan, dtype=torch.float32, device=dev)
            a.record_features = f.data_ptr()
        meas.append(m)
        feats.append(f)
    opts, prof, stats = _new_opts(lib, graph=graph, autotune=autotune, learned=learned,
                                  waves=waves,
                                  profile=profile, keep=keep)
    need = int(lib.lingam_batch_workspace_size(arr, njobs, ctypes.byref(opts)))
    if need == 0:
        raise LingamError(E_INVALID, last_error() or "invalid batch")
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    status = torch.zeros(njobs, dtype=torch.int32, device=dev)
    code = lib.lingam_batch_causal_order(arr, njobs, _ptr(status), ctypes.byref(opts),
                                         _ptr(workspace), workspace.numel(),
                                         _stream_ptr(torch, dev))
    if raise_on_error:
        _check(code)
    out = {"orders": orders, "status": status, "code": code, "workspace": workspace}
    if with_measures:
        out["measures"] = meas
    if record_features:
        out["features"] = feats
    if prof is not None:
        out["profile"] = _profile_of(prof)
    if stats is not None:
        out["learned_stats"] = _stats_of(stats)
    return out


# ---------------------------------------------------------------------------
# the proposer network
# ---------------------------------------------------------------------------

def _check_features(torch, F):
    if not (isinstance(F, torch.Tensor) and F.is_cuda and F.dtype == torch.float32
            and F.is_contiguous() and F.dim() == 2 and F.shape[1] == N_FEATURES):
        raise TypeError("features must be a contiguous CUDA float32 tensor of shape (rows, 16)")


def _check_proposer(torch, p):
    if not (isinstance(p, torch.Tensor) and p.is_cuda and p.dtype == torch.float32
            and p.is_contiguous() and p.numel() == PROPOSER_SIZE):
        raise TypeError(f"proposer must be a contiguous CUDA float32 tensor of "
                        f"{PROPOSER_SIZE} values")


def proposer_scores(proposer, features):
    """Network scores of feature rows (CUDA float32 (rows, 16)) -> (rows,)."""
    import torch

    lib = load()
    _check_proposer(torch, proposer)
    _check_features(torch, features)
    rows = features.shape[0]
    dev = features.device
    scores = torch.empty(rows, dtype=torch.float32, device=dev)
    ws = torch.empty(int(lib.lingam_proposer_scores_workspace_size()), dtype=torch.uint8,
                     device=dev)
    _check(lib.lingam_proposer_scores(_ptr(proposer), _ptr(features), rows, _ptr(scores),
                                      _ptr(ws), ws.numel(), _stream_ptr(torch, dev)))
    return scores


def proposer_grad(proposer, features, offsets, targets=None, *, weights=None, workspace=None):
    """Listwise softmax cross-entropy and its gradient.

    ``offsets`` (int64, n_lists + 1) delimit the lists of feature rows;
    ``targets`` (int64, n_lists) name each list's target row, or ``weights``
    (float32 per row, >= 0) give each list a soft target distribution (its
    rows' weights over their sum; ``lingam_proposer_grad_soft``).  Returns
    ``(loss, grad, scores, workspace)`` with ``grad`` of N_PARAMS values.
    """
    import torch

    lib = load()
    _check_proposer(torch, proposer)
    _check_features(torch, features)
    if (targets is None) == (weights is None):
        raise ValueError("give exactly one of targets and weights")
    dev = features.device
    rows = features.shape[0]
    off = torch.as_tensor(offsets, dtype=torch.int64).to(dev).contiguous()
    nl = off.numel() - 1
    if targets is not None:
        tg = torch.as_tensor(targets, dtype=torch.int64).to(dev).contiguous()
        if tg.numel() != nl:
            raise ValueError("offsets must have n_lists + 1 entries")
    else:
        wt = torch.as_tensor(weights, dtype=torch.float32).to(dev).contiguous()
        if wt.numel() != rows:
            raise ValueError("weights must have one value per feature row")
    if nl < 1:
        raise LingamError(E_INVALID, "empty training batch")
    need = int(lib.lingam_proposer_grad_workspace_size(rows, nl))
    if need == 0:
        raise LingamError(E_INVALID, "empty training batch")
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    grad = torch.empty(N_PARAMS, dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    scores = torch.empty(rows, dtype=torch.float32, device=dev)
    if targets is not None:
        code = lib.lingam_proposer_grad(_ptr(proposer), _ptr(features), rows, _ptr(off),
                                        _ptr(tg), nl, _ptr(grad), _ptr(loss), _ptr(scores),
                                        _ptr(workspace), workspace.numel(),
                                        _stream_ptr(torch, dev))
    else:
        code = lib.lingam_proposer_grad_soft(_ptr(proposer), _ptr(features), rows, _ptr(off),
                                             _ptr(wt), nl, _ptr(grad), _ptr(loss), _ptr(scores),
                                             _ptr(workspace), workspace.numel(),
                                             _stream_ptr(torch, dev))
    _check(code)
    return loss, grad, scores, workspace


def proposer_adam(proposer, grad, m1, m2, step: int, lr: float = 1e-3, beta1: float = 0.9,
                  beta2: float = 0.999, eps: float = 1e-8):
    """One Adam step on the proposer's trainable values, in place."""
    import torch

    lib = load()
    _check_proposer(torch, proposer)
    _check(lib.lingam_proposer_adam(_ptr(proposer), _ptr(grad), _ptr(m1), _ptr(m2), int(step),
                                    float(lr), float(beta1), float(beta2), float(eps),
                                    _stream_ptr(torch, proposer.device)))
    return proposer
