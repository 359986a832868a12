"""ctypes binding of ``liblingam_mi355x.so``.

Only argument marshalling lives here.  Tensors must already be on the GPU;
the binding hands the library their device pointers and the current HIP
stream of PyTorch, allocates the workspace the library asks for, and turns
non-OK status codes into :class:`LingamError`.
"""
from __future__ import annotations

import ctypes
import os
import threading
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblingam_mi355x.so")

OK, E_INVALID, E_DEGENERATE, E_HIP, E_WORKSPACE, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
FLAG_NO_SYNC = 1

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
        lib.lingam_opts_init.argtypes = [ctypes.POINTER(_Opts)]
        lib.lingam_opts_init.restype = None
        lib.lingam_workspace_size.argtypes = [i64, i64, ctypes.POINTER(_Opts)]
        lib.lingam_workspace_size.restype = sz
        lib.lingam_causal_order.argtypes = [P, i64, i64, i64, P, ctypes.POINTER(_Opts), P, sz, P]
        lib.lingam_causal_order.restype = ctypes.c_int
        lib.lingam_residualize_workspace_size.argtypes = [i64, i64]
        lib.lingam_residualize_workspace_size.restype = sz
        lib.lingam_residualize.argtypes = [P, i64, i64, i64, P, i32, i32, P, sz, P]
        lib.lingam_residualize.restype = ctypes.c_int
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


def workspace_size(n: int, d: int) -> int:
    return int(load().lingam_workspace_size(int(n), int(d), None))


def residualize_workspace_size(n: int, d: int) -> int:
    return int(load().lingam_residualize_workspace_size(int(n), int(d)))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def causal_order(X, *, forced=None, with_measures: bool = False, profile: bool = False,
                 workspace=None, sync: bool = True):
    """DirectLiNGAM causal order of the columns of ``X`` (a CUDA float32 tensor, n x d).

    Returns ``order`` (int32 CUDA tensor, original column ids, exogenous first),
    or a dict with ``order``, ``measures`` ((d-1) x d FP64, NaN for columns
    already ordered), ``gaps`` and ``profile`` when ``with_measures`` or
    ``profile`` is set.  ``forced`` (sequence or tensor of column ids) fixes the
    first ``len(forced)`` choices (teacher forcing).
    """
    import torch

    lib = load()
    if not (isinstance(X, torch.Tensor) and X.is_cuda and X.dtype == torch.float32):
        raise TypeError("X must be a CUDA float32 tensor")
    if X.dim() != 2 or X.stride(1) != 1:
        raise ValueError("X must be 2-D with unit column stride")
    n, d = X.shape
    ldx = X.stride(0) if n > 1 else d
    dev = X.device
    order = torch.empty(d, dtype=torch.int32, device=dev)
    opts = _Opts()
    lib.lingam_opts_init(ctypes.byref(opts))
    if not sync:
        opts.flags |= FLAG_NO_SYNC
    keep = []
    if forced is not None:
        f = torch.as_tensor(forced, dtype=torch.int32).to(dev).contiguous()
        keep.append(f)
        opts.forced_order = f.data_ptr()
        opts.forced_len = f.numel()
    meas = gaps = None
    if with_measures and d > 1:
        meas = torch.empty((d - 1, d), dtype=torch.float64, device=dev)
        gaps = torch.empty(d - 1, dtype=torch.float64, device=dev)
        opts.step_measures = meas.data_ptr()
        opts.step_gap = gaps.data_ptr()
    prof = _Profile() if profile else None
    if prof is not None:
        opts.profile = ctypes.pointer(prof)
    need = int(lib.lingam_workspace_size(n, d, ctypes.byref(opts)))
    if need == 0:
        raise LingamError(E_UNSUPPORTED, f"unsupported size n={n} d={d}")
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    code = lib.lingam_causal_order(_ptr(X), n, d, ldx, _ptr(order), ctypes.byref(opts),
                                   _ptr(workspace), workspace.numel(), _stream_ptr(torch, dev))
    _check(code)
    if not (with_measures or profile):
        return order
    out = {"order": order, "measures": meas, "gaps": gaps}
    if prof is not None:
        out["profile"] = Profile(**{k: getattr(prof, k) for k, _ in _Profile._fields_})
    return out


def residualize(X, active, exo: int):
    """In place: regress column ``exo`` out of every other ``active`` column of X."""
    import torch

    lib = load()
    if not (isinstance(X, torch.Tensor) and X.is_cuda and X.dtype == torch.float32):
        raise TypeError("X must be a CUDA float32 tensor")
    if X.dim() != 2 or X.stride(1) != 1:
        raise ValueError("X must be 2-D with unit column stride")
    n, d = X.shape
    a = torch.as_tensor(active, dtype=torch.int32).to(X.device).contiguous()
    need = int(lib.lingam_residualize_workspace_size(n, d))
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=X.device)
    code = lib.lingam_residualize(_ptr(X), n, d, X.stride(0), _ptr(a), a.numel(), int(exo),
                                  _ptr(ws), ws.numel(), _stream_ptr(torch, X.device))
    _check(code)
    return X
