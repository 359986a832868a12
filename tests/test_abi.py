"""Host-side checks of the C ABI that need no GPU.

* the shared library loads and exports every function ``include/lingam.h``
  declares;
* argument errors the host can see are returned synchronously, before any
  device work (so they are testable without a GPU);
* the workspace query rejects unsupported sizes.
"""
import ctypes
import os
import re
import subprocess

import pytest

import paper_2403_03772_amd as pkg
from paper_2403_03772_amd import lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lingam.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:[A-Za-z_][\w\s\*]*?)\b(lingam_\w+|varlingam_\w+)\s*\(", text,
                       flags=re.M)
    return sorted(set(names))


def test_library_is_built():
    assert os.path.exists(pkg.LIB_PATH), "run `python -m paper_2403_03772_amd.build` first"


def test_exports_every_declared_symbol():
    names = _declared_functions()
    assert "lingam_causal_order" in names and "lingam_residualize" in names
    lib = pkg.load()
    for name in names:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", pkg.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing


def test_version_and_last_error():
    assert "gfx950" in pkg.version()
    assert isinstance(pkg.last_error(), str)


def _opts():
    o = L._Opts()
    pkg.load().lingam_opts_init(ctypes.byref(o))
    return o


def test_opts_init_sets_struct_size():
    o = _opts()
    assert o.struct_size == ctypes.sizeof(L._Opts)
    assert o.flags == 0 and o.forced_len == 0


def _call(X=1, n=100, d=5, ldx=5, order=1, opts=None, ws=1, ws_bytes=1 << 30):
    lib = pkg.load()
    return lib.lingam_causal_order(
        ctypes.c_void_p(X) if X else None, n, d, ldx,
        ctypes.c_void_p(order) if order else None,
        ctypes.byref(opts) if opts is not None else None,
        ctypes.c_void_p(ws) if ws else None, ws_bytes, None)


@pytest.mark.parametrize("kw,msg", [
    (dict(X=0), "non-NULL"),
    (dict(order=0), "non-NULL"),
    (dict(n=1), "n >= 2"),
    (dict(n=0), "n >= 2"),
    (dict(d=0), "d >= 1"),
    (dict(ldx=4), "ldx"),
])
def test_host_argument_errors(kw, msg):
    assert _call(**kw) == L.E_INVALID
    assert msg in pkg.last_error()


def test_bad_struct_size_and_forcing():
    o = _opts()
    o.struct_size = 8
    assert _call(opts=o) == L.E_INVALID
    o = _opts()
    o.forced_len = 6
    assert _call(opts=o) == L.E_INVALID
    o = _opts()
    o.forced_len = 2
    assert _call(opts=o) == L.E_INVALID  # forced_order is NULL


def test_unsupported_sizes():
    assert _call(d=1 << 20, ldx=1 << 20) == L.E_UNSUPPORTED
    lib = pkg.load()
    assert lib.lingam_workspace_size(1, 10, None) == 0
    assert lib.lingam_workspace_size(100, 0, None) == 0
    assert lib.lingam_residualize_workspace_size(1, 3) == 0


def test_residualize_argument_errors():
    lib = pkg.load()
    c = lambda **k: lib.lingam_residualize(
        ctypes.c_void_p(1) if k.get("X", 1) else None, k.get("n", 10), k.get("d", 3),
        k.get("ldx", 3), ctypes.c_void_p(1) if k.get("active", 1) else None,
        k.get("n_active", 2), k.get("exo", 0), ctypes.c_void_p(1), 1 << 20, None)
    assert c(X=0) == L.E_INVALID
    assert c(active=0) == L.E_INVALID
    assert c(n=1) == L.E_INVALID
    assert c(ldx=2) == L.E_INVALID
    assert c(n_active=0) == L.E_INVALID
    assert c(n_active=4) == L.E_INVALID
    assert c(exo=3) == L.E_INVALID
    assert c(exo=-1) == L.E_INVALID


def test_adjacency_argument_errors():
    """Host-side checks of lingam_adjacency / varlingam_lagged_effects (no GPU call)."""
    lib = pkg.load()
    v = ctypes.c_void_p(1)
    c = lambda **k: lib.lingam_adjacency(
        v if k.get("X", 1) else None, k.get("n_rows", 10), k.get("ldx", 3),
        v if k.get("rows", 0) else None, k.get("n", 10), k.get("d", 3),
        v if k.get("order", 1) else None, v if k.get("B", 1) else None, v,
        k.get("ws", 1 << 30), None)
    assert c(X=0) == L.E_INVALID
    assert c(order=0) == L.E_INVALID
    assert c(B=0) == L.E_INVALID
    assert c(n=1) == L.E_INVALID
    assert c(d=0) == L.E_INVALID
    assert c(ldx=2) == L.E_INVALID
    assert c(n=11) == L.E_INVALID          # more samples than rows, no row map
    assert c(n_rows=0, rows=1) == L.E_INVALID
    assert c(d=1 << 20, ldx=1 << 20) == L.E_UNSUPPORTED
    assert c(ws=16) == L.E_WORKSPACE
    pr = lambda **k: lib.lingam_adjacency_pruned(
        v, k.get("n_rows", 100), 3, None, k.get("n", 100), k.get("d", 3), v, k.get("ma", 64), v,
        v, k.get("ws", 1 << 30), None)
    assert pr(ma=0) == L.E_INVALID
    assert pr(ma=65) == L.E_INVALID
    assert pr(n=4, n_rows=4) == L.E_DEGENERATE     # n <= d + 1
    assert pr(ws=16) == L.E_WORKSPACE
    assert lib.lingam_adjacency_pruned_workspace_size(1, 3) == 0
    a = lambda **k: lib.lingam_bootstrap_accumulate(
        v if k.get("order", 1) else None, v if k.get("B", 1) else None, k.get("d", 3),
        k.get("thr", 0.0), v if k.get("oc", 1) else None, v if k.get("ec", 1) else None,
        None, None)
    assert a(order=0) == L.E_INVALID
    assert a(B=0) == L.E_INVALID
    assert a(oc=0) == L.E_INVALID
    assert a(ec=0) == L.E_INVALID
    assert a(d=0) == L.E_INVALID
    assert a(thr=-1.0) == L.E_INVALID
    assert a(thr=float("nan")) == L.E_INVALID
    assert a(d=1 << 20) == L.E_UNSUPPORTED
    f = lambda **k: lib.lingam_bootstrap_finalize(
        v if k.get("oc", 1) else None, v if k.get("ec", 1) else None,
        v if k.get("cs", 0) else None, k.get("d", 3), k.get("R", 4),
        v if k.get("op", 1) else None, v if k.get("ep", 1) else None,
        v if k.get("cm", 0) else None, None)
    assert f(oc=0) == L.E_INVALID
    assert f(ec=0) == L.E_INVALID
    assert f(op=0) == L.E_INVALID
    assert f(ep=0) == L.E_INVALID
    assert f(cs=1) == L.E_INVALID       # a coefficient sum needs its output
    assert f(d=0) == L.E_INVALID
    assert f(R=0) == L.E_INVALID
    assert f(d=1 << 20) == L.E_UNSUPPORTED
    assert lib.lingam_adjacency_workspace_size(1, 3) == 0
    assert lib.lingam_adjacency_workspace_size(10, 0) == 0
    # n = 100, d = 8: covariance, factor and inverse columns dominate
    assert lib.lingam_adjacency_workspace_size(100, 8) >= 8 * (9 * 128 + 2 * 64)
    t = lambda **k: lib.lingam_total_effects(
        v if k.get("B", 1) else None, k.get("d", 3), v if k.get("order", 1) else None,
        ctypes.c_void_p(k.get("T", 2)), v, k.get("ws", 1 << 30), None)
    assert t(B=0) == L.E_INVALID
    assert t(order=0) == L.E_INVALID
    assert t(T=0) == L.E_INVALID
    assert t(T=1) == L.E_INVALID       # aliases B
    assert t(d=0) == L.E_INVALID
    assert t(d=1 << 20) == L.E_UNSUPPORTED
    assert t(ws=16) == L.E_WORKSPACE
    assert lib.lingam_total_effects_workspace_size(0) == 0
    assert lib.lingam_total_effects_workspace_size(100) >= 2 * 100 * 100 * 8
    e = lambda **k: lib.varlingam_lagged_effects(
        v if k.get("M", 1) else None, v if k.get("B0", 1) else None, k.get("d", 3),
        k.get("lags", 1), ctypes.c_void_p(k.get("theta", 2)), None)
    assert e(M=0) == L.E_INVALID
    assert e(B0=0) == L.E_INVALID
    assert e(d=0) == L.E_INVALID
    assert e(lags=0) == L.E_INVALID
    assert e(theta=1) == L.E_INVALID  # aliases M
    assert e(d=1 << 20) == L.E_UNSUPPORTED


def test_product_path_has_no_oracle_dependency():
    """The binding and the library never load the oracle."""
    src = open(os.path.join(ROOT, "paper_2403_03772_amd", "lib.py")).read()
    assert "oracle" not in src.replace("# ", "")
    out = subprocess.run(["ldd", pkg.LIB_PATH], capture_output=True, text=True).stdout
    assert "oracle" not in out


def test_batch_argument_errors():
    lib = pkg.load()
    J = (L._Job * 2)()
    for k in range(2):
        J[k].X, J[k].n_rows, J[k].ldx, J[k].n, J[k].d, J[k].order = 1, 100, 5, 100, 5, 1
    assert lib.lingam_batch_workspace_size(J, 0, None) == 0
    J[1].n = 200                      # more samples than rows, no row map
    assert lib.lingam_batch_workspace_size(J, 2, None) == 0
    assert lib.lingam_batch_causal_order(J, 2, None, None, ctypes.c_void_p(1), 1 << 30, None) \
        == L.E_INVALID
    assert "job 1" in pkg.last_error()
    J[1].n = 100
    o = _opts()
    o.forced_len = 1
    o.forced_order = 1
    assert lib.lingam_batch_causal_order(J, 2, None, ctypes.byref(o), ctypes.c_void_p(1),
                                         1 << 30, None) == L.E_INVALID


def test_learned_options_are_validated():
    lib = pkg.load()
    o = _opts()
    assert o.topk == 64 and o.audit_every == 0 and o.learned_min_m == 128
    assert o.max_suspects == 1024 and o.extension == 0
    o.proposer = 1
    assert lib.lingam_workspace_size(1000, 300, ctypes.byref(o)) > \
        lib.lingam_workspace_size(1000, 300, None)
    for field, bad in (("topk", 12), ("topk", 0), ("topk", 264), ("audit_every", -1),
                       ("learned_min_m", 32), ("extension", -8), ("extension", 12),
                       ("extension", 264)):
        o = _opts()
        o.proposer = 1
        setattr(o, field, bad)
        assert lib.lingam_workspace_size(1000, 300, ctypes.byref(o)) == 0, field
        assert _call(opts=o) == L.E_INVALID, field
    o = _opts()
    o.proposer = 1
    o.margin = float("nan")
    assert _call(opts=o) == L.E_INVALID
    # extension columns: single orderings only
    J = (L._Job * 1)()
    J[0].X, J[0].n_rows, J[0].ldx, J[0].n, J[0].d, J[0].order = 1, 1000, 300, 1000, 300, 1
    o = _opts()
    o.proposer = 1
    o.extension = 64
    assert lib.lingam_batch_workspace_size(J, 1, ctypes.byref(o)) == 0
    assert lib.lingam_batch_causal_order(J, 1, None, ctypes.byref(o), ctypes.c_void_p(1),
                                         1 << 30, None) == L.E_UNSUPPORTED
    assert "single orderings" in pkg.last_error()
    o.extension = 0
    assert lib.lingam_batch_workspace_size(J, 1, ctypes.byref(o)) > 0


def test_launch_shape_is_validated():
    """waves_all / waves_rows: 0 (default or autotuned), 1, 2 or 4 waves per
    workgroup; anything else is refused on the host."""
    lib = pkg.load()
    o = _opts()
    assert o.waves_all == 0 and o.waves_rows == 0
    for w in (1, 2, 4):
        o = _opts()
        o.waves_all, o.waves_rows = w, w
        assert lib.lingam_workspace_size(1000, 300, ctypes.byref(o)) == \
            lib.lingam_workspace_size(1000, 300, None)
    for field, bad in (("waves_all", 3), ("waves_all", 8), ("waves_rows", -1), ("waves_rows", 5)):
        o = _opts()
        setattr(o, field, bad)
        assert lib.lingam_workspace_size(1000, 300, ctypes.byref(o)) == 0, field
        assert _call(opts=o) == L.E_INVALID, field
        assert "waves" in pkg.last_error()


def test_proposer_argument_errors():
    lib = pkg.load()
    P = ctypes.c_void_p(1)
    assert lib.lingam_proposer_scores_workspace_size() >= 38016
    assert lib.lingam_proposer_scores(None, P, 10, P, P, 1 << 20, None) == L.E_INVALID
    assert lib.lingam_proposer_scores(P, P, 0, P, P, 1 << 20, None) == L.E_INVALID
    assert lib.lingam_proposer_scores(P, P, 10, P, P, 16, None) == L.E_WORKSPACE
    assert lib.lingam_proposer_grad_workspace_size(0, 1) == 0
    assert lib.lingam_proposer_grad_workspace_size(100, 0) == 0
    assert lib.lingam_proposer_grad_workspace_size(100, 3) > 0
    assert lib.lingam_proposer_grad(P, P, 100, P, P, 0, P, None, None, P, 1 << 30,
                                    None) == L.E_INVALID
    assert lib.lingam_proposer_grad(P, P, 100, None, P, 3, P, None, None, P, 1 << 30,
                                    None) == L.E_INVALID
    assert lib.lingam_proposer_grad(P, P, 100, P, P, 3, P, None, None, P, 8,
                                    None) == L.E_WORKSPACE
    assert lib.lingam_proposer_grad_soft(P, P, 100, P, None, 3, P, None, None, P, 1 << 30,
                                         None) == L.E_INVALID
    assert lib.lingam_proposer_grad(P, P, 100, P, None, 3, P, None, None, P, 1 << 30,
                                    None) == L.E_INVALID
    assert lib.lingam_proposer_grad_soft(P, P, 100, P, P, 3, P, None, None, P, 8,
                                         None) == L.E_WORKSPACE
    assert lib.lingam_proposer_adam(P, P, P, P, 0, 1e-3, 0.9, 0.999, 1e-8, None) == L.E_INVALID
    assert lib.lingam_proposer_adam(P, P, P, P, 1, 1e-3, 1.0, 0.999, 1e-8, None) == L.E_INVALID
    assert lib.lingam_proposer_adam(P, P, None, P, 1, 1e-3, 0.9, 0.999, 1e-8,
                                    None) == L.E_INVALID


def test_struct_layouts_match_header():
    """ctypes mirrors of the ABI structs have the sizes the library expects."""
    o = _opts()
    assert o.struct_size == ctypes.sizeof(L._Opts)
    assert ctypes.sizeof(L._Profile) == 13 * 8
    assert ctypes.sizeof(L._LearnedStats) == 48
    assert ctypes.sizeof(L._Job) == 10 * 8


def test_binding_rejects_host_tensors():
    """The Python functions refuse host tensors before any device call."""
    import torch
    X = torch.zeros((100, 4), dtype=torch.float32)
    B = torch.zeros((4, 4), dtype=torch.float64)
    for call in (lambda: pkg.causal_order(X), lambda: pkg.adjacency(X, [0, 1, 2, 3]),
                 lambda: pkg.adjacency_pruned(X, [0, 1, 2, 3])):
        with pytest.raises(TypeError):
            call()
    with pytest.raises(ValueError):
        pkg.total_effects(B, [0, 1, 2, 3])


def test_header_is_plain_c(tmp_path):
    """include/lingam.h compiles as C99 (pedantic) and a C program links the
    library and calls it (no device call: the options initializer)."""
    import shutil
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "use.c"
    src.write_text('#include "lingam.h"\n'
                   "int main(void) {\n"
                   "  lingam_opts o;\n"
                   "  lingam_opts_init(&o);\n"
                   "  return (o.struct_size == sizeof(lingam_opts) && o.topk == 64) ? 0 : 1;\n"
                   "}\n")
    exe = tmp_path / "use"
    libdir = os.path.dirname(pkg.LIB_PATH)
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
                        "-I", os.path.join(ROOT, "include"), str(src), "-L", libdir,
                        "-llingam_mi355x", f"-Wl,-rpath,{libdir}", "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    assert subprocess.run([str(exe)]).returncode == 0


def test_ctypes_mirrors_match_c_offsets(tmp_path):
    """Every field of the ctypes mirrors sits at the offset the C compiler
    gives the same field of the header's struct, and the sizes agree."""
    import shutil
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no C compiler")
    mirrors = {"lingam_opts": L._Opts, "lingam_profile": L._Profile,
               "lingam_learned_stats": L._LearnedStats, "lingam_job": L._Job}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "lingam.h"',
             "int main(void) {"]
    for cname, mirror in mirrors.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in mirror._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "offsets.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "offsets"
    r = subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src),
                        "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, mirror in mirrors.items():
        assert got[(cname, "size")] == ctypes.sizeof(mirror), cname
        for f, _ in mirror._fields_:
            assert got[(cname, f)] == getattr(mirror, f).offset, (cname, f)


def test_binding_declares_every_signature():
    """The binding gives every declared entry point its argument types and the
    header's result type (64-bit sizes and pointers must not pass through
    ctypes' int default)."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    ret = dict((n, t.replace(" ", "")) for t, n in re.findall(
        r"^(size_t|int|const char\s*\*|void)\s*\b((?:lingam|varlingam)_\w+)\s*\(", text,
        flags=re.M))
    want = {"size_t": ctypes.c_size_t, "int": ctypes.c_int, "constchar*": ctypes.c_char_p,
            "void": None}
    lib = pkg.load()
    names = _declared_functions()
    assert set(ret) == set(names)
    for name in names:
        fn = getattr(lib, name)
        assert fn.argtypes is not None, name
        assert fn.restype is want[ret[name]], (name, ret[name], fn.restype)
