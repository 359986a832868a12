"""Build the gfx950 shared library ``liblingam_mi355x.so`` in-tree with hipcc.

Usage: ``python -m paper_2403_03772_amd.build`` (or call :func:`build`).
Every HIP source is compiled for gfx950 only, with packed-FP32 instruction
selection switched off (``-packed-fp32-ops``).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "liblingam_mi355x.so")
SOURCES = ["lingam_kernels.hip", "lingam_learned.hip", "lingam_linalg.hip", "lingam_noalloc.hip",
           "lingam_abi.cpp"]
# the issue-rate probe that bench.py uses for the pair kernel's roofline; a
# library of its own, not part of the ordering library
PROBE_LIB = os.path.join(HERE, "liblingam_probe.so")
PROBE_SOURCE = "lingam_probe.hip"
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-I", INCLUDE,
]


def _hipcc(cmd, what):
    r = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass warns that it does not know the packed-fp32 feature
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {what}:\n{err}")
    return err


def build_probe(verbose: bool = False) -> str:
    """Compile the issue-rate probe library. Returns its path."""
    tmp = PROBE_LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, *COMMON, "-shared", "-o", tmp, os.path.join(CSRC, PROBE_SOURCE)]
    if verbose:
        print(" ".join(cmd), flush=True)
    _hipcc(cmd, PROBE_SOURCE)
    os.replace(tmp, PROBE_LIB)
    return PROBE_LIB


def build(verbose: bool = False) -> str:
    """Compile every source and link the shared library (and the probe
    library). Returns the library's path."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC, *COMMON, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        err = _hipcc(cmd, src)
        if verbose and err.strip():
            print(err, file=sys.stderr)
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    build_probe(verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
