"""Host checks of the launch plan's index arithmetic, compiled for the CPU.

Every pair-kernel launch is built from two pieces of host/device code in
``csrc/lingam_internal.h``: the order in which the all-pairs kernel walks the
upper triangle of 8 x 8 variable blocks (``decode_tile_st``) and the sample
split of a pair pass (``split_for``); a step's plan (``job_step_base``) sets
the FP64 path, the tile count and the learned pass's candidates.  A mistake
there makes a kernel skip or repeat work, or read out of bounds.
``tests/plan_host_check.cpp`` checks them on the CPU:

* ``decode_tile_st`` maps [0, nb (nb + 1) / 2) one to one onto the blocks
  bi <= bj < nb, super-rows in order, each super-row's diagonal triangle
  before the blocks to its right: every nb up to 300, and around the largest
  supported d (32768 variables: nb = 4096);
* ``split_for`` covers [0, n_pad) with whole 64-sample quanta, the last split
  non-empty, no split shorter than ``min_iters`` quanta, never more splits
  than ``min_iters`` allows, workgroup counts within int32, items x splits
  at most items + CUs x target (the suspect pass's workspace bound), the
  most aggressive policy splitting the most (the policy the workspace is
  sized for), and never more splits for more items (so the host's launch
  bound from one job's items bounds the device's plan from the batch's),
  over item counts up to the
  largest tile count, n_pad up to 2^30 and every policy the autotuner can
  pick;
* ``job_step_base``: the FP64 path for m <= 64, blocks and tiles covering the
  active variables, candidates between min(32, K) and K;
* ``suspect_cap`` / ``ext_count``: suspects a multiple of 8 within the
  layout's room and only while the second pass stays cheaper than the full
  step; extension columns m - K clamped to the cap.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "plan_host_check.cpp")


def test_plan_index_arithmetic(tmp_path):
    from paper_2403_03772_amd import build as b
    hipcc = b.HIPCC if os.path.exists(b.HIPCC) else shutil.which("hipcc")
    if not hipcc:
        pytest.skip("hipcc not found")
    exe = str(tmp_path / "plan_host_check")
    r = subprocess.run([hipcc, "-std=c++17", "-O2", "-I", b.INCLUDE, "-I", b.CSRC, SRC,
                        "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout[-2000:])
    assert r.returncode == 0 and r.stdout.strip().splitlines()[-1].startswith("ok"), r.stdout
