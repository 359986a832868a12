"""The committed rocprofv3 summaries stay usable, on the CPU:

* every summary under profiles/ gives the full command that made it, and
  every bench.py option in those commands exists (so the command still runs
  against the committed bench.py);
* the k_pair traffic summary was taken on the current kernel sources (its
  recorded sha256 matches), so bench.py reports its HBM bytes rather than
  null.
"""
import glob
import os
import re
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md")))


def _bench_options():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    return set(re.findall(r"--[a-z][a-z0-9-]*", r.stdout))


def _commands(path):
    """bench.py invocations in the fenced blocks of a summary (continuation
    lines joined)."""
    text = open(path).read()
    cmds = []
    for block in re.findall(r"```\n(.*?)```", text, flags=re.S):
        joined = re.sub(r"\\\n\s*", " ", block)
        cmds += [line for line in joined.splitlines() if "bench.py" in line]
    return cmds


def test_profiles_exist():
    assert PROFILES, "no rocprofv3 summaries committed"


@pytest.mark.parametrize("path", PROFILES, ids=os.path.basename)
def test_profile_commands_use_existing_options(path):
    cmds = _commands(path)
    assert cmds, f"{os.path.basename(path)} gives no bench.py command"
    opts = _bench_options()
    for c in cmds:
        assert "rocprofv3" in c, c
        tail = c.split("bench.py", 1)[1]
        for flag in re.findall(r"--[a-z][a-z0-9-]*", tail):
            assert flag in opts, (os.path.basename(path), flag)


def test_traffic_summary_matches_current_kernels():
    t = bench.measured_traffic(1024, 8192)
    assert t is not None, ("profiles/k_pair_d1024_n8192_traffic.md was taken on other kernel "
                           "sources: re-run its two counter passes")
    assert t > 0
