"""Writes tests/golden/gene_d1024_n8192_seed0.json: the oracle's free-running
DirectLiNGAM order (Section 2.2, Algorithm 1, table mode, FP64) of the
gene-expression-scale workload (d = 1024, n = 8192, seed 0), with per-step
measures to check the library against.  It calls only the oracle and the seeded
input generators.  Run from the repo root:

    python tests/golden/make_gene_order.py [--checkpoint PATH] [--chunk STEPS]

The whole ordering is about 2.9e12 sample-pair evaluations (several hours on
eight host cores), so the run advances in chunks of steps; after every chunk
the state goes to the checkpoint file (resumed from if it exists) and the JSON
is rewritten with the steps done so far (``steps_done``).

Per step t the JSON holds (M = -k, by original variable id):
  * ``order[t]``: the oracle's choice (the first maximum of M, ties to the
    smaller id);
  * ``top``: the four largest M with their ids (best first);
  * ``max_abs``: max |M| over the active variables (the tolerance floor is
    1e-3 of it);
  * ``sample``: M of up to twelve active ids drawn by a seeded generator;
  * every measure at the steps in FULL_STEPS.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2403_03772_amd import synth  # noqa: E402

D, N, SEED = 1024, 8192, 0
FULL_STEPS = (0, 1, 2, 100, 300, 600, 1000, 1022)
OUT = os.path.join(HERE, "gene_d1024_n8192_seed0.json")


def summarize(run: "oracle.OrderRun") -> dict:
    done = run.steps_done
    rng = np.random.default_rng(12345)
    steps = []
    for t in range(done):
        M = run.measures[t]
        act = np.flatnonzero(np.isfinite(M))
        # descending M, ties to the smaller id (stable sort on -M)
        srt = act[np.argsort(-M[act], kind="stable")]
        top = srt[:4]
        pick = np.sort(rng.choice(act, size=min(12, act.size), replace=False))
        rec = {
            "t": t,
            "choice": int(run.order[t]),
            "top_ids": [int(v) for v in top],
            "top_M": [float(M[v]) for v in top],
            "max_abs": float(np.max(np.abs(M[act]))),
            "sample_ids": [int(v) for v in pick],
            "sample_M": [float(M[v]) for v in pick],
        }
        if t in FULL_STEPS:
            rec["all_ids"] = [int(v) for v in act]
            rec["all_M"] = [float(M[v]) for v in act]
        steps.append(rec)
    return {
        "source": ("oracle.OrderRun (table mode, FP64) on "
                   "synth.workload_gene_scale(seed=0, d=1024, n=8192) cast to FP32"),
        "d": D, "n": N, "seed": SEED,
        "steps_done": done,
        "finished": bool(run.finished),
        "order": [int(v) for v in run.order[:done]] + (
            [int(run.order[D - 1])] if run.finished else []),
        "steps": steps,
    }


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--checkpoint", default="/tmp/gene_d1024_n8192_seed0_ckpt.npz")
    ap.add_argument("--chunk", type=int, default=8)
    ap.add_argument("--out", default=OUT)
    args = ap.parse_args()
    if os.path.exists(args.checkpoint):
        run = oracle.OrderRun.load(args.checkpoint)
    else:
        X = synth.workload_gene_scale(seed=SEED, d=D, n=N).X.astype(np.float32)
        run = oracle.OrderRun(X, mode="table")
    print(f"threads {oracle.num_threads()}, starting at step {run.steps_done}", flush=True)
    while not run.finished:
        t0 = time.time()
        run.run(args.chunk)
        tmp = args.checkpoint + ".tmp.npz"
        run.save(tmp)
        os.replace(tmp, args.checkpoint)
        with open(args.out + ".tmp", "w") as f:
            json.dump(summarize(run), f, separators=(",", ":"))
        os.replace(args.out + ".tmp", args.out)
        print(f"step {run.steps_done}/{D - 1} ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
