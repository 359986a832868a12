"""Benchmark: DirectLiNGAM causal ordering on one MI355X.

One "step" is one full causal ordering (all d - 1 search steps: pair moments,
entropies and likelihood ratios, per-variable measures, selection,
residualisation) of the gene-expression-scale workload: a synthetic linear
non-Gaussian SEM with d = 1024 variables and n = 8192 samples (ER DAG,
expected in-degree 4, |w| in [0.5, 2], per-variable noise from {uniform,
Laplace, exponential - 1}, unit variance).  The input is resident in HBM
before the timed region.

Metric: sample-pair evaluations per second, where one evaluation is one
residual-entropy term (log cosh and Gaussian-weighted moment) of one ordered
pair at one sample; an ordering does n (d^3 - d) / 3 of them.  Also reported:
the full-ordering time (ms_per_step), the roofline of the pair-moment kernel
(timed with HIP events on the launch stream over the timed region; 12 flops
per evaluation against the published FP32 vector peak, and the kernel's own
issue model from live-measured instruction rates) and the FP64 oracle (table
mode) timed on steps 0-1 of the same workload on the host cores.

Also reported (when the trained network is present): the learned-proposal
form on the same input -- time per ordering, speed-up over the plain form,
Kendall tau to the plain order, its decisions, and the same form with an
untrained network (ablation) --, the learned form against the plain one at
d = 4096, n = 16384 (learned_large), a batched bootstrap workload, the
adjacency, VarLiNGAM and bootstrap-statistics records, and the cost of one
phase boundary of a step (a graph-replayed launch against a grid-wide barrier
in one persistent launch).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload gene|large|batch]
                       [--no-cpu-baseline] [--no-batch] [--no-learned] [--no-large]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Pair-kernel roofline.  The kernel is bound by vector-ALU issue (not by HBM
# and not by the matrix cores).  Its algorithmic cost per evaluation (one
# residual direction of one pair at one sample) is 3 transcendentals (exp,
# log, exp) + 9 FP32 VALU operations = 12 flops; priced against the published
# FP32 vector peak of the MI355X (157.3 TFLOP/s: 256 CUs x 2.4 GHz x 256
# flops/clk/CU, which counts packed FP32 FMAs).
N_CU, CLOCK_HZ = 256, 2.4e9
FLOPS_PER_EVAL = 12
PEAK_FP32_TFLOPS = 157.3
# Secondary figure, the issue model of the kernel's own instruction stream:
# an evaluation issues 7 unpacked FP32 VALU instructions and 2 v_exp_f32 (the
# log of a product is taken once per 32 samples), so it costs
# 7 / R_fma + 2 / R_exp seconds per lane, with R_fma and R_exp the FP32 FMA
# and v_exp_f32 lane-operation rates that the probe library measures live.
VALU_PER_EVAL, TRANS_PER_EVAL = 7, 2


def issue_rates():
    """FP32 FMA lane-ops/s, v_exp_f32 lane-ops/s and evaluation-shaped units/s
    (7 FMA + 2 exp2) measured by liblingam_probe.so on the current device."""
    import ctypes

    from paper_2403_03772_amd import build as b

    if not os.path.exists(b.PROBE_LIB):
        return None
    lib = ctypes.CDLL(b.PROBE_LIB)
    lib.lingam_probe_rates.argtypes = [ctypes.c_void_p]
    lib.lingam_probe_rates.restype = ctypes.c_int
    out = (ctypes.c_double * 3)()
    if lib.lingam_probe_rates(out) != 0:
        return None
    return {"fma_lane_ops_per_s": out[0], "exp_lane_ops_per_s": out[1],
            "eval_mix_per_s": out[2]}


def sync_probe(rounds: int = 2000):
    """Cost of one phase boundary of the ordering step, measured by
    liblingam_probe.so over the step kernels' grid (4 workgroups per CU): a
    launch boundary in a replayed HIP graph, an eager launch boundary, and a
    grid-wide barrier in one cooperative (persistent) launch."""
    import ctypes

    from paper_2403_03772_amd import build as b

    if not os.path.exists(b.PROBE_LIB):
        return None
    lib = ctypes.CDLL(b.PROBE_LIB)
    lib.lingam_probe_sync.argtypes = [ctypes.c_int, ctypes.c_void_p]
    lib.lingam_probe_sync.restype = ctypes.c_int
    out = (ctypes.c_double * 7)()
    code = lib.lingam_probe_sync(rounds, out)
    if code != 0:
        return {"error": code}
    return {"graph_launch_us": out[0], "eager_launch_us": out[1],
            "grid_barrier_us": out[2], "grid_barrier_8_groups_us": out[3],
            "grid_barrier_8_groups_1_per_cu_us": out[4], "workgroups": int(out[5]),
            "barrier_waits_at_poll_limit": int(out[6]), "rounds": rounds}


def pair_roofline(evals_per_s: float, rates) -> dict:
    """roofline record of the pair kernel from its measured evaluation rate."""
    tflops = evals_per_s * FLOPS_PER_EVAL / 1e12
    rec = {"bound": "alu", "achieved": tflops, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
           "frac": tflops / PEAK_FP32_TFLOPS, "evals_per_s": evals_per_s,
           "flops_per_eval": FLOPS_PER_EVAL}
    if rates:
        model = 1.0 / (VALU_PER_EVAL / rates["fma_lane_ops_per_s"]
                       + TRANS_PER_EVAL / rates["exp_lane_ops_per_s"])
        rec["issue_model"] = {
            "evals_per_s": model, "valu_per_eval": VALU_PER_EVAL,
            "trans_per_eval": TRANS_PER_EVAL, "probe": rates,
            "fma_lane_ops_per_clk_per_cu": rates["fma_lane_ops_per_s"] / (N_CU * CLOCK_HZ),
            "exp_lane_ops_per_clk_per_cu": rates["exp_lane_ops_per_s"] / (N_CU * CLOCK_HZ)}
        rec["issue_model_frac"] = evals_per_s / model
        rec["eval_mix_frac"] = evals_per_s / rates["eval_mix_per_s"]
    return rec


def evals_per_ordering(n: int, d: int) -> float:
    return float(n) * (d ** 3 - d) / 3.0


def measured_traffic(d: int, n: int):
    """HBM bytes per k_pair launch from the committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy kernel), or None when the
    summary is for another shape or the kernel sources changed since."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"k_pair_d{d}_n{n}_traffic.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(("|", "#", " ")):
            k, _, v = line.partition(":")
            fields[k.strip()] = v.strip()
    src = os.path.join(ROOT, "paper_2403_03772_amd", "csrc")
    h = hashlib.sha256(b"".join(open(os.path.join(src, f), "rb").read() for f in
                                ("lingam_kernels.hip", "lingam_internal.h",
                                 "lingam_device.h"))).hexdigest()
    if fields.get("kernel_sources_sha256") != h or "traffic_bytes_per_launch" not in fields:
        return None
    return float(fields["traffic_bytes_per_launch"])


def host_cpu() -> dict:
    """The host's logical CPU count, the CPUs this process may use and the CPU
    model name (from /proc/cpuinfo, the field lscpu prints as "Model name")."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)),
            "model": model}


def cpu_baseline(X32, n: int, d: int) -> dict:
    """Time the FP64 oracle in table mode (each ordered residual entropy once
    per step, OpenMP over candidates) on steps 0 and 1 of the workload:
    m (m - 1) n sample-pair evaluations per step, m = d - t."""
    import oracle

    threads = oracle.num_threads()
    run = oracle.OrderRun(X32, mode="table")
    steps = 2
    t0 = time.perf_counter()
    run.run(steps)
    dt = time.perf_counter() - t0
    pairs = sum((d - t) * (d - t - 1) for t in range(steps))
    evals = float(pairs) * n
    cpu = host_cpu()
    return {"value": evals / dt, "unit": "sample-pair evals/s", "cores": threads,
            "kind": "oracle",
            "sample": f"steps 0-{steps - 1} ({pairs} ordered pairs) of the d={d}, n={n} "
                      f"workload, oracle table mode, FP64, {threads} OpenMP threads, "
                      f"{dt:.1f} s",
            "host": cpu}


def bench_batch(steps: int, warmup: int, seed: int, rates=None) -> dict:
    """Batched orderings: 256 bootstrap resamples of one d = 200 base sample
    (n ~ U[500, 5000] rows each, gathered on the device) plus 64 independent
    SEMs with d ~ U[50, 400], n ~ U[500, 5000], all in one graph-captured run."""
    import torch

    import paper_2403_03772_amd as lg
    from paper_2403_03772_amd import synth

    wl = synth.workload_bootstrap_batch(seed=seed)
    base = torch.as_tensor(np.ascontiguousarray(wl.base.X, dtype=np.float32), device="cuda:0")
    jobs = [{"X": base, "rows": torch.as_tensor(r, device="cuda:0")} for r in wl.rows]
    jobs += [{"X": torch.as_tensor(np.ascontiguousarray(s.X, dtype=np.float32),
                                   device="cuda:0")} for s in wl.sems]
    evals = sum(evals_per_ordering(r.size, wl.base.X.shape[1]) for r in wl.rows)
    evals += sum(evals_per_ordering(*s.X.shape) for s in wl.sems)
    # the library's autotuner picks the launch shape on the first call and
    # records it in this file (untimed); later calls reuse it
    import tempfile
    cache = os.path.join(tempfile.gettempdir(), f"lingam_tune_{os.getpid()}.txt")
    os.environ["LINGAM_AUTOTUNE_CACHE"] = cache
    ws = None
    t_tune = time.perf_counter()
    for _ in range(max(warmup, 1)):  # the first call tunes, then captures the graph
        ws = lg.batch_causal_order(jobs, graph=True, autotune=True, workspace=ws)["workspace"]
    torch.cuda.synchronize()
    t_tune = time.perf_counter() - t_tune
    t0 = time.perf_counter()
    for _ in range(steps):
        out = lg.batch_causal_order(jobs, graph=True, autotune=True, workspace=ws)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    assert int(out["status"].abs().sum()) == 0
    # one more, profiled (not graph-captured) call: the pair kernel's share
    # and its evaluation rate against the roofline
    p = lg.batch_causal_order(jobs, autotune=True, workspace=ws, profile=True)["profile"]
    pair = dict(pair_roofline(p.pair_evals / (p.pair_ms * 1e-3), rates), kernel="k_pair",
                share_of_batch=p.pair_ms / p.total_ms) if p.pair_ms else None
    tuned = {}
    if os.path.exists(cache):
        for line in open(cache):
            f = line.split()
            if len(f) == 5:
                tuned[f[0]] = {"target_per_cu": int(f[1]), "min_iters": int(f[2]),
                               "waves_all": int(f[3]), "waves_rows": int(f[4])}
        os.remove(cache)
    return {"workload": "256 bootstrap resamples (d=200, n~U[500,5000]) + 64 SEMs "
                        "(d~U[50,400], n~U[500,5000]), one graph-captured batch",
            "jobs": len(jobs), "evals": evals, "ms": dt * 1e3, "value": evals / dt,
            "unit": "sample-pair evals/s", "workspace_bytes": int(ws.numel()),
            "autotuned_shape": tuned, "warmup_and_tuning_s": t_tune,
            "pair_kernel": pair,
            "issue_model_frac": (evals / dt) / pair["issue_model"]["evals_per_s"]
            if pair and "issue_model" in pair else None}


def bench_bootstrap(seed: int) -> dict:
    """Bootstrap statistics of the d = 200 base sample over its 256 resamples:
    batched orderings (graph-captured) plus one adjacency and one count update
    per resample; one untimed call first."""
    import torch

    import paper_2403_03772_amd as lg
    from paper_2403_03772_amd import synth

    wl = synth.workload_bootstrap_batch(seed=seed)
    base = torch.as_tensor(np.ascontiguousarray(wl.base.X, dtype=np.float32), device="cuda:0")
    res = [torch.as_tensor(r, device="cuda:0") for r in wl.rows]
    lg.bootstrap(base, res, threshold=0.01, graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = lg.bootstrap(base, res, threshold=0.01, graph=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    true_edges = wl.base.B != 0
    ep = out["edge_prob"].cpu().numpy()
    return {"workload": "256 bootstrap resamples of one d=200 sample (n~U[500,5000])",
            "ms": dt * 1e3, "resamples": len(res), "threshold": 0.01,
            "mean_edge_prob_true_edges": float(ep[true_edges].mean()),
            "mean_edge_prob_other": float(ep[~true_edges].mean())}


def kendall_tau(a, b) -> float:
    """Kendall rank correlation of two orders of the same items."""
    from scipy import stats

    pa = np.empty(len(a))
    pb = np.empty(len(b))
    pa[np.asarray(a)] = np.arange(len(a))
    pb[np.asarray(b)] = np.arange(len(b))
    return float(stats.kendalltau(pa, pb)[0])


def reversed_edges(order, B) -> int:
    """Edges of the generating DAG (B[child, parent] != 0) that `order` places
    child first."""
    pos = np.empty(len(order), dtype=np.int64)
    pos[np.asarray(order)] = np.arange(len(order))
    child, parent = np.nonzero(B)
    return int(np.sum(pos[parent] > pos[child]))


def run_learned(lg, X, n, d, steps, warmup, cfg, plain_order, plain_ms, B=None, rates=None,
                profile=True):
    """The learned-proposal form on the same input: time per ordering, speed-up
    over the plain form, Kendall tau to the plain order, decisions, the work
    actually performed and the candidate-row kernels against the roofline."""
    import torch

    ws = torch.empty(lg.workspace_size(n, d, cfg), dtype=torch.uint8, device="cuda:0")
    for _ in range(warmup):
        lg.causal_order(X, learned=cfg, workspace=ws)
    torch.cuda.synchronize()
    # timed without the library's per-kernel events (they add ~2-8%); one
    # more, profiled, ordering gives the kernel figures
    t0 = time.perf_counter()
    for i in range(steps):
        out = lg.causal_order(X, learned=cfg, workspace=ws)
        progress(f"learned ordering {i + 1}/{steps}")
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    order = out["order"].cpu().numpy()
    st = out["learned_stats"]
    rec = {}
    if profile:
        p = lg.causal_order(X, learned=cfg, workspace=ws, profile=True)["profile"]
        cand_ms, cand_evals, pair_ms, pair_evals = p.cand_ms, p.cand_evals, p.pair_ms, p.pair_evals
        small = sum(m * (m - 1) * float(n) for m in range(2, min(64, d) + 1))
        done = cand_evals + pair_evals + small
        rec = {
            "evals_done": done,
            "evals_done_per_s": done / dt,
            "cand_kernel": dict(pair_roofline(cand_evals / (cand_ms * 1e-3), rates),
                                kernel="k_pair_cand + k_pair_ext + k_pair_susp",
                                ms_per_ordering=cand_ms) if cand_ms else None,
            "full_pair_ms_per_ordering": pair_ms,
        }
    return {
        "ms_per_ordering": dt * 1e3,
        "speedup_vs_plain": plain_ms / (dt * 1e3),
        "kendall_tau": kendall_tau(order, plain_order),
        "orders_identical": bool(np.array_equal(order, plain_order)),
        "reversed_edges": reversed_edges(order, B) if B is not None else None,
        "topk": cfg.topk, "audit_every": cfg.audit_every,
        "margin": cfg.margin if np.isfinite(cfg.margin) else str(cfg.margin),
        "max_suspects": cfg.max_suspects,
        "extension": cfg.extension,
        "stats": {"learned_steps": st.learned_steps, "certified": st.certified,
                  "expanded": st.expanded, "fallbacks": st.fallbacks, "audits": st.audits,
                  "audit_agree": st.audit_agree,
                  "suspects_mean": st.suspects_sum / max(st.learned_steps, 1),
                  "cleared": st.cleared,
                  "rows_mean": st.rows_sum / max(st.learned_steps, 1)},
        **rec,
    }


def run_large(lg, tp, seed: int, rates) -> dict:
    """The learned form's target workload, d = 4096, n = 16384 (the gene family):
    one plain ordering, then the exact learned ordering, and the exact form
    with a full-step audit every 32 steps (top-K = 64): time, speed-up over the
    plain ordering and Kendall tau to the plain order."""
    import torch
    from paper_2403_03772_amd import synth

    d, n = 4096, 16384
    progress(f"large workload: generating d={d}, n={n}")
    sem = synth.workload_gene_scale(seed=seed, d=d, n=n)
    X = torch.as_tensor(np.ascontiguousarray(sem.X, dtype=np.float32), device="cuda:0")
    B = sem.B
    del sem
    ws = torch.empty(lg.workspace_size(n, d), dtype=torch.uint8, device="cuda:0")
    progress("large workload: plain ordering (about two minutes)")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = lg.causal_order(X, workspace=ws, profile=True)
    torch.cuda.synchronize()
    plain_ms = (time.perf_counter() - t0) * 1e3
    plain_order = out["order"].cpu().numpy()
    prof = out["profile"]
    del ws
    progress(f"large workload: plain {plain_ms / 1e3:.1f} s")
    prop = tp.default_proposer()
    rec = {"workload": "gene-expression-scale SEM", "d": d, "n": n, "seed": seed,
           "plain_ms": plain_ms, "plain_evals_per_s": evals_per_ordering(n, d) / (plain_ms * 1e-3),
           "plain_reversed_edges": reversed_edges(plain_order, B),
           "plain_fp64_ties": {"steps": prof.tie_steps, "rows": prof.tie_rows,
                               "overflow_steps": prof.tie_overflow}}
    for name, cfg in (("exact", lg.Learned(prop, topk=64)),
                      ("audited_every_32", lg.Learned(prop, topk=64, audit_every=32))):
        progress(f"large workload: learned ({name})")
        rec[name] = run_learned(lg, X, n, d, 1, 0, cfg, plain_order, plain_ms, B, rates,
                                profile=False)
        progress(f"large workload: learned ({name}) {rec[name]['ms_per_ordering'] / 1e3:.1f} s, "
                 f"{rec[name]['speedup_vs_plain']:.2f}x, tau {rec[name]['kendall_tau']:.4f}")
    return rec


def progress(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_adjacency(lg, X, n, d, order, reps=5):
    """lingam_adjacency on the ordering's input along its order: mean ms per call
    (the call synchronizes) and FP64 rate against the algorithmic flops:
    covariance n d (d + 1) (upper triangle, one multiply-add per sample), the
    Cholesky d^3 / 3 and the inverse-factor recurrence d^3 / 3."""
    import torch

    ws = torch.empty(int(lg.load().lingam_adjacency_workspace_size(n, d)), dtype=torch.uint8,
                     device=X.device)
    lg.adjacency(X, order, workspace=ws)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        lg.adjacency(X, order, workspace=ws)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    flops = float(n) * d * (d + 1) + 2.0 * d ** 3 / 3.0
    return {"ms": ms, "bound": "mfma", "achieved": flops / (ms * 1e-3) / 1e12, "peak": 78.6,
            "unit": "TFLOP/s (fp64)", "frac": flops / (ms * 1e-3) / 78.6e12,
            "flops": flops, "reps": reps}


def run_total_effects(lg, X, order, reps=10):
    """lingam_total_effects on the adjacency along the plain order: mean ms per
    call (the call synchronizes once, for its order check) and the FP64 rate
    of the blocked triangular inverse against its algorithmic d^3 / 3 flops."""
    import torch

    B = lg.adjacency(X, order)
    d = B.shape[0]
    ws = torch.empty(int(lg.load().lingam_total_effects_workspace_size(d)), dtype=torch.uint8,
                     device=X.device)
    lg.total_effects(B, order, workspace=ws)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        lg.total_effects(B, order, workspace=ws)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    flops = d ** 3 / 3.0
    return {"ms": ms, "bound": "mfma", "achieved": flops / (ms * 1e-3) / 1e12, "peak": 78.6,
            "unit": "TFLOP/s (fp64)", "frac": flops / (ms * 1e-3) / 78.6e12, "flops": flops,
            "reps": reps}


def run_adjacency_pruned(lg, X, order, B_true, reps=3):
    """lingam_adjacency_pruned along the plain order: mean ms per call and the
    edges it keeps against the generating DAG (precision, recall)."""
    import torch

    lg.adjacency_pruned(X, order)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        B = lg.adjacency_pruned(X, order)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    kept = B.cpu().numpy() != 0
    true = np.asarray(B_true) != 0
    tp = int(np.sum(kept & true))
    return {"ms": ms, "reps": reps, "edges_kept": int(kept.sum()), "edges_true": int(true.sum()),
            "precision": tp / max(int(kept.sum()), 1), "recall": tp / max(int(true.sum()), 1)}


def run_varlingam(lg, reps=3):
    """varlingam_fit on the stock-shaped series (d = 487, T = 1258, VAR(1)):
    mean ms per fit, lagged effects included."""
    import torch
    from paper_2403_03772_amd import synth

    v = synth.var_series(d=487, T=1258, seed=0)
    X = torch.as_tensor(np.ascontiguousarray(v.X, dtype=np.float32), device="cuda:0")
    lg.varlingam_fit(X, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        lg.varlingam_fit(X, 1)
    torch.cuda.synchronize()
    return {"ms": (time.perf_counter() - t0) * 1e3 / reps, "d": 487, "T": 1258, "lags": 1,
            "reps": reps}


def run_plain(lg, X, n, d, steps, warmup):
    import torch

    ws = torch.empty(lg.workspace_size(n, d), dtype=torch.uint8, device="cuda:0")
    torch.cuda.synchronize()
    for _ in range(warmup):
        lg.causal_order(X, workspace=ws)
    torch.cuda.synchronize()
    acc = dict(pair_ms=0.0, pair_evals=0.0, pair_launches=0, gram_ms=0.0, gram_flops=0.0,
               resid_ms=0.0, resid_bytes=0.0, tie_steps=0, tie_rows=0, tie_overflow=0)
    orders = []
    t0 = time.perf_counter()
    for i in range(steps):
        out = lg.causal_order(X, workspace=ws, profile=True)
        p = out["profile"]
        for k in acc:
            acc[k] += getattr(p, k)
        orders.append(out["order"])
        progress(f"plain ordering {i + 1}/{steps}: {p.total_ms:.0f} ms")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    o0 = orders[0].cpu().numpy()
    for o in orders[1:]:
        assert np.array_equal(o.cpu().numpy(), o0), "orderings differ between steps"
    acc["dt"] = dt
    acc["order"] = o0
    return acc


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=("gene", "large", "batch"), default="gene",
                    help="gene: d=1024, n=8192 (default); large: d=4096, n=16384 "
                         "(learned vs plain at scale; one plain ordering takes ~2 min); "
                         "batch: the bootstrap batch alone")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched bootstrap workload")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-proposal form")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the learned-vs-plain record at d=4096, n=16384 (about "
                         "three minutes)")
    ap.add_argument("--learned-only", action="store_true",
                    help="with --workload large: only the exact learned ordering (one, "
                         "untimed warm-up none; for kernel profiles of the learned form)")
    ap.add_argument("--exact-only", action="store_true",
                    help="of the learned forms, run only the exact one (for its profile)")
    ap.add_argument("--no-aux", action="store_true",
                    help="skip the adjacency, VarLiNGAM, bootstrap and phase-boundary "
                         "records (their kernels would mix into a profile of the plain "
                         "ordering)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the run, copy 1 GiB device-to-device with a plain copy "
                         "kernel (reference for the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the ordering is single-GPU here); "
              f"got --gpus {args.gpus}", file=sys.stderr)
        return 2

    import torch

    import paper_2403_03772_amd as lg
    from paper_2403_03772_amd import synth
    from paper_2403_03772_amd import train_proposer as tp

    if args.workload == "batch":
        b = bench_batch(max(1, args.steps), args.warmup, args.seed, issue_rates())
        rec = {"metric": "sample-pair evals/s (batched bootstrap orderings)",
               "value": b["value"], "unit": b["unit"], "n_gpus": 1, "steps": args.steps,
               "warmup": args.warmup, "ms_per_step": b["ms"], "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
               "config": {"workload": b["workload"], "jobs": b["jobs"]}, "batch": b}
        print(json.dumps(rec), flush=True)
        return 0

    if args.workload == "large" and args.learned_only:
        d, n = 4096, 16384
        sem = synth.workload_gene_scale(seed=args.seed, d=d, n=n)
        X = torch.as_tensor(np.ascontiguousarray(sem.X, dtype=np.float32), device="cuda:0")
        cfg = lg.Learned(tp.default_proposer(), topk=64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = lg.causal_order(X, learned=cfg)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = out["learned_stats"]
        print(json.dumps({"workload": "learned exact ordering only", "d": d, "n": n,
                          "ms": dt * 1e3, "learned_steps": st.learned_steps,
                          "certified": st.certified, "expanded": st.expanded,
                          "suspects_mean": st.suspects_sum / max(st.learned_steps, 1),
                          "rows_mean": st.rows_sum / max(st.learned_steps, 1),
                          "reversed_edges": reversed_edges(out["order"].cpu().numpy(), sem.B)}),
              flush=True)
        return 0
    d, n = (1024, 8192) if args.workload == "gene" else (4096, 16384)
    if args.workload == "large" and args.steps == 3 and args.warmup == 1:
        args.steps, args.warmup = 1, 0  # one plain ordering takes about two minutes
    sem = synth.workload_gene_scale(seed=args.seed, d=d, n=n)
    X32 = np.ascontiguousarray(sem.X, dtype=np.float32)
    X = torch.as_tensor(X32, device="cuda:0")

    pl = run_plain(lg, X, n, d, args.steps, args.warmup)
    dt = pl["dt"]
    ms_per_step = dt * 1e3 / args.steps
    evals = evals_per_ordering(n, d)
    value = evals * args.steps / dt
    achieved = pl["pair_evals"] / (pl["pair_ms"] * 1e-3)
    progress("issue-rate probe")
    rates = issue_rates()
    launches = max(pl["pair_launches"], 1)
    # algorithmic bytes of one k_pair launch: one pass over the active FP32
    # rows (4 n bytes per variable), mean over the launches of an ordering
    # (steps with m > 64 active variables; smaller steps run the FP64 path)
    alg_bytes = 4.0 * n * np.mean(np.arange(65, d + 1)) if d > 64 else 0.0
    traffic = measured_traffic(d, n)
    rec = {
        "metric": f"sample-pair evals/s (plain DirectLiNGAM ordering, d={d}, n={n})",
        "reversed_edges": reversed_edges(pl["order"], sem.B),
        "value": value,
        "unit": "sample-pair evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "full_ordering_ms": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "gene-expression-scale linear non-Gaussian SEM, plain ordering",
                   "d": d, "n": n, "seed": args.seed, "indeg": 4, "form": "plain"},
        "roofline": dict(
            pair_roofline(achieved, rates),
            kernel="k_pair",
            traffic=traffic,
            traffic_unit="HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled)",
            algorithmic_bytes=alg_bytes,
            traffic_over_algorithmic=traffic / alg_bytes if traffic and alg_bytes else None,
            avg_launch_ms=pl["pair_ms"] / launches,
            launches=pl["pair_launches"],
            share_of_step=pl["pair_ms"] / (dt * 1e3),
        ),
        "gram": {"bound": "mfma", "ms": pl["gram_ms"] / args.steps,
                 "achieved": pl["gram_flops"] / (pl["gram_ms"] * 1e-3) / 1e12
                 if pl["gram_ms"] else None,
                 "peak": 78.6, "unit": "TFLOP/s (fp64)"},
        # residual update: algorithmic 8 B per sample and remaining variable
        # (read and write the FP32 residual); the kernel moves 28 B (FP64
        # master copy read and written, FP32 copy written)
        "resid": {"bound": "hbm", "ms": pl["resid_ms"] / args.steps,
                  "achieved": pl["resid_bytes"] * 8.0 / 28.0 / (pl["resid_ms"] * 1e-3) / 1e9
                  if pl["resid_ms"] else None,
                  "peak": 8000.0, "unit": "GB/s",
                  "moved_gb_per_s": pl["resid_bytes"] / (pl["resid_ms"] * 1e-3) / 1e9
                  if pl["resid_ms"] else None},
        # near-ties decided in FP64 (per ordering)
        "fp64_ties": {"steps": pl["tie_steps"] // args.steps,
                      "rows": pl["tie_rows"] // args.steps,
                      "overflow_steps": pl["tie_overflow"] // args.steps},
        "learned": None,
    }
    if not args.no_learned and not os.path.exists(tp.WEIGHTS):
        rec["learned"] = {"error": f"no trained proposer at {tp.WEIGHTS}"}
    elif not args.no_learned:
        prop = tp.default_proposer()
        _, meta = tp.load_weights()
        lw = max(1, args.warmup)
        K = 64
        B = sem.B
        # exact form (the default): certified, suspects evaluated, or a full step
        exact = lg.Learned(prop, topk=K)
        progress("learned (exact)")
        rec["learned"] = run_learned(lg, X, n, d, args.steps, lw, exact, pl["order"],
                                     ms_per_step, B, rates)
        rec["learned"]["proposer"] = {k: meta.get(k) for k in
                                      ("sems", "d", "n", "big_sems", "big_d", "target",
                                       "lists", "holdout", "holdout_big")}
        if "stage2" in meta:  # streamed fine-tuning on further SEMs
            rec["learned"]["proposer"]["stage2"] = {
                k: meta["stage2"].get(k) for k in ("sems", "d", "n", "updates", "holdout",
                                                   "holdout_big")}
        # fast form: no second pass, the best candidate is always taken
        fast = lg.Learned(prop, topk=K, margin=-np.inf, max_suspects=0, audit_every=32)
        if not args.exact_only:
            progress("learned (fast)")
            rec["learned"]["fast"] = run_learned(lg, X, n, d, args.steps, lw, fast,
                                                 pl["order"], ms_per_step, B, rates)
        if args.workload == "large" and not args.exact_only:
            # the exact form with a full-step audit every 32 steps (the audits
            # only repeat exact decisions; this records what they cost)
            progress("learned (exact, audited)")
            rec["learned"]["audited"] = run_learned(
                lg, X, n, d, args.steps, lw, lg.Learned(prop, topk=K, audit_every=32),
                pl["order"], ms_per_step, B, rates)
        if args.workload == "gene" and not args.exact_only:
            # ablation: the exact form with an untrained (random) network (not on
            # the large workload, where it runs about as long as the plain form)
            raw = prop.clone()
            raw[32:] = torch.as_tensor(tp.init_weights(1), device=raw.device)
            progress("learned (untrained)")
            rec["learned"]["untrained"] = run_learned(lg, X, n, d, 1, 0,
                                                      lg.Learned(raw, topk=K), pl["order"],
                                                      ms_per_step, B, rates)
    if args.workload == "gene" and not args.no_aux:
        progress("adjacency along the plain order")
        rec["adjacency"] = run_adjacency(lg, X, n, d, torch.as_tensor(pl["order"]).cuda())
        progress("total effects along the plain order")
        rec["total_effects"] = run_total_effects(lg, X, torch.as_tensor(pl["order"]).cuda())
        progress("adaptive-lasso pruning along the plain order")
        rec["adjacency_pruned"] = run_adjacency_pruned(lg, X, torch.as_tensor(pl["order"]).cuda(),
                                                       sem.B)
        progress("varlingam (stock shape)")
        rec["varlingam"] = run_varlingam(lg)
        progress("phase-boundary probe (launch vs grid barrier)")
        rec["phase_boundary"] = sync_probe()
    if not args.no_batch and args.workload == "gene":
        rec["batch"] = bench_batch(max(1, args.steps), args.warmup, args.seed, rates)
        if not args.no_aux:
            progress("bootstrap statistics")
            rec["bootstrap"] = bench_bootstrap(args.seed)
    if (args.workload == "gene" and not args.no_learned and not args.no_large
            and os.path.exists(tp.WEIGHTS)):
        rec["learned_large"] = run_large(lg, tp, args.seed, rates)
    if args.copy_calibration:
        src = torch.ones(256 << 20, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        rec["copy_calibration_bytes"] = src.numel() * 4
    if not args.no_cpu_baseline and args.workload == "gene":
        rec["cpu_baseline"] = cpu_baseline(X32, n, d)
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
