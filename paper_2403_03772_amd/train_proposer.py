"""Training of the proposer network of the learned-proposal form.

The network learns to rank the active variables of a step by the plain
search's measure k (small k first), from orderings the plain search produces
on synthetic linear non-Gaussian SEMs.  Its inputs are the 16 features the
library records at every step (``record_features``).  The loss is the
listwise softmax cross-entropy of each step's scores against a soft target
q_i proportional to (2 k_min / (k_i + k_min))^2 (k from the plain run's
per-step measures): every variable whose k is near the step's minimum gets
a large share, because the learned form is exact only when all of them are
among its candidates (``--target choice`` trains on the plain choice alone).
The optimiser is Adam.  All arithmetic runs in the library's kernels (the plain search,
``lingam_proposer_grad`` and ``lingam_proposer_adam``); this module only
draws the SEMs, samples the steps and drives the loop.

Usage (writes the weights the package ships):

    python -m paper_2403_03772_amd.train_proposer --sems 1000 --out weights.npz
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import lib as L
from . import synth

N_FEAT = L.N_FEATURES

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "proposer_weights.npz")


def _gen(spec):
    d, n, seed = spec
    s = synth.er_sem(d, n, indeg=4.0, wlo=0.5, whi=2.0,
                     noise_family=("uniform", "laplace", "exp"), seed=seed)
    return s.X.astype(np.float32)


def soft_weights(k) -> np.ndarray:
    """Soft target weights of one list from its variables' k values."""
    k = np.asarray(k, dtype=np.float64)
    k = np.where(np.isfinite(k) & (k >= 0.0), k, np.inf)  # no weight for a bad value
    kmin = max(float(np.min(k)), 1e-30)
    return ((2.0 * kmin) / (k + kmin)) ** 2


def sem_specs(n_sems: int, d_lo: int, d_hi: int, n_lo: int, n_hi: int, seed: int):
    """(d, n, seed) of ``n_sems`` SEMs: d ~ U[d_lo, d_hi], n log-uniform in
    [n_lo, n_hi] and at least 2 d."""
    rng = np.random.default_rng(seed)
    specs = []
    for _ in range(n_sems):
        d = int(rng.integers(d_lo, d_hi + 1))
        n = int(round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))))
        specs.append((d, max(n, 2 * d), int(rng.integers(1 << 31))))  # n >= 2 d
    return specs


def label_batches(specs, steps_per_sem: int = 32, m_floor: int = 64, batch: int = 16,
                  workers: int = 8, log=print):
    """Training lists from plain GPU orderings of the SEMs ``specs`` (a draw
    the plain search finds degenerate is skipped), one batched ordering of
    ``batch`` SEMs at a time.  At up to ``steps_per_sem`` steps with at least
    ``m_floor`` active variables (drawn from the SEM's own seed), a list holds
    the features of the active variables; its target is the plain choice, and
    its variables' k values give the soft target weights.  SEMs are drawn by
    a pool of ``workers`` processes ahead of the GPU.  Yields, per batch,
    the number of SEMs it took and its lists (features float32 [rows, 16],
    offsets int64, targets int64, weights float32 [rows]; empty when every
    SEM of the batch was skipped)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    import torch

    n_sems = len(specs)
    pool = ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn"))
    futs = [pool.submit(_gen, sp) for sp in specs[:2 * batch]]
    nxt = len(futs)
    done = 0
    try:
        while done < n_sems:
            cnt = min(batch, n_sems - done)
            Xs = [futs[done + k].result() for k in range(cnt)]
            for _ in range(cnt):
                if nxt < n_sems:
                    futs.append(pool.submit(_gen, specs[nxt]))
                    nxt += 1
            jobs = [{"X": torch.as_tensor(X, device="cuda")} for X in Xs]
            out = L.batch_causal_order(jobs, record_features=True, with_measures=True,
                                       raise_on_error=False)
            status = out["status"].cpu().numpy()
            feats, offs, tgs, wts = [], [0], [], []
            for k, X in enumerate(Xs):
                d = X.shape[1]
                futs[done + k] = None
                if status[k] != 0:  # a degenerate draw (collinear residuals): skip it
                    log(f"label: SEM {done + k} skipped (status {int(status[k])})")
                    continue
                order = out["orders"][k].cpu().numpy()
                R = out["features"][k]
                Mk = out["measures"][k]
                last = d - m_floor  # steps t <= last have m >= m_floor
                if last < 0:
                    continue
                rng = np.random.default_rng(specs[done + k][2])
                ts = np.sort(rng.choice(last + 1, size=min(steps_per_sem, last + 1),
                                        replace=False))
                Rt = R[torch.as_tensor(ts, device=R.device)].cpu().numpy()
                Mt = Mk[torch.as_tensor(ts, device=Mk.device)].cpu().numpy()
                for i, t in enumerate(ts):
                    act = np.flatnonzero(~np.isnan(Rt[i, :, 0]))
                    w = soft_weights(-Mt[i, act])
                    if not np.isfinite(w).all() or not w.sum() > 0.0:
                        continue
                    feats.append(Rt[i, act])
                    wts.append(w.astype(np.float32))
                    tgs.append(offs[-1] + int(np.flatnonzero(act == order[t])[0]))
                    offs.append(offs[-1] + act.size)
            done += cnt
            del out, jobs
            F = (np.concatenate(feats) if feats else np.zeros((0, N_FEAT))).astype(np.float32)
            W = (np.concatenate(wts) if wts else np.zeros(0)).astype(np.float32)
            yield cnt, (F, np.asarray(offs, np.int64), np.asarray(tgs, np.int64), W)
    finally:
        pool.shutdown(cancel_futures=True)


def collect(n_sems: int, d_lo: int = 100, d_hi: int = 1000, n_lo: int = 2048,
            n_hi: int = 16384, steps_per_sem: int = 32, m_floor: int = 64, seed: int = 0,
            batch: int = 16, workers: int = 8, log=print):
    """Training lists of ``n_sems`` SEMs (``sem_specs``, ``label_batches``),
    all held at once.  Returns (features float32 [rows, 16], offsets int64,
    targets int64, weights float32 [rows])."""
    t0 = time.time()
    sets, lists = [], 0
    specs = sem_specs(n_sems, d_lo, d_hi, n_lo, n_hi, seed)
    for _, part in label_batches(specs, steps_per_sem, m_floor, batch, workers, log):
        sets.append(part)
        lists += len(part[2])
        log(f"collect: {lists} lists, {time.time() - t0:.0f} s")
    return _concat(sets)


def _lists(F, offs, tgs, W):
    """A list set as per-list tuples (features, target row, weights)."""
    return [(F[offs[i]:offs[i + 1]], int(tgs[i] - offs[i]), W[offs[i]:offs[i + 1]])
            for i in range(len(tgs))]


def _stack(items):
    """Per-list tuples -> one list set."""
    sizes = np.array([f.shape[0] for f, _, _ in items], dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return (np.concatenate([f for f, _, _ in items]), offs,
            offs[:-1] + np.array([t for _, t, _ in items], dtype=np.int64),
            np.concatenate([w for _, _, w in items]))


def stream_train(prop, specs, state: dict, *, lr: float, lr_end: float, total_updates: int,
                 updates_per_batch: int = 4, replay_lists: int = 4096,
                 lists_per_batch: int = 256, batch: int = 16, steps_per_sem: int = 32,
                 workers: int = 8, time_budget: float = float("inf"), log=print):
    """Train ``prop`` while its data is labeled: after each batched plain
    ordering of ``batch`` SEMs, ``updates_per_batch`` Adam steps on the soft
    listwise cross-entropy, each on ``lists_per_batch`` lists drawn from a
    buffer of the newest ``replay_lists`` lists (the full set of 10^4 SEMs
    would not fit in memory).  The learning rate falls from ``lr`` to
    ``lr_end`` on a cosine over ``total_updates``.  ``state`` (Adam moments,
    step, next SEM index into ``specs``, losses) is updated in place so that a
    run can stop after ``time_budget`` seconds and resume."""
    import torch

    P = torch.as_tensor(prop, device="cuda")
    m1 = torch.as_tensor(state["m1"], device="cuda")
    m2 = torch.as_tensor(state["m2"], device="cuda")
    buf = []
    t0 = time.time()
    ws = None
    todo = specs[int(state["next_sem"]):]
    for cnt, part in label_batches(todo, steps_per_sem, batch=batch, workers=workers, log=log):
        state["next_sem"] += cnt
        buf.extend(_lists(*part))
        if not buf:
            continue
        del buf[:max(0, len(buf) - replay_lists)]
        rng = np.random.default_rng([int(state["seed"]), int(state["step"])])
        losses = []
        for _ in range(updates_per_batch):
            sel = rng.choice(len(buf), size=min(lists_per_batch, len(buf)), replace=False)
            Fb, bo, _, Wb = _stack([buf[i] for i in sel])
            state["step"] += 1
            frac = min(1.0, state["step"] / max(total_updates, 1))
            lr_t = lr_end + 0.5 * (lr - lr_end) * (1.0 + np.cos(np.pi * frac))
            loss, g, _, ws = L.proposer_grad(P, torch.as_tensor(Fb, device="cuda"), bo,
                                             weights=torch.as_tensor(Wb, device="cuda"),
                                             workspace=ws)
            L.proposer_adam(P, g, m1, m2, state["step"], lr=lr_t)
            losses.append(float(loss.item()))
        state["loss"].append(float(np.mean(losses)))
        log(f"stream: SEMs {state['next_sem']}/{len(specs)}, update {state['step']}, "
            f"loss {state['loss'][-1]:.4f}, buffer {len(buf)} lists, {time.time() - t0:.0f} s")
        if time.time() - t0 > time_budget:
            break
    state["m1"], state["m2"] = m1.cpu().numpy(), m2.cpu().numpy()
    return P.cpu().numpy()


def normalization(F) -> np.ndarray:
    """Feature mean and scale (std, floored) of the training rows."""
    mu = F.mean(axis=0, dtype=np.float64)
    sd = F.std(axis=0, dtype=np.float64)
    sd = np.maximum(sd, 1e-2 * np.maximum(1.0, np.abs(mu)))
    return np.concatenate([mu, sd]).astype(np.float32)


def init_weights(seed: int) -> np.ndarray:
    """He-uniform weights, zero biases (flat, FP32)."""
    rng = np.random.default_rng(seed)
    H, Fn = L.HIDDEN, L.N_FEATURES
    parts = [rng.uniform(-1, 1, (H, Fn)) * np.sqrt(6.0 / Fn), np.zeros(H),
             rng.uniform(-1, 1, (H, H)) * np.sqrt(6.0 / H), np.zeros(H),
             rng.uniform(-1, 1, H) * np.sqrt(6.0 / H), np.zeros(1)]
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


def _batches(n_lists, lists_per_batch, rng):
    idx = rng.permutation(n_lists)
    for a in range(0, n_lists, lists_per_batch):
        yield idx[a:a + lists_per_batch]


def train(F, offs, tgs, W=None, *, epochs: int = 20, lr: float = 2e-3,
          lists_per_batch: int = 256, seed: int = 0, log=print):
    """Adam on the listwise cross-entropy (soft targets when the row weights
    ``W`` are given, else the plain choice).  Returns the proposer block
    (numpy float32, LINGAM_PROPOSER_SIZE values) and the per-epoch mean
    losses."""
    import torch

    rng = np.random.default_rng(seed)
    prop = np.concatenate([normalization(F), init_weights(seed)])
    P = torch.as_tensor(prop, device="cuda")
    Fd = torch.as_tensor(F, device="cuda")
    Wd = torch.as_tensor(W, device="cuda") if W is not None else None
    m1 = torch.zeros(L.N_PARAMS, device="cuda")
    m2 = torch.zeros(L.N_PARAMS, device="cuda")
    sizes = np.diff(offs)
    step, ws, hist = 0, None, []
    for ep in range(epochs):
        tot, nb = 0.0, 0
        for sel in _batches(len(tgs), lists_per_batch, rng):
            # gather the batch's lists into contiguous rows (device plumbing)
            sz = sizes[sel]
            bo = np.concatenate([[0], np.cumsum(sz)]).astype(np.int64)
            rows = np.concatenate([np.arange(offs[i], offs[i + 1]) for i in sel])
            ridx = torch.as_tensor(rows, device="cuda")
            Fb = Fd.index_select(0, ridx).contiguous()
            step += 1
            if Wd is not None:
                loss, g, _, ws = L.proposer_grad(P, Fb, bo, weights=Wd.index_select(0, ridx),
                                                 workspace=ws)
            else:
                bt = bo[:-1] + (tgs[sel] - offs[sel])
                loss, g, _, ws = L.proposer_grad(P, Fb, bo, bt, workspace=ws)
            L.proposer_adam(P, g, m1, m2, step, lr=lr)
            tot += float(loss.item())
            nb += 1
        hist.append(tot / max(nb, 1))
        log(f"train: epoch {ep + 1}/{epochs} loss {hist[-1]:.4f}")
    return P.cpu().numpy(), hist


def evaluate(prop, F, offs, tgs, W=None, K: int = 64) -> dict:
    """Top-1 accuracy and top-K recall of the plain choice (GPU scores); with
    the soft weights ``W``, also the mean share of each list's near-minimal
    variables (weight >= 0.25, i.e. k <= 3 k_min) ranked within its top
    max(K, m / 16)."""
    import torch

    s = L.proposer_scores(torch.as_tensor(prop, device="cuda"),
                          torch.as_tensor(F, device="cuda")).cpu().numpy()
    top1 = recall = 0
    near = []
    for i in range(len(tgs)):
        seg = s[offs[i]:offs[i + 1]]
        tgt = tgs[i] - offs[i]
        rank = int(np.sum(seg > seg[tgt]))
        top1 += rank == 0
        recall += rank < K
        if W is not None:
            w = W[offs[i]:offs[i + 1]]
            kk = max(K, int(np.ceil(seg.size / 16)))
            top = np.argsort(-seg, kind="stable")[:kk]
            cl = np.flatnonzero(w >= 0.25)
            near.append(np.isin(cl, top).mean() if cl.size else 1.0)
    out = {"top1": top1 / len(tgs), f"top{K}_recall": recall / len(tgs), "lists": len(tgs)}
    if W is not None:
        out["near_min_recall"] = float(np.mean(near))
    return out


def save(path: str, prop, meta: dict) -> None:
    np.savez(path, proposer=np.asarray(prop, dtype=np.float32),
             meta=np.array(json.dumps(meta, sort_keys=True)))


def load_weights(path: str = WEIGHTS):
    """(proposer float32 array, metadata dict) of a saved network."""
    with np.load(path, allow_pickle=False) as z:
        prop = z["proposer"].astype(np.float32)
        meta = json.loads(str(z["meta"]))
    if prop.size != L.PROPOSER_SIZE:
        raise ValueError(f"{path}: expected {L.PROPOSER_SIZE} values, got {prop.size}")
    return prop, meta


def default_proposer(device="cuda"):
    """The shipped trained network as a CUDA tensor (raises if absent)."""
    import torch

    prop, _ = load_weights(WEIGHTS)
    return torch.as_tensor(prop, device=device)


def _split(F, offs, tgs, W, frac):
    """(train, holdout) of a list set: the last ``frac`` of its lists (whole
    SEMs, since lists are in SEM order) are held out."""
    nl = len(tgs)
    cut = nl - int(nl * frac)
    tr = (F[:offs[cut]], offs[:cut + 1], tgs[:cut], W[:offs[cut]])
    te = (F[offs[cut]:], offs[cut:] - offs[cut], tgs[cut:] - offs[cut], W[offs[cut]:])
    return tr, te


def _concat(sets):
    """One list set from several (offsets and targets rebased)."""
    Fs, os_, ts, Ws = [], [np.zeros(1, np.int64)], [], []
    base = 0
    for F, o, t, W in sets:
        Fs.append(F)
        os_.append(o[1:] + base)
        ts.append(t + base)
        Ws.append(W)
        base += int(o[-1])
    return (np.concatenate(Fs), np.concatenate(os_), np.concatenate(ts), np.concatenate(Ws))


def _save_state(path: str, prop, state: dict) -> None:
    """Write the resumable state of a streamed run to ``path`` (as named: the
    file handle keeps numpy from appending a suffix), replacing it whole."""
    scal = {k: v for k, v in state.items() if k not in ("m1", "m2")}
    tmp = path + ".tmp"
    with open(tmp, "wb") as f:
        np.savez(f, proposer=np.asarray(prop, np.float32),
                 m1=np.asarray(state["m1"], np.float32), m2=np.asarray(state["m2"], np.float32),
                 state=np.array(json.dumps(scal)))
    os.replace(tmp, path)


def _load_state(path: str):
    with np.load(path, allow_pickle=False) as z:
        state = json.loads(str(z["state"]))
        state["m1"], state["m2"] = z["m1"].astype(np.float32), z["m2"].astype(np.float32)
        return z["proposer"].astype(np.float32), state


def stream_main(a, log) -> int:
    """Stage two: fine-tune a trained network on ``--sems`` SEMs labeled while
    it trains (``stream_train``), resumable through ``--ckpt``; once every
    training SEM is done, evaluate on the held-out SEMs and write ``--out``."""
    t0 = time.time()
    specs = sem_specs(a.sems, a.d_lo, a.d_hi, a.n_lo, a.n_hi, a.seed)
    n_train = a.sems - a.holdout_sems
    if a.ckpt and os.path.exists(a.ckpt):
        prop, state = _load_state(a.ckpt)
        log(f"stream: resuming at SEM {state['next_sem']}, update {state['step']}")
    else:
        prop, meta0 = load_weights(a.init)
        state = {"m1": np.zeros(L.N_PARAMS, np.float32), "m2": np.zeros(L.N_PARAMS, np.float32),
                 "step": 0, "next_sem": 0, "loss": [], "seed": a.seed, "seconds": 0.0,
                 "init_meta": meta0}
    total = -(-n_train // a.batch) * a.updates
    if state["next_sem"] < n_train:
        prop = stream_train(prop, specs[:n_train], state, lr=a.lr, lr_end=a.lr_end,
                            total_updates=total, updates_per_batch=a.updates,
                            replay_lists=a.replay, batch=a.batch,
                            steps_per_sem=a.steps_per_sem, workers=a.workers,
                            time_budget=a.time_budget, log=log)
        state["seconds"] = float(state["seconds"]) + (time.time() - t0)
        if a.ckpt:
            _save_state(a.ckpt, prop, state)
    if state["next_sem"] < n_train:
        log(f"stream: stopped at SEM {state['next_sem']} of {n_train} (resume with --ckpt)")
        return 0
    log("stream: evaluating on the held-out SEMs")
    hold = _concat([p for _, p in label_batches(specs[n_train:], a.steps_per_sem,
                                                batch=a.batch, workers=a.workers, log=log)])
    init_prop, _ = load_weights(a.init)
    big = None
    if a.big_holdout > 0:
        bs = sem_specs(a.big_holdout, a.big_d_lo, a.big_d_hi, a.big_n_lo, a.big_n_hi,
                       a.seed + 7)
        big = _concat([p for _, p in label_batches(bs, a.steps_per_sem, batch=2,
                                                   workers=a.workers, log=log)])
    meta = dict(state["init_meta"])
    meta["stage2"] = {
        "sems": n_train, "holdout_sems": a.holdout_sems, "d": [a.d_lo, a.d_hi],
        "n": [a.n_lo, a.n_hi], "steps_per_sem": a.steps_per_sem, "batch": a.batch,
        "updates_per_batch": a.updates, "replay_lists": a.replay, "lr": [a.lr, a.lr_end],
        "updates": int(state["step"]), "loss": state["loss"][::10],
        "seconds": round(float(state["seconds"]), 1),
        "holdout": evaluate(prop, *hold), "holdout_stage1_net": evaluate(init_prop, *hold)}
    if big is not None:
        meta["stage2"]["holdout_big"] = evaluate(prop, *big)
        meta["stage2"]["holdout_big_stage1_net"] = evaluate(init_prop, *big)
    save(a.out, prop, meta)
    log(json.dumps({k: v for k, v in meta["stage2"].items() if k != "loss"}))
    return 0


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--sems", type=int, default=1000)
    ap.add_argument("--d-lo", type=int, default=100)
    ap.add_argument("--d-hi", type=int, default=1000)
    ap.add_argument("--n-lo", type=int, default=2048)
    ap.add_argument("--n-hi", type=int, default=16384)
    ap.add_argument("--big-sems", type=int, default=0,
                    help="additional SEMs with d in [--big-d-lo, --big-d-hi]")
    ap.add_argument("--big-d-lo", type=int, default=1500)
    ap.add_argument("--big-d-hi", type=int, default=4096)
    ap.add_argument("--big-n-lo", type=int, default=4096)
    ap.add_argument("--big-n-hi", type=int, default=8192)
    ap.add_argument("--steps-per-sem", type=int, default=32)
    ap.add_argument("--target", choices=("soft", "choice"), default="soft")
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--holdout", type=float, default=0.1)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--out", default=WEIGHTS)
    # stage two (streamed fine-tuning)
    ap.add_argument("--stream", action="store_true",
                    help="fine-tune --init on --sems SEMs labeled while it trains")
    ap.add_argument("--init", default=WEIGHTS)
    ap.add_argument("--ckpt", default=None, help="resumable state of a streamed run")
    ap.add_argument("--holdout-sems", type=int, default=200)
    ap.add_argument("--big-holdout", type=int, default=0)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--updates", type=int, default=4)
    ap.add_argument("--replay", type=int, default=4096)
    ap.add_argument("--lr-end", type=float, default=1e-4)
    ap.add_argument("--time-budget", type=float, default=float("inf"))
    a = ap.parse_args(argv)
    log = lambda msg: print(msg, flush=True)  # noqa: E731
    if a.stream:
        return stream_main(a, log)
    t0 = time.time()
    sets = [collect(a.sems, a.d_lo, a.d_hi, a.n_lo, a.n_hi, a.steps_per_sem,
                    seed=a.seed, workers=a.workers, log=log)]
    if a.big_sems > 0:
        sets.append(collect(a.big_sems, a.big_d_lo, a.big_d_hi, a.big_n_lo, a.big_n_hi,
                            a.steps_per_sem, seed=a.seed + 1, batch=2, workers=a.workers,
                            log=log))
    parts = [_split(*st, a.holdout) for st in sets]
    Ftr, otr, ttr, Wtr = _concat([tr for tr, _ in parts])
    soft = a.target == "soft"
    prop, hist = train(Ftr, otr, ttr, Wtr if soft else None, epochs=a.epochs, lr=a.lr,
                       seed=a.seed, log=log)
    ev_tr = evaluate(prop, Ftr, otr, ttr, Wtr)
    ev_te = [evaluate(prop, *te) if len(te[2]) else {} for _, te in parts]
    meta = {"sems": a.sems, "d": [a.d_lo, a.d_hi], "n": [a.n_lo, a.n_hi],
            "big_sems": a.big_sems, "big_d": [a.big_d_lo, a.big_d_hi],
            "big_n": [a.big_n_lo, a.big_n_hi], "target": a.target,
            "steps_per_sem": a.steps_per_sem,
            "epochs": a.epochs, "lr": a.lr, "seed": a.seed,
            "lists": int(sum(len(st[2]) for st in sets)),
            "rows": int(sum(st[1][-1] for st in sets)), "loss": hist, "train": ev_tr,
            "holdout": ev_te[0], "holdout_big": ev_te[1] if len(ev_te) > 1 else {},
            "seconds": round(time.time() - t0, 1)}
    save(a.out, prop, meta)
    log(json.dumps({k: meta[k] for k in ("lists", "rows", "train", "holdout", "holdout_big",
                                         "seconds")}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
