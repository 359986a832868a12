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


def collect(n_sems: int, d_lo: int = 100, d_hi: int = 1000, n_lo: int = 2048,
            n_hi: int = 16384, steps_per_sem: int = 32, m_floor: int = 64, seed: int = 0,
            batch: int = 16, workers: int = 8, log=print):
    """Training lists from plain GPU orderings of ``n_sems`` SEMs (d ~ U[d_lo,
    d_hi], n log-uniform in [n_lo, n_hi] and at least 2 d, gene-expression-scale
    family; a draw the plain search finds degenerate is skipped).  At up to
    ``steps_per_sem`` steps with at least ``m_floor`` active variables, a list
    holds the features of the active variables; its target is the plain
    choice, and its variables' k values give the soft target weights.  SEMs
    are drawn by a pool of ``workers`` processes ahead of the GPU.  Returns
    (features float32 [rows, 16], offsets int64, targets int64, weights
    float32 [rows])."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    import torch

    rng = np.random.default_rng(seed)
    specs = []
    for _ in range(n_sems):
        d = int(rng.integers(d_lo, d_hi + 1))
        n = int(round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))))
        specs.append((d, max(n, 2 * d), int(rng.integers(1 << 31))))  # n >= 2 d
    feats, offs, tgs, wts = [], [0], [], []
    done = 0
    t0 = time.time()
    pool = ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn"))
    futs = [pool.submit(_gen, sp) for sp in specs[:2 * batch]]
    nxt = len(futs)
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
        for k, X in enumerate(Xs):
            d = X.shape[1]
            futs[done + k] = None
            if status[k] != 0:  # a degenerate draw (collinear residuals): skip it
                log(f"collect: SEM {done + k} skipped (status {int(status[k])})")
                continue
            order = out["orders"][k].cpu().numpy()
            R = out["features"][k]
            Mk = out["measures"][k]
            last = d - m_floor  # steps t <= last have m >= m_floor
            if last < 0:
                continue
            ts = np.sort(rng.choice(last + 1, size=min(steps_per_sem, last + 1), replace=False))
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
        log(f"collect: {done}/{n_sems} SEMs, {len(tgs)} lists, {offs[-1]} rows, "
            f"{time.time() - t0:.0f} s")
    pool.shutdown()
    return (np.concatenate(feats).astype(np.float32), np.asarray(offs, np.int64),
            np.asarray(tgs, np.int64), np.concatenate(wts).astype(np.float32))


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
    a = ap.parse_args(argv)
    log = lambda msg: print(msg, flush=True)  # noqa: E731
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
