"""Training of the proposer network of the learned-proposal form.

The network learns which active variable the exact (plain) search takes at a
step, from orderings the plain search produces on synthetic linear
non-Gaussian SEMs.  Its inputs are the 16 features the library records at
every step (``record_features``); the loss is the listwise softmax
cross-entropy of each step's scores against the plain choice; the optimiser
is Adam.  All arithmetic runs in the library's kernels (the plain search,
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


def collect(n_sems: int, d_lo: int = 100, d_hi: int = 1000, n_lo: int = 2048,
            n_hi: int = 16384, steps_per_sem: int = 32, m_floor: int = 64, seed: int = 0,
            batch: int = 16, workers: int = 8, log=print):
    """Training lists from plain GPU orderings of ``n_sems`` SEMs (d ~ U[d_lo,
    d_hi], n log-uniform in [n_lo, n_hi], gene-expression-scale family).  At up to
    ``steps_per_sem`` steps with at least ``m_floor`` active variables, a list
    holds the features of the active variables; its target is the plain
    choice.  SEMs are drawn by a pool of ``workers`` processes ahead of the
    GPU.  Returns (features float32 [rows, 16], offsets int64, targets
    int64)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    import torch

    rng = np.random.default_rng(seed)
    specs = [(int(rng.integers(d_lo, d_hi + 1)),
              int(round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi))))),
              int(rng.integers(1 << 31))) for _ in range(n_sems)]
    feats, offs, tgs = [], [0], []
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
        out = L.batch_causal_order(jobs, record_features=True)
        for k, X in enumerate(Xs):
            d = X.shape[1]
            futs[done + k] = None
            order = out["orders"][k].cpu().numpy()
            R = out["features"][k]
            last = d - m_floor  # steps t <= last have m >= m_floor
            if last < 0:
                continue
            ts = np.sort(rng.choice(last + 1, size=min(steps_per_sem, last + 1), replace=False))
            Rt = R[torch.as_tensor(ts, device=R.device)].cpu().numpy()
            for i, t in enumerate(ts):
                act = np.flatnonzero(~np.isnan(Rt[i, :, 0]))
                feats.append(Rt[i, act])
                tgs.append(offs[-1] + int(np.flatnonzero(act == order[t])[0]))
                offs.append(offs[-1] + act.size)
        done += cnt
        del out, jobs
        log(f"collect: {done}/{n_sems} SEMs, {len(tgs)} lists, {offs[-1]} rows, "
            f"{time.time() - t0:.0f} s")
    pool.shutdown()
    return (np.concatenate(feats).astype(np.float32), np.asarray(offs, np.int64),
            np.asarray(tgs, np.int64))


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


def train(F, offs, tgs, *, epochs: int = 20, lr: float = 2e-3, lists_per_batch: int = 256,
          seed: int = 0, log=print):
    """Adam on the listwise cross-entropy.  Returns the proposer block (numpy
    float32, LINGAM_PROPOSER_SIZE values) and the per-epoch mean losses."""
    import torch

    rng = np.random.default_rng(seed)
    prop = np.concatenate([normalization(F), init_weights(seed)])
    P = torch.as_tensor(prop, device="cuda")
    Fd = torch.as_tensor(F, device="cuda")
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
            Fb = Fd.index_select(0, torch.as_tensor(rows, device="cuda")).contiguous()
            bt = bo[:-1] + (tgs[sel] - offs[sel])
            step += 1
            loss, g, _, ws = L.proposer_grad(P, Fb, bo, bt, workspace=ws)
            L.proposer_adam(P, g, m1, m2, step, lr=lr)
            tot += float(loss.item())
            nb += 1
        hist.append(tot / max(nb, 1))
        log(f"train: epoch {ep + 1}/{epochs} loss {hist[-1]:.4f}")
    return P.cpu().numpy(), hist


def evaluate(prop, F, offs, tgs, K: int = 64) -> dict:
    """Top-1 accuracy and top-K recall of the plain choice (GPU scores)."""
    import torch

    s = L.proposer_scores(torch.as_tensor(prop, device="cuda"),
                          torch.as_tensor(F, device="cuda")).cpu().numpy()
    top1 = recall = 0
    for i in range(len(tgs)):
        seg = s[offs[i]:offs[i + 1]]
        tgt = tgs[i] - offs[i]
        rank = int(np.sum(seg > seg[tgt]))
        top1 += rank == 0
        recall += rank < K
    return {"top1": top1 / len(tgs), f"top{K}_recall": recall / len(tgs), "lists": len(tgs)}


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


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--sems", type=int, default=1000)
    ap.add_argument("--d-lo", type=int, default=100)
    ap.add_argument("--d-hi", type=int, default=1000)
    ap.add_argument("--n-lo", type=int, default=2048)
    ap.add_argument("--n-hi", type=int, default=16384)
    ap.add_argument("--steps-per-sem", type=int, default=32)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--holdout", type=float, default=0.1)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--out", default=WEIGHTS)
    a = ap.parse_args(argv)
    log = lambda msg: print(msg, flush=True)  # noqa: E731
    t0 = time.time()
    F, offs, tgs = collect(a.sems, a.d_lo, a.d_hi, a.n_lo, a.n_hi, a.steps_per_sem,
                           seed=a.seed, workers=a.workers, log=log)
    nl = len(tgs)
    nh = int(nl * a.holdout)
    # hold out the last lists (whole SEMs, since lists are in SEM order)
    cut = nl - nh
    Ftr, otr, ttr = F[:offs[cut]], offs[:cut + 1], tgs[:cut]
    Fte, ote, tte = F[offs[cut]:], offs[cut:] - offs[cut], tgs[cut:] - offs[cut]
    prop, hist = train(Ftr, otr, ttr, epochs=a.epochs, lr=a.lr, seed=a.seed, log=log)
    ev_tr = evaluate(prop, Ftr, otr, ttr)
    ev_te = evaluate(prop, Fte, ote, tte) if nh else {}
    meta = {"sems": a.sems, "d": [a.d_lo, a.d_hi], "n": [a.n_lo, a.n_hi],
            "steps_per_sem": a.steps_per_sem,
            "epochs": a.epochs, "lr": a.lr, "seed": a.seed, "lists": nl,
            "rows": int(offs[-1]), "loss": hist, "train": ev_tr, "holdout": ev_te,
            "seconds": round(time.time() - t0, 1)}
    save(a.out, prop, meta)
    log(json.dumps({k: meta[k] for k in ("lists", "rows", "train", "holdout", "seconds")}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
