"""GPU learned-proposal form against the FP64 oracle, through the C ABI.

* network scores (BF16 MFMA, FP32 accumulation) vs the oracle forward pass
  with the same BF16 rounding points;
* the training gradient vs the oracle's FP64 backward pass at the same
  BF16-rounded weights and inputs (relative error per parameter block);
* Adam vs the oracle's Adam;
* the 16 features recorded during a plain search vs the oracle's features of
  the residuals along the same order;
* orderings: the exact mode (margin = +inf) and all-audit runs give the plain
  order, with the FP64 resolution of near-ties and with FP32 tie decisions;
  the pure learned order (margin = -inf) equals the oracle's learned order
  up to the first near-tie;
* training on recorded plain orderings lowers the loss.
"""
import os

import numpy as np
import pytest

import oracle
from oracle import proposer as OP
from paper_2403_03772_amd import synth

pytestmark = pytest.mark.gpu


def _t(a, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=dtype or np.float32)).cuda()


def _proposer(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    norm = np.concatenate([rng.normal(scale=0.3, size=16), rng.uniform(0.5, 2.0, 16)])
    return np.concatenate([norm, OP.init_params(seed) * scale])


def test_scores_match_oracle(lib):
    rng = np.random.default_rng(0)
    prop = _proposer(1)
    for rows in (1, 63, 64, 1000, 4099):
        F = rng.normal(size=(rows, 16)).astype(np.float32)
        print(f"scores rows={rows}", flush=True)
        g = lib.proposer_scores(_t(prop), _t(F)).cpu().numpy().astype(np.float64)
        ref, _ = OP.forward(prop[32:], OP.normalize(F, prop[:32]), emulate_bf16=True)
        scale = max(1.0, np.max(np.abs(ref)))
        assert np.max(np.abs(g - ref)) <= 2e-5 * scale, rows


def _lists(rng, sizes):
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    tg = np.array([offs[L] + rng.integers(sizes[L]) for L in range(len(sizes))],
                  dtype=np.int64)
    return offs, tg


def test_grad_matches_oracle(lib):
    rng = np.random.default_rng(2)
    prop = _proposer(3)
    sizes = [int(x) for x in rng.integers(2, 300, 40)]
    offs, tg = _lists(rng, sizes)
    rows = int(offs[-1])
    F = rng.normal(size=(rows, 16)).astype(np.float32)
    print(f"grad rows={rows} lists={len(sizes)}", flush=True)
    loss, grad, scores, _ = lib.proposer_grad(_t(prop), _t(F), _t(offs, np.int64),
                                              _t(tg, np.int64))
    g = grad.cpu().numpy().astype(np.float64)
    # oracle at the BF16-rounded weights and inputs the kernels use
    flat = prop[32:].copy()
    p = OP.unpack(flat)
    for k in ("W1", "W2", "w3"):
        p[k] = OP.bf16(p[k])
    flat_b = OP.pack(p)
    s, cache = OP.forward(flat_b, OP.bf16(OP.normalize(F, prop[:32])), emulate_bf16=True)
    ref_loss, ds = OP.listwise_ce(s.astype(np.float32).astype(np.float64), offs, tg)
    ref = OP.backward(flat_b, cache, ds)
    assert abs(float(loss.item()) - ref_loss) <= 1e-4 * max(1.0, abs(ref_loss))
    o = 0
    for name, shp in OP.SHAPES:
        k = int(np.prod(shp))
        a, b = g[o:o + k], ref[o:o + k]
        o += k
        if name == "b3":
            # d loss / d b3 = sum of ds = 0 exactly (softmax gradients sum to
            # zero over every list): only rounding remains
            print(f"  b3: {a[0]:.2e} (exact 0)", flush=True)
            assert abs(a[0]) <= 1e-6
            continue
        err = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-12)
        print(f"  {name}: rel err {err:.2e}", flush=True)
        assert err <= 1e-2, name


def test_grad_soft_matches_oracle(lib):
    """Soft target distributions: loss and gradient against the oracle's
    soft cross-entropy at the BF16-rounded weights; one-hot weights give the
    hard-target call's loss and gradient."""
    rng = np.random.default_rng(7)
    prop = _proposer(4)
    sizes = [int(x) for x in rng.integers(2, 200, 30)]
    offs, tg = _lists(rng, sizes)
    rows = int(offs[-1])
    F = rng.normal(size=(rows, 16)).astype(np.float32)
    w = (rng.uniform(size=rows) ** 4).astype(np.float32)
    print(f"grad soft rows={rows} lists={len(sizes)}", flush=True)
    loss, grad, _, _ = lib.proposer_grad(_t(prop), _t(F), _t(offs, np.int64), weights=_t(w))
    g = grad.cpu().numpy().astype(np.float64)
    flat = prop[32:].copy()
    p = OP.unpack(flat)
    for k in ("W1", "W2", "w3"):
        p[k] = OP.bf16(p[k])
    flat_b = OP.pack(p)
    s, cache = OP.forward(flat_b, OP.bf16(OP.normalize(F, prop[:32])), emulate_bf16=True)
    ref_loss, ds = OP.listwise_ce_soft(s.astype(np.float32).astype(np.float64), offs,
                                       w.astype(np.float64))
    ref = OP.backward(flat_b, cache, ds)
    assert abs(float(loss.item()) - ref_loss) <= 1e-4 * max(1.0, abs(ref_loss))
    o = 0
    for name, shp in OP.SHAPES:
        k = int(np.prod(shp))
        a, b = g[o:o + k], ref[o:o + k]
        o += k
        if name == "b3":
            assert abs(a[0]) <= 1e-6  # softmax minus a distribution sums to 0
            continue
        err = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-12)
        print(f"  {name}: rel err {err:.2e}", flush=True)
        assert err <= 1e-2, name
    onehot = np.zeros(rows, dtype=np.float32)
    onehot[tg] = 3.0
    l1, g1, _, _ = lib.proposer_grad(_t(prop), _t(F), _t(offs, np.int64), weights=_t(onehot))
    l0, g0, _, _ = lib.proposer_grad(_t(prop), _t(F), _t(offs, np.int64), _t(tg, np.int64))
    assert abs(float(l1.item()) - float(l0.item())) <= 1e-6 * max(1.0, abs(float(l0.item())))
    assert float((g1 - g0).abs().max()) <= 1e-6 * max(1e-3, float(g0.abs().max()))
    bad = w.copy()
    bad[offs[1]:offs[2]] = 0.0  # a list with no mass
    with pytest.raises(lib.LingamError):
        lib.proposer_grad(_t(prop), _t(F), _t(offs, np.int64), weights=_t(bad))
    bad = w.copy()
    bad[3] = -1.0
    with pytest.raises(lib.LingamError):
        lib.proposer_grad(_t(prop), _t(F), _t(offs, np.int64), weights=_t(bad))


def test_adam_matches_oracle(lib):
    import torch
    rng = np.random.default_rng(4)
    prop = _proposer(5)
    P = _t(prop)
    m1 = torch.zeros(OP.N_PARAMS, device="cuda")
    m2 = torch.zeros(OP.N_PARAMS, device="cuda")
    opt = OP.Adam(lr=3e-3)
    w = prop[32:].copy()
    for step in range(1, 4):
        g = rng.normal(size=OP.N_PARAMS).astype(np.float32)
        lib.proposer_adam(P, _t(g), m1, m2, step, lr=3e-3)
        w = opt.step(w, g.astype(np.float64))
    got = P.cpu().numpy().astype(np.float64)
    assert np.array_equal(got[:32], prop[:32].astype(np.float32).astype(np.float64))
    assert np.max(np.abs(got[32:] - w)) <= 1e-6 * max(1.0, np.max(np.abs(w)))


def test_features_match_oracle(lib):
    s = synth.er_sem(40, 2000, indeg=2.0, noise_family=("uniform", "laplace", "exp"), seed=8)
    X32 = s.X.astype(np.float32)
    out = lib.causal_order(_t(X32), record_features=True)
    order = out["order"].cpu().numpy()
    feats = out["features"].cpu().numpy()
    Xc = X32.astype(np.float64)
    U = list(range(40))
    for t in range(39):
        if t in (0, 1, 5, 20, 37):
            F = OP.features(Xc, U, t, 40)
            G = feats[t][U].astype(np.float64)
            cont = [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 12, 13, 14, 15]
            err = np.abs(G[:, cont] - F[:, cont]) / np.maximum(np.abs(F[:, cont]), 1e-3)
            assert np.max(err) <= 1e-5, (t, np.unravel_index(np.argmax(err), err.shape))
            assert np.array_equal(G[:, 10], F[:, 10].astype(np.float32)), t
            assert np.array_equal(G[:, 11], F[:, 11].astype(np.float32)), t
            inactive = np.setdiff1d(np.arange(40), U)
            assert np.all(np.isnan(feats[t][inactive]))
        Xc = oracle.residualize(Xc, U, int(order[t]))
        U.remove(int(order[t]))


def _sem(d, n, seed):
    return synth.er_sem(d, n, indeg=3.0, noise_family=("uniform", "laplace", "exp"), seed=seed)


def test_exact_mode_and_audits_give_plain_order(lib):
    s = _sem(180, 3000, 11)
    X = _t(s.X)
    plain = lib.causal_order(X, with_measures=True)
    po = plain["order"].cpu().numpy()
    P = _t(_proposer(6))
    for margin, audit in ((np.inf, 0), (-np.inf, 1)):
        print(f"learned margin={margin} audit={audit}", flush=True)
        out = lib.causal_order(X, learned=lib.Learned(P, topk=16, audit_every=audit,
                                                      margin=float(margin), min_m=64))
        lo = out["order"].cpu().numpy()
        st = out["learned_stats"]
        print(st, flush=True)
        assert st.learned_steps == 180 - 64
        if audit == 1:
            assert st.audits == st.learned_steps
        else:  # every step certified, decided by the suspect pass, or a full step
            assert st.certified + st.expanded + st.fallbacks == st.learned_steps
        diff = np.flatnonzero(lo != po)
        if diff.size:
            t = int(diff[0])
            mv = plain["measures"].cpu().numpy()[t]
            a, b = mv[po[t]], mv[lo[t]]
            assert abs(a - b) <= 2e-4 * max(abs(a), 1e-3 * np.nanmax(np.abs(mv))), (t, a, b)


@pytest.mark.parametrize("fp32_ties", [False, True])
def test_exact_form_equals_plain_with_either_tie_rule(lib, fp32_ties):
    """The exact learned form returns the plain order under both tie rules:
    with the FP64 resolution of near-ties (its row passes then take their own
    sample splits, and near-ties are decided from the FP64 residuals in both
    forms) and with FP32 decisions (the row passes then take the full step's
    split, so every row they measure equals the full step's bit for bit).
    Shipped network, d = 600, n = 6000, two seeds."""
    from paper_2403_03772_amd import train_proposer as TP
    if not os.path.exists(TP.WEIGHTS):
        pytest.skip("no trained network shipped")
    P = TP.default_proposer()
    for seed in (5, 6):
        s = _sem(600, 6000, seed)
        X = _t(s.X)
        plain = lib.causal_order(X, fp32_ties=fp32_ties).cpu().numpy()
        out = lib.causal_order(X, learned=lib.Learned(P, topk=64), fp32_ties=fp32_ties)
        st = out["learned_stats"]
        print(f"seed {seed} fp32_ties={fp32_ties}: {st}", flush=True)
        assert st.learned_steps > 0 and st.fallbacks == 0
        assert np.array_equal(out["order"].cpu().numpy(), plain), seed


def test_autotuned_exact_form_equals_plain(lib):
    """The launch-shape autotuner on a learned call (split policy and row
    waves timed on the candidate pass, all-pairs waves on the full step)
    keeps the exact form's order equal to the plain order, on the tuning call
    and on a later call that reuses the tuned shape.  Shipped network,
    d = 600, n = 6000."""
    from paper_2403_03772_amd import train_proposer as TP
    if not os.path.exists(TP.WEIGHTS):
        pytest.skip("no trained network shipped")
    s = _sem(600, 6000, 7)
    X = _t(s.X)
    plain = lib.causal_order(X).cpu().numpy()
    cfg = lib.Learned(TP.default_proposer(), topk=64)
    for rep in range(2):
        out = lib.causal_order(X, learned=cfg, autotune=True)
        st = out["learned_stats"]
        print(f"autotuned learned call {rep}: {st}", flush=True)
        assert st.learned_steps > 0 and st.fallbacks == 0
        assert np.array_equal(out["order"].cpu().numpy(), plain), rep


def _oracle_step(X32, prefix, prop, K):
    """Oracle scores and exact k at the state after `prefix`."""
    Xc = X32.astype(np.float64)
    U = list(range(X32.shape[1]))
    for e in prefix:
        Xc = oracle.residualize(Xc, U, int(e))
        U.remove(int(e))
    F = OP.features(Xc, U, len(prefix), X32.shape[1])
    s, _ = OP.forward(prop[32:], OP.normalize(F, prop[:32]), emulate_bf16=True)
    D = oracle.pair_matrix(Xc, U)
    k = np.sum(np.minimum(D, 0) ** 2, axis=1)
    return np.array(U), s.astype(np.float32).astype(np.float64), k


@pytest.mark.parametrize("max_suspects", [1024, 0])
def test_pure_learned_order_matches_oracle(lib, max_suspects):
    """margin = -inf: the learned choice is never handed to a full step; with
    the second pass (max_suspects 1024) or without it (0, the fast form)."""
    d, n, K = 110, 1500, 8
    s = _sem(d, n, 12)
    X32 = s.X.astype(np.float32)
    prop = _proposer(7)
    out = lib.causal_order(_t(X32), learned=lib.Learned(_t(prop), topk=K, audit_every=0,
                                                        margin=-np.inf, min_m=64,
                                                        max_suspects=max_suspects))
    go = out["order"].cpu().numpy()
    st = out["learned_stats"]
    assert st.fallbacks == 0 and st.audits == 0
    if max_suspects == 0:
        assert st.expanded == 0
    ro, info = OP.learned_order(X32, prop, K=K, delta=-np.inf, audit_every=0, min_m=64,
                                max_suspects=max_suspects)
    diff = np.flatnonzero(go != ro)
    if diff.size == 0:
        return
    t = int(diff[0])
    U, sc, k = _oracle_step(X32, ro[:t], prop, K)
    srt = np.sort(sc)[::-1]
    boundary_tie = abs(srt[K - 1] - srt[K]) <= 1e-4 * max(1.0, np.max(np.abs(sc)))
    pa, pb = np.flatnonzero(U == ro[t])[0], np.flatnonzero(U == go[t])[0]
    k_tie = abs(k[pa] - k[pb]) <= 2e-4 * max(k[pa], k[pb], 1e-12)
    assert boundary_tie or k_tie, (t, ro[t], go[t], k[pa], k[pb])


def test_batch_learned_equals_single(lib):
    P = _t(_proposer(8))
    cfg = lib.Learned(P, topk=8, audit_every=8, margin=1.0, min_m=64)
    Xs = [_sem(d, n, 30 + d) .X for d, n in ((100, 800), (150, 1200), (70, 600), (30, 500))]
    out = lib.batch_causal_order([{"X": _t(X)} for X in Xs], learned=cfg)
    for k, X in enumerate(Xs):
        single = lib.causal_order(_t(X), learned=cfg)["order"].cpu().numpy()
        assert np.array_equal(out["orders"][k].cpu().numpy(), single), k


def test_many_job_learned_batch_equals_single(lib):
    """More than 64 jobs in the exact learned form (the suspect schedule then
    scans the jobs one wave per kind): 70 jobs with d in [130, 200], every
    one with its single-job order, which is the plain order."""
    from paper_2403_03772_amd import train_proposer as TP
    if not os.path.exists(TP.WEIGHTS):
        pytest.skip("no trained network shipped")
    P = TP.default_proposer()
    cfg = lib.Learned(P, topk=64)
    rng = np.random.default_rng(71)
    Xs = [_sem(int(rng.integers(130, 201)), int(rng.integers(800, 1500)), 3000 + k).X
          for k in range(70)]
    print("case 70 learned jobs", flush=True)
    out = lib.batch_causal_order([{"X": _t(X)} for X in Xs], learned=cfg)
    assert int(out["status"].abs().sum()) == 0
    st = out["learned_stats"]
    assert st.learned_steps > 0 and st.fallbacks == 0
    for k, X in enumerate(Xs):
        single = lib.causal_order(_t(X), learned=cfg)["order"].cpu().numpy()
        plain = lib.causal_order(_t(X)).cpu().numpy()
        assert np.array_equal(out["orders"][k].cpu().numpy(), single), k
        assert np.array_equal(single, plain), k


def test_bad_proposer_and_lists_rejected(lib):
    import torch
    prop = _proposer(9)
    bad = prop.copy()
    bad[40] = np.nan
    X = _t(_sem(100, 500, 1).X)
    with pytest.raises(lib.LingamError) as e:
        lib.causal_order(X, learned=lib.Learned(_t(bad), topk=8, min_m=64))
    assert e.value.code == -1
    F = _t(np.zeros((10, 16)))
    with pytest.raises(lib.LingamError):
        lib.proposer_grad(_t(prop), F, np.array([0, 5, 12]), np.array([1, 6]))
    with pytest.raises(lib.LingamError):
        lib.proposer_grad(_t(prop), F, np.array([0, 5, 10]), np.array([1, 3]))
    # a good call after the rejected ones
    loss, g, _, _ = lib.proposer_grad(_t(prop), F, np.array([0, 5, 10]), np.array([1, 6]))
    assert np.isfinite(loss.item()) and torch.isfinite(g).all()


def test_training_lowers_loss(lib):
    """A few Adam steps on lists recorded from plain orderings."""
    import torch
    feats, offs, tgs = [], [0], []
    for seed in range(6):
        s = _sem(120, 1500, 100 + seed)
        out = lib.causal_order(_t(s.X), record_features=True)
        order = out["order"].cpu().numpy()
        R = out["features"].cpu().numpy()
        for t in range(0, 100, 5):
            act = np.flatnonzero(~np.isnan(R[t, :, 0]))
            feats.append(R[t, act])
            tgs.append(offs[-1] + int(np.flatnonzero(act == order[t])[0]))
            offs.append(offs[-1] + act.size)
    F = np.concatenate(feats).astype(np.float32)
    mu, sd = F.mean(axis=0), F.std(axis=0) + 1e-3
    prop = np.concatenate([mu, sd, OP.init_params(0)]).astype(np.float32)
    P = _t(prop)
    Ft = _t(F)
    m1 = torch.zeros(OP.N_PARAMS, device="cuda")
    m2 = torch.zeros(OP.N_PARAMS, device="cuda")
    ws = None
    losses = []
    for step in range(1, 61):
        loss, g, _, ws = lib.proposer_grad(P, Ft, np.array(offs), np.array(tgs), workspace=ws)
        losses.append(float(loss.item()))
        lib.proposer_adam(P, g, m1, m2, step, lr=3e-3)
    print("loss", losses[0], "->", losses[-1], flush=True)
    assert losses[-1] < 0.8 * losses[0]


def test_step_log_matches_stats(lib):
    """The per-step decision log agrees with the counters and the schedule."""
    s = _sem(200, 2000, 21)
    P = _t(_proposer(10))
    out = lib.causal_order(_t(s.X), learned=lib.Learned(P, topk=16, audit_every=8, min_m=64,
                                                        extension=64),
                           step_log=True)
    log = out["step_log"].cpu().numpy()
    st = out["learned_stats"]
    kind, nsus, rows = log & 15, (log >> 4) & 0xFFF, log >> 16
    m = 200 - np.arange(200)
    learned = (m > 64) & (np.arange(200) < 199)
    assert np.all(kind[~learned] == 0)
    assert np.all(kind[learned] > 0)
    assert int(np.sum(kind == 3)) == st.audits == int(np.sum(learned & (np.arange(200) % 8 == 0)))
    assert int(np.sum(kind == 4)) == st.expanded
    assert int(np.sum(kind == 2)) == st.fallbacks
    assert int(np.sum(kind == 1)) + st.expanded + st.fallbacks + st.audits == st.learned_steps
    assert np.all(nsus[kind == 4] > 0) and np.all(nsus[kind != 4] == 0)
    assert np.all(nsus[kind == 4] <= np.maximum((m[kind == 4] // 2 - 16) // 8 * 8, 0))
    # the extension columns leave some of the suspects for the rows pass
    assert np.all(rows <= nsus) and np.all(rows[kind != 4] == 0)
    assert int(np.sum(rows)) == st.rows_sum
    assert int(np.sum((kind == 4) & (rows == 0))) == st.cleared


def test_exact_decisions_match_oracle(lib):
    """Exact mode step by step against the oracle's learned form (same
    network, K, witnesses, extension columns): the plain order, and at every
    learned step the same decision (certified by the bound, or a second pass
    over the same number of suspects, of which the same number have their
    rows measured after the extension columns).  The bound compares
    FP32-path measures on the GPU with FP64 ones in the oracle, so a step
    whose counts differ is accepted only where some oracle bound lies within
    1e-3 of the best candidate's k of the suspects' threshold (the best
    candidate's k widened by the near-tie limit of the FP64 tie resolution)."""
    d, n, K = 130, 2500, 16
    s = _sem(d, n, 31)
    X32 = s.X.astype(np.float32)
    prop = _proposer(11)
    out = lib.causal_order(_t(X32), learned=lib.Learned(_t(prop), topk=K, min_m=64,
                                                        extension=32),
                           step_log=True)
    go = out["order"].cpu().numpy()
    log = out["step_log"].cpu().numpy()
    ro, info = OP.learned_order(X32, prop, K=K, delta=np.inf, audit_every=0, min_m=64,
                                n_ext=32)
    assert np.array_equal(go, ro)
    mism = 0
    rows_checked = 0
    for st in info:
        if st.kind == "plain":
            assert log[st.t] & 15 == 0
            continue
        g_kind, g_sus = int(log[st.t] & 15), int((log[st.t] >> 4) & 0xFFF)
        g_rows = int(log[st.t] >> 16)
        o_sus = 0 if st.certified else st.suspects
        same = (g_kind == 1) == st.certified and g_sus == o_sus
        if same and (g_kind != 4 or g_rows == st.rows):
            rows_checked += g_kind == 4
            continue
        mism += 1
        # the oracle's bounds at this step: some must sit at the best
        # candidate's k within the FP32 path's error
        Xc = X32.astype(np.float64)
        U = list(range(d))
        for e in ro[:st.t]:
            Xc = oracle.residualize(Xc, U, int(e))
            U.remove(int(e))
        D = oracle.pair_matrix(Xc, U)
        k = np.sum(np.minimum(D, 0) ** 2, axis=1)
        C = np.asarray(st.candidates)
        wit = OP.witnesses(Xc, U, 8)
        lb = OP.lower_bounds(D, C, wit)
        kb = np.min(k[C])
        lim = kb * (1.0 + OP.TIE_REL) + OP.TIE_ABS  # the suspects' threshold
        notc = np.setdiff1d(np.arange(len(U)), C)
        if same:   # same suspects, a different count of measured rows
            sus = notc[~(lb[notc] > lim)]
            lb = OP.extension_bounds(D, lb, sus, st.extension, wit)
            notc = sus
        near = np.abs(lb[notc] - lim) <= 1e-3 * kb
        assert near.any(), (st.t, g_kind, g_sus, g_rows, st.certified, o_sus, st.rows)
    print(f"exact decisions: {len(info)} steps, {mism} with different counts, "
          f"{rows_checked} second passes with equal measured rows", flush=True)
    assert rows_checked > 0


def test_extension_columns_only_shrink_the_rows(lib):
    """The extension columns change only how many suspects' rows are
    measured: with and without them the order is the plain order and the
    decisions and suspects of every step are the same; without them every
    suspect's row is measured, with them fewer (shipped network, d = 400)."""
    from paper_2403_03772_amd import train_proposer as TP
    s = _sem(400, 4000, 41)
    X = _t(s.X)
    P = TP.default_proposer()
    plain = lib.causal_order(X).cpu().numpy()
    runs = {}
    for ext in (0, 128, 8):
        print(f"extension {ext}", flush=True)
        out = lib.causal_order(X, learned=lib.Learned(P, topk=32, extension=ext),
                               step_log=True)
        assert np.array_equal(out["order"].cpu().numpy(), plain), ext
        runs[ext] = (out["learned_stats"], out["step_log"].cpu().numpy())
    (a, la), (b, lb), (c, lc) = runs[0], runs[128], runs[8]
    for st, lg_ in ((b, lb), (c, lc)):
        assert np.array_equal(lg_ & 0xFFFF, la & 0xFFFF)
        assert (st.certified, st.expanded, st.suspects_sum) == \
            (a.certified, a.expanded, a.suspects_sum)
    assert a.rows_sum == a.suspects_sum and a.cleared == 0
    assert b.rows_sum <= c.rows_sum <= a.rows_sum
    assert a.expanded > 0 and b.rows_sum < a.rows_sum
    print(f"rows measured: none {a.rows_sum}, 8 columns {c.rows_sum}, 128 columns "
          f"{b.rows_sum} (cleared {b.cleared} of {b.expanded})", flush=True)


def test_graph_cache_follows_the_proposer(lib):
    """Two graph-mode calls that differ only in the proposer buffer (same
    input, output and workspace buffers) must not share a captured graph: the
    second call's decisions follow its own network, as the eager calls show."""
    import torch
    from paper_2403_03772_amd import train_proposer as TP
    s = _sem(300, 3000, 43)
    X = _t(s.X)
    trained = TP.default_proposer()
    raw = _t(_proposer(9))
    cfg = {p: lib.Learned(q, topk=32) for p, q in (("trained", trained), ("raw", raw))}
    eager = {k: lib.causal_order(X, learned=c)["learned_stats"] for k, c in cfg.items()}
    assert eager["trained"].certified != eager["raw"].certified  # the networks differ
    ws = torch.empty(lib.workspace_size(3000, 300, cfg["trained"]), dtype=torch.uint8,
                     device="cuda")
    out = torch.empty(300, dtype=torch.int32, device="cuda")
    for k in ("trained", "raw", "trained", "raw"):
        print(f"graph call with the {k} network", flush=True)
        got = lib.causal_order(X, learned=cfg[k], graph=True, workspace=ws,
                               out=out)["learned_stats"]
        ref = eager[k]
        assert (got.certified, got.expanded, got.suspects_sum, got.fallbacks) == \
            (ref.certified, ref.expanded, ref.suspects_sum, ref.fallbacks), k
