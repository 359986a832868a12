"""Pins of the proposer oracle (CPU): every part is checked against something
other than itself -- a library routine, a closed form, finite differences, or
the plain search it must reduce to."""
import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import proposer as P
from paper_2403_03772_amd import synth


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=5000) * 10.0 ** rng.integers(-8, 8, 5000),
                        # exact halfway cases between two BF16 values (ties to even)
                        np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -1.0 - 2.0 ** -8])])
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(P.bf16(x), ref)


def _grid(dist, n=200001):
    q = (np.arange(n) + 0.5) / n
    return dist.ppf(q)


@pytest.mark.parametrize("name,dist,e_lc,H,e3,ex4,eabs", [
    ("gauss", stats.norm(), 0.3745672075, 1.4189385326, 0.0, 0.0, np.sqrt(2 / np.pi)),
    ("uniform", stats.uniform(-np.sqrt(3), 2 * np.sqrt(3)), 0.4013378931, 1.3622997688, 0.0,
     -1.2, np.sqrt(3) / 2),
    ("laplace", stats.laplace(scale=1 / np.sqrt(2)), 0.3382367723, 1.3145883171, 0.0, 3.0,
     1 / np.sqrt(2)),
    ("exp", stats.expon(loc=-1.0), 0.3301432991, 1.0879312472, 2.0, 6.0, 2 / np.e),
])
def test_moment_features_closed_forms(name, dist, e_lc, H, e3, ex4, eabs):
    """Features 1-7 of one column drawn on a quantile grid equal the
    distribution's moments (closed forms; the grid error is far below the
    tolerances, which allow for the truncated tails of the 4th moment)."""
    x = _grid(dist)
    F = P.features(x[:, None], [0], t=0, d=1)[0]
    assert abs(F[0] - e_lc) < 2e-5
    assert abs(F[2] - H) < 1e-4
    assert abs(F[3] - e3) < 2e-3 * max(1.0, abs(e3))
    assert abs(F[4] - ex4) < 5e-3 * max(1.0, abs(ex4))
    assert abs(F[5] - eabs) < 3e-5
    assert abs(F[6] - F[3] ** 2) < 1e-15
    assert F[12] == 0.0 and F[13] == 1.0 and abs(F[14] - np.log(x.size)) < 1e-12


def test_correlation_features_brute_force():
    """Features 3, 8-12 and 16 against np.corrcoef, the C oracle's entropy and
    scipy's ordinal ranks."""
    s = synth.er_sem(7, 300, indeg=2.0, noise_family=("uniform", "laplace", "exp"), seed=4)
    X = s.X.astype(np.float64)
    U = [0, 2, 3, 5, 6]
    F = P.features(X, U, t=2, d=7)
    rho = np.corrcoef(X[:, U].T)
    H = np.array([oracle.entropy((X[:, v] - X[:, v].mean()) / X[:, v].std()) for v in U])
    m = len(U)
    ranks = stats.rankdata(H, method="ordinal") - 1
    for p in range(m):
        r = np.delete(rho[p], p)
        Ho = np.delete(H, p)
        assert abs(F[p, 2] - H[p]) < 1e-12
        assert abs(F[p, 7] - np.abs(r).max()) < 1e-12
        assert abs(F[p, 8] - (r ** 2).sum() / m) < 1e-12
        assert abs(F[p, 9] - np.abs(r).mean()) < 1e-12
        assert F[p, 10] == np.mean(np.abs(r) > 0.5)
        assert F[p, 11] == ranks[p] / m
        assert abs(F[p, 15] - (r ** 2 * Ho).sum() / (r ** 2).sum()) < 1e-12
        assert F[p, 12] == 2 / 7 and F[p, 13] == m / 7


def _lists(rng, sizes):
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    tg = np.array([offs[L] + rng.integers(sizes[L]) for L in range(len(sizes))])
    return offs, tg


def _torch_net(flat, bf16: bool):
    """The network as torch modules, with the parameters sliced from the flat
    layout the header states (W1[128][16], b1[128], W2[128][128], b2[128],
    w3[128], b3[1]); BF16 rounding by torch's own conversion."""
    import torch
    f = torch.tensor(np.asarray(flat, dtype=np.float64))
    sizes = [128 * 16, 128, 128 * 128, 128, 128, 1]
    W1, b1, W2, b2, w3, b3 = torch.split(f, sizes)
    rnd = (lambda t: t.to(torch.bfloat16).to(torch.float64)) if bf16 else (lambda t: t)
    l1 = torch.nn.Linear(16, 128, dtype=torch.float64)
    l2 = torch.nn.Linear(128, 128, dtype=torch.float64)
    l3 = torch.nn.Linear(128, 1, dtype=torch.float64)
    with torch.no_grad():
        l1.weight.copy_(rnd(W1.view(128, 16)))
        l1.bias.copy_(b1)
        l2.weight.copy_(rnd(W2.view(128, 128)))
        l2.bias.copy_(b2)
        l3.weight.copy_(rnd(w3.view(1, 128)))
        l3.bias.copy_(b3)

    def run(x):
        with torch.no_grad():
            h1 = torch.relu(l1(rnd(torch.tensor(x, dtype=torch.float64))))
            h2 = torch.relu(l2(rnd(h1)))
            return l3(h2)[:, 0].numpy()
    return run


@pytest.mark.parametrize("bf16", [False, True])
def test_forward_matches_torch_modules(bf16):
    """forward() against torch.nn.Linear / ReLU built from the same flat
    parameters (non-zero biases, so a dropped bias or a misplaced ReLU fails)."""
    rng = np.random.default_rng(7)
    flat = P.init_params(5) + rng.normal(scale=0.05, size=P.N_PARAMS)
    Xn = rng.normal(size=(300, P.N_FEAT)) * 2.0
    s, _ = P.forward(flat, Xn, emulate_bf16=bf16)
    ref = _torch_net(flat, bf16)(Xn)
    assert np.max(np.abs(s - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))
    assert np.std(ref) > 0.1  # the scores actually vary


def test_forward_hand_cases():
    """A network whose output is known in closed form: unit 0 of each layer
    passes x0 - 1 through both ReLUs, the output adds b3."""
    p = {name: np.zeros(shp) for name, shp in P.SHAPES}
    p["W1"][0, 0] = 1.0
    p["b1"][0] = -1.0
    p["W2"][0, 0] = 2.0
    p["b2"][0] = 0.5
    p["w3"][0] = 3.0
    p["b3"][0] = 0.25
    x = np.zeros((4, P.N_FEAT))
    x[:, 0] = [-2.0, 0.5, 1.0, 3.0]
    s, _ = P.forward(P.pack(p), x)
    # h1 = relu(x0 - 1), h2 = relu(2 h1 + 0.5), s = 3 h2 + 0.25
    h1 = np.maximum(x[:, 0] - 1.0, 0.0)
    assert np.array_equal(s, 3.0 * np.maximum(2.0 * h1 + 0.5, 0.0) + 0.25)
    assert list(s) == [1.75, 1.75, 1.75, 3.0 * 4.5 + 0.25]


def test_gradient_central_differences():
    rng = np.random.default_rng(1)
    flat = P.init_params(3) + rng.normal(scale=0.01, size=P.N_PARAMS)
    offs, tg = _lists(rng, [9, 15, 6])
    Xn = rng.normal(size=(offs[-1], P.N_FEAT))

    def loss(f):
        s, _ = P.forward(f, Xn)
        return P.listwise_ce(s, offs, tg)[0]

    s, cache = P.forward(flat, Xn)
    _, ds = P.listwise_ce(s, offs, tg)
    g = P.backward(flat, cache, ds)
    idx = np.concatenate([rng.choice(P.N_PARAMS, 300, replace=False),
                          [P.N_PARAMS - 1, 2048, 18560, 18700]])  # every block
    h = 1e-6
    for i in idx:
        e = np.zeros(P.N_PARAMS)
        e[i] = h
        fd = (loss(flat + e) - loss(flat - e)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])), (i, fd, g[i])


def test_listwise_ce_closed_forms():
    rng = np.random.default_rng(2)
    sizes = [5, 8, 3]
    offs, tg = _lists(rng, sizes)
    loss, ds = P.listwise_ce(np.zeros(offs[-1]), offs, tg)
    assert abs(loss - np.mean(np.log(sizes))) < 1e-15
    for L, m in enumerate(sizes):
        seg = ds[offs[L]:offs[L + 1]]
        assert abs(seg.sum()) < 1e-15
        assert abs(ds[tg[L]] - (1 / m - 1) / 3) < 1e-15
    # a dominant target score gives a loss near 0
    s = np.zeros(offs[-1])
    s[tg] = 50.0
    assert P.listwise_ce(s, offs, tg)[0] < 1e-20


def test_listwise_ce_soft_pins():
    """Soft targets: one-hot weights give the hard loss and gradient; uniform
    weights on zero scores give loss log m (cross-entropy of a uniform target
    against a uniform prediction) and zero gradient; scaling a list's weights
    changes nothing; the gradient matches central differences of the loss."""
    rng = np.random.default_rng(4)
    sizes = [6, 11, 4]
    offs, tg = _lists(rng, sizes)
    s = rng.normal(size=offs[-1])
    w = np.zeros(offs[-1])
    w[tg] = 1.0
    l_h, d_h = P.listwise_ce(s, offs, tg)
    l_s, d_s = P.listwise_ce_soft(s, offs, w)
    assert abs(l_h - l_s) < 1e-14 and np.max(np.abs(d_h - d_s)) < 1e-15
    l_u, d_u = P.listwise_ce_soft(np.zeros(offs[-1]), offs, np.ones(offs[-1]))
    assert abs(l_u - np.mean(np.log(sizes))) < 1e-15 and np.max(np.abs(d_u)) < 1e-16
    w2 = rng.uniform(0.0, 2.0, size=offs[-1])
    sc = w2.copy()
    for L in range(len(sizes)):
        sc[offs[L]:offs[L + 1]] *= 10.0 ** L
    a = P.listwise_ce_soft(s, offs, w2)
    b = P.listwise_ce_soft(s, offs, sc)
    assert abs(a[0] - b[0]) < 1e-13 and np.max(np.abs(a[1] - b[1])) < 1e-15
    h = 1e-6
    for i in range(offs[-1]):
        e = np.zeros(offs[-1])
        e[i] = h
        fd = (P.listwise_ce_soft(s + e, offs, w2)[0] - P.listwise_ce_soft(s - e, offs, w2)[0]) / (2 * h)
        assert abs(fd - a[1][i]) < 1e-8


def test_lower_bounds_are_bounds():
    """The learned step's bound never exceeds k, adding witness columns never
    lowers it, and when the candidates and witnesses cover every column it is
    k itself (for every non-candidate)."""
    s = synth.er_sem(14, 1500, indeg=2.5, noise_family=("uniform", "laplace"), seed=9)
    U = list(range(14))
    X = s.X.astype(np.float32).astype(np.float64)
    D = oracle.pair_matrix(X, U)
    neg = np.minimum(D, 0.0)
    k = np.sum(neg * neg, axis=1)
    C = np.array([2, 7, 11])
    lb0 = P.lower_bounds(D, C)
    lb4 = P.lower_bounds(D, C, P.witnesses(X, U, 4))
    full = P.lower_bounds(D, C, P.witnesses(X, U, 13))
    notc = np.setdiff1d(np.arange(14), C)
    assert np.all(lb0[notc] <= lb4[notc] + 1e-18)
    assert np.all(lb4[notc] <= k[notc] * (1 + 1e-12))
    assert np.max(np.abs(full[notc] - k[notc])) <= 1e-12 * np.max(k)
    wit = P.witnesses(X, U, 3)
    Z = (X - X.mean(0)) / X.std(0)
    a = np.abs(Z.T @ Z / X.shape[0])
    for p in range(14):
        others = [q for q in range(14) if q != p]
        top = sorted(others, key=lambda q: -a[p, q])[:3]
        assert list(wit[p]) == top


def test_extension_bounds_pins():
    """The extension columns keep the bound a bound: it never exceeds k; with
    candidates, witnesses and extension covering every column it is k itself
    (a witness inside the extension is counted once, not twice); only the
    listed suspects change; and a hand-made 4 x 4 case gives the sum of the
    negative squares of the added, non-witness columns."""
    s = synth.er_sem(16, 1500, indeg=2.5, noise_family=("uniform", "laplace"), seed=12)
    U = list(range(16))
    X = s.X.astype(np.float32).astype(np.float64)
    D = oracle.pair_matrix(X, U)
    k = np.sum(np.minimum(D, 0.0) ** 2, axis=1)
    C = np.array([1, 5, 9])
    notc = np.setdiff1d(np.arange(16), C)
    wit = P.witnesses(X, U, 3)
    lb = P.lower_bounds(D, C, wit)
    S = notc[::2]
    E = notc[:6]
    lb2 = P.extension_bounds(D, lb, S, E, wit)
    assert np.all(lb2[notc] <= k[notc] * (1 + 1e-12))
    assert np.all(lb2[S] >= lb[S]) and np.array_equal(np.delete(lb2, S), np.delete(lb, S))
    full = P.extension_bounds(D, lb, notc, notc, wit)     # every column covered
    assert np.max(np.abs(full[notc] - k[notc])) <= 1e-12 * np.max(k)
    # hand case: R antisymmetric, candidate {0}, suspect 2 with witness 3
    R = np.array([[0.0, 0.5, 0.2, 0.1],
                  [-0.5, 0.0, 0.3, -0.4],
                  [-0.2, -0.3, 0.0, -0.7],
                  [-0.1, 0.4, 0.7, 0.0]])
    w = np.array([[-1], [-1], [3], [-1]])
    lb_h = P.lower_bounds(R, np.array([0]), w)
    assert abs(lb_h[2] - (0.2 ** 2 + 0.7 ** 2)) < 1e-15   # max(0, R(0,2))^2 + min(0, R(2,3))^2
    got = P.extension_bounds(R, lb_h, [2], [1, 2, 3], w)
    assert abs(got[2] - (lb_h[2] + 0.3 ** 2)) < 1e-15      # only column 1 is new
    assert got[1] == lb_h[1] and got[3] == lb_h[3]


def test_adam_first_step_and_convergence():
    rng = np.random.default_rng(3)
    x = rng.normal(size=50)
    g = rng.normal(size=50)
    opt = P.Adam(lr=0.01)
    x1 = opt.step(x, g)
    # bias-corrected first step: -lr * g / (|g| + eps)
    assert np.allclose(x1 - x, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    # minimises a convex quadratic
    c = rng.normal(size=50)
    opt = P.Adam(lr=0.05)
    y = np.zeros(50)
    for _ in range(3000):
        y = opt.step(y, 2 * (y - c))
    assert np.max(np.abs(y - c)) < 5e-3  # from O(1) at the start


def test_topk_brute_force():
    rng = np.random.default_rng(4)
    s = rng.integers(0, 20, 200).astype(np.float64)  # many ties
    slots = rng.permutation(200)
    C = P.topk(s, slots, 37)
    ref = sorted(range(200), key=lambda p: (-s[p], slots[p]))[:37]
    assert list(C) == ref


def test_certificate_is_sound():
    """LB_l <= k_l for every excluded l, and a certified best candidate is the
    plain choice (checked on the full measure matrix at several steps)."""
    s = synth.er_sem(14, 1500, indeg=2.0, noise_family=("uniform", "laplace", "exp"), seed=7)
    X = s.X.astype(np.float64)
    rng = np.random.default_rng(5)
    U = list(range(14))
    checked = 0
    for step in range(6):
        D = oracle.pair_matrix(X, U)
        k = np.sum(np.minimum(D, 0) ** 2, axis=1)
        for trial in range(20):
            C = rng.choice(len(U), 4, replace=False)
            excl = np.setdiff1d(np.arange(len(U)), C)
            lb = np.sum(np.maximum(D[C], 0) ** 2, axis=0)
            assert np.all(lb[excl] <= k[excl] + 1e-15)
            best = C[np.argmin(k[C])]
            if np.all(lb[excl] > k[best]):
                assert best == int(np.argmin(k))
                checked += 1
        e = U[int(np.argmin(k))]
        X = oracle.residualize(X, U, e)
        U.remove(e)
    assert checked > 0


def test_step_topk():
    assert P.step_topk(4096, 256) == 256
    assert P.step_topk(2000, 256) == 128
    assert P.step_topk(1024, 256) == 64
    assert P.step_topk(300, 256) == 32
    assert P.step_topk(600, 64) == 40
    assert P.step_topk(4096, 64) == 64
    assert P.step_topk(100, 8) == 8
    assert P.step_topk(1000, 3) == 3


def test_suspect_cap():
    assert P.suspect_cap(200, 64) == 32
    assert P.suspect_cap(130, 64) == 0
    assert P.suspect_cap(4096, 64) == 1024
    assert P.suspect_cap(1000, 8) == 488


@pytest.mark.parametrize("seed", [0, 1])
def test_learned_order_reduces_to_plain(seed):
    """With delta = +inf (suspects evaluated, or the full step), or with an
    audit at every step, the learned form must give exactly the plain order."""
    s = synth.er_sem(12, 1000, indeg=2.0, noise_family=("uniform", "laplace", "exp"),
                     seed=20 + seed)
    plain = oracle.causal_order(s.X, mode="table")
    prop = np.concatenate([np.zeros(16), np.ones(16), P.init_params(seed)])
    o1, info1 = P.learned_order(s.X, prop, K=3, delta=np.inf, audit_every=0, min_m=3)
    assert np.array_equal(o1, plain)
    kinds = {i.kind for i in info1}
    assert "learned" in kinds or "fallback" in kinds
    o2, info2 = P.learned_order(s.X, prop, K=3, delta=-np.inf, audit_every=1, min_m=3)
    assert np.array_equal(o2, plain)
    o3, info3 = P.learned_order(s.X, prop, K=3, delta=-np.inf, audit_every=0, min_m=3)
    assert sorted(o3) == list(range(12))
    assert all(i.kind in ("learned", "plain", "expanded") for i in info3)
    # certified and expanded steps take the plain choice of that step
    assert all(i.learned_choice == i.plain_choice for i in info3 if i.certified)
    assert all(i.chosen == i.plain_choice for i in info3 if i.kind == "expanded")
    # without the second pass (cap 0) uncertified steps follow the margin rule
    o4, info4 = P.learned_order(s.X, prop, K=3, delta=np.inf, audit_every=0, min_m=3,
                                max_suspects=0)
    assert np.array_equal(o4, plain)
    assert not any(i.kind == "expanded" for i in info4)
    # the extension columns only shrink the rows measured, never the order
    o5, info5 = P.learned_order(s.X, prop, K=3, delta=np.inf, audit_every=0, min_m=3,
                                n_ext=2)
    assert np.array_equal(o5, plain)
    ex1 = [i for i in info1 if i.kind == "expanded"]
    ex5 = [i for i in info5 if i.kind == "expanded"]
    assert [i.suspects for i in ex1] == [i.suspects for i in ex5]
    assert all(i.rows == i.suspects for i in ex1)
    assert all(i.rows <= i.suspects for i in ex5)


def test_kendall_tau_matches_scipy():
    rng = np.random.default_rng(6)
    n = 300
    a = rng.permutation(n)
    assert P.kendall_tau(a, a) == 1.0
    assert P.kendall_tau(a, a[::-1]) == -1.0
    for _ in range(5):
        b = a.copy()
        sw = rng.choice(n - 1, 30)
        for i in sw:
            b[i], b[i + 1] = b[i + 1], b[i]
        pa = np.empty(n)
        pb = np.empty(n)
        pa[a] = np.arange(n)
        pb[b] = np.arange(n)
        assert abs(P.kendall_tau(a, b) - stats.kendalltau(pa, pb)[0]) < 1e-12
