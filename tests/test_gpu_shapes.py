"""Launch shapes of the pair kernels (waves per workgroup: 1, 2 or 4) change
only how the 4 x 4 quadrants of a tile are grouped into workgroups, never the
samples a wave sums or their order, so every result must be bit for bit the
same under every shape: the plain ordering's order and every measure, the
learned form's order, decisions and recorded measures, and a batch.  Each
case prints its shape before running."""
import numpy as np
import pytest

from paper_2403_03772_amd import synth

pytestmark = pytest.mark.gpu

SHAPES = [(4, 4), (2, 2), (1, 1), (1, 4), (4, 1)]


def _plain(lib, X, waves):
    out = lib.causal_order(X, with_measures=True, waves=waves)
    return out["order"].cpu().numpy(), out["measures"].cpu().numpy()


def test_plain_ordering_is_shape_invariant(lib):
    import torch
    s = synth.er_sem(130, 1000, indeg=2.0, noise_family=("uniform", "laplace", "exp"), seed=11)
    X = torch.as_tensor(s.X.astype(np.float32)).cuda()
    ref = None
    for w in SHAPES:
        print(f"plain d=130 n=1000 waves={w}", flush=True)
        o, m = _plain(lib, X, w)
        if ref is None:
            ref = (o, m)
            continue
        assert np.array_equal(o, ref[0]), w
        assert np.array_equal(m, ref[1], equal_nan=True), w


def test_learned_form_is_shape_invariant(lib):
    import torch
    from oracle import proposer as op
    s = synth.er_sem(300, 3000, indeg=2.0, noise_family=("uniform", "laplace", "exp"), seed=12)
    X = torch.as_tensor(s.X.astype(np.float32)).cuda()
    prop = torch.zeros(lib.PROPOSER_SIZE, dtype=torch.float32, device="cuda")
    prop[16:32] = 1.0
    prop[32:] = torch.as_tensor(op.init_params(3).astype(np.float32)).cuda()
    cfg = lib.Learned(prop, topk=16, min_m=128, audit_every=7)
    ref = None
    for w in SHAPES:
        print(f"learned d=300 n=3000 waves={w}", flush=True)
        out = lib.causal_order(X, learned=cfg, with_measures=True, step_log=True, waves=w)
        st = out["learned_stats"]
        got = (out["order"].cpu().numpy(), out["measures"].cpu().numpy(),
               out["step_log"].cpu().numpy(),
               (st.learned_steps, st.certified, st.expanded, st.audits, st.rows_sum))
        if ref is None:
            ref = got
            assert st.learned_steps > 0 and st.expanded > 0
            continue
        assert np.array_equal(got[0], ref[0]), w
        assert np.array_equal(got[1], ref[1], equal_nan=True), w
        assert np.array_equal(got[2], ref[2]), w
        assert got[3] == ref[3], w


def test_batch_is_shape_invariant(lib):
    import torch
    sems = [synth.er_sem(d, n, indeg=2.0, noise_family=("uniform", "laplace"), seed=d)
            for d, n in ((70, 900), (150, 2000), (33, 640))]
    jobs = [{"X": torch.as_tensor(s.X.astype(np.float32)).cuda()} for s in sems]
    ref = None
    for w in SHAPES:
        print(f"batch of 3 waves={w}", flush=True)
        out = lib.batch_causal_order(jobs, with_measures=True, waves=w)
        got = [o.cpu().numpy() for o in out["orders"]], \
            [m.cpu().numpy() for m in out["measures"]]
        if ref is None:
            ref = got
            continue
        for a, b in zip(got[0], ref[0]):
            assert np.array_equal(a, b), w
        for a, b in zip(got[1], ref[1]):
            assert np.array_equal(a, b, equal_nan=True), w
