"""lingam_causal_order_noalloc (the ordering for callers that cannot allocate)
against lingam_causal_order, through the C ABI: two calls in a row, the second
on a smaller input, then a learned-form call and a larger one again (the
scratch array keeps the previous call's contents, which must not leak into the
next result); sizes beyond the scratch array and the options that would
allocate are refused before any device work."""
import numpy as np
import pytest

from paper_2403_03772_amd import synth

pytestmark = pytest.mark.gpu


def _pair(lib, X, **kw):
    ref = lib.causal_order(X, with_measures=True, **kw)
    got = lib.causal_order_noalloc(X, with_measures=True, **kw)
    return ref, got


def _check(ref, got, label):
    o_ref, o_got = ref["order"].cpu().numpy(), got["order"].cpu().numpy()
    assert np.array_equal(o_ref, o_got), label
    m_ref, m_got = ref["measures"].cpu().numpy(), got["measures"].cpu().numpy()
    assert np.array_equal(np.isnan(m_ref), np.isnan(m_got)), label
    fin = np.isfinite(m_ref)
    # same kernels and launch plan, other workspace address: the same numbers
    assert np.array_equal(m_ref[fin], m_got[fin]), label
    print(f"{label}: order and every measure identical", flush=True)


@pytest.mark.parametrize("seed", [0])
def test_noalloc_matches_causal_order(lib, seed):
    import torch
    cases = [(200, 3000), (37, 777), (300, 4000)]
    for k, (d, n) in enumerate(cases):
        s = synth.er_sem(d, n, indeg=2.0, noise_family=("uniform", "laplace", "exp"),
                         seed=seed * 100 + k)
        X = torch.as_tensor(s.X.astype(np.float32)).cuda()
        print(f"noalloc case d={d} n={n}", flush=True)
        ref, got = _pair(lib, X)
        _check(ref, got, f"d={d} n={n}")
    # the learned form (exact mode) through the scratch array
    s = synth.er_sem(260, 3000, indeg=2.0, noise_family=("uniform", "laplace", "exp"), seed=7)
    X = torch.as_tensor(s.X.astype(np.float32)).cuda()
    raw = torch.zeros(lib.PROPOSER_SIZE, dtype=torch.float32, device="cuda")
    raw[16:32] = 1.0
    from oracle import proposer as op
    raw[32:] = torch.as_tensor(op.init_params(0).astype(np.float32)).cuda()
    cfg = lib.Learned(raw, topk=16, min_m=128)
    print("noalloc case learned d=260 n=3000", flush=True)
    ref, got = _pair(lib, X, learned=cfg)
    _check(ref, got, "learned d=260 n=3000")


def test_noalloc_refuses_what_it_cannot_hold(lib):
    import torch
    X = torch.zeros((8192, 1024), dtype=torch.float32, device="cuda")
    with pytest.raises(lib.LingamError) as e:
        lib.causal_order_noalloc(X)
    from paper_2403_03772_amd import lib as L
    assert e.value.code == L.E_UNSUPPORTED and "scratch" in str(e.value)
    X = torch.randn((500, 20), dtype=torch.float32, device="cuda")
    from paper_2403_03772_amd import lib as L
    with pytest.raises(lib.LingamError) as e:
        L.causal_order(X, graph=True, _noalloc=True)
    assert e.value.code == L.E_UNSUPPORTED
