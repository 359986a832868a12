"""GPU VarLiNGAM (Section 3.2) against the FP64 oracle, through the C ABI.

The oracle receives the same FP32 series (cast to FP64).  VAR coefficients
and B0 are compared element by element; the residual ordering is compared
teacher-forced along the GPU order with the measure tolerance of the
ordering tests, and the free-running orders must agree outside near-ties.
"""
import numpy as np
import pytest

import oracle
from paper_2403_03772_amd import synth
from gpu_helpers import check_step

pytestmark = pytest.mark.gpu


def _gpu(lib, X32, lags, **kw):
    import torch
    out = lib.varlingam_fit(torch.as_tensor(X32).cuda(), lags, **kw)
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items()}


@pytest.mark.parametrize("d,T,lags,seed", [(5, 400, 1, 0), (12, 1000, 2, 1), (70, 900, 1, 2),
                                           (33, 2000, 3, 3)])
def test_varlingam_matches_oracle(lib, d, T, lags, seed):
    v = synth.var_series(d=d, T=T, seed=seed)
    X32 = v.X.astype(np.float32)
    print(f"case d={d} T={T} lags={lags}", flush=True)
    g = _gpu(lib, X32, lags, with_measures=True)
    ref = oracle.varlingam(X32.astype(np.float64), lags=lags)
    # VAR coefficients and residuals
    scale = np.max(np.abs(ref["M"]))
    assert np.max(np.abs(g["M"] - ref["M"])) <= 1e-9 * max(scale, 1.0)
    assert np.max(np.abs(g["resid"] - ref["resid"])) <= 1e-5 * np.max(np.abs(ref["resid"]))
    # ordering of the residuals, teacher-forced along the GPU order
    order = g["order"]
    assert sorted(order.tolist()) == list(range(d))
    o_ref, mr, _ = oracle._order_fp64(ref["resid"], order, True)
    for t in range(d - 1):
        bad, ok = check_step(g["measures"][t], mr[t], order[t])
        assert bad == 0, f"step {t}: {bad} measures outside tolerance"
        assert ok, f"step {t}: choice outside a near-tie"
    # B0 on the GPU order
    b_ref = oracle.ols_adjacency(ref["resid"], order)
    assert np.max(np.abs(g["B0"] - b_ref)) <= 1e-8 * max(1.0, np.max(np.abs(b_ref)))
    # lagged effects (I - B0) M_tau from the GPU's own M and B0
    th_ref = oracle.var_lagged_effects(g["M"], g["B0"])
    assert np.max(np.abs(g["theta"] - th_ref)) <= 1e-12 * max(1.0, np.max(np.abs(th_ref)))


STOCK_STEPS = (0, 1, 2, 50, 150, 300, 420, 480, 485)


def test_varlingam_stock_shape(lib):
    """The stock-shaped workload (d = 487, T = 1258, VAR(1), t4 noise; Section
    3.2): VAR coefficients, B0 over 16 Cholesky panels, and the ordering of the
    residuals: at sampled steps the oracle (table mode, FP64 residuals of its
    own VAR fit) measures every active variable, teacher-forced along the GPU
    order; every measure must be within tolerance and the GPU's choice must
    be the oracle's argmax outside near-ties."""
    d = 487
    v = synth.var_series(d=d, T=1258, seed=0)
    X32 = v.X.astype(np.float32)
    g = _gpu(lib, X32, 1, with_measures=True)
    coef, resid = oracle.var_fit(X32.astype(np.float64), 1)
    assert np.max(np.abs(g["M"][0] - coef[1:].T)) <= 1e-8 * max(1.0, np.max(np.abs(coef)))
    order = g["order"]
    assert sorted(order.tolist()) == list(range(d))
    b_ref = oracle.ols_adjacency(resid, order)
    assert np.max(np.abs(g["B0"] - b_ref)) <= 1e-8 * max(1.0, np.max(np.abs(b_ref)))
    worst = 0.0
    for t in STOCK_STEPS:
        print(f"stock shape: oracle step {t}", flush=True)
        ref = oracle.step_measures_all(resid, order[:t], fp64=True)
        got = g["measures"][t]
        bad, ok = check_step(got, ref, order[t])
        ids = np.flatnonzero(np.isfinite(ref))
        s_t = 1e-3 * np.max(np.abs(ref[ids]))
        err = np.abs(got[ids] - ref[ids]) / np.maximum(np.abs(ref[ids]), s_t)
        worst = max(worst, float(err.max()))
        assert bad == 0, f"step {t}: {bad} measures outside tolerance (worst {err.max():.2e})"
        assert ok, f"step {t}: choice {order[t]} outside a near-tie of the oracle's argmax"
    print(f"stock shape: worst scaled measure error {worst:.3e} over steps {STOCK_STEPS}")


def test_varlingam_errors(lib):
    import torch
    X = torch.randn((10, 6), device="cuda")
    with pytest.raises(lib.LingamError):
        lib.varlingam_fit(X, 2)     # T - lags = 8 <= 1 + 2 * 6 regressors
    Y = torch.randn((300, 4), device="cuda")
    Y[:, 2] = Y[:, 1]               # collinear regressors
    with pytest.raises(lib.LingamError) as e:
        lib.varlingam_fit(Y, 1)
    assert e.value.code == -2
