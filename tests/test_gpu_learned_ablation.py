"""What the trained proposer gains over the same learned form without it.

The shipped network and an untrained (random) network run the learned form
with identical K, audit period and margin on a held-out SEM of the training
family.  The trained network must be certified more often, leave fewer
suspects for the second pass (less exact work: the suspects' rows are what
exactness costs beyond the candidates) and keep the order within Kendall tau
0.99 of the plain order.
"""
import os

import numpy as np
import pytest

from paper_2403_03772_amd import synth
from paper_2403_03772_amd import train_proposer as tp

pytestmark = pytest.mark.gpu


def _tau(a, b):
    from scipy import stats
    pa = np.empty(len(a))
    pb = np.empty(len(b))
    pa[a] = np.arange(len(a))
    pb[b] = np.arange(len(b))
    return float(stats.kendalltau(pa, pb)[0])


@pytest.mark.skipif(not os.path.exists(tp.WEIGHTS), reason="no trained network shipped")
def test_trained_network_beats_untrained(lib):
    import torch
    s = synth.workload_gene_scale(seed=7, d=512, n=4096)
    X = torch.as_tensor(np.ascontiguousarray(s.X, dtype=np.float32)).cuda()
    plain = lib.causal_order(X).cpu().numpy()
    prop = tp.default_proposer()
    raw = prop.clone()
    raw[32:] = torch.as_tensor(tp.init_weights(1), device=raw.device)
    res = {}
    for name, P in (("trained", prop), ("untrained", raw)):
        out = lib.causal_order(X, learned=lib.Learned(P))
        st = out["learned_stats"]
        res[name] = {"tau": _tau(out["order"].cpu().numpy(), plain),
                     "certified": st.certified, "fallbacks": st.fallbacks,
                     "suspects": st.suspects_sum, "steps": st.learned_steps,
                     "audits": st.audits, "audit_agree": st.audit_agree}
    print(res, flush=True)
    tr, un = res["trained"], res["untrained"]
    assert tr["certified"] > un["certified"]
    assert tr["suspects"] < un["suspects"]
    assert tr["fallbacks"] <= un["fallbacks"]
    assert tr["tau"] >= 0.99
