"""Host logic of the proposer's streamed training (no GPU): the SEM draws, the
list packing that feeds the replay buffer, and the resumable state."""
import numpy as np

from paper_2403_03772_amd import lib as L
from paper_2403_03772_amd import train_proposer as tp


def test_sem_specs_are_seeded_and_in_range():
    a = tp.sem_specs(200, 100, 1000, 2048, 8192, seed=3)
    b = tp.sem_specs(200, 100, 1000, 2048, 8192, seed=3)
    assert a == b and a != tp.sem_specs(200, 100, 1000, 2048, 8192, seed=4)
    d = np.array([s[0] for s in a])
    n = np.array([s[1] for s in a])
    assert d.min() >= 100 and d.max() <= 1000
    assert np.all(n >= 2 * d)                       # fewer samples would be collinear
    assert np.all((n >= 2048) & (n <= max(8192, 2 * d.max())))
    assert len({s[2] for s in a}) == len(a)         # every SEM its own seed


def test_lists_round_trip_through_the_buffer():
    rng = np.random.default_rng(0)
    sizes = rng.integers(1, 40, size=7)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    F = rng.standard_normal((offs[-1], L.N_FEATURES)).astype(np.float32)
    W = rng.random(offs[-1]).astype(np.float32)
    tg = offs[:-1] + np.array([rng.integers(0, s) for s in sizes])
    items = tp._lists(F, offs, tg, W)
    assert len(items) == len(sizes)
    F2, o2, t2, W2 = tp._stack(items)
    assert np.array_equal(F2, F) and np.array_equal(o2, offs)
    assert np.array_equal(t2, tg) and np.array_equal(W2, W)
    # a subset in another order keeps each list's rows, target and weights together
    sel = [4, 0, 6]
    F3, o3, t3, W3 = tp._stack([items[i] for i in sel])
    for k, i in enumerate(sel):
        assert np.array_equal(F3[o3[k]:o3[k + 1]], F[offs[i]:offs[i + 1]])
        assert t3[k] - o3[k] == tg[i] - offs[i]
        assert np.array_equal(W3[o3[k]:o3[k + 1]], W[offs[i]:offs[i + 1]])


def test_state_survives_a_restart(tmp_path):
    rng = np.random.default_rng(1)
    prop = rng.standard_normal(L.PROPOSER_SIZE).astype(np.float32)
    state = {"m1": rng.standard_normal(L.N_PARAMS).astype(np.float32),
             "m2": rng.random(L.N_PARAMS).astype(np.float32),
             "step": 123, "next_sem": 4672, "loss": [3.4, 3.3], "seed": 0,
             "seconds": 880.5, "init_meta": {"sems": 1000}}
    path = str(tmp_path / "state.bin")  # any name: no suffix is added
    tp._save_state(path, prop, state)
    assert (tmp_path / "state.bin").exists() and not (tmp_path / "state.bin.npz").exists()
    p2, s2 = tp._load_state(path)
    assert np.array_equal(p2, prop)
    assert np.array_equal(s2["m1"], state["m1"]) and np.array_equal(s2["m2"], state["m2"])
    for k in ("step", "next_sem", "loss", "seed", "seconds", "init_meta"):
        assert s2[k] == state[k]


def test_soft_weights_favour_the_minimum():
    w = tp.soft_weights([1.0, 1.0, 3.0, np.inf, -1.0, np.nan])
    assert w[0] == w[1] == 1.0
    assert np.isclose(w[2], (2.0 / 4.0) ** 2)
    assert w[3] == 0.0 and w[4] == 0.0 and w[5] == 0.0
