"""CPU: host logic of the guard-width model (run draws, features, splits, the choice with judge and fallback)."""

import math

import numpy as np

from oracle import mlp as omlp
from paper_1812_07357_amd import guard_model as gm


def test_run_draws_follow_the_stated_ranges():
    rng = np.random.default_rng(0)
    runs = [gm.draw_run(rng) for _ in range(2000)]
    orders = np.array([r.order for r in runs])
    inf_frac = np.mean(orders == 0)
    assert 0.07 < inf_frac < 0.13
    fin = orders[orders > 0]
    assert fin.min() >= 8 and fin.max() <= 256 and np.all(fin % 2 == 0)
    assert all(0.25 <= r.cdt <= 1.0 and 10 <= r.lam <= 40 and 0.05 <= r.width <= 0.3 for r in runs)


def test_features_agree_with_the_oracle_definition():
    rng = np.random.default_rng(1)
    n = 50
    args = (rng.choice([0, 8, 16, 100], n), rng.choice(gm.GUARDS, n), rng.uniform(0.25, 1, n),
            rng.uniform(10, 40, n), rng.uniform(0.05, 0.3, n), rng.choice(gm.CHECKPOINTS, n))
    assert np.allclose(gm.features(*args), omlp.features(*args), rtol=1e-6, atol=1e-7)


def test_init_params_layout():
    p = gm.init_params(np.random.default_rng(2))
    assert p.shape == (omlp.NPARAM,) and p.dtype == np.float32
    u = omlp.unpack(p.astype(np.float64))
    assert np.all(u["b1"] == 0) and np.all(u["b2"] == 0) and u["b3"][0] == 0
    assert abs(u["W2"].std() - 1 / 8) < 0.02


def test_split_by_run_is_disjoint():
    rid = np.repeat(np.arange(100), 21).astype(np.int32)
    tr, va, te = gm.split_runs(rid, np.random.default_rng(3))
    assert not np.any(tr & va) and not np.any(tr & te) and not np.any(va & te)
    assert np.all(tr | va | te)
    for mask in (tr, va, te):
        runs = set(rid[mask].tolist())
        assert all(np.all(mask[rid == r]) for r in runs)
    assert 75 <= len(set(rid[tr].tolist())) <= 85


def test_pick_guard_smallest_safe():
    guards = (4, 8, 16, 32)
    pred = [-3.0, -5.0, -7.5, -9.0]
    assert gm.pick_guard(pred, 0.0, 1e-6, guards) == 16
    assert gm.pick_guard(pred, 2.0, 1e-6, guards) == 32
    assert gm.pick_guard(pred, 0.0, 1e-12, guards) == 32  # none safe: largest


def test_judged_fallback_and_plain_scan():
    true = {4: -3.0, 8: -5.0, 16: -6.5, 32: -9.0}
    calls = []

    def judge(g):
        calls.append(g)
        return true[g]

    guards = (4, 8, 16, 32)
    # a too-optimistic pick is stepped up until the comparison passes
    g, n, e = gm.judged(8, judge, 1e-6, guards)
    assert (g, n, e) == (16, 2, -6.5) and calls == [8, 16]
    calls.clear()
    g, n, _ = gm.plain_scan(judge, 1e-6, guards)
    assert (g, n) == (16, 3) and calls == [4, 8, 16]
    g, n, e = gm.judged(4, judge, 1e-12, guards)
    assert g is None and n == 4 and e is None
    assert math.log10(1e-6) == -6.0
