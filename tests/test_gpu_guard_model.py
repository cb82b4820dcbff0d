"""GPU: what the trained guard-width network gains over the plain comparison.

The committed network (paper_1812_07357_amd/data/guard_model.npz, trained by
the library's own kernels on solver-generated runs) picks n_g for fresh runs;
the plain local-vs-global comparison judges the pick and steps n_g up until
it passes.  Against the plain method (scan n_g upwards, one comparison run per
candidate) the result must be just as safe -- it passes the tolerance whenever
the scan finds any passing n_g, and is never below the scan's smallest
passing n_g -- while needing fewer comparison runs in total.  Against the
trivial rule that always takes the largest candidate (safe in one call), it
must transform fewer cells: its boxes average under 0.9 of the largest
candidate's, and it lands on the scan's optimum or the next width up.
"""

import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MODEL = os.path.join(ROOT, "paper_1812_07357_amd", "data", "guard_model.npz")
DATA = os.path.join(ROOT, "paper_1812_07357_amd", "data", "guard_data.npz")


def test_network_choice_is_safe_and_needs_fewer_comparisons(lib):
    from paper_1812_07357_amd import guard_model as gm

    model = gm.load(MODEL)
    lvg = gm.LocalVsGlobal(domain=64, split=2, precision="fp64")
    runs = [gm.Run(16, 0.5, 16.0, 0.1), gm.Run(64, 0.7, 24.0, 0.2), gm.Run(128, 0.4, 12.0, 0.15)]
    tol, steps = 1e-4, 32
    calls_model = calls_plain = 0
    ratios, close = [], []
    for i, run in enumerate(runs):
        g1 = lvg.fields(run, synth.rng_for(600, i))
        r = gm.compare(model, lvg, run, g1, steps, tol)
        g_plain = r["plain"]["nguard"]
        g_model = r["model"]["nguard"]
        print(run, r["pick"], r["model"], r["plain"], r.get("cells_ratio_vs_largest"), flush=True)
        if g_plain is not None:
            assert g_model is not None and g_model >= g_plain
            assert r["model"]["log10_err"] <= np.log10(tol)
            # the choice is the scan's optimum or the next candidate up
            close.append(gm.GUARDS.index(g_model) - gm.GUARDS.index(g_plain) <= 1)
            ratios.append(r["cells_ratio_vs_largest"])
        calls_model += r["model"]["judge_calls"]
        calls_plain += r["plain"]["judge_calls"]
    assert calls_model < calls_plain, (calls_model, calls_plain)
    # Against the trivial rule "always take the largest guard" (one judge call, always safe,
    # cells ratio 1): the network's boxes are smaller, i.e. it saves transformed cells.
    print(f"judge calls {calls_model} vs {calls_plain}; box cells vs the largest guard: {ratios}", flush=True)
    assert ratios and float(np.mean(ratios)) < 0.9, ratios
    assert sum(close) >= len(close) - 1, close
    model.mlp.close()


def test_training_on_solver_data_generalises(lib):
    """The library's kernels fit the committed solver-generated data: held-out RMSE well below the label spread."""
    from paper_1812_07357_amd import guard_model as gm

    z = np.load(DATA, allow_pickle=False)
    model, (tr, va, te) = gm.train(z["X"], z["y"], z["run"], np.random.default_rng(11), steps=4000, batch=512)
    y = np.minimum(z["y"], gm.LABEL_CAP)
    spread = float(np.std(y[te]))
    assert model.metrics["rmse_test"] < 0.2 * spread, (model.metrics, spread)
    assert model.metrics["loss_last"] < 0.05 * model.metrics["loss_first"]
    model.mlp.close()
