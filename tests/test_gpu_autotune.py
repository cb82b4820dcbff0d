"""GPU: the schedule autotuner keeps results correct and caches its choices."""

import json
import os

import numpy as np
import pytest

import synth
from oracle import step

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_autotuned_plan_matches_oracle_and_cache_roundtrips(lib, tmp_path, precision):
    import torch

    interior, ng, order, d, dt = (56, 40, 36), 4, 16, 1.0, 0.5   # box 64 x 48 x 44
    path = str(tmp_path / "tune.json")
    plan = lib.Plan(*interior, nguard=ng, order=order, dx=d, dt=dt, precision=precision)
    plan.autotune(path)
    torch.cuda.synchronize()
    sched = [plan.schedule(a) for a in range(3)]
    for (radices, tile), n in zip(sched, plan.box):
        assert int(np.prod(radices)) == n and tile > 0
    with open(path) as f:
        cache = json.load(f)
    assert len(cache["entries"]) >= 3
    f = synth.random_fields(synth.rng_for(400, 0), plan.box_shape)
    ref = step.box_step(f, d, dt, order)
    g = torch.as_tensor(f, dtype=plan.dtype, device="cuda")
    plan.push_fields(g)
    torch.cuda.synchronize()
    err = np.abs(g[0:6].double().cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err <= (1e-12 if precision == "fp64" else 2e-5), err
    # a second plan of the same shape takes its schedules from the cache file
    plan2 = lib.Plan(*interior, nguard=ng, order=order, dx=d, dt=dt, precision=precision)
    plan2.autotune(path)
    assert [plan2.schedule(a) for a in range(3)] == sched
    plan.close()
    plan2.close()
    assert os.path.getsize(path) > 0
