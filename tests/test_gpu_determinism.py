"""GPU: the step is a pure function of the fields it is given.

* Run twice from the same input, the same plan gives bitwise the same fields.
* Checkpoint / resume: 2N steps equal N steps, a save of the eleven G1 arrays
  to a file, a fresh plan loading them, and N more steps -- bitwise.  The plan
  carries nothing from one step to the next besides its tables.
* Poisoned workspaces: a step on NaN-filled fields leaves NaN in every
  workspace byte the step writes; a following step on clean fields must equal
  a fresh plan's step bitwise (no step reads a workspace value it did not write
  in the same step).  The same for a batch, and for the no-allocation entry
  point's shared static workspace.
"""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

INTERIOR, NG, ORDER = (96, 80, 72), 8, 16


def _fields(shape, seed):
    return synth.random_fields(synth.rng_for(180, seed), shape, 11, 1.0)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_run_twice_and_checkpoint_resume_are_bitwise(lib, precision, tmp_path):
    import torch

    gshape = INTERIOR[::-1]
    host = _fields(gshape, 0)
    plan = lib.Plan(*INTERIOR, nguard=NG, order=ORDER, dx=1.0, dt=0.5, precision=precision)
    runs = []
    for _ in range(2):
        g = torch.as_tensor(host, dtype=plan.dtype, device="cuda")
        for _ in range(6):
            plan.step_g1(g, (0, 0, 0))
        torch.cuda.synchronize()
        runs.append(g.cpu().numpy())
    assert np.array_equal(runs[0], runs[1])
    g = torch.as_tensor(host, dtype=plan.dtype, device="cuda")
    for _ in range(3):
        plan.step_g1(g, (0, 0, 0))
    torch.cuda.synchronize()
    path = tmp_path / "checkpoint.npy"
    np.save(path, g.cpu().numpy())
    plan.close()
    del g
    plan2 = lib.Plan(*INTERIOR, nguard=NG, order=ORDER, dx=1.0, dt=0.5, precision=precision)
    g = torch.as_tensor(np.load(path), device="cuda")
    for _ in range(3):
        plan2.step_g1(g, (0, 0, 0))
    torch.cuda.synchronize()
    assert np.array_equal(g.cpu().numpy(), runs[0])
    plan2.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_poisoned_workspace_does_not_leak_into_the_next_step(lib, precision):
    import torch

    gshape = INTERIOR[::-1]
    host = _fields(gshape, 1)
    fresh = lib.Plan(*INTERIOR, nguard=NG, order=ORDER, dx=1.0, dt=0.5, precision=precision)
    ref = torch.as_tensor(host, dtype=fresh.dtype, device="cuda")
    fresh.step_g1(ref, (0, 0, 0))
    torch.cuda.synchronize()
    fresh.close()
    plan = lib.Plan(*INTERIOR, nguard=NG, order=ORDER, dx=1.0, dt=0.5, precision=precision)
    bad = torch.full((11,) + gshape, float("nan"), dtype=plan.dtype, device="cuda")
    plan.step_g1(bad, (0, 0, 0))
    torch.cuda.synchronize()
    assert bool(torch.isnan(bad[0:6]).all())
    g = torch.as_tensor(host, dtype=plan.dtype, device="cuda")
    plan.step_g1(g, (0, 0, 0))
    torch.cuda.synchronize()
    assert np.array_equal(g.cpu().numpy(), ref.cpu().numpy())
    plan.close()


def test_poisoned_batch_workspaces_do_not_leak(lib):
    import torch

    gdims = (44, 36, 30)
    boxes = [dict(origin=(0, 0, 0), interior=(20, 36, 30), nguard=6, order=8),
             dict(origin=(20, 0, 0), interior=(24, 17, 30), nguard=(4, 9, 3), order=0),
             dict(origin=(20, 17, 0), interior=(24, 19, 30), nguard=5, order=16)]
    host = _fields(gdims[::-1], 2)
    fresh = lib.Batch(boxes, gdims, dt=0.5)
    ref = torch.as_tensor(host, dtype=torch.float32, device="cuda")
    fresh.step(ref)
    torch.cuda.synchronize()
    fresh.close()
    batch = lib.Batch(boxes, gdims, dt=0.5)
    bad = torch.full((11,) + gdims[::-1], float("nan"), dtype=torch.float32, device="cuda")
    batch.step(bad)
    g = torch.as_tensor(host, dtype=torch.float32, device="cuda")
    batch.step(g)
    torch.cuda.synchronize()
    assert np.array_equal(g.cpu().numpy(), ref.cpu().numpy())
    batch.close()


def test_poisoned_static_workspace_does_not_leak(lib):
    import torch

    interior = (40, 36, 28)
    host = _fields(interior[::-1], 3)
    plan = lib.Plan(*interior, nguard=4, order=8, dt=0.5)
    ref = torch.as_tensor(host, dtype=torch.float32, device="cuda")
    plan.step_g1(ref, (0, 0, 0))
    bad = torch.full_like(ref, float("nan"))
    plan.step_g1_noalloc(bad, (0, 0, 0))
    g = torch.as_tensor(host, dtype=torch.float32, device="cuda")
    plan.step_g1_noalloc(g, (0, 0, 0))
    torch.cuda.synchronize()
    assert np.array_equal(g.cpu().numpy(), ref.cpu().numpy())
    plan.close()
