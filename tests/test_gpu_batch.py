"""GPU: batched steps of many uneven boxes (one persistent launch per pass, hipGraph replay).

Sec. 1.3 / Fig. 1(a) of arXiv:1812.07357: the global grid is split into
sub-domains with guard regions, each advanced independently with its own FFT;
guards are refreshed from the neighbours every step.  The oracle is the FP64
local-with-guards driver (every fill of a step reads the previous step's
fields, then every interior is merged).
"""

import numpy as np
import pytest

import synth
from oracle import domain, step

pytestmark = pytest.mark.gpu


def _to_gpu(a, dtype):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _small_decomposition():
    # 2 x 2 x 2 uneven split of a 30 x 26 x 22 grid; guards up to wider than a neighbour
    xs, ys, zs = (0, 17), (0, 11), (0, 9)
    wx, wy, wz = (17, 13), (11, 15), (9, 13)
    guards = [2, 5, 0, 12, 3, 7, 1, 16]
    orders = [8, 0, 4, 16, 2, 32, 6, 10]
    boxes, i = [], 0
    for k in range(2):
        for j in range(2):
            for l in range(2):
                boxes.append({"origin": (xs[l], ys[j], zs[k]), "interior": (wx[l], wy[j], wz[k]),
                              "nguard": guards[i], "order": orders[i]})
                i += 1
    return (30, 26, 22), boxes


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_step_matches_oracle(lib, precision):
    import torch

    gdims, boxes = _small_decomposition()
    gshape = gdims[::-1]
    d, dt = 1.0, 0.4
    g1 = synth.random_fields(synth.rng_for(300, 0), gshape)
    ref = domain.local_steps(g1, boxes, 2, d, dt)
    batch = lib.Batch(boxes, gdims, dx=d, dt=dt, precision=precision)
    g = _to_gpu(g1, batch.dtype)
    batch.step(g)
    batch.step(g)
    torch.cuda.synchronize()
    got = g.double().cpu().numpy()
    err = np.abs(got[0:6] - ref[0:6]).max() / np.abs(ref[0:6]).max()
    assert err <= (1e-12 if precision == "fp64" else 3e-5), err
    np.testing.assert_array_equal(got[6:], g1[6:].astype(np.float64 if precision == "fp64" else np.float32))
    batch.close()


def _edge_decomposition(case):
    if case == "single":
        # one box covering the whole grid, its guards wrapping onto itself
        return (12, 10, 8), [{"origin": (3, 4, 5), "interior": (12, 10, 8), "nguard": 3, "order": 4}]
    # a one-cell-wide slab next to a wide box
    return (9, 7, 5), [{"origin": (0, 0, 0), "interior": (1, 7, 5), "nguard": 2, "order": 8},
                       {"origin": (1, 0, 0), "interior": (8, 7, 5), "nguard": 1, "order": 0}]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", ["single", "slab"])
def test_batch_edge_decompositions_match_oracle(lib, precision, case):
    import torch

    gdims, boxes = _edge_decomposition(case)
    d, dt = 1.0, 0.5
    g1 = synth.random_fields(synth.rng_for(303, len(boxes)), gdims[::-1])
    ref = domain.local_steps(g1, boxes, 2, d, dt)
    batch = lib.Batch(boxes, gdims, dx=d, dt=dt, precision=precision)
    g = _to_gpu(g1, batch.dtype)
    batch.step(g)
    batch.step(g)
    torch.cuda.synchronize()
    got = g.double().cpu().numpy()
    err = np.abs(got[0:6] - ref[0:6]).max() / np.abs(ref[0:6]).max()
    assert err <= (1e-12 if precision == "fp64" else 3e-5), err
    batch.close()


def test_batch_equals_boxes_advanced_one_by_one(lib):
    """Each batched box gives bitwise the result of its own plan on a snapshot of the step-n fields."""
    import torch

    gdims, boxes = _small_decomposition()
    gshape = gdims[::-1]
    g1 = _to_gpu(synth.random_fields(synth.rng_for(301, 0), gshape), torch.float32)
    batch = lib.Batch(boxes, gdims, dt=0.5)
    got = g1.clone()
    batch.step(got)
    expect = g1.clone()
    for b in boxes:
        plan = lib.Plan(*b["interior"], nguard=b["nguard"], order=b["order"], dt=0.5)
        snap = g1.clone()
        plan.step_g1(snap, b["origin"])
        nx, ny, nz = b["interior"]
        ox, oy, oz = b["origin"]
        zi = (oz + torch.arange(nz, device="cuda")) % gshape[0]
        yi = (oy + torch.arange(ny, device="cuda")) % gshape[1]
        xi = (ox + torch.arange(nx, device="cuda")) % gshape[2]
        idx = (slice(0, 6), zi[:, None, None], yi[None, :, None], xi[None, None, :])
        expect[idx] = snap[idx]
        plan.close()
    torch.cuda.synchronize()
    assert torch.equal(got, expect)
    batch.close()


def test_graph_replays_equal_eager_steps(lib):
    """Every graph replay equals the same number of eager steps, with eager work between replays."""
    import torch

    gdims, boxes = _small_decomposition()
    gshape = gdims[::-1]
    batch = lib.Batch(boxes, gdims, dt=0.5)
    for rep in range(3):
        init = _to_gpu(synth.random_fields(synth.rng_for(302, rep), gshape), torch.float32)
        a = init.clone()
        b = init.clone()
        batch.run(a, 4)                     # replay (captured on the first call)
        for _ in range(4):
            batch.step(b)                   # eager
        torch.cuda.synchronize()
        assert torch.equal(a, b), f"replay {rep} differs from eager steps"
        # unrelated eager work and a host synchronisation between replays
        (init * 2.0).sum().item()
    batch.close()


def test_uneven_decomposition_full_size_sampled_boxes(lib):
    """64 boxes, edges 32..96 + guards 8..64, orders 16..64 (FP32): one step, oracle on three boxes."""
    import torch

    rng = synth.rng_for(3, 0)
    gdims, boxes = synth.uneven_decomposition(rng)
    gshape = gdims[::-1]
    d, dt = 1.0, 0.5
    g1 = synth.random_fields(synth.rng_for(3, 1), gshape).astype(np.float32)
    batch = lib.Batch(boxes, gdims, dx=d, dt=dt)
    g = torch.as_tensor(g1, device="cuda")
    batch.step(g)
    torch.cuda.synchronize()
    got = g[0:6].cpu().numpy()
    # the oracle advances a few boxes from the same step-n fields
    g1d = g1.astype(np.float64)
    for bi in (0, 21, 63):
        b = boxes[bi]
        box = domain.guard_fill(g1d, b["origin"], b["interior"], b["nguard"])
        eb = step.box_step(box, d, dt, b["order"])
        ng = b["nguard"]
        nx, ny, nz = b["interior"]
        ox, oy, oz = b["origin"]
        ref = eb[:, ng:ng + nz, ng:ng + ny, ng:ng + nx]
        zi = (oz + np.arange(nz)) % gshape[0]
        yi = (oy + np.arange(ny)) % gshape[1]
        xi = (ox + np.arange(nx)) % gshape[2]
        gv = got[:, zi[:, None, None], yi[None, :, None], xi[None, None, :]]
        rel = np.linalg.norm(gv - ref) / np.linalg.norm(ref)
        print(f"  box {bi} {b}: rel L2 {rel:.2e}", flush=True)
        assert rel <= 2e-6
    batch.close()
