"""GPU parity of the staggered (Yee) grid variant (PSATD_FLAG_STAGGERED) against the oracle.

The oracle's staggered step is pinned by the matrix exponential of the
real-space staggered semi-discrete system (tests/test_oracle_staggered.py).
Here the HIP path is compared element by element with it: the staggered
symbol tables, the box push on shapes with even (Nyquist) and odd edges,
chirp-z edges, both the run-time and the two-stage compile-time z kernels,
the fused step on G1 with guards (wrap, multi-hop), and a batch.  Tolerances
as for the collocated grid: FP64 1e-12 relative (max norm); FP32 2e-6
relative L2 and 2e-5 relative max norm per step.
"""

import numpy as np
import pytest

import synth
from oracle import diagnostics, domain, kspace, step

pytestmark = pytest.mark.gpu


def _close(got, ref, precision):
    err_max = float(np.abs(got - ref).max() / np.abs(ref).max())
    if precision == "fp64":
        assert err_max <= 1e-12, err_max
    else:
        err = diagnostics.rel_l2(got, ref)
        assert err <= 2e-6 and err_max <= 2e-5, (err, err_max)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("interior,ng,order", [((18, 12, 10), 3, 8), ((21, 15, 7), 0, 4), ((9, 13, 33), 1, 0),
                                               ((53, 29, 23), 0, 16), ((24, 16, 304), 8, 100)])
def test_staggered_push_matches_oracle(lib, precision, interior, ng, order):
    import torch

    d, dt, c, eps0 = (1.0, 0.9, 1.1), 0.45, 1.2, 0.8
    plan = lib.Plan(*interior, nguard=ng, order=order, dx=d, dt=dt, c=c, eps0=eps0, precision=precision,
                    staggered=True)
    NX, NY, NZ = plan.box
    coef, kx, ky, kz = plan.tables()
    tol = 1e-13 if precision == "fp64" else 1e-6
    for got, ref in ((kx, kspace.modified_k_staggered(NX, d[0], order)[: NX // 2 + 1]),
                     (ky, kspace.modified_k_staggered(NY, d[1], order)),
                     (kz, kspace.modified_k_staggered(NZ, d[2], order))):
        np.testing.assert_allclose(got.cpu().numpy(), ref, rtol=tol, atol=tol * np.abs(ref).max())
    f = synth.random_fields(synth.rng_for(140, sum(interior) + order), plan.box_shape)
    ref = step.box_step(f, d, dt, order, c, eps0, staggered=True)
    g = torch.as_tensor(f, dtype=plan.dtype, device="cuda")
    plan.push_fields(g)
    torch.cuda.synchronize()
    _close(g[0:6].double().cpu().numpy(), ref, precision)
    plan.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("gshape,interior,ng,origin,order", [
    ((16, 20, 24), (12, 10, 8), 3, (17, 13, 11), 16),   # box wrapping around the edges
    ((10, 12, 14), (6, 8, 4), 9, (5, 2, 7), 0),         # guards wider than the grid (multi-hop)
    ((304, 8, 16), (16, 8, 304), 8, (0, 0, 0), 32),     # z lines of 320 (two-stage z kernel)
])
def test_staggered_step_g1_matches_oracle(lib, precision, gshape, interior, ng, origin, order):
    import torch

    g1 = synth.random_fields(synth.rng_for(141, sum(gshape) + order), gshape)
    ref = domain.local_step(g1, [{"origin": origin, "interior": interior, "nguard": ng, "order": order,
                                  "staggered": True}], 1.0, 0.5)
    plan = lib.Plan(*interior, nguard=ng, order=order, precision=precision, staggered=True)
    g = torch.as_tensor(g1, dtype=plan.dtype, device="cuda")
    plan.step_g1(g, origin)
    torch.cuda.synchronize()
    _close(g[0:6].double().cpu().numpy(), ref[0:6], precision)
    plan.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_staggered_batch_matches_oracle(lib, precision):
    import torch

    gdims = (30, 26, 22)
    boxes = []
    for k, (oz, nz) in enumerate(((0, 9), (9, 13))):
        for j, (oy, ny) in enumerate(((0, 11), (11, 15))):
            for i, (ox, nx) in enumerate(((0, 17), (17, 13))):
                boxes.append({"origin": (ox, oy, oz), "interior": (nx, ny, nz), "nguard": 2 + i + 2 * j + 3 * k,
                              "order": (4, 8, 0, 16)[(i + j + k) % 4], "staggered": True})
    g1 = synth.random_fields(synth.rng_for(142, 0), gdims[::-1])
    ref = domain.local_steps(g1, boxes, 2, 1.0, 0.4)
    batch = lib.Batch(boxes, gdims, dx=1.0, dt=0.4, precision=precision)
    g = torch.as_tensor(g1, dtype=batch.dtype, device="cuda")
    batch.step(g)
    batch.step(g)
    torch.cuda.synchronize()
    got = g.double().cpu().numpy()
    err = np.abs(got[0:6] - ref[0:6]).max() / np.abs(ref[0:6]).max()
    assert err <= (1e-12 if precision == "fp64" else 3e-5), err
    batch.close()
