"""GPU parity on dense random fields through the kernels the benchmark runs at full length.

The full-size tests of the benchmark shapes use few-mode inputs, which leave most
(kx, ky) columns and lines of the spectral passes empty.  Here every array is
dense N(0, 1) noise, and the boxes are chosen so that the line lengths and the
tile shapes are those of the 576 x 320 x 320 benchmark box while the oracle
still finishes in seconds:

* 512 x 16 x 256 interior + 32 guards (box 576 x 80 x 320), order 100: x lines
  of 576 (the x passes with the periodic gather table and the interior scatter),
  z lines of 320 (the single-column z kernel);
* 8 x 312 x 136 + 4 (box 16 x 320 x 144): y lines of 320, and z lines of 144 in
  two-column z tiles whose block of 256 threads is shorter than two lines (the
  long-line branch of the multi-column z kernel);
* 8 x 6 x 180 + 4 (box 16 x 14 x 188, 188 = 4 x 47 by chirp-z): single-column z
  kernel on short x and y lines, on a periodic grid the box wraps around;
* 6 x 8 x 152 + 4 (box 14 x 16 x 160): the long-line multi-column branch on
  smooth z lines, infinite order.

Each runs the fused step on G1 (the call bench.py times) against the oracle's
local step (Sec. 1.1 push, Sec. 2.5.2 fill and merge of arXiv:1812.07357), in
FP64 (<= 1e-12 relative, max norm) and FP32 (<= 2e-6 relative L2, <= 2e-5
relative max norm).  The tile shapes are asserted through the plan's schedule.
"""

import numpy as np
import pytest

import synth
from oracle import diagnostics, domain

pytestmark = pytest.mark.gpu

CASES = [
    # interior (x, y, z), guards, order, global grid (x, y, z), origin, (kx, ky) columns per z tile
    ((512, 16, 256), 32, 100, (512, 16, 256), (0, 0, 0), 1),
    ((8, 312, 136), 4, 16, (8, 312, 136), (0, 0, 0), 2),
    ((8, 6, 180), 4, 8, (11, 9, 183), (5, 2, 100), 1),
    ((6, 8, 152), 4, 0, (6, 8, 152), (0, 0, 0), 2),
]

_REF = {}


def _reference(case):
    if case not in _REF:
        interior, ng, order, gdims, origin, _ = case
        g1 = synth.random_fields(synth.rng_for(110, sum(interior) + ng), gdims[::-1])
        box = {"origin": origin, "interior": interior, "nguard": ng, "order": order}
        _REF.clear()
        _REF[case] = (g1, domain.local_step(g1, [box], 1.0, 0.5))
    return _REF[case]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(str(v + 2 * c[1]) for v in c[0]))
def test_dense_fields_full_length_kernels(lib, case, precision):
    import torch

    interior, ng, order, gdims, origin, zcols = case
    g1, ref = _reference(case)
    plan = lib.Plan(*interior, nguard=ng, order=order, dx=1.0, dt=0.5, precision=precision)
    box = plan.box
    assert plan.query(lib.Q_Z_COLUMNS) == zcols
    g = torch.as_tensor(g1, dtype=plan.dtype, device="cuda")
    print(f"dense case box {box} p={order} {precision}", flush=True)
    plan.step_g1(g, origin)
    torch.cuda.synchronize()
    got = g.double().cpu().numpy()
    plan.close()
    err_max = float(np.abs(got[0:6] - ref[0:6]).max() / np.abs(ref[0:6]).max())
    if precision == "fp64":
        assert err_max <= 1e-12, err_max
    else:
        err_l2 = diagnostics.rel_l2(got[0:6], ref[0:6])
        assert err_l2 <= 2e-6 and err_max <= 2e-5, (err_l2, err_max)
    # sources untouched
    np.testing.assert_array_equal(got[6:], g1[6:].astype(np.float64 if precision == "fp64" else np.float32))
