"""GPU: the fused step without allocation (psatd_step_g1_noalloc) against psatd_step_g1.

The no-allocation entry point runs the same five passes with their spectral
workspaces in the library's static device scratch.  Two calls in a row, the
second on a smaller box, each compared with the allocating entry point on the
same inputs (bitwise: same kernels and schedules) and with the FP64 oracle
(Sec. 1.1 and 2.5.2 of arXiv:1812.07357, <= 1e-12 in FP64, 2e-6 relative L2 /
2e-5 max in FP32).  Boxes beyond the scratch are refused with PSATD_EINVAL.
"""

import numpy as np
import pytest

import synth
from oracle import diagnostics, domain

pytestmark = pytest.mark.gpu

CALLS = [  # (interior, guards, order, global grid, origin): the second call is smaller
    ((40, 36, 44), 6, 16, (48, 40, 44), (5, 3, 0)),
    ((10, 12, 9), 3, 8, (14, 12, 20), (7, 0, 15)),
]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_step_matches_the_allocating_step(lib, precision):
    import torch

    for k, (interior, ng, order, gdims, origin) in enumerate(CALLS):
        g1 = synth.random_fields(synth.rng_for(120, k), gdims[::-1])
        ref = domain.local_step(g1, [{"origin": origin, "interior": interior, "nguard": ng, "order": order}],
                                1.0, 0.5)
        ref_plan = lib.Plan(*interior, nguard=ng, order=order, precision=precision)
        lean = lib.Plan(*interior, nguard=ng, order=order, precision=precision,
                        flags=lib.PSATD_FLAG_NO_WORKSPACE)
        assert lean.query(lib.Q_WORKSPACE_BYTES) < ref_plan.query(lib.Q_WORKSPACE_BYTES)
        a = torch.as_tensor(g1, dtype=ref_plan.dtype, device="cuda")
        b = a.clone()
        c = a.clone()
        print(f"noalloc call {k}: box {lean.box} {precision}", flush=True)
        ref_plan.step_g1(a, origin)
        lean.step_g1_noalloc(b, origin)
        ref_plan.step_g1_noalloc(c, origin)  # a plan with its own workspace may use the scratch too
        torch.cuda.synchronize()
        assert torch.equal(a, b) and torch.equal(a, c)
        got = b.double().cpu().numpy()
        if precision == "fp64":
            assert np.abs(got[0:6] - ref[0:6]).max() <= 1e-12 * np.abs(ref[0:6]).max()
        else:
            assert diagnostics.rel_l2(got[0:6], ref[0:6]) <= 2e-6
            assert np.abs(got[0:6] - ref[0:6]).max() <= 2e-5 * np.abs(ref[0:6]).max()
        with pytest.raises(lib.PsatdError) as e:  # no workspace: only the static-scratch step
            lean.step_g1(b, origin)
        assert e.value.code == lib.PSATD_ESTATE
        ref_plan.close()
        lean.close()


def test_noalloc_rejects_boxes_beyond_the_scratch(lib):
    import torch

    with pytest.raises(lib.PsatdError) as e:
        lib.Plan(256, 256, 256, nguard=8, order=8, flags=lib.PSATD_FLAG_NO_WORKSPACE)
    assert e.value.code == lib.PSATD_EINVAL
    plan = lib.Plan(192, 192, 160, nguard=16, order=8)  # box 224 x 224 x 192: 1.1 GB of workspace
    g = torch.zeros((11, 160, 192, 192), dtype=torch.float32, device="cuda")
    with pytest.raises(lib.PsatdError) as e:
        plan.step_g1_noalloc(g, (0, 0, 0))
    assert e.value.code == lib.PSATD_EINVAL and "scratch" in str(e.value)
    plan.close()
