"""GPU: object state and resource errors of the C ABI.

* PSATD_ESTATE: a plan or batch owns its spectral workspace, so a step called
  on a second stream while the previous step is still running on the first
  must be refused (the two would overwrite each other's workspace).  Once the
  first stream has finished, the second may take over.
* PSATD_ENOMEM: with a device budget below what a plan needs, construction
  fails part-way through its allocations, and everything it had allocated is
  released (the library's device byte count returns to where it was).
"""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def test_plan_on_a_second_stream_while_busy_is_refused(lib):
    import torch

    plan = lib.Plan(512, 256, 256, nguard=32, order=100, dx=1.0, dt=0.5)
    g = torch.zeros((11, 256, 256, 512), dtype=torch.float32, device="cuda")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    for _ in range(8):  # about 40 ms of work queued on s1
        plan.step_g1(g, (0, 0, 0), stream=s1)
    with pytest.raises(lib.PsatdError) as e:
        plan.step_g1(g, (0, 0, 0), stream=s2)
    assert e.value.code == lib.PSATD_ESTATE
    plan.step_g1(g, (0, 0, 0), stream=s1)  # the same stream is always fine
    s1.synchronize()
    plan.step_g1(g, (0, 0, 0), stream=s2)  # the first stream has drained: the plan moves
    s2.synchronize()
    plan.close()


def test_batch_on_a_second_stream_while_busy_is_refused(lib):
    import torch

    gdims, boxes = synth.uneven_decomposition(synth.rng_for(3, 0))
    batch = lib.Batch(boxes, gdims, dx=1.0, dt=0.5)
    g = torch.zeros((11,) + tuple(gdims[::-1]), dtype=torch.float32, device="cuda")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    batch.run(g, 4, stream=s1)
    with pytest.raises(lib.PsatdError) as e:
        batch.step(g, stream=s2)
    assert e.value.code == lib.PSATD_ESTATE
    s1.synchronize()
    batch.step(g, stream=s2)
    s2.synchronize()
    batch.close()


def test_enomem_part_way_through_construction_releases_everything(lib):
    import torch

    boxes = [{"origin": (0, 0, 0), "interior": (32, 24, 20), "nguard": 8, "order": 16},
             {"origin": (32, 0, 0), "interior": (32, 24, 20), "nguard": 8, "order": 16}]
    torch.cuda.synchronize()
    before = lib.device_bytes_in_use()
    plan = lib.Plan(64, 48, 40, nguard=8, order=16, precision="fp64")
    need_plan = plan.query(lib.Q_WORKSPACE_BYTES)
    plan.close()
    batch = lib.Batch(boxes, (64, 24, 20), precision="fp64")
    need_batch = batch.query(lib.QB_WORKSPACE_BYTES)
    batch.close()
    assert lib.device_bytes_in_use() == before
    try:
        for frac in (0.1, 0.5, 0.9):
            lib.set_device_budget(before + int(frac * need_plan))
            with pytest.raises(lib.PsatdError) as e:
                lib.Plan(64, 48, 40, nguard=8, order=16, precision="fp64")
            assert e.value.code == lib.PSATD_ENOMEM
            assert lib.device_bytes_in_use() == before
            lib.set_device_budget(before + int(frac * need_batch))
            with pytest.raises(lib.PsatdError) as e:
                lib.Batch(boxes, (64, 24, 20), precision="fp64")
            assert e.value.code == lib.PSATD_ENOMEM
            assert lib.device_bytes_in_use() == before
        lib.set_device_budget(before + need_plan)
        plan = lib.Plan(64, 48, 40, nguard=8, order=16, precision="fp64")  # exactly enough
        assert lib.device_bytes_in_use() == before + need_plan
        plan.close()
    finally:
        lib.set_device_budget(None)
    assert lib.device_bytes_in_use() == before
    assert need_plan > 0 and need_batch > 0
