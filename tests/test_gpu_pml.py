"""GPU parity of the two-step PML (psatd_pml_set / psatd_pml_step) against the oracle.

The oracle (oracle/pml.py) is pinned in tests/test_oracle_pml.py by the ordinary
box when undamped, the matrix exponential of the split system mode by mode, and
the absorption of outgoing pulses.  Here the HIP path is compared with it
element by element over several steps on boxes with even, odd and chirp-z edges and
with 320 / 256-point lines (the two-stage x kernels and the two-stage PML z kernel),
layers on one, two or three axes, sources, non-unit c and eps0, FP64 (1e-12
relative, max norm) and FP32 (2e-6 relative L2 and 2e-5 max norm per step, grown
linearly with the steps); without layers the sums of the parts equal psatd_push;
a pulse sent into the layers at full length is absorbed like in the oracle.
"""

import numpy as np
import pytest

import synth
from oracle import pml

pytestmark = pytest.mark.gpu


def _check(got, ref, precision, nsteps):
    err_max = float(np.abs(got - ref).max() / np.abs(ref).max())
    if precision == "fp64":
        assert err_max <= 1e-12 * nsteps, err_max
    else:
        err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        assert err <= 2e-6 * nsteps and err_max <= 2e-5 * nsteps, (err, err_max)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("interior,ng,order,widths", [((40, 36, 30), 0, 8, (6, 0, 0)),
                                                       ((33, 20, 25), 2, 0, (5, 4, 3)),
                                                       ((47, 16, 18), 0, 16, (0, 3, 4)),
                                                       # x = 320, z = 256: two-stage x kernels and
                                                       # the two-stage PML z kernel
                                                       ((320, 12, 256), 0, 16, (16, 2, 24)),
                                                       # z = 180: one column per tile, run-time kernel
                                                       ((14, 10, 180), 0, 8, (3, 0, 20))])
def test_pml_steps_match_oracle(lib, precision, interior, ng, order, widths):
    import torch

    d, dt, c, eps0 = (1.0, 0.9, 1.1), 0.4, 1.2, 0.8
    plan = lib.Plan(*interior, nguard=ng, order=order, dx=d, dt=dt, c=c, eps0=eps0, precision=precision)
    shape = plan.box_shape
    rng = synth.rng_for(200, sum(interior) + order)
    parts = rng.normal(size=(12,) + shape)
    src = 0.2 * rng.normal(size=(5,) + shape)
    sigma_max, power = 1.5, 2.0
    plan.pml_set(widths, sigma_max, power)
    damp = pml.damping(shape, widths, sigma_max, power, dt)
    nsteps = 3
    ref = pml.pml_steps(parts, src, nsteps, d, dt, order, damp, c, eps0)
    g = torch.as_tensor(parts, dtype=plan.dtype, device="cuda")
    s = torch.as_tensor(src, dtype=plan.dtype, device="cuda")
    if precision == "fp32":
        parts = g.double().cpu().numpy()
        src = s.double().cpu().numpy()
        ref = pml.pml_steps(parts, src, nsteps, d, dt, order, damp, c, eps0)
    for _ in range(nsteps):
        plan.pml_step(g, s)
    torch.cuda.synchronize()
    _check(g.double().cpu().numpy(), ref, precision, nsteps)
    plan.close()


def test_without_layers_the_parts_add_up_to_the_ordinary_push(lib):
    import torch

    plan = lib.Plan(24, 20, 18, nguard=0, order=4, dt=0.5, precision="fp64")
    shape = plan.box_shape
    rng = synth.rng_for(201, 0)
    parts = rng.normal(size=(12,) + shape)
    src = 0.2 * rng.normal(size=(5,) + shape)
    plan.pml_set((0, 0, 0), 0.0)
    g = torch.as_tensor(parts, device="cuda")
    s = torch.as_tensor(src, device="cuda")
    plan.pml_step(g, s)
    full = torch.as_tensor(np.concatenate([parts[0:3] + parts[6:9], parts[3:6] + parts[9:12], src]),
                           device="cuda")
    plan.push_fields(full)
    torch.cuda.synchronize()
    sums = torch.cat([g[0:3] + g[6:9], g[3:6] + g[9:12]]).cpu().numpy()
    ref = full[0:6].cpu().numpy()
    assert np.abs(sums - ref).max() <= 1e-12 * np.abs(ref).max()
    plan.close()


def test_pml_state_and_arguments(lib):
    import torch

    plan = lib.Plan(16, 16, 16, nguard=0, order=4, dt=0.5, precision="fp64")
    z = torch.zeros((12, 16, 16, 16), dtype=torch.float64, device="cuda")
    src = torch.zeros((5, 16, 16, 16), dtype=torch.float64, device="cuda")
    with pytest.raises(lib.PsatdError) as e:
        plan.pml_step(z, src)
    assert e.value.code == lib.PSATD_ESTATE
    with pytest.raises(lib.PsatdError):
        plan.pml_set((9, 0, 0), 1.0)   # wider than half the box edge
    with pytest.raises(lib.PsatdError):
        plan.pml_set((2, 2, 2), -1.0)
    plan.close()
    stag = lib.Plan(16, 16, 16, nguard=0, order=4, dt=0.5, staggered=True)
    with pytest.raises(lib.PsatdError) as e:
        stag.pml_set((2, 2, 2), 1.0)
    assert e.value.code == lib.PSATD_EUNSUPPORTED
    stag.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_outgoing_pulse_is_absorbed(lib, precision):
    """A packet along x on a 320 x 16 x 16 box (the benchmark's line length, two-stage y/x
    kernels around the run-time z kernel) with 32-cell layers: after one crossing the
    interior holds less than 1 % of the peak, and the GPU matches the oracle."""
    import torch

    n, w, dt, c, order = 320, 32, 0.5, 1.0, 16
    plan = lib.Plan(n, 16, 16, nguard=0, order=order, dt=dt, c=c, precision=precision)
    shape = plan.box_shape
    x = np.arange(n, dtype=np.float64)
    env = np.exp(-((x - 0.5 * n) / 8.0) ** 2) * np.cos(0.6 * x)
    parts = np.zeros((12,) + shape)
    parts[7] = env[None, None, :]   # E_y driven along x: set B of y (E_yx)
    parts[5] = env[None, None, :]   # B_z driven along x: set A of z (B_zx)
    sigma_max = 3.0 * np.log(1e4) * c / (2 * w)
    plan.pml_set((w, 0, 0), sigma_max, 2.0)
    g = torch.as_tensor(parts, dtype=plan.dtype, device="cuda")
    s = torch.zeros((5,) + shape, dtype=plan.dtype, device="cuda")
    nsteps = int(n / (c * dt))
    for _ in range(nsteps):
        plan.pml_step(g, s)
    torch.cuda.synchronize()
    got = g.double().cpu().numpy()
    assert np.abs(got[..., w:n - w]).max() < 1e-2
    ref = pml.pml_steps(parts, np.zeros((5,) + shape), nsteps, 1.0, dt, order,
                        pml.damping(shape, (w, 0, 0), sigma_max, 2.0, dt), c)
    tol = 1e-10 if precision == "fp64" else 2e-3  # 640 FP32 steps
    assert np.abs(got - ref).max() <= tol
    plan.close()
