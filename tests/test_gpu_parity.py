"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Element-by-element comparisons on seeded inputs at sizes the oracle finishes in
seconds, spanning several tiles of every pass and ragged tails, with odd and
mixed-radix box edges.  Tolerances: FP64 path 1e-12 relative (max norm); FP32
path 2e-6 relative L2 and 2e-5 relative max norm for one step (single
precision round-off of ~17 transforms of length <= 64 plus the push; see the
precision budget in the design notes).
"""

import numpy as np
import pytest

import synth
from oracle import diagnostics, domain, kspace, step

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_L2 = 2e-6
FP32_MAX = 2e-5


def _to_gpu(a, dtype):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _rel_max(got, ref):
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def _assert_close(got, ref, precision):
    if precision == "fp64":
        assert _rel_max(got, ref) <= FP64_TOL, _rel_max(got, ref)
    else:
        assert diagnostics.rel_l2(got, ref) <= FP32_L2, diagnostics.rel_l2(got, ref)
        assert _rel_max(got, ref) <= FP32_MAX, _rel_max(got, ref)


def _boxes():
    return [
        ((32, 32, 32), 0, 0),
        ((18, 12, 10), 3, 8),        # box 24 x 18 x 16
        ((16, 30, 36), 2, 100),      # box 20 x 34 x 40  (34 = 2 * 17)
        ((21, 15, 7), 0, 4),         # odd edges 21 x 15 x 7
        ((44, 18, 40), 0, 16),       # box 44 x 18 x 40  (44 = 4 * 11)
        ((9, 13, 33), 1, 2),         # box 11 x 15 x 35  (primes 11, 13-ish mix)
        ((53, 29, 23), 0, 8),        # prime edges > 17 on every axis (chirp-z transforms)
        ((219, 40, 60), 2, 32),      # box 223 x 44 x 64: prime x edge of the uneven-box range
        ((33, 41, 45), 7, 64),       # box 47 x 55 x 59: 47, 59 prime; 55 = 5 * 11
        ((1, 6, 5), 0, 0),           # degenerate: one cell along x (half spectrum of one bin)
        ((2, 1, 3), 0, 2),           # degenerate: one cell along y, Nyquist-only x
        ((1, 1, 1), 0, 0),           # a single cell: only k = 0
    ]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("interior,ng,order", _boxes())
def test_tables_match_oracle(lib, precision, interior, ng, order):
    import torch

    d, dt, c = (1.0, 0.9, 1.1), 0.45, 1.3
    plan = lib.Plan(*interior, nguard=ng, order=order, dx=d, dt=dt, c=c, precision=precision)
    coef, kx, ky, kz = plan.tables()
    torch.cuda.synchronize()
    NX, NY, NZ = plan.box
    nxh = NX // 2 + 1
    Kx = kspace.modified_k(NX, d[0], order)[:nxh]
    Ky = kspace.modified_k(NY, d[1], order)
    Kz = kspace.modified_k(NZ, d[2], order)
    tol = 1e-14 if precision == "fp64" else 1e-7
    np.testing.assert_allclose(kx.cpu().numpy(), Kx, rtol=tol, atol=tol * max(1.0, np.abs(Kx).max()))
    np.testing.assert_allclose(ky.cpu().numpy(), Ky, rtol=tol, atol=tol * max(1.0, np.abs(Ky).max()))
    np.testing.assert_allclose(kz.cpu().numpy(), Kz, rtol=tol, atol=tol * max(1.0, np.abs(Kz).max()))
    ref = kspace.coefficients(Kx[:, None, None], Ky[None, :, None], Kz[None, None, :], dt, c)
    got = coef.cpu().numpy() * (NX * NY * NZ)
    ctol = 1e-12 if precision == "fp64" else 2e-7
    for i, name in enumerate(("C", "S1", "X1", "X2", "X3")):
        r = np.broadcast_to(ref[name], got[i].shape)
        err = np.abs(got[i] - r).max() / np.abs(r).max()
        assert err <= ctol, (name, err)
    plan.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("interior,ng,order", _boxes())
def test_push_matches_oracle(lib, precision, interior, ng, order):
    import torch

    d, dt, c, eps0 = 1.0, 0.5, 1.0, 1.0
    plan = lib.Plan(*interior, nguard=ng, order=order, dx=d, dt=dt, c=c, eps0=eps0, precision=precision)
    shape = plan.box_shape
    rng = synth.rng_for(100, sum(interior) + ng + order)
    f = synth.random_fields(rng, shape)
    ref = step.box_step(f, d, dt, order, c, eps0)
    g = _to_gpu(f, plan.dtype)
    plan.push_fields(g)
    torch.cuda.synchronize()
    got = g[0:6].double().cpu().numpy()
    _assert_close(got, ref, precision)
    # sources are read-only
    np.testing.assert_array_equal(g[6:].double().cpu().numpy(), f[6:].astype(
        np.float64 if precision == "fp64" else np.float32))
    plan.close()


def test_push_nonunit_constants_fp64(lib):
    import torch

    interior, ng, order = (14, 10, 12), 2, 6
    d, dt, c, eps0 = (0.7, 1.2, 0.9), 0.8, 1.7, 0.6
    plan = lib.Plan(*interior, nguard=ng, order=order, dx=d, dt=dt, c=c, eps0=eps0, precision="fp64")
    f = synth.random_fields(synth.rng_for(101, 0), plan.box_shape)
    ref = step.box_step(f, d, dt, order, c, eps0)
    g = _to_gpu(f, plan.dtype)
    plan.push_fields(g)
    torch.cuda.synchronize()
    _assert_close(g[0:6].cpu().numpy(), ref, "fp64")
    plan.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("gshape,interior,ng,origin,order", [
    ((20, 24, 28), (28, 24, 20), 4, (0, 0, 0), 8),        # one group covering the whole grid
    ((16, 20, 24), (12, 10, 8), 3, (17, 13, 11), 16),     # box wrapping around the edges
    ((10, 12, 14), (6, 8, 4), 9, (5, 2, 7), 0),           # guards wider than the grid (multi-hop)
    ((12, 18, 22), (22, 18, 12), 0, (0, 0, 0), 32),       # no guards: the global solve
    ((6, 8, 1), (1, 4, 3), 2, (0, 5, 4), 4),              # one-cell x axis: every x guard wraps onto it
])
def test_step_g1_matches_oracle(lib, precision, gshape, interior, ng, origin, order):
    import torch

    d, dt = 1.0, 0.6
    plan = lib.Plan(*interior, nguard=ng, order=order, dx=d, dt=dt, precision=precision)
    g1 = synth.random_fields(synth.rng_for(102, ng + order), gshape)
    box = {"origin": origin, "interior": interior, "nguard": ng, "order": order}
    ref = domain.local_step(g1, [box], d, dt)
    g = _to_gpu(g1, plan.dtype)
    plan.step_g1(g, origin)
    torch.cuda.synchronize()
    got = g.double().cpu().numpy()
    _assert_close(got[0:6], ref[0:6], precision)
    np.testing.assert_array_equal(got[6:], g1[6:].astype(np.float64 if precision == "fp64" else np.float32))
    plan.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_guard_fill_and_merge_are_exact(lib, precision):
    import torch

    gshape, interior, ng, origin = (9, 11, 13), (5, 7, 4), 5, (10, 3, 8)
    plan = lib.Plan(*interior, nguard=ng, order=4, precision=precision)
    g1 = synth.random_fields(synth.rng_for(103, 0), gshape, nfields=3)
    g = _to_gpu(g1, plan.dtype)
    box = [torch.zeros(plan.box_shape, dtype=plan.dtype, device="cuda") for _ in range(3)]
    plan.guard_fill(list(g), box, origin)
    torch.cuda.synchronize()
    ref = domain.guard_fill(np.asarray(g.cpu().numpy()), origin, interior, ng)
    for i in range(3):
        np.testing.assert_array_equal(box[i].cpu().numpy(), ref[i])
    # copy merge of a fresh box
    nb = synth.random_fields(synth.rng_for(103, 1), plan.box_shape, nfields=3)
    nbg = [_to_gpu(nb[i], plan.dtype) for i in range(3)]
    tgt = _to_gpu(np.zeros((3,) + gshape), plan.dtype)
    plan.guard_merge(nbg, list(tgt), origin, mode=0)
    torch.cuda.synchronize()
    expect = np.zeros((3,) + gshape)
    domain.guard_merge(np.stack([t.cpu().numpy() for t in nbg]).astype(np.float64), expect, origin, interior, ng)
    np.testing.assert_array_equal(tgt.cpu().numpy(), expect)
    # add merge: every box cell (guards included) summed into its wrapped cell
    tgt2 = _to_gpu(np.zeros((3,) + gshape), plan.dtype)
    plan.guard_merge(nbg, list(tgt2), origin, mode=1)
    torch.cuda.synchronize()
    nbh = np.stack([t.cpu().numpy() for t in nbg]).astype(np.float64)
    expect2 = np.zeros((3,) + gshape)
    NZ, NY, NX = gshape
    bz, by, bx = plan.box_shape
    for k in range(bz):
        for j in range(by):
            zi, yi = (origin[2] - ng + k) % NZ, (origin[1] - ng + j) % NY
            xi = (origin[0] - ng + np.arange(bx)) % NX
            np.add.at(expect2, (slice(None), zi, yi, xi), nbh[:, k, j, :])
    tol = 1e-12 if precision == "fp64" else 1e-5
    np.testing.assert_allclose(tgt2.cpu().numpy(), expect2, rtol=tol, atol=tol * np.abs(expect2).max())
    plan.close()


def test_config1_ten_steps_fp64(lib):
    """32^3 periodic grid, infinite order, dt = dx/2, 10 steps (plane waves + Gaussian current)."""
    import torch

    shape, d, dt, order = (32, 32, 32), 1.0, 0.5, 0
    rng = synth.rng_for(1, 0)
    pw = synth.plane_wave_modes(rng, shape, 4)
    from oracle import modes

    kvec = modes.mode_wavevectors(pw["m"], (32, 32, 32), d)
    ev, bv = [], []
    for j in range(4):
        e = synth.transverse_unit(pw["u"][j], kvec[j])
        ev.append(e)
        bv.append(np.cross(kvec[j], e) / np.linalg.norm(kvec[j]))
    E, B = synth.plane_wave_sum(shape, d, pw["m"], pw["amp"], pw["phase"], ev, bv)
    J = synth.gaussian_blob(shape, d, (16.0, 16.0, 16.0), 3.0, 0.1, rng.normal(size=3))
    rho_old = diagnostics.rho_from_gauss(E, d, order)
    rho_new = diagnostics.rho_continuity(rho_old, J, dt, d, order)
    f = np.concatenate([E, B, J, rho_old[None], rho_new[None]])
    ref = step.box_steps(f, 10, d, dt, order)
    plan = lib.Plan(32, 32, 32, nguard=0, order=0, dx=d, dt=dt, precision="fp64")
    g = _to_gpu(f, torch.float64)
    for _ in range(10):
        plan.step_g1(g, (0, 0, 0))
    torch.cuda.synchronize()
    got = g[0:6].cpu().numpy()
    assert diagnostics.rel_l2(got[0:3], ref[0:3]) <= 1e-12
    assert diagnostics.rel_l2(got[3:6], ref[3:6]) <= 1e-12
    plan.close()
