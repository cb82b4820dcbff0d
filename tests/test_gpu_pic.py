"""GPU parity of the particle side of the PIC cycle (psatd_pic_*) against the oracle.

The oracle (oracle/pic.py) is pinned in tests/test_oracle_pic.py by the tent
function, the truncated-power form of the B-splines, their moments, exact charge
conservation, gather/deposit adjointness, exact linear interpolation and Boris
closed forms.  Here the HIP kernels are compared with it element by element on
seeded warm-plasma particles (edge cases included: nodes, the periodic edge, tile
corners) on collocated and staggered grids, for particle shapes of degree 1, 2
and 3, with D1 tiles that divide the grid and tiles that leave a ragged tail, a
grid smaller than one tile, an empty particle set, and a full PIC cycle (push,
deposit, Maxwell step on the FFT boxes) against the oracle's cycle.

Tolerances.  FP64: 1e-12 relative (max norm); the deposit's atomic sums change
only the order of rounding.  FP32: positions and momenta to 2e-6 of their scale
(a few ulps of the gather of up to 64 terms and the Boris step), grid sums to
2e-5 of the largest cell value (fp32 positions set the weights to ~1e-6 absolute
and a cell sums up to a few hundred weighted terms).
"""

import numpy as np
import pytest

import synth
from oracle import domain, pic

pytestmark = pytest.mark.gpu

G1 = (24, 20, 16)  # (GX, GY, GZ)
D = (1.0, 0.9, 1.1)
DT, C = 0.4, 1.0


def _lengths(gdims, d):
    return np.array([gdims[0] * d[0], gdims[1] * d[1], gdims[2] * d[2]])


def _as_inputs(x, u, precision, L):
    """Host arrays rounded to the kernel precision (both sides see the same values), positions < L."""
    dt = np.float64 if precision == "fp64" else np.float32
    x = x.astype(dt)
    x = np.minimum(x, np.nextafter(L.astype(dt), dt(0)))
    return x.astype(np.float64), u.astype(dt).astype(np.float64)


def _gpu(a, lib_obj):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a), dtype=lib_obj.dtype, device="cuda")


def _periodic_diff(a, b, L):
    return (a - b + 0.5 * L) % L - 0.5 * L


def _g1_fields(seed, gdims, scale=0.3):
    gshape = (gdims[2], gdims[1], gdims[0])
    return synth.random_fields(synth.rng_for(seed, 0), gshape, 11, scale)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("staggered", [False, True])
@pytest.mark.parametrize("shape", [1, 2, 3])
def test_push_matches_oracle(lib, precision, staggered, shape):
    import torch

    L = _lengths(G1, D)
    x, u = synth.plasma_particles(synth.rng_for(160, int(staggered)), 6000, L, 0.8)
    x, u = _as_inputs(x, u, precision, L)
    g1 = _g1_fields(161, G1)
    qm = -1.3
    xr, ur = pic.push(x, u, g1, g1.shape[1:], D, qm, DT, C, staggered=staggered, order=shape)
    p = lib.Pic(G1, dx=D, dt=DT, c=C, q=1.0, q_over_m=qm, max_particles=len(x), tile=8, precision=precision,
                staggered=staggered, shape=shape)
    g = _gpu(g1, p)
    xg, ug = _gpu(x.T, p), _gpu(u.T, p)
    xo = torch.empty_like(xg)
    p.push(g, xg, ug, xo)
    torch.cuda.synchronize()
    assert np.array_equal(xo.double().cpu().numpy(), x.T)
    tol = 1e-12 if precision == "fp64" else 2e-6
    du = np.abs(ug.double().cpu().numpy().T - ur).max() / np.abs(ur).max()
    dx = np.abs(_periodic_diff(xg.double().cpu().numpy().T, xr, L)).max() / L.max()
    assert du <= tol and dx <= tol, (du, dx)
    assert float(xg.min()) >= 0.0 and bool((xg.double().cpu().numpy().T < L).all())
    p.close()


def _deposit_case(lib, precision, staggered, gdims, tile, n, seed, shape=1):
    import torch

    L = _lengths(gdims, D)
    x0, u = synth.plasma_particles(synth.rng_for(seed, tile), n, L, 0.7)
    # a particle moves at most c dt (< one cell) per step
    x0, u = _as_inputs(x0, u, precision, L)
    gam = np.sqrt(1.0 + np.sum(u * u, axis=1, keepdims=True) / C**2)
    x1 = np.mod(x0 + DT * u / gam, L)
    x1, _ = _as_inputs(x1, u, precision, L)
    gshape = (gdims[2], gdims[1], gdims[0])
    q = -0.37
    J, r0, r1 = pic.sources(x0, x1, u, q, gshape, D, DT, C, staggered=staggered, order=shape)
    ref = np.concatenate([J, r0[None], r1[None]])
    p = lib.Pic(gdims, dx=D, dt=DT, c=C, q=q, q_over_m=1.0, max_particles=max(n, 1), tile=tile, precision=precision,
                staggered=staggered, shape=shape)
    g1 = _g1_fields(seed + 1, gdims)
    g = _gpu(g1, p)
    p.deposit(g, _gpu(x0.T, p), _gpu(x1.T, p), _gpu(u.T, p))
    torch.cuda.synchronize()
    got = g.double().cpu().numpy()
    p.close()
    return got, g1, ref


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("staggered", [False, True])
@pytest.mark.parametrize("tile", [8, 5])
@pytest.mark.parametrize("shape", [1, 2, 3])
def test_deposit_matches_oracle(lib, precision, staggered, tile, shape):
    got, g1, ref = _deposit_case(lib, precision, staggered, G1, tile, 20000, 162, shape)
    assert np.array_equal(got[0:6], g1[0:6].astype(np.float32 if precision == "fp32" else np.float64))
    tol = 1e-12 if precision == "fp64" else 2e-5
    err = np.abs(got[6:] - ref).max() / np.abs(ref).max()
    assert err <= tol, err
    # total charge: the deposits of every particle sum to n q at both ends
    vol = np.prod(D)
    for k in (9, 10):
        assert abs(got[k].sum() * vol - 20000 * -0.37) <= (1e-10 if precision == "fp64" else 1e-4) * 20000 * 0.37


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("staggered", [False, True])
@pytest.mark.parametrize("shape,gdims,tile", [(2, (40, 20, 30), 5), (2, (20, 10, 30), 5), (3, (32, 16, 16), 8),
                                              (1, (16, 16, 24), 8)])
def test_deposit_through_tile_blocks_matches_oracle(lib, precision, staggered, shape, gdims, tile):
    """Shapes of degree 2 and 3 with tiles that divide the grid, at least two per axis
    (exactly two along some axes) and guards no wider than a tile: the blocks are stored per
    tile and gathered cell by cell without atomics; every cell of the source slots is
    written, the field slots are not touched.  (Degree 1 on the same kind of grid: the
    atomic merge.)"""
    import torch

    got, _, ref = _deposit_case(lib, precision, staggered, gdims, tile, 12000, 169, shape)
    tol = 1e-12 if precision == "fp64" else 2e-5
    assert np.abs(got[6:] - ref).max() / np.abs(ref).max() <= tol
    L = _lengths(gdims, D)
    x0, u = synth.plasma_particles(synth.rng_for(170, tile), 12000, L, 0.7)
    x0, u = _as_inputs(x0, u, precision, L)
    gam = np.sqrt(1.0 + np.sum(u * u, axis=1, keepdims=True) / C**2)
    x1, _ = _as_inputs(np.mod(x0 + DT * u / gam, L), u, precision, L)
    p = lib.Pic(gdims, dx=D, dt=DT, c=C, q=0.3, max_particles=len(x0), tile=tile, precision=precision,
                staggered=staggered, shape=shape)
    a, b = (torch.full((11, gdims[2], gdims[1], gdims[0]), float(k), dtype=p.dtype, device="cuda")
            for k in (1, 2))
    args = [_gpu(x0.T, p), _gpu(x1.T, p), _gpu(u.T, p)]
    p.deposit(a, *args)
    p.deposit(b, *args)
    torch.cuda.synchronize()
    # the same sources whatever the arrays held before (the order of a tile's particle list,
    # and so the rounding of the per-thread sums, may differ between the calls)
    d = (a[6:] - b[6:]).abs().max().item() / a[6:].abs().max().item()
    assert d <= (1e-13 if precision == "fp64" else 1e-6), d
    assert bool((a[0:6] == 1).all()) and bool((b[0:6] == 2).all())
    p.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [1, 3])
def test_deposit_on_a_grid_smaller_than_a_tile(lib, precision, shape):
    # with shape 3 the 4-point stencil covers more than the 3 cells along z: the
    # periodic images of one point add up
    got, _, ref = _deposit_case(lib, precision, True, (6, 5, 3), 8, 700, 163, shape)
    tol = 1e-12 if precision == "fp64" else 2e-5
    assert np.abs(got[6:] - ref).max() / np.abs(ref).max() <= tol


@pytest.mark.parametrize("shape,gdims,tile", [(1, G1, 8), (2, (40, 20, 30), 5)])
def test_deposit_of_no_particles_clears_the_sources(lib, shape, gdims, tile):
    # (degree 2 on a grid the tiles divide: the path with per-tile blocks)
    import torch

    p = lib.Pic(gdims, dx=D, dt=DT, c=C, max_particles=10, tile=tile, precision="fp64", shape=shape)
    g1 = _g1_fields(164, gdims)
    g = _gpu(g1, p)
    e = torch.empty((3, 0), dtype=torch.float64, device="cuda")
    p.deposit(g, e, e, e)
    p.push(g, e, e, e)
    torch.cuda.synchronize()
    got = g.cpu().numpy()
    assert np.array_equal(got[0:6], g1[0:6]) and not got[6:].any()
    with pytest.raises(lib.PsatdError):
        big = torch.zeros((3, 11), dtype=torch.float64, device="cuda")
        p.deposit(g, big, big, big)  # more than max_particles
    p.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("staggered,shape", [(False, 1), (True, 1), (False, 2), (True, 3)])
def test_pic_cycle_matches_oracle(lib, precision, staggered, shape):
    """Three PIC cycles: gather + push, deposit, local PSATD step on four FFT boxes (D2)
    whose edges differ from the D1 tiles, against the same cycle in the oracle; on the
    collocated and on the staggered (Yee) grid, with linear and higher-order shapes."""
    import torch

    gdims, d, dt, c = (32, 24, 20), (1.0, 1.0, 1.0), 0.45, 1.0
    L = _lengths(gdims, d)
    gshape = (gdims[2], gdims[1], gdims[0])
    boxes = [dict(origin=(0, 0, 0), interior=(18, 24, 20), nguard=4, order=8, staggered=staggered),
             dict(origin=(18, 0, 0), interior=(14, 11, 20), nguard=(4, 5, 3), order=8, staggered=staggered),
             dict(origin=(18, 11, 0), interior=(14, 13, 9), nguard=6, order=16, staggered=staggered),
             dict(origin=(18, 11, 9), interior=(14, 13, 11), nguard=3, order=0, staggered=staggered)]
    x, u = synth.plasma_particles(synth.rng_for(165, 0), 4000, L, 0.3)
    x, u = _as_inputs(x, u, precision, L)
    q, qm = -0.05, -1.0
    f = 0.05 * synth.random_fields(synth.rng_for(166, 0), gshape, 11, 1.0)
    f[6:] = 0.0
    p = lib.Pic(gdims, dx=d, dt=dt, c=c, q=q, q_over_m=qm, max_particles=len(x), tile=8, precision=precision,
                staggered=staggered, shape=shape)
    batch = lib.Batch(boxes, gdims, dx=d, dt=dt, precision=precision)
    g = _gpu(f, p)
    f = g.double().cpu().numpy()
    xg, ug = _gpu(x.T, p), _gpu(u.T, p)
    xo = torch.empty_like(xg)
    for _ in range(3):
        p.push(g, xg, ug, xo)
        p.deposit(g, xo, xg, ug)
        batch.step(g)
        xn, u = pic.push(x, u, f, gshape, d, qm, dt, c, staggered=staggered, order=shape)
        J, r0, r1 = pic.sources(x, xn, u, q, gshape, d, dt, c, staggered=staggered, order=shape)
        f[6:9], f[9], f[10] = J, r0, r1
        f = domain.local_step(f, boxes, d, dt, c)
        x = xn
    torch.cuda.synchronize()
    tol = 1e-11 if precision == "fp64" else 1e-4
    got = g.double().cpu().numpy()
    assert np.abs(got - f).max() / np.abs(f).max() <= tol
    assert np.abs(ug.double().cpu().numpy().T - u).max() / np.abs(u).max() <= tol
    assert np.abs(_periodic_diff(xg.double().cpu().numpy().T, x, L)).max() / L.max() <= tol
    batch.close()
    p.close()


@pytest.mark.parametrize("precision,shape", [("fp32", 1), ("fp64", 1), ("fp32", 3)])
def test_deposit_at_scale_sampled_cells(lib, precision, shape):
    """256 x 128 x 128 cells, 8 particles per cell (33.5 M): total charge exact to rounding,
    and 48 sampled cells of every slot against the oracle's deposit of the particles
    whose stencil reaches them."""
    import torch

    gdims = (256, 128, 128)
    gshape = (gdims[2], gdims[1], gdims[0])
    d, dt, c, q = (1.0, 1.0, 1.0), 0.5, 1.0, 0.01
    n = 8 * gdims[0] * gdims[1] * gdims[2]
    p = lib.Pic(gdims, dx=d, dt=dt, c=c, q=q, max_particles=n, tile=8, precision=precision, shape=shape)
    gen = torch.Generator(device="cuda").manual_seed(167)
    L = torch.tensor(_lengths(gdims, d), dtype=p.dtype, device="cuda")[:, None]
    x0 = torch.rand((3, n), generator=gen, dtype=p.dtype, device="cuda") * L
    x0 = torch.minimum(x0, torch.nextafter(L, torch.zeros_like(L)))
    u = 0.5 * torch.randn((3, n), generator=gen, dtype=p.dtype, device="cuda")
    gam = torch.sqrt(1.0 + (u * u).sum(0, keepdim=True) / c**2)
    x1 = torch.remainder(x0 + dt * u / gam, L)
    x1 = torch.minimum(x1, torch.nextafter(L, torch.zeros_like(L)))
    g = torch.zeros((11,) + gshape, dtype=p.dtype, device="cuda")
    p.deposit(g, x0, x1, u)
    torch.cuda.synchronize()
    vol = float(np.prod(d))
    for k in (9, 10):
        tot = float(g[k].double().sum()) * vol
        assert abs(tot - n * q) <= (1e-9 if precision == "fp64" else 2e-5) * n * q, (k, tot)
    rng = synth.rng_for(168, 0)
    cells = np.stack([rng.integers(0, gdims[a], 48) for a in range(3)], axis=1)
    cells[0] = 0
    cells[1] = np.array(gdims) - 1
    sub = None
    for cx, cy, cz in cells:
        ctr = torch.tensor([cx * d[0], cy * d[1], cz * d[2]], dtype=p.dtype, device="cuda")[:, None]
        dist0 = torch.remainder(x0 - ctr + 0.5 * L, L) - 0.5 * L
        dist1 = torch.remainder(x1 - ctr + 0.5 * L, L) - 0.5 * L
        # every particle whose stencil can reach the cell: start (rho_old, and the mid-point
        # of J within a quarter cell of it) or end (rho_new) within 2.5 cells (the cubic
        # stencil reaches 2 cells)
        m = (dist0.abs() <= 2.5).all(0) | (dist1.abs() <= 2.5).all(0)
        sub = m if sub is None else sub | m
    idx = torch.nonzero(sub).squeeze(1)
    xs0, xs1, us = (t[:, idx].double().cpu().numpy().T for t in (x0, x1, u))
    J, r0, r1 = pic.sources(xs0, xs1, us, q, gshape, d, dt, c, order=shape)
    ref = np.concatenate([J, r0[None], r1[None]])
    got = g[6:].double().cpu().numpy()
    scale = np.abs(got).max()
    tol = 1e-12 if precision == "fp64" else 2e-5
    for cx, cy, cz in cells:
        err = np.abs(got[:, cz, cy, cx] - ref[:, cz, cy, cx]).max() / scale
        assert err <= tol, ((cx, cy, cz), err)
    p.close()
