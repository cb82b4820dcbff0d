"""Pins of the oracle's whole step: transforms + push on a box, guards, local vs global.

arXiv:1812.07357:
* Sec. 1.1: PSATD propagates resolved vacuum modes without numerical
  dispersion at infinite order; a finite order p propagates them with the
  dispersion of its modified wavenumber.  Gauss's law is kept with
  charge-conserving sources.
* Sec. 1.3: the local solver's only error is a truncation error at sub-domain
  boundaries when the stencil half width exceeds the guard width; it falls as
  guards widen, and a finite order can beat infinite order at fixed guards.
* Sec. 2.5.2: guards of G2 are filled from G1; the interior is copied back.
"""

import numpy as np
import pytest

import synth
from oracle import diagnostics, domain, kspace, modes, step


def _plane_waves(shape, d, order, c, nmodes, seed, t=0.0):
    """Forward-propagating vacuum plane waves of the order-p solver (closed form)."""
    rng = np.random.default_rng(seed)
    pw = synth.plane_wave_modes(rng, shape, nmodes)
    nz, ny, nx = shape
    dims = (nx, ny, nz)
    kvec = modes.mode_wavevectors(pw["m"], dims, d)
    ev, bv, om = [], [], []
    for j in range(nmodes):
        K = np.array([kspace.modified_k_at(abs(kvec[j, a]), d, order) * np.sign(kvec[j, a]) for a in range(3)])
        e = synth.transverse_unit(pw["u"][j], K)
        w = c * np.linalg.norm(K)
        ev.append(e)
        bv.append(np.cross(K, e) / w)
        om.append(w)
    return synth.plane_wave_sum(shape, d, pw["m"], pw["amp"], pw["phase"], ev, bv, om, t)


@pytest.mark.parametrize("order", [2, 4, 16, 100, 0])
def test_plane_waves_follow_closed_form_dispersion(order):
    shape, d, dt, c, nsteps = (12, 20, 18), 1.0, 0.7, 1.0, 10
    E0, B0 = _plane_waves(shape, d, order, c, 4, seed=order + 1)
    E1, B1 = _plane_waves(shape, d, order, c, 4, seed=order + 1, t=nsteps * dt)
    f = np.zeros((11,) + shape)
    f[0:3], f[3:6] = E0, B0
    out = step.box_steps(f, nsteps, d, dt, order, c)
    ref = np.concatenate([E1, B1])
    assert diagnostics.rel_l2(out, ref) <= 1e-12


def test_plane_wave_nonunit_c_and_anisotropic_spacing():
    shape, d, dt, c, order = (10, 14, 16), (0.8, 1.1, 1.3), 0.4, 2.3, 8
    rng = np.random.default_rng(5)
    pw = synth.plane_wave_modes(rng, shape, 3)
    nz, ny, nx = shape
    kvec = modes.mode_wavevectors(pw["m"], (nx, ny, nz), d)
    ev, bv, om = [], [], []
    for j in range(3):
        K = np.array([kspace.modified_k_at(abs(kvec[j, a]), d[a], order) * np.sign(kvec[j, a]) for a in range(3)])
        e = synth.transverse_unit(pw["u"][j], K)
        w = c * np.linalg.norm(K)
        ev.append(e), bv.append(np.cross(K, e) / w), om.append(w)
    E0, B0 = synth.plane_wave_sum(shape, d, pw["m"], pw["amp"], pw["phase"], ev, bv, om, 0.0)
    E1, B1 = synth.plane_wave_sum(shape, d, pw["m"], pw["amp"], pw["phase"], ev, bv, om, 5 * dt)
    f = np.zeros((11,) + shape)
    f[0:3], f[3:6] = E0, B0
    out = step.box_steps(f, 5, d, dt, order, c)
    assert diagnostics.rel_l2(out, np.concatenate([E1, B1])) <= 1e-12


def _config1_fields(shape=(32, 32, 32), d=1.0, dt=0.5, order=0, seed=1):
    """Config-1 style inputs: 4 vacuum plane waves + a Gaussian current blob, consistent rho."""
    rng = synth.rng_for(1, seed)
    pw = synth.plane_wave_modes(rng, shape, 4)
    nz, ny, nx = shape
    kvec = modes.mode_wavevectors(pw["m"], (nx, ny, nz), d)
    ev, bv = [], []
    for j in range(4):
        K = np.array([kspace.modified_k_at(abs(kvec[j, a]), d, order) * np.sign(kvec[j, a]) for a in range(3)])
        e = synth.transverse_unit(pw["u"][j], K)
        ev.append(e), bv.append(np.cross(K, e) / np.linalg.norm(K))
    E, B = synth.plane_wave_sum(shape, d, pw["m"], pw["amp"], pw["phase"], ev, bv)
    direction = rng.normal(size=3)
    J = synth.gaussian_blob(shape, d, (nx * d / 2, ny * d / 2, nz * d / 2), 3.0, 0.1, direction)
    rho_old = diagnostics.rho_from_gauss(E, d, order)
    rho_new = diagnostics.rho_continuity(rho_old, J, dt, d, order)
    return np.concatenate([E, B, J, rho_old[None], rho_new[None]])


@pytest.mark.parametrize("order", [0, 8])
def test_gauss_law_kept_over_ten_steps(order):
    d, dt = 1.0, 0.5
    shape = (16, 20, 24)
    f = _config1_fields(shape=shape, order=order)
    # add an electrostatic (non-solenoidal) blob so that rho is not zero
    f[0:3] += synth.gaussian_blob(shape, d, (9.0, 11.0, 7.0), 2.5, 0.7, (1.0, -0.5, 0.3))
    f[9] = diagnostics.rho_from_gauss(f[0:3], d, order)
    f[10] = diagnostics.rho_continuity(f[9], f[6:9], dt, d, order)
    assert diagnostics.gauss_residual(f[0:3], f[9], d, order) <= 1e-13
    for _ in range(10):
        f[0:6] = step.box_step(f, d, dt, order)
        # rho advances by continuity with the same (constant) current
        f[9] = f[10]
        f[10] = diagnostics.rho_continuity(f[9], f[6:9], dt, d, order)
        assert diagnostics.gauss_residual(f[0:3], f[9], d, order) <= 1e-12
        assert diagnostics.div_b(f[3:6], d, order) <= 1e-13


def test_vacuum_energy_conserved_over_100_steps():
    shape, d, dt, order = (12, 10, 14), 1.0, 0.9, 16
    rng = np.random.default_rng(21)
    E = diagnostics.project_divfree(rng.standard_normal((3,) + shape), d, order)
    B = diagnostics.project_divfree(rng.standard_normal((3,) + shape), d, order)
    f = np.zeros((11,) + shape)
    f[0:3], f[3:6] = E, B
    w0 = diagnostics.energy(E, B)
    for _ in range(100):
        f[0:6] = step.box_step(f, d, dt, order)
    assert abs(diagnostics.energy(f[0:3], f[3:6]) - w0) <= 1e-13 * w0


def _brute_fill(g1, origin, interior, ng):
    nf, NZ, NY, NX = g1.shape
    nx, ny, nz = interior
    box = np.zeros((nf, nz + 2 * ng, ny + 2 * ng, nx + 2 * ng))
    for k in range(nz + 2 * ng):
        for j in range(ny + 2 * ng):
            for i in range(nx + 2 * ng):
                box[:, k, j, i] = g1[:, (origin[2] - ng + k) % NZ, (origin[1] - ng + j) % NY,
                                     (origin[0] - ng + i) % NX]
    return box


@pytest.mark.parametrize("origin,interior,ng", [((0, 0, 0), (4, 3, 5), 0), ((2, 5, 1), (3, 4, 2), 2),
                                                ((6, 1, 3), (2, 2, 2), 9)])
def test_guard_fill_and_merge_brute_force(origin, interior, ng):
    rng = np.random.default_rng(3)
    g1 = rng.standard_normal((2, 5, 6, 7))
    box = domain.guard_fill(g1, origin, interior, ng)
    np.testing.assert_array_equal(box, _brute_fill(g1, origin, interior, ng))
    tgt = np.zeros_like(g1)
    newbox = rng.standard_normal(box.shape)
    domain.guard_merge(newbox, tgt, origin, interior, ng)
    nf, NZ, NY, NX = g1.shape
    expect = np.zeros_like(g1)
    nx, ny, nz = interior
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                expect[:, (origin[2] + k) % NZ, (origin[1] + j) % NY, (origin[0] + i) % NX] = \
                    newbox[:, ng + k, ng + j, ng + i]
    np.testing.assert_array_equal(tgt, expect)


def test_single_box_without_guards_equals_global_solve():
    f = _config1_fields(shape=(16, 12, 20))
    boxes = [{"origin": (0, 0, 0), "interior": (20, 12, 16), "nguard": 0, "order": 0}]
    a = domain.local_steps(f, boxes, 3, 1.0, 0.5)
    b = domain.global_steps(f, 3, 1.0, 0.5, 0)
    np.testing.assert_array_equal(a, b)


def _truncation_error(order, ng, nsteps=6, seed=0):
    """max |local - global| / max |global| on a 2x2x2 split of a 32^3 periodic grid."""
    shape, d, dt = (32, 32, 32), 1.0, 0.5
    rng = np.random.default_rng(seed)
    x = np.arange(32)
    # a smooth, band-limited pulse so that truncation (not resolution) dominates
    g = np.exp(-((x - 16.0) / 4.0) ** 2)
    E = np.zeros((3,) + shape)
    E[1] = g[None, None, :] * np.cos(2 * np.pi * x / 8.0)[None, None, :] * np.ones((32, 32, 1))
    B = np.zeros((3,) + shape)
    B[2] = E[1]
    f = np.zeros((11,) + shape)
    f[0:3], f[3:6] = E, B
    del rng
    boxes = [{"origin": (ox, oy, oz), "interior": (16, 16, 16), "nguard": ng, "order": order}
             for oz in (0, 16) for oy in (0, 16) for ox in (0, 16)]
    loc = domain.local_steps(f, boxes, nsteps, d, dt)[0:6]
    glo = domain.global_steps(f, nsteps, d, dt, order)[0:6]
    return np.abs(loc - glo).max() / np.abs(glo).max()


def test_local_error_falls_with_guards_and_finite_order_helps():
    e = {ng: _truncation_error(16, ng) for ng in (2, 4, 8)}
    assert e[2] > e[4] > e[8]
    assert e[8] < 1e-3
    # at fixed guards a moderate finite order truncates less than infinite order
    assert _truncation_error(16, 4) < _truncation_error(0, 4)
