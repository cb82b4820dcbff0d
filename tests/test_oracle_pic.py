"""Pins of the oracle's particle side of the PIC cycle (arXiv:1812.07357, Sec. 2.5.1).

Linear (cloud-in-cell) weights are checked against the tent function evaluated on
every grid point of a tiny periodic grid (an independent formulation), charge
deposition against exact conservation, gathering against exact interpolation of
linear fields and against its adjoint relation to deposition, and the Boris push
against closed forms: a pure electric field adds q E dt / m to u every step, a
pure magnetic field rotates u by exactly 2 atan(q B dt / (2 m gamma)) per step
without changing |u|, and crossed fields produce the E x B drift.
"""

import numpy as np
import pytest

import synth
from oracle import pic


def _tent_weights(pos, gshape, d, offset):
    """Weight of every grid point for every particle: prod over axes of max(0, 1 - |s - i|)
    with s the particle's coordinate in cells (minus the offset), over periodic images."""
    nz, ny, nx = gshape
    out = np.zeros((pos.shape[0],) + tuple(gshape))
    for p in range(pos.shape[0]):
        ax = []
        for a, n in enumerate((nx, ny, nz)):
            s = pos[p, a] / d[a] - 0.5 * offset[a]
            i = np.arange(n)
            w = np.zeros(n)
            for img in (-1, 0, 1):  # periodic images of the grid
                w += np.maximum(0.0, 1.0 - np.abs(s - (i + img * n)))
            ax.append(w)
        out[p] = ax[2][:, None, None] * ax[1][None, :, None] * ax[0][None, None, :]
    return out


@pytest.mark.parametrize("offset", [(0, 0, 0), (1, 0, 0), (0, 1, 1), (1, 1, 1)])
def test_cic_weights_equal_the_tent_function(offset):
    gshape, d = (5, 4, 6), (0.7, 1.1, 0.9)
    rng = synth.rng_for(150, sum(offset))
    L = np.array([gshape[2] * d[0], gshape[1] * d[1], gshape[0] * d[2]])
    pos = rng.uniform(0, 1, size=(40, 3)) * L
    pos[0] = [0.0, 0.0, 0.0]                   # on a node
    pos[1] = L - 1e-12                         # at the periodic edge
    idx, w = pic.cic(pos, gshape, d, offset)
    got = np.zeros((pos.shape[0], int(np.prod(gshape))))
    for p in range(pos.shape[0]):
        np.add.at(got[p], idx[p], w[p])
    ref = _tent_weights(pos, gshape, d, offset).reshape(pos.shape[0], -1)
    np.testing.assert_allclose(got, ref, atol=1e-12)


def test_deposit_conserves_charge_and_is_adjoint_to_gather():
    gshape, d = (8, 6, 10), (1.0, 0.8, 1.2)
    rng = synth.rng_for(151, 0)
    L = np.array([gshape[2] * d[0], gshape[1] * d[1], gshape[0] * d[2]])
    pos = rng.uniform(0, 1, size=(500, 3)) * L
    q = rng.normal(size=500)
    vol = np.prod(d)
    for off in ((0, 0, 0), (1, 0, 1)):
        rho = pic.deposit(q, pos, gshape, d, off)
        assert abs(rho.sum() * vol - q.sum()) <= 1e-12 * np.abs(q).sum()
        F = rng.normal(size=gshape)
        lhs = float(np.sum(F * rho) * vol)
        rhs = float(np.sum(q * pic.gather(F, pos, d, off)))
        assert abs(lhs - rhs) <= 1e-12 * np.abs(q).sum() * np.abs(F).max()


def test_gather_interpolates_linear_fields_exactly():
    gshape, d = (6, 7, 8), (0.5, 1.0, 2.0)
    nz, ny, nx = gshape
    a, b = 0.3, np.array([1.7, -0.4, 0.9])
    for off in ((0, 0, 0), (1, 1, 0)):
        x = (np.arange(nx) + 0.5 * off[0]) * d[0]
        y = (np.arange(ny) + 0.5 * off[1]) * d[1]
        z = (np.arange(nz) + 0.5 * off[2]) * d[2]
        F = a + b[0] * x[None, None, :] + b[1] * y[None, :, None] + b[2] * z[:, None, None]
        rng = synth.rng_for(152, off[0])
        # positions whose stencil does not wrap (a linear field is not periodic)
        lo = np.array([0.5 * off[0] * d[0], 0.5 * off[1] * d[1], 0.5 * off[2] * d[2]])
        hi = lo + np.array([(nx - 1) * d[0], (ny - 1) * d[1], (nz - 1) * d[2]])
        pos = lo + rng.uniform(0.01, 0.99, size=(100, 3)) * (hi - lo)
        got = pic.gather(F, pos, d, off)
        np.testing.assert_allclose(got, a + pos @ b, rtol=0, atol=1e-12)


def test_boris_pure_electric_field_kicks_exactly():
    rng = synth.rng_for(153, 0)
    u = rng.normal(size=(10, 3))
    E = rng.normal(size=(10, 3))
    out = pic.boris(u, E, np.zeros((10, 3)), q_over_m=-1.3, dt=0.2, c=1.0)
    np.testing.assert_allclose(out, u + (-1.3) * 0.2 * E, rtol=0, atol=1e-14)


def test_boris_pure_magnetic_field_rotates_by_the_boris_angle():
    u0 = np.array([[0.3, 0.1, 0.05]])
    B = np.array([[0.0, 0.0, 2.0]])
    qm, dt, c, n = 1.0, 0.1, 1.0, 400
    gamma = np.sqrt(1 + np.sum(u0 ** 2) / c ** 2)
    u = u0.copy()
    for _ in range(n):
        u = pic.boris(u, np.zeros((1, 3)), B, qm, dt, c)
    assert abs(np.linalg.norm(u) - np.linalg.norm(u0)) <= 1e-13
    theta = 2 * np.arctan(0.5 * qm * dt * B[0, 2] / gamma)  # per step, clockwise for q B_z > 0
    ang = np.arctan2(u0[0, 1], u0[0, 0]) - n * theta
    ref = np.array([np.hypot(u0[0, 0], u0[0, 1]) * np.cos(ang), np.hypot(u0[0, 0], u0[0, 1]) * np.sin(ang),
                    u0[0, 2]])
    np.testing.assert_allclose(u[0], ref, atol=1e-12)


def test_boris_crossed_fields_drift_at_e_cross_b():
    E = np.array([[0.0, 1e-3, 0.0]])
    B = np.array([[0.0, 0.0, 1.0]])
    qm, dt, c = 1.0, 0.05, 1.0
    u = np.zeros((1, 3))
    vs = []
    for _ in range(20000):  # ~160 gyro periods
        u = pic.boris(u, E, B, qm, dt, c)
        vs.append(u[0] / np.sqrt(1 + np.sum(u ** 2)))
    drift = np.mean(vs, axis=0)
    np.testing.assert_allclose(drift, np.cross(E[0], B[0]) / np.dot(B[0], B[0]), rtol=0, atol=2e-5)


def test_sources_of_resting_and_moving_particles():
    gshape, d, dt = (6, 6, 6), (1.0, 1.0, 1.0), 0.5
    rng = synth.rng_for(154, 0)
    x = rng.uniform(0, 6, size=(50, 3))
    u = np.zeros((50, 3))
    J, r0, r1 = pic.sources(x, x, u, 0.2, gshape, d, dt)
    assert np.abs(J).max() == 0.0
    np.testing.assert_allclose(r0, r1, atol=0)
    u = np.tile([0.6, 0.0, 0.0], (50, 1))
    v = 0.6 / np.sqrt(1 + 0.36)
    xn = np.mod(x + dt * np.array([v, 0, 0]), 6.0)
    J, r0, r1 = pic.sources(x, xn, u, 0.2, gshape, d, dt)
    # a uniform drift along x: total current = N q v, none across
    assert abs(J[0].sum() - 50 * 0.2 * v) <= 1e-12
    assert abs(J[1]).max() == 0.0 and abs(J[2]).max() == 0.0
    assert abs(r1.sum() - r0.sum()) <= 1e-12


def _bspline(x, k):
    """Centred cardinal B-spline of degree k from the truncated-power formula
    B(x) = (1/k!) sum_j (-1)^j C(k+1, j) (x + (k+1)/2 - j)_+^k (independent of shape_1d)."""
    from math import comb, factorial

    out = np.zeros_like(x, dtype=np.float64)
    for j in range(k + 2):
        t = x + 0.5 * (k + 1) - j
        out += (-1) ** j * comb(k + 1, j) * np.where(t > 0, t, 0.0) ** k
    return out / factorial(k)


@pytest.mark.parametrize("order", [1, 2, 3])
def test_shape_weights_equal_the_centred_b_spline(order):
    rng = synth.rng_for(155, order)
    s = np.concatenate([rng.uniform(-3.0, 7.0, 400), [0.0, 0.5, 1.0, -0.5, 2.25]])
    first, w = pic.shape_1d(s, order)
    for p in range(len(s)):
        i = np.arange(first[p] - 2, first[p] + order + 3)
        ref = _bspline(s[p] - i, order)
        got = np.zeros_like(ref)
        got[2:2 + order + 1] = w[p]
        np.testing.assert_allclose(got, ref, atol=1e-13)


@pytest.mark.parametrize("order", [1, 2, 3])
def test_shape_moments(order):
    """sum w = 1 and sum w (i - s) = 0 for every position; for degree >= 2, which reproduces
    quadratics, also sum w (i - s)^2 = (order + 1) / 12, the B-spline's variance."""
    s = synth.rng_for(156, order).uniform(-5.0, 5.0, 1000)
    first, w = pic.shape_1d(s, order)
    i = first[:, None] + np.arange(order + 1)[None, :]
    np.testing.assert_allclose(w.sum(1), 1.0, atol=1e-14)
    np.testing.assert_allclose((w * (i - s[:, None])).sum(1), 0.0, atol=1e-13)
    if order >= 2:
        np.testing.assert_allclose((w * (i - s[:, None]) ** 2).sum(1), (order + 1) / 12.0, atol=1e-13)


@pytest.mark.parametrize("order", [2, 3])
def test_higher_order_deposit_conserves_charge_and_is_adjoint(order):
    gshape, d = (8, 6, 10), (1.0, 0.8, 1.2)
    rng = synth.rng_for(157, order)
    L = np.array([gshape[2] * d[0], gshape[1] * d[1], gshape[0] * d[2]])
    pos = rng.uniform(0, 1, size=(300, 3)) * L
    q = rng.normal(size=300)
    vol = np.prod(d)
    for off in ((0, 0, 0), (1, 0, 1)):
        rho = pic.deposit(q, pos, gshape, d, off, order)
        assert abs(rho.sum() * vol - q.sum()) <= 1e-12 * np.abs(q).sum()
        F = rng.normal(size=gshape)
        lhs = float(np.sum(F * rho) * vol)
        rhs = float(np.sum(q * pic.gather(F, pos, d, off, order)))
        assert abs(lhs - rhs) <= 1e-12 * np.abs(q).sum() * np.abs(F).max()
