"""Pins of the oracle's staggered (Yee) grid variant.

arXiv:1812.07357, Sec. 1.1 and 1.3: the solver of order p takes its derivatives
from a stencil of half width p/2 and p -> inf is spectral; the production codes
the paper builds on keep E and B on a staggered grid.  The oracle's staggered
step (half-cell shift factors around a push with the real staggered symbol) is
pinned here by routes that share none of its code:

* the staggered weights against the textbook table and against the exact
  moment equations solved in rationals;
* the whole step against the matrix exponential of the semi-discrete Maxwell
  system written in REAL space with the staggered difference stencils on a tiny
  periodic grid (even and odd sizes, so Nyquist modes are included), with
  sources held constant over the step and charges consistent with the
  discrete Gauss law and continuity; the collocated variant is pinned the same
  way with centred stencils;
* plane waves sampled at each component's own half-cell position, against
  their closed-form evolution at the staggered dispersion relation.
"""

import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import kspace, modes, step

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "staggered_difference_weights.txt")


def _golden():
    out = {}
    for line in open(GOLDEN):
        line = line.strip()
        if line and not line.startswith("#"):
            p, rest = line.split(":")
            out[int(p)] = [Fraction(t) for t in rest.split()]
    return out


def test_staggered_weights_match_textbook_table():
    for p, w in _golden().items():
        assert kspace.staggered_weights(p) == w


@pytest.mark.parametrize("p", [2, 4, 6, 10, 16, 32])
def test_staggered_weights_solve_moment_equations(p):
    """Exact for polynomials through degree p: sum_l alpha_l 2 ((2l-1)/2)^(2q+1) = [q == 0]."""
    m = p // 2
    A = [[Fraction(2) * Fraction(2 * l - 1, 2) ** (2 * q + 1) for l in range(1, m + 1)] for q in range(m)]
    b = [Fraction(int(q == 0)) for q in range(m)]
    for i in range(m):  # exact Gauss-Jordan elimination
        piv = next(r for r in range(i, m) if A[r][i] != 0)
        A[i], A[piv], b[i], b[piv] = A[piv], A[i], b[piv], b[i]
        for r in range(m):
            if r != i and A[r][i] != 0:
                f = A[r][i] / A[i][i]
                A[r] = [A[r][c] - f * A[i][c] for c in range(m)]
                b[r] -= f * b[i]
    assert [b[i] / A[i][i] for i in range(m)] == kspace.staggered_weights(p)


def test_staggered_symbol_limits():
    k = np.linspace(-np.pi, np.pi, 101)
    np.testing.assert_allclose(kspace.staggered_k_at(k, 1.0, 2), 2 * np.sin(k / 2), rtol=0, atol=1e-15)
    err = [np.abs(kspace.staggered_k_at(k, 1.0, p) - k).max() for p in (2, 8, 32, 128)]
    assert all(a > b for a, b in zip(err, err[1:])), err
    # at the Nyquist wavenumber the staggered symbol tends to pi (not zero, unlike the centred one)
    ny = [float(kspace.staggered_k_at(np.pi, 1.0, p)) for p in (2, 4, 16, 64, 256)]
    assert ny[0] == pytest.approx(2.0) and ny[1] == pytest.approx(2 * (9 / 8 + 1 / 24))
    assert all(a < b < np.pi for a, b in zip(ny, ny[1:]))
    assert np.pi - ny[-1] < 0.15  # slow (algebraic) approach to pi


# ------------------------------------------------------------------ real-space semi-discrete system
def _diff_1d(n, d, order, kind):
    """Dense n x n periodic difference matrix along one axis.

    kind 'c': centred, nodes to nodes; 'p': staggered, nodes (i) to half points (i + 1/2,
    stored at i); 'm': staggered, half points (i + 1/2 at i) to nodes (i).
    """
    D = np.zeros((n, n))
    if kind == "c":
        for l, a in enumerate(kspace.fd_weights(order), start=1):
            for i in range(n):
                D[i, (i + l) % n] += float(a) / d
                D[i, (i - l) % n] -= float(a) / d
    else:
        for l, a in enumerate(kspace.staggered_weights(order), start=1):
            for i in range(n):
                if kind == "p":
                    D[i, (i + l) % n] += float(a) / d
                    D[i, (i - l + 1) % n] -= float(a) / d
                else:
                    D[i, (i + l - 1) % n] += float(a) / d
                    D[i, (i - l) % n] -= float(a) / d
    return D


def _axis_ops(shape, d, order, kind):
    """Difference along x, y, z on flattened (nz, ny, nx) arrays (x fastest)."""
    nz, ny, nx = shape
    dx, dy, dz = d
    Ix, Iy, Iz = np.eye(nx), np.eye(ny), np.eye(nz)
    return (np.kron(Iz, np.kron(Iy, _diff_1d(nx, dx, order, kind))),
            np.kron(Iz, np.kron(_diff_1d(ny, dy, order, kind), Ix)),
            np.kron(_diff_1d(nz, dz, order, kind), np.kron(Iy, Ix)))


def _real_space_step(shape, d, order, staggered, dt, c, eps0, rng):
    """Inputs and the exact one-step result of the real-space semi-discrete system."""
    N = int(np.prod(shape))
    if staggered:
        P = _axis_ops(shape, d, order, "p")  # node -> half point
        M = _axis_ops(shape, d, order, "m")  # half point -> node
    else:
        P = M = _axis_ops(shape, d, order, "c")
    Z = np.zeros((N, N))
    # curl of E-located fields (gives B-located ones) and of B-located fields (gives E-located)
    curl_e = np.block([[Z, -P[2], P[1]], [P[2], Z, -P[0]], [-P[1], P[0], Z]])
    curl_b = np.block([[Z, -M[2], M[1]], [M[2], Z, -M[0]], [-M[1], M[0], Z]])
    div_e = np.hstack([M[0], M[1], M[2]])
    E = rng.normal(size=3 * N)
    J = rng.normal(size=3 * N)
    B = curl_e @ rng.normal(size=3 * N)  # divergence-free by construction
    rho_old = eps0 * (div_e @ E)
    rho_new = rho_old - dt * (div_e @ J)
    # d/dt (E, B) = (c^2 curl B - J / eps0, -curl E), J constant: augmented matrix exponential
    A = np.zeros((6 * N + 1, 6 * N + 1))
    A[:3 * N, 3 * N:6 * N] = c * c * curl_b
    A[3 * N:6 * N, :3 * N] = -curl_e
    A[:3 * N, 6 * N] = -J / eps0
    u = scipy.linalg.expm(A * dt) @ np.concatenate([E, B, [1.0]])
    fields = np.concatenate([E, B, J, rho_old, rho_new]).reshape((11,) + tuple(shape))
    return fields, u[:6 * N].reshape((6,) + tuple(shape))


@pytest.mark.parametrize("staggered", [True, False])
@pytest.mark.parametrize("shape,order", [((4, 5, 6), 2), ((6, 4, 5), 4), ((5, 6, 4), 6), ((3, 4, 8), 8)])
def test_step_equals_matrix_exponential_of_the_real_space_system(staggered, shape, order):
    d, dt, c, eps0 = (0.9, 1.1, 0.8), 0.37, 1.3, 0.7
    fields, exact = _real_space_step(shape, d, order, staggered, dt, c, eps0,
                                     synth.rng_for(130, order + 10 * staggered))
    got = step.box_step(fields, d, dt, order, c, eps0, staggered=staggered)
    err = np.abs(got - exact).max() / np.abs(exact).max()
    assert err <= 1e-12, err


@pytest.mark.parametrize("order", [2, 4, 16, 0])
def test_staggered_plane_waves_follow_the_staggered_dispersion(order):
    """Plane waves sampled at each component's half-cell position, 10 steps, closed form."""
    shape, d, dt = (12, 10, 16), 1.0, 0.45
    nz, ny, nx = shape
    rng = synth.rng_for(131, order)
    m = np.array([[3, -2, 1], [-5, 4, 2], [1, 1, -6], [7, 0, 3]])
    kvec = modes.mode_wavevectors(m, (nx, ny, nz), d)
    ks = np.stack([kspace.staggered_k_at(kvec[:, a], d, order) for a in range(3)], axis=1)
    coefs = np.zeros((11, len(m)), dtype=np.complex128)
    for j in range(len(m)):
        u = rng.normal(size=3) + 1j * rng.normal(size=3)
        kh = ks[j] / np.linalg.norm(ks[j])
        e = u - kh * (kh @ u)  # transverse to K_s: no charge
        coefs[0:3, j] = e
        coefs[3:6, j] = np.cross(kh, e)
    grid = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"), -1)
    grid = grid.transpose(2, 1, 0, 3).reshape(-1, 3).astype(np.float64)  # (z, y, x) order, x fastest

    def sample(cf):
        out = np.zeros((cf.shape[0],) + shape)
        for f in range(cf.shape[0]):
            pos = (grid + 0.5 * np.array(kspace.STAGGER_OFFSETS[f])) * d
            out[f] = modes.synthesize(kvec, cf[f:f + 1], pos)[0].reshape(shape)
        return out

    fields = sample(coefs)
    got = step.box_steps(fields, 10, d, dt, order, staggered=True)
    exact = sample(modes.push_modes(kvec, coefs, d, dt, order, nsteps=10, staggered=True))
    err = np.abs(got - exact).max() / np.abs(exact).max()
    assert err <= 1e-12, err
    # the same waves are not solutions of the collocated solver (the pin sees the staggering)
    wrong = step.box_steps(fields, 10, d, dt, order, staggered=False)
    assert np.abs(wrong - exact).max() / np.abs(exact).max() > 1e-3
