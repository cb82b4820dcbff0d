"""Pins of the oracle's two-step PML (oracle/pml.py; arXiv:1812.07357, Sec. 2.6).

* Without damping the split box is the ordinary box: the sums of the split parts
  after several steps equal ``step.box_step`` (pinned elsewhere against closed
  forms), for arbitrary fields and sources.
* The split of each increment between its two parts is checked against the
  matrix exponential of the split system itself, mode by mode: the twelve split
  amplitudes of one Fourier mode obey a linear ODE with constant sources (each
  part driven by its own derivative of the full fields, the source drive -J/eps0
  on set A), integrated exactly by scipy's expm of the augmented 13 x 13 matrix.
  Charges follow Gauss's law and continuity, and the full B is divergence-free, so
  that the rho-form step is the exact solution of that system.
* A pulse launched into the layers is absorbed (the residual after it would have
  wrapped around the periodic box is below 1 % of its peak; without the layers the
  whole pulse comes back), for propagation along each axis: damping applied along
  the wrong axis for any split part leaves that part unabsorbed.
* The conductivity profile: zero inside, sigma_max at the outer cells, the
  stated power law.
"""

import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import kspace, pml, step


def test_profile():
    s = pml.sigma_profile(20, 4, 2.0, 2.0)
    assert np.all(s[4:16] == 0.0)
    np.testing.assert_allclose(s[:4], 2.0 * (np.array([4, 3, 2, 1]) / 4.0) ** 2)
    np.testing.assert_allclose(s[16:], 2.0 * (np.array([1, 2, 3, 4]) / 4.0) ** 2)


@pytest.mark.parametrize("order", [4, 0])
def test_undamped_split_box_is_the_ordinary_box(order):
    shape = (10, 12, 14)
    rng = synth.rng_for(190, order)
    split = rng.normal(size=(12,) + shape)
    src = 0.3 * rng.normal(size=(5,) + shape)
    d, dt, c, eps0 = (1.0, 0.8, 1.2), 0.4, 1.1, 0.9
    damp = pml.damping(shape, (0, 0, 0), 0.0, 2.0, dt)
    got = pml.pml_steps(split, src, 3, d, dt, order, damp, c, eps0)
    full = np.concatenate([split[0:3] + split[6:9], split[3:6] + split[9:12], src])
    ref = step.box_steps(full, 3, d, dt, order, c, eps0)
    sums = np.concatenate([got[0:3] + got[6:9], got[3:6] + got[9:12]])
    np.testing.assert_allclose(sums, ref[0:6], atol=1e-12 * np.abs(ref[0:6]).max())


def _split_matrix(K, c, eps0):
    """Affine ODE of one mode: state [EA(3), BA(3), EB(3), BB(3), 1], sources J via the last column."""
    M = np.zeros((13, 13), dtype=np.complex128)
    c2 = c * c
    EA, BA, EB, BB = 0, 3, 6, 9
    for a in range(3):
        b, cc = (a + 1) % 3, (a + 2) % 3
        # each part is driven by its derivative of the FULL field (set A + set B):
        # dE_a^A/dt = i c^2 K_b B_c, dE_a^B/dt = -i c^2 K_c B_b
        for s in (BA, BB):
            M[EA + a, s + cc] += 1j * c2 * K[b]
            M[EB + a, s + b] += -1j * c2 * K[cc]
        # dB_a^A/dt = -i K_b E_c, dB_a^B/dt = +i K_c E_b
        for s in (EA, EB):
            M[BA + a, s + cc] += -1j * K[b]
            M[BB + a, s + b] += 1j * K[cc]
    return M


@pytest.mark.parametrize("order", [8, 0])
def test_split_increments_equal_the_exact_split_evolution(order):
    shape, d, dt, c, eps0 = (6, 8, 10), (1.0, 0.9, 1.1), 0.45, 1.3, 0.7
    kx, ky, kz = kspace.k_grids(shape, d, order)
    rng = synth.rng_for(191, order)
    checked = 0
    for (iz, iy, ix) in [(1, 2, 3), (0, 3, 1), (2, 0, 0), (5, 7, 9), (3, 4, 5), (0, 0, 0)]:
        K = np.array([kx[0, 0, ix], ky[0, iy, 0], kz[iz, 0, 0]])
        coef = kspace.coefficients(K[0], K[1], K[2], dt, c)
        EA = rng.normal(size=3) + 1j * rng.normal(size=3)
        EB = rng.normal(size=3) + 1j * rng.normal(size=3)
        BA = rng.normal(size=3) + 1j * rng.normal(size=3)
        BB = rng.normal(size=3) + 1j * rng.normal(size=3)
        J = rng.normal(size=3) + 1j * rng.normal(size=3)
        # div B = 0 for the full field (the rho-form step scales a longitudinal B by C,
        # the exact system keeps it): move the longitudinal part of set A onto set B
        k2 = float(K @ K)
        if k2 > 0:
            BA = BA - K * (K @ (BA + BB)) / k2
        E, Bf = EA + EB, BA + BB
        ro = 1j * eps0 * (K @ E)                 # Gauss's law
        rn = ro - 1j * dt * (K @ J)              # continuity
        M = _split_matrix(K, c, eps0)
        for a in range(3):
            M[a, 12] = -J[a] / eps0              # source drive on set A
        x0 = np.concatenate([EA, BA, EB, BB, [1.0]])
        x1 = scipy.linalg.expm(M * dt) @ x0
        inc = x1[:12] - x0[:12]
        dEA, dBA, dEB, dBB = pml.split_increments(list(E), list(Bf), list(J), ro, rn, list(K), coef, dt, c, eps0)
        got = np.concatenate([dEA, dBA, dEB, dBB]).astype(np.complex128)
        scale = np.abs(inc).max() + 1e-300
        assert np.abs(got - inc).max() <= 1e-11 * max(scale, 1.0), (iz, iy, ix, np.abs(got - inc).max())
        checked += 1
    assert checked == 6


def _pulse(shape, axis, d, c, width_cells=6.0, k0=0.6):
    """A plane-wave packet travelling along +axis: E along the next axis, B along the third."""
    nz, ny, nx = shape
    n = (nx, ny, nz)[axis]
    coord = np.arange(n) * d
    env = np.exp(-((coord - 0.5 * n * d) / (width_cells * d)) ** 2) * np.cos(k0 * coord)
    f = np.zeros((12,) + shape)
    e_comp, b_comp = (axis + 1) % 3, (axis + 2) % 3
    if axis == 0:
        prof = env[None, None, :]
    elif axis == 1:
        prof = env[None, :, None]
    else:
        prof = env[:, None, None]
    # E_{e_comp} is driven by the derivative along `axis` = e_comp + 2 -> set B;
    # B_{b_comp} by the derivative along `axis` = b_comp + 1 -> set A.
    f[6 + e_comp] = np.broadcast_to(prof, shape)
    f[3 + b_comp] = np.broadcast_to(prof, shape) / c
    return f


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_layers_absorb_an_outgoing_pulse(axis):
    n_long, n_short, w = 128, 4, 24
    shape = [n_short, n_short, n_short]
    shape[2 - axis] = n_long
    shape = tuple(shape)
    d, dt, c, order = 1.0, 0.5, 1.0, 16
    widths = [0, 0, 0]
    widths[axis] = w
    f0 = _pulse(shape, axis, d, c)
    src = np.zeros((5,) + shape)
    peak = np.abs(f0).max()
    nsteps = int(1.0 * n_long * d / (c * dt))   # the packet crosses the box once
    inner = [slice(None)] * 3
    inner[2 - axis] = slice(w, n_long - w)
    inner = tuple(inner)
    free = pml.pml_steps(f0, src, nsteps, d, dt, order, pml.damping(shape, (0, 0, 0), 0.0, 2.0, dt), c)
    assert np.abs(free[(slice(None),) + inner]).max() > 0.5 * peak    # it wrapped around
    sigma_max = 3.0 * np.log(1e4) * c / (2 * w * d)
    out = pml.pml_steps(f0, src, nsteps, d, dt, order, pml.damping(shape, widths, sigma_max, 2.0, dt), c)
    assert np.abs(out[(slice(None),) + inner]).max() < 1e-2 * peak
