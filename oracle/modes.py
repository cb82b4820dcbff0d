"""Oracle (test infrastructure): exact step output for inputs made of a few grid modes.

When every input field is a finite sum of Fourier modes that are periodic on
the box being transformed, the box DFT is exactly zero away from those modes,
so the PSATD step (Sec. 1.1 of arXiv:1812.07357: analytic integration in
k-space, exact for resolved modes) acts on each mode independently.  The
output at any grid point is then a short sum that costs O(number of modes),
which lets the tests check the GPU path point by point on grids far too large
for a full FP64 CPU transform.

A field is represented as f(x) = sum_j 2 Re(c_j exp(i k_j . x)) with k_j the
physical wave vector of mode j; the modes must be pairwise distinct, not
negatives of one another, and never the zero or a Nyquist mode of the box.
"""

from __future__ import annotations

import numpy as np

from . import kspace


def mode_wavevectors(m, dims, d):
    """Physical wave vectors 2 pi m / (N d) for integer modes ``m`` (nm, 3) on a grid ``dims`` (nx, ny, nz)."""
    m = np.asarray(m, dtype=np.float64)
    dx, dy, dz = (d, d, d) if np.isscalar(d) else d
    return np.stack([2 * np.pi * m[:, 0] / (dims[0] * dx),
                     2 * np.pi * m[:, 1] / (dims[1] * dy),
                     2 * np.pi * m[:, 2] / (dims[2] * dz)], axis=1)


def push_modes(kvec, coef_in, d, dt: float, order, nsteps: int = 1, c: float = 1.0, eps0: float = 1.0,
               staggered: bool = False):
    """Advance the complex mode amplitudes by ``nsteps`` PSATD steps, sources fixed.

    kvec: (nm, 3) physical wave vectors; coef_in: (11, nm) complex amplitudes of
    Ex Ey Ez Bx By Bz Jx Jy Jz rho_old rho_new.  ``order`` scalar or per axis.
    Returns (6, nm) complex amplitudes of E', B'.

    ``staggered``: the amplitudes describe each component at its own staggered
    position (``synthesize`` with the component's offset), where every
    staggered difference acts on a mode as i times the real staggered symbol.
    """
    dx, dy, dz = (d, d, d) if np.isscalar(d) else d
    px, py, pz = (order, order, order) if np.isscalar(order) else order
    sym = kspace.staggered_k_at if staggered else kspace.modified_k_at
    K = (sym(kvec[:, 0], dx, px),
         sym(kvec[:, 1], dy, py),
         sym(kvec[:, 2], dz, pz))
    coef = kspace.coefficients(K[0], K[1], K[2], dt, c)
    a = np.array(coef_in, dtype=np.complex128, copy=True)
    for _ in range(nsteps):
        En, Bn = kspace.push(a[0:3], a[3:6], a[6:9], a[9], a[10], K, coef, c, eps0)
        a[0:3] = En
        a[3:6] = Bn
    return a[0:6].copy()


def synthesize(kvec, coefs, positions):
    """Evaluate f(x) = sum_j 2 Re(c_j e^{i k_j.x}) at ``positions`` (npts, 3) (x, y, z lengths).

    coefs: (nf, nm) complex.  Returns (nf, npts) float64.
    """
    phase = np.exp(1j * (np.asarray(positions, dtype=np.float64) @ np.asarray(kvec).T))  # (npts, nm)
    return 2.0 * (np.asarray(coefs) @ phase.T).real


def synthesize_grid(kvec, coefs, shape, d, origin=(0, 0, 0)):
    """Evaluate the mode sum on every node of a (nz, ny, nx) grid, node (i,j,k) at ((origin+i) d, ...).

    Separable evaluation: exp(i k.x) = exp(i kx x) exp(i ky y) exp(i kz z).
    Returns (nf, nz, ny, nx) float64.
    """
    nz, ny, nx = shape
    dx, dy, dz = (d, d, d) if np.isscalar(d) else d
    x = (origin[0] + np.arange(nx)) * dx
    y = (origin[1] + np.arange(ny)) * dy
    z = (origin[2] + np.arange(nz)) * dz
    kvec = np.asarray(kvec)
    coefs = np.asarray(coefs)
    out = np.zeros((coefs.shape[0], nz, ny, nx))
    for j in range(kvec.shape[0]):
        ex = np.exp(1j * kvec[j, 0] * x)
        ey = np.exp(1j * kvec[j, 1] * y)
        ez = np.exp(1j * kvec[j, 2] * z)
        plane = ez[:, None, None] * ey[None, :, None] * ex[None, None, :]
        for f in range(coefs.shape[0]):
            if coefs[f, j] != 0:
                out[f] += 2.0 * (coefs[f, j] * plane).real
    return out
