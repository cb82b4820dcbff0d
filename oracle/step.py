"""Oracle (test infrastructure): one PSATD step on one periodic box, FP64.

Sec. 1.1 of arXiv:1812.07357: the fields are Fourier-transformed in space,
advanced analytically over dt in k-space, and transformed back.  Fig. 1(a):
with the local decomposition each guard-padded box is treated as a periodic
domain of its own and transformed with a shared-memory (here: single-host)
FFT.  Reading: forward transform sum_x f(x) e^{-i k.x} (unnormalised), inverse
with 1/N; complex C2C throughout.
"""

from __future__ import annotations

import os

import numpy as np
import scipy.fft as sfft

from . import kspace

# Threads handed to the library FFT; the rest of the oracle is single-threaded numpy.
WORKERS = max(1, int(os.environ.get("ORACLE_FFT_WORKERS", "1")))


def fft3(a):
    """Forward complex 3D DFT over the last three axes (z, y, x), unnormalised."""
    return sfft.fftn(np.asarray(a, dtype=np.complex128), axes=(-3, -2, -1), workers=WORKERS)


def ifft3(a):
    """Inverse complex 3D DFT over the last three axes, with the 1/N factor."""
    return sfft.ifftn(a, axes=(-3, -2, -1), workers=WORKERS)


def real_part(z, rel_tol: float = 1e-12, scale: float = 0.0):
    """Real part of an inverse transform whose input is Hermitian up to round-off.

    Raises if the imaginary part exceeds ``rel_tol`` times max(max|Re z|, scale)
    (it would mean the push broke the Hermitian symmetry of real fields);
    ``scale`` is the magnitude of the data the transform came from.
    """
    re = z.real
    ref = max(float(np.abs(re).max()), float(scale), 1e-300)
    im = float(np.abs(z.imag).max())
    if im > rel_tol * ref:
        raise AssertionError(f"inverse transform not real: max|Im|={im:.3e}, reference {ref:.3e}")
    return re.copy()


def box_step(fields, d, dt: float, order, c: float = 1.0, eps0: float = 1.0, imag_tol: float = 1e-12,
             staggered: bool = False):
    """Advance E, B of one periodic box by one step.

    ``fields``: array (11, nz, ny, nx) in the order Ex Ey Ez Bx By Bz Jx Jy Jz
    rho_old rho_new (J at the half step, rho at the start and at the end of the
    step).  ``d`` and ``order`` are scalars or per-axis (x, y, z) triples; order 0
    is the infinite-order (spectral) solver.  Returns (6, nz, ny, nx): E', B'.

    ``staggered``: components on the staggered (Yee) grid of
    kspace.STAGGER_OFFSETS with staggered order-p differences.  Each spectrum is
    first moved to the component's true position (times the conjugate half-cell
    shifts of its offset axes); there every derivative is i K_s with the real
    staggered symbol, so the push is the one above with K = K_s; the results are
    moved back to their own grid positions before the inverse transform.
    """
    fields = np.asarray(fields, dtype=np.float64)
    shape = fields.shape[1:]
    F = [fft3(fields[i]) for i in range(11)]
    if staggered:
        K, Sh = kspace.k_grids_staggered(shape, d, order)

        def shift(f):
            o = kspace.STAGGER_OFFSETS[f]
            return (Sh[0] if o[0] else 1.0) * (Sh[1] if o[1] else 1.0) * (Sh[2] if o[2] else 1.0)

        F = [F[f] * np.conj(shift(f)) for f in range(11)]
    else:
        K = kspace.k_grids(shape, d, order)
    coef = kspace.coefficients(K[0], K[1], K[2], dt, c)
    En, Bn = kspace.push(F[0:3], F[3:6], F[6:9], F[9], F[10], K, coef, c, eps0)
    del F
    out = En + Bn
    if staggered:
        out = [out[f] * shift(f) for f in range(6)]
    scale = float(np.abs(fields).max())
    return np.stack([real_part(ifft3(X), imag_tol, scale) for X in out])


def box_steps(fields, nsteps: int, d, dt: float, order, c: float = 1.0, eps0: float = 1.0,
              staggered: bool = False):
    """``nsteps`` box steps with the sources (J, rho_old, rho_new) held fixed.

    Returns the final (6, nz, ny, nx) E, B.
    """
    f = np.array(fields, dtype=np.float64, copy=True)
    for _ in range(nsteps):
        f[0:6] = box_step(f, d, dt, order, c, eps0, staggered=staggered)
    return f[0:6].copy()
