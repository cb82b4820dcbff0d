"""Oracle (test infrastructure): diagnostics and consistent-source fixtures, FP64.

arXiv:1812.07357, Sec. 1.1: the PSATD solver is exact for resolved modes, so
with charge-conserving sources it keeps Gauss's law and div B = 0 to round-off
and conserves the vacuum field energy.  The helpers here measure those
quantities and build inputs that satisfy the constraints (Gauss's law at the
start of the step, continuity between rho_old and rho_new, div B = 0), all with
the solver's own modified wave vector K.
"""

from __future__ import annotations

import numpy as np

from . import kspace
from .step import fft3, ifft3, real_part


def rel_l2(f, ref):
    """||f - ref||_2 / ||ref||_2 over all elements."""
    f = np.asarray(f, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm((f - ref).ravel()) / max(np.linalg.norm(ref.ravel()), 1e-300))


def energy(E, B, c: float = 1.0):
    """Field energy sum over nodes of |E|^2 + c^2 |B|^2 (units with eps0 = 1, factor 1/2 dropped)."""
    return float(np.sum(np.square(E)) + c * c * np.sum(np.square(B)))


def gauss_residual(E, rho, d, order, eps0: float = 1.0):
    """||i K.E^ - rho^/eps0|| / ||rho^/eps0|| in k-space."""
    shape = np.shape(rho)
    K = kspace.k_grids(shape, d, order)
    Eh = [fft3(E[i]) for i in range(3)]
    rh = fft3(rho) / eps0
    res = 1j * (K[0] * Eh[0] + K[1] * Eh[1] + K[2] * Eh[2]) - rh
    return float(np.linalg.norm(res.ravel()) / max(np.linalg.norm(rh.ravel()), 1e-300))


def div_b(B, d, order):
    """||K.B^|| / || |K| |B^| || in k-space (zero for a divergence-free B)."""
    shape = np.shape(B[0])
    K = kspace.k_grids(shape, d, order)
    Bh = [fft3(B[i]) for i in range(3)]
    kdotb = K[0] * Bh[0] + K[1] * Bh[1] + K[2] * Bh[2]
    kabs = np.sqrt(K[0] ** 2 + K[1] ** 2 + K[2] ** 2)
    nb = np.sqrt(np.abs(Bh[0]) ** 2 + np.abs(Bh[1]) ** 2 + np.abs(Bh[2]) ** 2)
    return float(np.linalg.norm(kdotb.ravel()) / max(np.linalg.norm((kabs * nb).ravel()), 1e-300))


def project_divfree(V, d, order):
    """Remove the longitudinal part of the vector field V (3, ...): V^ - K (K.V^)/|K|^2."""
    shape = np.shape(V[0])
    K = kspace.k_grids(shape, d, order)
    Vh = [fft3(V[i]) for i in range(3)]
    k2 = K[0] ** 2 + K[1] ** 2 + K[2] ** 2
    inv = np.where(k2 > 0, 1.0 / np.where(k2 > 0, k2, 1.0), 0.0)
    kdotv = (K[0] * Vh[0] + K[1] * Vh[1] + K[2] * Vh[2]) * inv
    scale = float(np.abs(V).max())
    return np.stack([real_part(ifft3(Vh[i] - K[i] * kdotv), scale=scale) for i in range(3)])


def rho_from_gauss(E, d, order, eps0: float = 1.0):
    """rho = eps0 div_p E, i.e. rho^ = eps0 i K.E^ (Gauss's law with the solver's K)."""
    shape = np.shape(E[0])
    K = kspace.k_grids(shape, d, order)
    Eh = [fft3(E[i]) for i in range(3)]
    scale = eps0 * float(np.abs(E).max()) * float(max(np.abs(K[0]).max(), np.abs(K[1]).max(), np.abs(K[2]).max()))
    return real_part(ifft3(eps0 * 1j * (K[0] * Eh[0] + K[1] * Eh[1] + K[2] * Eh[2])), scale=scale)


def rho_continuity(rho_old, J, dt: float, d, order):
    """rho_new = rho_old - dt div_p J, i.e. rho_new^ = rho_old^ - dt i K.J^."""
    shape = np.shape(rho_old)
    K = kspace.k_grids(shape, d, order)
    Jh = [fft3(J[i]) for i in range(3)]
    scale = float(np.abs(J).max()) * float(max(np.abs(K[0]).max(), np.abs(K[1]).max(), np.abs(K[2]).max()))
    return rho_old - dt * real_part(ifft3(1j * (K[0] * Jh[0] + K[1] * Jh[1] + K[2] * Jh[2])), scale=scale)
