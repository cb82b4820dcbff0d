"""Oracle (test infrastructure): two-step perfectly matched layers around a PSATD box, FP64.

arXiv:1812.07357, Sec. 2.6: the FFT-based solver of the paper is combined with
absorbing boundaries built as the two-step PML of Shapoval, Vay and Vincenti
(2019): in the layers the fields are split by the direction of the derivative
that drives them (Berenger's split fields), the split fields are first advanced
over the step without absorption by the analytic (PSATD) solution, then each is
damped in real space by exp(-sigma dt) with the conductivity of its own
direction.

Readings (the paper gives no formulas):
* Split fields everywhere on the box.  Component a has two parts: set A, driven
  by the derivative along axis a+1, and set B, along a+2 (axes mod 3); e.g.
  E_x = E_xy + E_xz, E_y = E_yz + E_yx.  The twelve arrays are ordered
  [E_xy, E_yz, E_zx, B_xy, B_yz, B_zx, E_xz, E_yx, E_zy, B_xz, B_yx, B_zy].
* Undamped advance: each part gains the integral over the step of its own
  right-hand side along the exact evolution of the full fields.  With the
  sources held constant, set B of E_a gains -i c^2 K_{a+2} IB_{a+1} and set B of
  B_a gains +i K_{a+2} IE_{a+1}, where IB and IE are the integrals of B(t) and
  E(t) over the step:
      IB = S1 B_T + dt B_L - i X1 (K x E) + i (dt X2 / eps0) (K x J),
      IE = S1 E_T + dt E_L + i c^2 X1 (K x B) - (X1/eps0) J_T - (dt^2 / 2 eps0) J_L,
  (T, L: parts transverse and parallel to K).  Set A takes the rest of the
  step's increment, so the two parts always add up to the rho-form step of
  ``kspace.push`` (with no damping the split box is exactly the ordinary box).
* Damping: the part of set A of component a is multiplied by d_{a+1}, set B by
  d_{a+2}, with d(i) = exp(-sigma(i) dt) per axis; sigma rises as
  sigma_max ((depth)/w)^m through a layer of w cells at each end of the axis
  (depth w at the outer cell, 1 at the innermost) and is zero inside.
* Collocated grid only; the box is periodic for the transforms, the layers keep
  waves from wrapping around.
"""

from __future__ import annotations

import numpy as np

from . import kspace
from .step import fft3, ifft3


def sigma_profile(n: int, width: int, sigma_max: float, power: float):
    """Conductivity per cell of an axis of n cells with layers of ``width`` cells at both ends."""
    s = np.zeros(n)
    for i in range(n):
        if i < width:
            s[i] = sigma_max * ((width - i) / width) ** power
        elif i >= n - width:
            s[i] = sigma_max * ((i - (n - width) + 1) / width) ** power
    return s


def damping(shape, widths, sigma_max: float, power: float, dt: float):
    """(dx, dy, dz) 1D damping factors exp(-sigma dt) for a box of shape (nz, ny, nx)."""
    nz, ny, nx = shape
    return tuple(np.exp(-sigma_profile(n, w, sigma_max, power) * dt) for n, w in zip((nx, ny, nz), widths))


def _axis_factor(damp, axis, shape):
    nz, ny, nx = shape
    if axis == 0:
        return damp[0][None, None, :]
    if axis == 1:
        return damp[1][None, :, None]
    return damp[2][:, None, None]


def split_increments(E, B, J, rho_old, rho_new, K, coef, dt: float, c: float = 1.0, eps0: float = 1.0):
    """Spectral increments of the twelve split parts over one undamped step.

    Returns (dEA, dBA, dEB, dBB), each a list of three spectra.
    """
    C, S1, X1, X2 = coef["C"], coef["S1"], coef["X1"], coef["X2"]
    k2 = K[0] ** 2 + K[1] ** 2 + K[2] ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = np.where(k2 > 0, 1.0 / np.where(k2 > 0, k2, 1.0), 0.0)

    def parts(V):
        kv = (K[0] * V[0] + K[1] * V[1] + K[2] * V[2]) * inv
        L = [K[i] * kv for i in range(3)]
        return [V[i] - L[i] for i in range(3)], L

    cross = kspace._cross
    ET, EL = parts(E)
    BT, BL = parts(B)
    JT, JL = parts(J)
    kxe, kxb, kxj = cross(K, E), cross(K, B), cross(K, J)
    c2 = c * c
    IB = [S1 * BT[i] + dt * BL[i] - 1j * X1 * kxe[i] + 1j * (dt * X2 / eps0) * kxj[i] for i in range(3)]
    IE = [S1 * ET[i] + dt * EL[i] + 1j * c2 * X1 * kxb[i] - (X1 / eps0) * JT[i] - (dt * dt / (2 * eps0)) * JL[i]
          for i in range(3)]
    dEB = [-1j * c2 * K[(a + 2) % 3] * IB[(a + 1) % 3] for a in range(3)]
    dBB = [1j * K[(a + 2) % 3] * IE[(a + 1) % 3] for a in range(3)]
    En, Bn = kspace.push(E, B, J, rho_old, rho_new, K, coef, c, eps0)
    dEA = [En[a] - E[a] - dEB[a] for a in range(3)]
    dBA = [Bn[a] - B[a] - dBB[a] for a in range(3)]
    return dEA, dBA, dEB, dBB


def pml_step(split, sources, d, dt: float, order, damp, c: float = 1.0, eps0: float = 1.0,
             imag_tol: float = 1e-10):
    """One two-step PML step of a box: ``split`` (12, nz, ny, nx) as ordered above,
    ``sources`` (5, ...) = Jx Jy Jz rho_old rho_new, ``damp`` from ``damping``.
    Returns the new (12, ...) split fields."""
    split = np.asarray(split, dtype=np.float64)
    shape = split.shape[1:]
    E = [fft3(split[a] + split[6 + a]) for a in range(3)]
    B = [fft3(split[3 + a] + split[9 + a]) for a in range(3)]
    J = [fft3(sources[a]) for a in range(3)]
    ro, rn = fft3(sources[3]), fft3(sources[4])
    K = kspace.k_grids(shape, d, order)
    coef = kspace.coefficients(*K, dt, c)
    dEA, dBA, dEB, dBB = split_increments(E, B, J, ro, rn, K, coef, dt, c, eps0)
    scale = float(np.abs(split).max()) + float(np.abs(np.asarray(sources)).max())
    out = np.empty_like(split)
    for a in range(3):
        for idx, inc, axis in ((a, dEA[a], a + 1), (3 + a, dBA[a], a + 1), (6 + a, dEB[a], a + 2),
                               (9 + a, dBB[a], a + 2)):
            z = ifft3(inc)
            im = float(np.abs(z.imag).max())
            if im > imag_tol * max(scale, 1e-300):
                raise AssertionError(f"split increment {idx} not real: {im:.3e}")
            out[idx] = (split[idx] + z.real) * _axis_factor(damp, axis % 3, shape)
    return out


def pml_steps(split, sources, nsteps: int, d, dt: float, order, damp, c: float = 1.0, eps0: float = 1.0):
    """``nsteps`` PML steps with the sources held fixed."""
    f = np.array(split, dtype=np.float64, copy=True)
    for _ in range(nsteps):
        f = pml_step(f, sources, d, dt, order, damp, c, eps0)
    return f
