"""Oracle (test infrastructure): wavenumbers, modified wavenumbers, PSATD coefficients, push.

FP64.  Paper: Kallala, Vay & Vincenti, arXiv:1812.07357.

* Sec. 1.1: the PSATD solver Fourier-transforms Maxwell's equations in space
  and integrates them analytically in time over one step; it is exact for the
  resolved modes, has no Courant limit and no numerical dispersion.  The
  equations themselves are only cited there (Haber et al. 1973), so the update
  below is derived here from
      dE/dt = i c^2 K x B - J / eps0,      dB/dt = -i K x E,
  with J held constant over the step, Gauss's law i K.E = rho / eps0 and the
  continuity equation rho_new - rho_old = -dt i K.J.
* Sec. 1.1 and 1.3: a solver of order p uses a centred stencil of half width
  p/2; the infinite-order limit p -> inf is the spectral derivative.  Replacing
  i k by i k_p (the symbol of the order-p centred difference) gives the
  finite-order solver.  Readings: collocated (nodal) grid, centred stencil,
  k_p = 0 at the Nyquist index.
"""

from __future__ import annotations

from fractions import Fraction
from math import factorial

import numpy as np

# Below this value of theta = omega dt the coefficients use their Taylor series.
THETA_SERIES = 0.1


def signed_index(n: int):
    """Signed mode number of each DFT index and a Nyquist mask.

    Index m maps to m for m < n/2 and to m - n for m > n/2; for even n the
    index n/2 is the Nyquist mode, returned as +n/2 with its mask entry True.
    """
    m = np.arange(n, dtype=np.int64)
    ms = np.where(2 * m <= n, m, m - n)
    nyq = (2 * m == n)
    return ms, nyq


def wavenumbers(n: int, d: float):
    """Exact wavenumbers k = 2 pi m' / (n d) of the DFT indices, Nyquist set to zero."""
    ms, nyq = signed_index(n)
    k = 2.0 * np.pi * ms.astype(np.float64) / (n * d)
    k[nyq] = 0.0
    return k


def fd_weights(order: int):
    """Weights a_l (l = 1..p/2) of the centred order-p first-derivative stencil.

    f'(x) ~ sum_l a_l (f(x + l d) - f(x - l d)) / d with the classical closed form
    a_l = (-1)^(l+1) (m!)^2 / (l (m-l)! (m+l)!), m = p/2, evaluated in exact
    rational arithmetic.  (Sec. 1.1: order p, stencil half width p/2.)
    """
    if order <= 0 or order % 2:
        raise ValueError("order must be a positive even integer")
    m = order // 2
    return [Fraction((-1) ** (l + 1) * factorial(m) ** 2, l * factorial(m - l) * factorial(m + l))
            for l in range(1, m + 1)]


def modified_k(n: int, d: float, order: int):
    """Modified wavenumber k_p of each DFT index along one axis (Sec. 1.1, 1.3).

    order == 0 means infinite order (k_p = k).  For finite even order,
    k_p = sum_l a_l 2 sin(l k d) / d.  Evaluated for |m'| and given the sign of
    m' so that k_p(-k) = -k_p(k) holds exactly; the Nyquist index gets 0.
    """
    ms, nyq = signed_index(n)
    kabs = 2.0 * np.pi * np.abs(ms).astype(np.float64) / (n * d)
    kp = modified_k_at(kabs, d, order)
    kp = np.where(ms < 0, -kp, kp)
    kp[nyq] = 0.0
    return kp


def modified_k_at(k, d: float, order: int):
    """k_p at arbitrary wavenumbers k: k itself for order 0, else sum_l a_l 2 sin(l k d) / d."""
    k = np.asarray(k, dtype=np.float64)
    if order == 0:
        return k.copy()
    kp = np.zeros_like(k)
    for l, a in enumerate(fd_weights(order), start=1):
        kp += float(a) * 2.0 * np.sin(l * k * d) / d
    return kp


# ------------------------------------------------------------------ staggered (Yee) grid
# Reading for the staggered variant (the grid of the production PSATD codes the
# paper builds on, Sec. 1.1 and 1.3): each component lives half a cell off the
# nodes along the axes listed below, in slot order Ex Ey Ez Bx By Bz Jx Jy Jz
# rho_old rho_new; array index i of a component stores its value at
# (i + offset) d.  Derivatives are order-p staggered differences between
# half-cell-shifted points.
STAGGER_OFFSETS = ((1, 0, 0), (0, 1, 0), (0, 0, 1),
                   (0, 1, 1), (1, 0, 1), (1, 1, 0),
                   (1, 0, 0), (0, 1, 0), (0, 0, 1),
                   (0, 0, 0), (0, 0, 0))


def staggered_weights(order: int):
    """Weights alpha_l (l = 1..p/2) of the order-p staggered first-derivative stencil.

    f'(x) ~ sum_l alpha_l (f(x + (l - 1/2) d) - f(x - (l - 1/2) d)) / d, with the
    closed form alpha_l = 1/(2l-1) prod_{j != l} (2j-1)^2 / ((2j-1)^2 - (2l-1)^2)
    (derivative of the Lagrange interpolant on the nodes +-(2j-1)/2), in exact
    rational arithmetic: 1 for p = 2; 9/8, -1/24 for p = 4.
    """
    if order <= 0 or order % 2:
        raise ValueError("order must be a positive even integer")
    m = order // 2
    out = []
    for l in range(1, m + 1):
        a = Fraction(1, 2 * l - 1)
        for j in range(1, m + 1):
            if j != l:
                a *= Fraction((2 * j - 1) ** 2, (2 * j - 1) ** 2 - (2 * l - 1) ** 2)
        out.append(a)
    return out


def staggered_k_at(k, d: float, order: int):
    """Symbol of the staggered difference at wavenumbers k: k for order 0, else
    sum_l alpha_l 2 sin((2l - 1) k d / 2) / d."""
    k = np.asarray(k, dtype=np.float64)
    if order == 0:
        return k.copy()
    ks = np.zeros_like(k)
    for l, a in enumerate(staggered_weights(order), start=1):
        ks += float(a) * 2.0 * np.sin((2 * l - 1) * k * d / 2.0) / d
    return ks


def modified_k_staggered(n: int, d: float, order: int):
    """Staggered modified wavenumber k_s of each DFT index along one axis.

    The Nyquist index of an even axis is taken at k = +pi/d; unlike the centred
    stencil, the staggered symbol does not vanish there (its value is the limit
    of the two half-cell shift factors below, which keep real fields real).
    """
    ms, _ = signed_index(n)
    k = 2.0 * np.pi * ms.astype(np.float64) / (n * d)
    return staggered_k_at(k, d, order)


def half_cell_shift(n: int, d: float):
    """exp(i k d / 2) at the exact wavenumber of each DFT index (Nyquist at +pi/d, i.e. +i).

    A component stored half a cell up (value at (i + 1/2) d under index i) has
    grid-index spectrum exp(i k d / 2) times the spectrum of its values at the
    true positions."""
    ms, _ = signed_index(n)
    k = 2.0 * np.pi * ms.astype(np.float64) / (n * d)
    return np.exp(0.5j * k * d)


def k_grids_staggered(shape, d, order):
    """(Kx, Ky, Kz) staggered symbols and (Sx, Sy, Sz) half-cell shifts, broadcastable on (nz, ny, nx)."""
    nz, ny, nx = shape
    dx, dy, dz = (d, d, d) if np.isscalar(d) else d
    px, py, pz = (order, order, order) if np.isscalar(order) else order
    K = (modified_k_staggered(nx, dx, px)[None, None, :], modified_k_staggered(ny, dy, py)[None, :, None],
         modified_k_staggered(nz, dz, pz)[:, None, None])
    Sh = (half_cell_shift(nx, dx)[None, None, :], half_cell_shift(ny, dy)[None, :, None],
          half_cell_shift(nz, dz)[:, None, None])
    return K, Sh


def k_grids(shape, d, order):
    """Broadcastable (Kx, Ky, Kz) for a box of shape (nz, ny, nx); ``d`` and ``order`` scalar or per axis (x, y, z)."""
    nz, ny, nx = shape
    dx, dy, dz = (d, d, d) if np.isscalar(d) else d
    px, py, pz = (order, order, order) if np.isscalar(order) else order
    kx = modified_k(nx, dx, px)[None, None, :]
    ky = modified_k(ny, dy, py)[None, :, None]
    kz = modified_k(nz, dz, pz)[:, None, None]
    return kx, ky, kz


def coefficients(kx, ky, kz, dt: float, c: float = 1.0):
    """PSATD coefficients at wave vector K = (kx, ky, kz) (broadcast), FP64.

    omega = c |K|, theta = omega dt and
      C  = cos(theta)
      S1 = sin(theta) / omega
      X1 = (1 - C) / omega^2
      X2 = (1 - S1 / dt) / omega^2
      X3 = (C - S1 / dt) / omega^2
    For theta < THETA_SERIES the Taylor series in theta^2 is used (terms through
    theta^8); at omega = 0 they reduce to dt, dt^2/2, dt^2/6 and -dt^2/3.
    """
    k2 = kx * kx + ky * ky + kz * kz
    omega = c * np.sqrt(k2)
    theta = omega * abs(dt)
    th2 = (omega * dt) ** 2
    C = np.cos(omega * dt)
    small = theta < THETA_SERIES
    # Series: S1/dt = sum (-1)^n th^2n/(2n+1)!, X1/dt^2 = sum (-1)^n th^2n/(2n+2)!,
    # X2/dt^2 = sum (-1)^n th^2n/(2n+3)!, X3/dt^2 = sum_{n>=1} (-1)^n 2n th^(2n-2)/(2n+1)!.
    s1_ser = dt * (1 - th2 / 6 + th2**2 / 120 - th2**3 / 5040 + th2**4 / 362880)
    x1_ser = dt * dt * (1 / 2 - th2 / 24 + th2**2 / 720 - th2**3 / 40320 + th2**4 / 3628800)
    x2_ser = dt * dt * (1 / 6 - th2 / 120 + th2**2 / 5040 - th2**3 / 362880 + th2**4 / 39916800)
    x3_ser = dt * dt * (-1 / 3 + th2 / 30 - th2**2 / 840 + th2**3 / 45360 - th2**4 / 3991680)
    with np.errstate(divide="ignore", invalid="ignore"):
        om = np.where(small, 1.0, omega)
        om2 = om * om
        s1_dir = np.sin(om * dt) / om
        x1_dir = (1 - np.cos(om * dt)) / om2
        x2_dir = (1 - s1_dir / dt) / om2
        x3_dir = (np.cos(om * dt) - s1_dir / dt) / om2
    return {
        "C": C,
        "S1": np.where(small, s1_ser, s1_dir),
        "X1": np.where(small, x1_ser, x1_dir),
        "X2": np.where(small, x2_ser, x2_dir),
        "X3": np.where(small, x3_ser, x3_dir),
    }


def _cross(a, b):
    return (a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0])


def push(E, B, J, rho_old, rho_new, K, coef, c: float = 1.0, eps0: float = 1.0):
    """Analytic PSATD update of the spectra over one step ("rho form").

    E' = C E + i c^2 S1 (K x B) - (S1/eps0) J + i (c^2/eps0) K (X3 rho_old - X2 rho_new)
    B' = C B - i S1 (K x E) + i (X1/eps0) (K x J)
    E, B, J: sequences of three complex arrays; K: (Kx, Ky, Kz) broadcastable.
    Returns (E', B') as lists of three arrays.
    """
    C, S1, X1, X2, X3 = (coef[n] for n in ("C", "S1", "X1", "X2", "X3"))
    kxb = _cross(K, B)
    kxe = _cross(K, E)
    kxj = _cross(K, J)
    rho_term = X3 * rho_old - X2 * rho_new
    c2 = c * c
    En = [C * E[i] + 1j * c2 * S1 * kxb[i] - (S1 / eps0) * J[i] + 1j * (c2 / eps0) * K[i] * rho_term
          for i in range(3)]
    Bn = [C * B[i] - 1j * S1 * kxe[i] + 1j * (X1 / eps0) * kxj[i] for i in range(3)]
    return En, Bn


def push_jform(E, B, J, K, coef, dt: float, c: float = 1.0, eps0: float = 1.0):
    """Same update written with the longitudinal projector instead of rho ("J form").

    E' = C E + i c^2 S1 K x B - (S1/eps0) J + (1 - C) Kh (Kh.E) + (S1 - dt) Kh (Kh.J) / eps0,
    B' as in ``push``; Kh = K/|K| (zero at K = 0).  Equal to ``push`` whenever
    Gauss's law holds for E and rho_old and continuity links rho_new to J.
    """
    C, S1, X1 = coef["C"], coef["S1"], coef["X1"]
    k2 = K[0] ** 2 + K[1] ** 2 + K[2] ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = np.where(k2 > 0, 1.0 / np.where(k2 > 0, k2, 1.0), 0.0)
    kdote = K[0] * E[0] + K[1] * E[1] + K[2] * E[2]
    kdotj = K[0] * J[0] + K[1] * J[1] + K[2] * J[2]
    kxb = _cross(K, B)
    kxe = _cross(K, E)
    kxj = _cross(K, J)
    c2 = c * c
    En = [C * E[i] + 1j * c2 * S1 * kxb[i] - (S1 / eps0) * J[i]
          + (1 - C) * K[i] * kdote * inv + (S1 - dt) * K[i] * kdotj * inv / eps0 for i in range(3)]
    Bn = [C * B[i] - 1j * S1 * kxe[i] + 1j * (X1 / eps0) * kxj[i] for i in range(3)]
    return En, Bn
