"""Oracle (test infrastructure): the particle side of the PIC cycle around the Maxwell step, FP64.

arXiv:1812.07357, Sec. 2.5.1 (the PIC cycle of Fig. 4): particles are pushed with
the fields at their positions, their current and charge are deposited on the grid
with linear (or higher order) interpolation, Maxwell's equations are solved, and
the new fields are gathered back to the particles with the same interpolation.
Sec. 2.5.2: particle-mesh work runs on the grid G1 (decomposition D1, guard cells
as wide as the interpolation stencil), the Maxwell solve on the FFT boxes of G2
(decomposition D2), coupled by the guard fill and interior copy of ``domain``.

Readings (the paper fixes none of them):
* linear (cloud-in-cell) weights by default; the paper allows higher orders for
  the deposit and a gather at the same order, read as the centred B-splines of
  degree 2 (triangular-shaped cloud) and 3 (cubic), ``order`` = 1, 2, 3; a
  quantity of a component that sits at offset o (0 or 1/2 cell per axis,
  kspace.STAGGER_OFFSETS on staggered grids) is attached to the grid points
  (i + o) d of the periodic grid G1;
* charge density rho = q S / (dx dy dz) at the particles' start and end
  positions, current J = q v S / (dx dy dz) at the mid-point of the step with
  the half-step velocity (not charge-conserving for order-p derivatives; the
  step stays exact for the sources it is given);
* relativistic Boris push of the momentum per mass u = gamma v with the fields
  gathered at the start positions, then x_new = x + dt u / gamma.
"""

from __future__ import annotations

import numpy as np

from . import kspace


def shape_1d(s, order: int = 1):
    """Centred B-spline weights of degree ``order`` at coordinates ``s`` (in cells).

    Returns (first grid index (n,), weights (n, order + 1)) for the points first .. first+order:
      1: first = floor(s), f = s - first: (1 - f, f);
      2: first = round(s) - 1, t = s - round(s) in [-1/2, 1/2):
         ((1/2 - t)^2 / 2, 3/4 - t^2, (1/2 + t)^2 / 2);
      3: first = floor(s) - 1, f = s - floor(s):
         ((1 - f)^3, 4 - 6 f^2 + 3 f^3, 1 + 3 f + 3 f^2 - 3 f^3, f^3) / 6.
    """
    s = np.asarray(s, dtype=np.float64)
    if order == 1:
        i0 = np.floor(s)
        f = s - i0
        return i0.astype(np.int64), np.stack([1.0 - f, f], axis=-1)
    if order == 2:
        i0 = np.floor(s + 0.5)
        t = s - i0
        return (i0 - 1).astype(np.int64), np.stack([0.5 * (0.5 - t) ** 2, 0.75 - t * t, 0.5 * (0.5 + t) ** 2], axis=-1)
    if order == 3:
        i0 = np.floor(s)
        f = s - i0
        return (i0 - 1).astype(np.int64), np.stack(
            [(1 - f) ** 3, 4 - 6 * f * f + 3 * f ** 3, 1 + 3 * f + 3 * f * f - 3 * f ** 3, f ** 3], axis=-1) / 6.0
    raise ValueError(f"shape order {order} not in 1..3")


def cic(pos, gshape, d, offset=(0, 0, 0), order: int = 1):
    """Weights of particles at ``pos`` (n, 3) (x, y, z lengths) on a periodic grid.

    Returns (idx (n, (order+1)^3) flat indices into a (nz, ny, nx) array, w (same) weights);
    the grid point (i, j, k) of a quantity with the given half-cell offsets sits at
    ((i + ox/2) dx, (j + oy/2) dy, (k + oz/2) dz).  Order 1 is cloud in cell.
    """
    nz, ny, nx = gshape
    dx, dy, dz = d
    fx, wx = shape_1d(pos[:, 0] / dx - 0.5 * offset[0], order)
    fy, wy = shape_1d(pos[:, 1] / dy - 0.5 * offset[1], order)
    fz, wz = shape_1d(pos[:, 2] / dz - 0.5 * offset[2], order)
    idx, w = [], []
    for cz in range(order + 1):
        for cy in range(order + 1):
            for cx in range(order + 1):
                ix = (fx + cx) % nx
                iy = (fy + cy) % ny
                iz = (fz + cz) % nz
                idx.append((iz * ny + iy) * nx + ix)
                w.append(wx[:, cx] * wy[:, cy] * wz[:, cz])
    return np.stack(idx, axis=1), np.stack(w, axis=1)


def deposit(values, pos, gshape, d, offset=(0, 0, 0), order: int = 1):
    """Grid array sum_p values_p S(x - pos_p) / (dx dy dz) (periodic), plain scatter-add."""
    idx, w = cic(pos, gshape, d, offset, order)
    out = np.zeros(int(np.prod(gshape)))
    np.add.at(out, idx.ravel(), (w * values[:, None]).ravel() / float(np.prod(d)))
    return out.reshape(gshape)


def gather(field, pos, d, offset=(0, 0, 0), order: int = 1):
    """Field values interpolated at ``pos`` with the same weights."""
    idx, w = cic(pos, field.shape, d, offset, order)
    return np.sum(field.ravel()[idx] * w, axis=1)


def offsets(staggered: bool):
    """Half-cell offsets of the eleven slots (all on the nodes for the collocated grid)."""
    return kspace.STAGGER_OFFSETS if staggered else ((0, 0, 0),) * 11


def boris(u, E, B, q_over_m: float, dt: float, c: float = 1.0):
    """Relativistic Boris step of u = gamma v (n, 3) in the fields E, B (n, 3) at the particles.

    Half an electric kick, a rotation about B by the angle of the magnetic force at the
    mid-step gamma, the other half kick (Boris, 1970).
    """
    h = 0.5 * q_over_m * dt
    um = u + h * E
    gm = np.sqrt(1.0 + np.sum(um * um, axis=1, keepdims=True) / (c * c))
    t = h * B / gm
    s = 2.0 * t / (1.0 + np.sum(t * t, axis=1, keepdims=True))
    up = um + np.cross(um, t)
    upl = um + np.cross(up, s)
    return upl + h * E


def push(x, u, g1, gshape, d, q_over_m: float, dt: float, c: float = 1.0, staggered: bool = False,
         order: int = 1):
    """Gather E, B (slots 0..5 of g1) at x, Boris-push u, move x; returns (x_new, u_new), x wrapped."""
    off = offsets(staggered)
    E = np.stack([gather(g1[k], x, d, off[k], order) for k in range(3)], axis=1)
    B = np.stack([gather(g1[3 + k], x, d, off[3 + k], order) for k in range(3)], axis=1)
    un = boris(u, E, B, q_over_m, dt, c)
    gam = np.sqrt(1.0 + np.sum(un * un, axis=1, keepdims=True) / (c * c))
    L = np.array([gshape[2] * d[0], gshape[1] * d[1], gshape[0] * d[2]])
    xn = np.mod(x + dt * un / gam, L)
    return xn, un


def sources(x_old, x_new, u, q: float, gshape, d, dt: float, c: float = 1.0, staggered: bool = False,
            order: int = 1):
    """(J (3, ...), rho_old, rho_new) of particles moving from x_old to x_new with half-step u.

    J = q v S at the mid-point x_old + v dt / 2 (v = u / gamma), rho at both ends.
    """
    off = offsets(staggered)
    gam = np.sqrt(1.0 + np.sum(u * u, axis=1, keepdims=True) / (c * c))
    v = u / gam
    L = np.array([gshape[2] * d[0], gshape[1] * d[1], gshape[0] * d[2]])
    xm = np.mod(x_old + 0.5 * dt * v, L)
    J = np.stack([deposit(q * v[:, k], xm, gshape, d, off[6 + k], order) for k in range(3)])
    qs = np.full(x_old.shape[0], q)
    return J, deposit(qs, x_old, gshape, d, off[9], order), deposit(qs, x_new, gshape, d, off[10], order)
