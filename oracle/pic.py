"""Oracle (test infrastructure): the particle side of the PIC cycle around the Maxwell step, FP64.

arXiv:1812.07357, Sec. 2.5.1 (the PIC cycle of Fig. 4): particles are pushed with
the fields at their positions, their current and charge are deposited on the grid
with linear (or higher order) interpolation, Maxwell's equations are solved, and
the new fields are gathered back to the particles with the same interpolation.
Sec. 2.5.2: particle-mesh work runs on the grid G1 (decomposition D1, guard cells
as wide as the interpolation stencil), the Maxwell solve on the FFT boxes of G2
(decomposition D2), coupled by the guard fill and interior copy of ``domain``.

Readings (the paper fixes none of them):
* linear (cloud-in-cell) weights; a quantity of a component that sits at
  offset o (0 or 1/2 cell per axis, kspace.STAGGER_OFFSETS on staggered grids)
  is attached to the grid points (i + o) d of the periodic grid G1;
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


def cic(pos, gshape, d, offset=(0, 0, 0)):
    """Linear weights of particles at ``pos`` (n, 3) (x, y, z lengths) on a periodic grid.

    Returns (idx (n, 8) flat indices into a (nz, ny, nx) array, w (n, 8) weights); the
    grid point (i, j, k) of a quantity with the given half-cell offsets sits at
    ((i + ox/2) dx, (j + oy/2) dy, (k + oz/2) dz).
    """
    nz, ny, nx = gshape
    dx, dy, dz = d
    xi = np.stack([pos[:, 0] / dx - 0.5 * offset[0], pos[:, 1] / dy - 0.5 * offset[1],
                   pos[:, 2] / dz - 0.5 * offset[2]], axis=1)
    i0 = np.floor(xi).astype(np.int64)
    f = xi - i0
    idx, w = [], []
    for cz in (0, 1):
        for cy in (0, 1):
            for cx in (0, 1):
                wx = f[:, 0] if cx else 1.0 - f[:, 0]
                wy = f[:, 1] if cy else 1.0 - f[:, 1]
                wz = f[:, 2] if cz else 1.0 - f[:, 2]
                ix = (i0[:, 0] + cx) % nx
                iy = (i0[:, 1] + cy) % ny
                iz = (i0[:, 2] + cz) % nz
                idx.append((iz * ny + iy) * nx + ix)
                w.append(wx * wy * wz)
    return np.stack(idx, axis=1), np.stack(w, axis=1)


def deposit(values, pos, gshape, d, offset=(0, 0, 0)):
    """Grid array sum_p values_p S(x - pos_p) / (dx dy dz) (periodic), plain scatter-add."""
    idx, w = cic(pos, gshape, d, offset)
    out = np.zeros(int(np.prod(gshape)))
    np.add.at(out, idx.ravel(), (w * values[:, None]).ravel() / float(np.prod(d)))
    return out.reshape(gshape)


def gather(field, pos, d, offset=(0, 0, 0)):
    """Field values interpolated at ``pos`` with the same linear weights."""
    idx, w = cic(pos, field.shape, d, offset)
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


def push(x, u, g1, gshape, d, q_over_m: float, dt: float, c: float = 1.0, staggered: bool = False):
    """Gather E, B (slots 0..5 of g1) at x, Boris-push u, move x; returns (x_new, u_new), x wrapped."""
    off = offsets(staggered)
    E = np.stack([gather(g1[k], x, d, off[k]) for k in range(3)], axis=1)
    B = np.stack([gather(g1[3 + k], x, d, off[3 + k]) for k in range(3)], axis=1)
    un = boris(u, E, B, q_over_m, dt, c)
    gam = np.sqrt(1.0 + np.sum(un * un, axis=1, keepdims=True) / (c * c))
    L = np.array([gshape[2] * d[0], gshape[1] * d[1], gshape[0] * d[2]])
    xn = np.mod(x + dt * un / gam, L)
    return xn, un


def sources(x_old, x_new, u, q: float, gshape, d, dt: float, c: float = 1.0, staggered: bool = False):
    """(J (3, ...), rho_old, rho_new) of particles moving from x_old to x_new with half-step u.

    J = q v S at the mid-point x_old + v dt / 2 (v = u / gamma), rho at both ends.
    """
    off = offsets(staggered)
    gam = np.sqrt(1.0 + np.sum(u * u, axis=1, keepdims=True) / (c * c))
    v = u / gam
    L = np.array([gshape[2] * d[0], gshape[1] * d[1], gshape[0] * d[2]])
    xm = np.mod(x_old + 0.5 * dt * v, L)
    J = np.stack([deposit(q * v[:, k], xm, gshape, d, off[6 + k]) for k in range(3)])
    qs = np.full(x_old.shape[0], q)
    return J, deposit(qs, x_old, gshape, d, off[9]), deposit(qs, x_new, gshape, d, off[10])
