"""Oracle (test infrastructure): guard fill / merge and the local-with-guards driver.

arXiv:1812.07357:
* Fig. 1(a) and Sec. 1.3: each sub-domain carries guard cells holding copies
  of its neighbours' fields and is advanced independently with a local FFT;
  guards are refreshed every step.
* Sec. 2.1: the hybrid solver puts guards only around a group of sub-domains;
  on one device a whole group is one box.
* Sec. 2.5.2 (coupling of G1 and G2): (1) G1 is copied to G2 including the
  group guards, which are filled from G1 itself; (2) Maxwell's equations are
  solved on G2; (3) the interior (no guards) is copied back from G2 to G1.
Readings: the global grid is periodic, so a guard cell takes the value of the
G1 cell at (origin - nguard + i) mod N on every axis, also when the guard is
wider than the neighbouring sub-domain; the merge copies the interior of E and
B only; every fill of a step reads the fields of the previous step (Jacobi
order); J and rho are filled but never merged.
"""

from __future__ import annotations

import numpy as np

from . import step as _step

# Arrays are (..., Nz, Ny, Nx); origins, interiors and guards are (x, y, z) triples.


def _axis_index(origin, count, n_global):
    return (origin + np.arange(count)) % n_global


def guard_fill(g1, origin, interior, nguard):
    """Gather one box (interior plus guards) from the periodic global arrays ``g1``.

    g1: (nf, NZ, NY, NX).  Returns (nf, nz + 2 gz, ny + 2 gy, nx + 2 gx) with
    box[f, k, j, i] = g1[f, (oz - gz + k) mod NZ, (oy - gy + j) mod NY, (ox - gx + i) mod NX].
    """
    g1 = np.asarray(g1)
    NZ, NY, NX = g1.shape[-3:]
    gx, gy, gz = _triple(nguard)
    ix = _axis_index(origin[0] - gx, interior[0] + 2 * gx, NX)
    iy = _axis_index(origin[1] - gy, interior[1] + 2 * gy, NY)
    iz = _axis_index(origin[2] - gz, interior[2] + 2 * gz, NZ)
    return g1[..., iz[:, None, None], iy[None, :, None], ix[None, None, :]]


def guard_merge(box, g1, origin, interior, nguard):
    """Copy the interior of ``box`` back into the global arrays ``g1`` in place.

    g1[f, (oz + k) mod NZ, (oy + j) mod NY, (ox + i) mod NX] = box[f, gz + k, gy + j, gx + i]
    for 0 <= (i, j, k) < interior.
    """
    NZ, NY, NX = g1.shape[-3:]
    gx, gy, gz = _triple(nguard)
    nx, ny, nz = interior
    ix = _axis_index(origin[0], nx, NX)
    iy = _axis_index(origin[1], ny, NY)
    iz = _axis_index(origin[2], nz, NZ)
    g1[..., iz[:, None, None], iy[None, :, None], ix[None, None, :]] = \
        box[..., gz:gz + nz, gy:gy + ny, gx:gx + nx]


def _triple(v):
    return (v, v, v) if np.isscalar(v) else tuple(v)


def local_step(g1, boxes, d, dt: float, c: float = 1.0, eps0: float = 1.0):
    """One step of the local (or hybrid, one box per group) solver on the global grid.

    g1: (11, NZ, NY, NX) fields of step n.  boxes: iterable of dicts with keys
    origin, interior, nguard (scalar or triple), order and optionally staggered.  Every box is filled
    from step-n fields, pushed with its own order, and its interior E, B are
    written to a copy of g1, which is returned (sources unchanged).
    """
    g1 = np.asarray(g1, dtype=np.float64)
    out = g1.copy()
    for b in boxes:
        box = guard_fill(g1, b["origin"], b["interior"], b["nguard"])
        eb = _step.box_step(box, d, dt, b["order"], c, eps0, staggered=b.get("staggered", False))
        guard_merge(eb, out[0:6], b["origin"], b["interior"], b["nguard"])
    return out


def local_steps(g1, boxes, nsteps: int, d, dt: float, c: float = 1.0, eps0: float = 1.0):
    """``nsteps`` local steps with fixed sources; returns the final (11, ...) fields."""
    f = np.asarray(g1, dtype=np.float64)
    for _ in range(nsteps):
        f = local_step(f, boxes, d, dt, c, eps0)
    return f


def global_steps(g1, nsteps: int, d, dt: float, order, c: float = 1.0, eps0: float = 1.0,
                 staggered: bool = False):
    """The undecomposed periodic solve (no guards) for ``nsteps``; returns (11, ...)."""
    f = np.array(g1, dtype=np.float64, copy=True)
    for _ in range(nsteps):
        f[0:6] = _step.box_step(f, d, dt, order, c, eps0, staggered=staggered)
    return f
