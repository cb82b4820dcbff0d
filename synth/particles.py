"""Seeded macro-particles of a warm plasma: uniform positions in the periodic box,
Gaussian momenta per mass (u = gamma v), plus a few particles placed on the edges
that a particle-mesh kernel has to handle (nodes, the periodic edge, tile corners).
Plain random draws only."""

from __future__ import annotations

import numpy as np


def plasma_particles(rng: np.random.Generator, n: int, lengths, u_rms: float, edge_cases: bool = True):
    """(x (n, 3), u (n, 3)) in fp64; ``lengths`` = (Lx, Ly, Lz)."""
    L = np.asarray(lengths, dtype=np.float64)
    x = rng.uniform(0.0, 1.0, size=(n, 3)) * L
    u = rng.normal(0.0, u_rms, size=(n, 3))
    if edge_cases and n >= 6:
        x[0] = 0.0                       # on the origin node
        x[1] = L * (1.0 - 1e-7)          # just below the periodic edge
        x[2] = 0.5 * L                   # a node in the middle
        x[3] = [L[0] * (1.0 - 1e-7), 0.0, 0.5 * L[2]]
        u[4] = 0.0                       # at rest
        u[5] = [3.0 * u_rms, -3.0 * u_rms, 3.0 * u_rms]
    return x, u
