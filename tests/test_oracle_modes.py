"""Pins of the oracle's few-mode evaluator (used for point checks on very large grids).

For inputs made of a few modes periodic on the transformed box, the step acts
on each mode on its own (Sec. 1.1 of arXiv:1812.07357: the update is exact and
local in k).  The evaluator must therefore agree with the full transform-based
oracle, both for a periodic box and for a guard-padded box whose size is
commensurate with the modes (then the guards carry no truncation error).
"""

import numpy as np
import pytest

from oracle import domain, modes, step


def _random_modes(rng, lattice, nmodes):
    """Distinct integer modes (not 0, not negatives of one another) with |m_a| < lattice_a / 2."""
    seen, out = set(), []
    while len(out) < nmodes:
        lim = (np.array(lattice) - 1) // 2
        m = tuple(int(v) for v in rng.integers(-lim, lim + 1))
        if m == (0, 0, 0) or m in seen or tuple(-v for v in m) in seen:
            continue
        seen.add(m)
        out.append(m)
    return np.array(out)


@pytest.mark.parametrize("order", [0, 6, 32])
def test_modes_match_full_oracle_on_periodic_box(order):
    rng = np.random.default_rng(order + 3)
    shape, d, dt = (10, 12, 14), 1.0, 0.6
    nz, ny, nx = shape
    m = _random_modes(rng, (nx, ny, nz), 7)
    kvec = modes.mode_wavevectors(m, (nx, ny, nz), d)
    coefs = rng.standard_normal((11, len(m))) + 1j * rng.standard_normal((11, len(m)))
    fields = modes.synthesize_grid(kvec, coefs, shape, d)
    ref = step.box_steps(fields, 3, d, dt, order)
    got = modes.synthesize_grid(kvec, modes.push_modes(kvec, coefs, d, dt, order, nsteps=3), shape, d)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    # point evaluation agrees with grid evaluation
    pts = np.array([[1.0, 2.0, 3.0], [13.0, 0.0, 9.0]])
    vals = modes.synthesize(kvec, coefs[0:2], pts)
    np.testing.assert_allclose(vals[:, 0], fields[0:2, 3, 2, 1], rtol=0, atol=1e-12)
    np.testing.assert_allclose(vals[:, 1], fields[0:2, 9, 0, 13], rtol=0, atol=1e-12)


def test_commensurate_modes_through_guarded_box_are_exact():
    # G1 of 16 x 12 x 8 cells, one box with 4 guards: box 24 x 20 x 16.  Modes of
    # period 4 cells are periodic on both, so the local solve is exact.
    rng = np.random.default_rng(9)
    g1_shape, d, dt, order, ng = (8, 12, 16), 1.0, 0.5, 8, 4
    period = 4
    m = _random_modes(rng, (period, period, period), 5)
    kvec = modes.mode_wavevectors(m, (period, period, period), d)
    coefs = rng.standard_normal((11, len(m))) + 1j * rng.standard_normal((11, len(m)))
    g1 = modes.synthesize_grid(kvec, coefs, g1_shape, d)
    box = {"origin": (0, 0, 0), "interior": (16, 12, 8), "nguard": ng, "order": order}
    out = domain.local_step(g1, [box], d, dt)[0:6]
    exact = modes.synthesize_grid(kvec, modes.push_modes(kvec, coefs, d, dt, order), g1_shape, d)
    assert np.abs(out - exact).max() <= 1e-12 * np.abs(exact).max()
