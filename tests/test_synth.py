"""Seeded input generators: reproducible, right shapes, charge of the deposit conserved."""

import numpy as np

import synth


def test_streams_are_reproducible_and_independent():
    a = synth.rng_for(2, 0).normal(size=5)
    b = synth.rng_for(2, 0).normal(size=5)
    c = synth.rng_for(2, 1).normal(size=5)
    np.testing.assert_array_equal(a, b)
    assert not np.allclose(a, c)


def test_macro_particle_deposit_conserves_charge():
    rng = synth.rng_for(2, 3)
    shape = (6, 7, 8)
    J, ro, rn = synth.macro_particle_deposit(rng, shape, 1.0, 0.5, 1000, q=0.1)
    assert J.shape == (3,) + shape and ro.shape == shape
    np.testing.assert_allclose(ro.sum(), 100.0, rtol=1e-12)
    np.testing.assert_allclose(rn.sum(), 100.0, rtol=1e-12)


def test_uneven_decomposition_tiles_the_grid():
    gdims, boxes = synth.uneven_decomposition(synth.rng_for(3, 0))
    assert len(boxes) == 64
    cells = sum(np.prod(b["interior"]) for b in boxes)
    assert cells == np.prod(gdims)
    for b in boxes:
        assert all(32 <= s <= 96 for s in b["interior"])
        assert b["nguard"] in (8, 16, 32, 64) and b["order"] in (16, 32, 64)


def test_laser_pulse_shape():
    E, B = synth.laser_pulse((8, 10, 64), 1.0, 16.0, 4.0, 12.0, 32.0)
    assert E.shape == (3, 8, 10, 64)
    np.testing.assert_array_equal(B[2], E[1])
    assert np.abs(E[0]).max() == 0 and np.abs(E[1]).max() <= 1.0
