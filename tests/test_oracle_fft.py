"""Pins of the oracle's Fourier transform (a library primitive) against brute force.

The oracle takes the library's complex 3D DFT as one step of the method (the
forward transform of Sec. 1.1 of arXiv:1812.07357).  Here it is checked against
a direct O(N^2) sum over all nodes, Parseval's identity and the shift theorem.
"""

import numpy as np
import pytest

from oracle.step import fft3, ifft3

SHAPES = [(1, 1, 1), (2, 3, 5), (3, 5, 7), (4, 6, 8), (5, 11, 2), (7, 4, 13), (8, 8, 17), (12, 1, 9)]


def brute_dft(f, sign=-1.0):
    """F(k) = sum_x f(x) exp(sign i 2 pi (kx x/nx + ky y/ny + kz z/nz)), one k at a time."""
    nz, ny, nx = f.shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    F = np.zeros(f.shape, dtype=np.complex128)
    for kz in range(nz):
        for ky in range(ny):
            for kx in range(nx):
                ph = 2 * np.pi * (kx * x / nx + ky * y / ny + kz * z / nz)
                F[kz, ky, kx] = np.sum(f * np.exp(sign * 1j * ph))
    return F


@pytest.mark.parametrize("shape", SHAPES)
def test_fft_matches_direct_sum(shape):
    rng = np.random.default_rng(11)
    f = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    ref = brute_dft(f)
    got = fft3(f)
    scale = np.abs(ref).max()
    assert np.abs(got - ref).max() <= 1e-13 * max(scale, 1.0)


@pytest.mark.parametrize("shape", SHAPES)
def test_inverse_matches_direct_sum(shape):
    rng = np.random.default_rng(12)
    F = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    ref = brute_dft(F, sign=+1.0) / F.size
    assert np.abs(ifft3(F) - ref).max() <= 1e-13 * max(np.abs(ref).max(), 1.0)


def test_parseval_and_shift():
    rng = np.random.default_rng(13)
    f = rng.standard_normal((10, 14, 18))
    F = fft3(f)
    assert abs(np.sum(np.abs(F) ** 2) / f.size - np.sum(f**2)) <= 1e-12 * np.sum(f**2)
    # shift theorem: f(x - s) <-> F(k) exp(-i k.s)
    s = (3, 5, 7)  # (z, y, x)
    g = np.roll(f, s, axis=(0, 1, 2))
    nz, ny, nx = f.shape
    kz = np.arange(nz)[:, None, None]
    ky = np.arange(ny)[None, :, None]
    kx = np.arange(nx)[None, None, :]
    ph = np.exp(-2j * np.pi * (kz * s[0] / nz + ky * s[1] / ny + kx * s[2] / nx))
    assert np.abs(fft3(g) - F * ph).max() <= 1e-12 * np.abs(F).max()
