"""Pins of the oracle's modified wavenumbers, PSATD coefficients and k-space push.

arXiv:1812.07357, Sec. 1.1: the PSATD update integrates Maxwell's equations
analytically over a step in k-space (exact for resolved modes, no Courant limit,
no dispersion); order p means a centred stencil of half width p/2 and p -> inf
is the spectral limit (Sec. 1.3).  Nothing here re-types the oracle's formulas:
each check goes through an independent route (textbook weights, exact rational
moment equations, 40-digit arithmetic, numerical ODE integration, conservation
laws).
"""

import os
from fractions import Fraction

import mpmath
import numpy as np
import pytest

from oracle import kspace

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "central_difference_weights.txt")


def _golden_weights():
    out = {}
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        p, rest = line.split(":")
        out[int(p)] = [Fraction(t) for t in rest.split()]
    return out


def test_fd_weights_match_textbook_table():
    for p, w in _golden_weights().items():
        assert kspace.fd_weights(p) == w


def _moment_solve(m):
    """Solve sum_l a_l 2 l^(2q+1) = [q == 0], q = 0..m-1, by exact Gaussian elimination."""
    A = [[Fraction(2 * l ** (2 * q + 1)) for l in range(1, m + 1)] for q in range(m)]
    b = [Fraction(1 if q == 0 else 0) for q in range(m)]
    n = m
    for i in range(n):
        piv = next(r for r in range(i, n) if A[r][i] != 0)
        A[i], A[piv] = A[piv], A[i]
        b[i], b[piv] = b[piv], b[i]
        for r in range(n):
            if r != i and A[r][i] != 0:
                f = A[r][i] / A[i][i]
                A[r] = [A[r][c] - f * A[i][c] for c in range(n)]
                b[r] -= f * b[i]
    return [b[i] / A[i][i] for i in range(n)]


@pytest.mark.parametrize("p", [2, 4, 6, 10, 16, 24, 32])
def test_fd_weights_solve_moment_equations(p):
    # An order-p centred first derivative is exact on polynomials up to degree p:
    # odd moments 1, 3, ..., p-1 give a linear system with a unique solution.
    assert kspace.fd_weights(p) == _moment_solve(p // 2)


@pytest.mark.parametrize("p", [2, 8, 50, 64, 100, 128])
def test_fd_weights_consistency(p):
    assert sum(2 * l * a for l, a in enumerate(kspace.fd_weights(p), start=1)) == 1


def test_modified_k_low_orders_closed_form():
    n, d = 24, 0.7
    k = kspace.wavenumbers(n, d)
    kd = k * d
    np.testing.assert_allclose(kspace.modified_k(n, d, 2), np.sin(kd) / d, rtol=0, atol=1e-14)
    np.testing.assert_allclose(kspace.modified_k(n, d, 4), (8 * np.sin(kd) - np.sin(2 * kd)) / (6 * d),
                               rtol=0, atol=1e-14)


@pytest.mark.parametrize("n", [1, 2, 7, 16, 33, 64])
@pytest.mark.parametrize("p", [0, 2, 6, 100])
def test_modified_k_symmetry_and_nyquist(n, p):
    kp = kspace.modified_k(n, 1.3, p)
    ms, nyq = kspace.signed_index(n)
    assert kp[0] == 0.0
    for i in range(n):
        j = (-i) % n
        assert kp[j] == -kp[i] or (nyq[i] and kp[i] == 0.0)
    assert np.all(kp[nyq] == 0.0)
    if n % 2 == 0:
        assert nyq.sum() == 1


def test_modified_k_converges_to_k():
    n, d = 64, 1.0
    k = kspace.wavenumbers(n, d)
    inner = np.abs(k * d) < 0.9 * np.pi
    prev = None
    for p in (2, 4, 8, 16, 32, 64, 100):
        err = np.abs(kspace.modified_k(n, d, p) - k)[inner].max()
        # centred differences under-estimate |k| for 0 < |k d| < pi
        assert np.all(np.abs(kspace.modified_k(n, d, p))[inner] <= np.abs(k[inner]) + 1e-15)
        if prev is not None:
            assert err < prev
        prev = err
    half = np.abs(k * d) <= 0.5 * np.pi
    assert np.abs(kspace.modified_k(n, d, 100) - k)[half].max() < 1e-10
    np.testing.assert_array_equal(kspace.modified_k(n, d, 0), k)


def _mp_coefs(theta, dt):
    mpmath.mp.dps = 40
    th = mpmath.mpf(theta)
    dtm = mpmath.mpf(dt)
    om = th / dtm
    C = mpmath.cos(th)
    S1 = mpmath.sin(th) / om
    X1 = (1 - C) / om**2
    X2 = (1 - S1 / dtm) / om**2
    X3 = (C - S1 / dtm) / om**2
    return {k: float(v) for k, v in dict(C=C, S1=S1, X1=X1, X2=X2, X3=X3).items()}


@pytest.mark.parametrize("theta", [1e-6, 1e-3, 0.01, 0.05, 0.0999, 0.1, 0.2, 0.7, 1.5, 3.0, 7.5])
def test_coefficients_against_40_digit_values(theta):
    dt = 0.37
    k = theta / dt  # c = 1, K along x
    got = kspace.coefficients(np.array([k]), np.array([0.0]), np.array([0.0]), dt, 1.0)
    ref = _mp_coefs(theta, dt)
    # Below theta = 0.1 the series is accurate to ~1e-16; just above it the
    # direct formulas lose about log10(6/theta^2) digits to cancellation.
    tol = 2e-15 if theta < 0.1 else 1e-12 * max(1.0, 0.1 / theta) ** 2
    for name in ("C", "S1", "X1", "X2", "X3"):
        assert abs(got[name][0] - ref[name]) <= tol * abs(ref[name]), name


def test_coefficients_zero_k_limits_and_c_scaling():
    dt = 0.25
    z = np.zeros(1)
    got = kspace.coefficients(z, z, z, dt, 3.0)
    assert got["C"][0] == 1.0
    assert got["S1"][0] == dt
    assert got["X1"][0] == dt * dt / 2
    assert got["X2"][0] == dt * dt / 6
    assert got["X3"][0] == -dt * dt / 3
    # omega = c |K|: scaling c by 2 and K by 1/2 leaves every coefficient unchanged
    a = kspace.coefficients(np.array([0.8]), np.array([0.3]), np.array([-1.1]), dt, 2.0)
    b = kspace.coefficients(np.array([1.6]), np.array([0.6]), np.array([-2.2]), dt, 1.0)
    for name in a:
        np.testing.assert_allclose(a[name], b[name], rtol=1e-15)


# ---------------------------------------------------------------- single-mode push

def _mode(rng, c, eps0, dt, order=8, with_sources=True):
    k = rng.uniform(-2.5, 2.5, size=3)
    K = kspace.modified_k_at(np.abs(k), 1.0, order) * np.sign(k)
    E = rng.standard_normal(3) + 1j * rng.standard_normal(3)
    B = rng.standard_normal(3) + 1j * rng.standard_normal(3)
    B = B - K * (K @ B) / (K @ K)  # div B = 0
    J = (rng.standard_normal(3) + 1j * rng.standard_normal(3)) if with_sources else np.zeros(3, complex)
    rho_old = eps0 * 1j * (K @ E)  # Gauss
    rho_new = rho_old - dt * 1j * (K @ J)  # continuity
    return K, E, B, J, rho_old, rho_new


def _push1(K, E, B, J, ro, rn, dt, c, eps0):
    coef = kspace.coefficients(np.array([K[0]]), np.array([K[1]]), np.array([K[2]]), dt, c)
    Kt = (np.array([K[0]]), np.array([K[1]]), np.array([K[2]]))
    En, Bn = kspace.push([np.array([e]) for e in E], [np.array([b]) for b in B], [np.array([j]) for j in J],
                         np.array([ro]), np.array([rn]), Kt, coef, c, eps0)
    return np.array([e[0] for e in En]), np.array([b[0] for b in Bn])


def _rk4(K, E, B, J, dt, c, eps0, nsub=4000):
    def rhs(e, b):
        return 1j * c * c * np.cross(K, b) - J / eps0, -1j * np.cross(K, e)
    h = dt / nsub
    e, b = E.astype(complex), B.astype(complex)
    for _ in range(nsub):
        k1 = rhs(e, b)
        k2 = rhs(e + h / 2 * k1[0], b + h / 2 * k1[1])
        k3 = rhs(e + h / 2 * k2[0], b + h / 2 * k2[1])
        k4 = rhs(e + h * k3[0], b + h * k3[1])
        e = e + h / 6 * (k1[0] + 2 * k2[0] + 2 * k3[0] + k4[0])
        b = b + h / 6 * (k1[1] + 2 * k2[1] + 2 * k3[1] + k4[1])
    return e, b


@pytest.mark.parametrize("seed,dt,c,eps0", [(1, 0.5, 1.0, 1.0), (2, 1.3, 1.7, 0.8), (3, 0.05, 0.6, 2.5),
                                            (4, 2.9, 1.0, 1.0)])
def test_push_equals_numerical_integration(seed, dt, c, eps0):
    rng = np.random.default_rng(seed)
    K, E, B, J, ro, rn = _mode(rng, c, eps0, dt)
    En, Bn = _push1(K, E, B, J, ro, rn, dt, c, eps0)
    er, br = _rk4(K, E, B, J, dt, c, eps0)
    scale = np.abs(np.concatenate([er, br * c])).max()
    assert np.abs(En - er).max() <= 1e-11 * scale
    assert np.abs(Bn - br).max() * c <= 1e-11 * scale


@pytest.mark.parametrize("seed", range(5))
def test_rho_form_equals_j_form(seed):
    rng = np.random.default_rng(100 + seed)
    dt, c, eps0 = 0.8, 1.3, 0.7
    K, E, B, J, ro, rn = _mode(rng, c, eps0, dt)
    En, Bn = _push1(K, E, B, J, ro, rn, dt, c, eps0)
    coef = kspace.coefficients(np.array([K[0]]), np.array([K[1]]), np.array([K[2]]), dt, c)
    Kt = (np.array([K[0]]), np.array([K[1]]), np.array([K[2]]))
    Ej, Bj = kspace.push_jform([np.array([e]) for e in E], [np.array([b]) for b in B],
                               [np.array([j]) for j in J], Kt, coef, dt, c, eps0)
    Ej = np.array([e[0] for e in Ej])
    assert np.abs(En - Ej).max() <= 1e-13 * np.abs(En).max()


@pytest.mark.parametrize("seed", range(5))
def test_gauss_and_div_b_preserved(seed):
    rng = np.random.default_rng(200 + seed)
    dt, c, eps0 = 1.1, 1.0, 1.4
    K, E, B, J, ro, rn = _mode(rng, c, eps0, dt)
    En, Bn = _push1(K, E, B, J, ro, rn, dt, c, eps0)
    assert abs(1j * (K @ En) - rn / eps0) <= 1e-13 * abs(rn / eps0) + 1e-15
    assert abs(K @ Bn) <= 1e-13 * np.linalg.norm(K) * np.abs(Bn).max()


@pytest.mark.parametrize("seed", range(5))
def test_vacuum_energy_conserved(seed):
    rng = np.random.default_rng(300 + seed)
    dt, c, eps0 = 0.9, 1.6, 1.0
    K, E, B, J, ro, rn = _mode(rng, c, eps0, dt, with_sources=False)
    E = E - K * (K @ E) / (K @ K)  # transverse, rho = 0
    z = np.zeros(3, complex)
    En, Bn = _push1(K, E, B, z, 0j, 0j, dt, c, eps0)
    w0 = np.sum(np.abs(E) ** 2) + c * c * np.sum(np.abs(B) ** 2)
    w1 = np.sum(np.abs(En) ** 2) + c * c * np.sum(np.abs(Bn) ** 2)
    assert abs(w1 - w0) <= 1e-14 * w0


@pytest.mark.parametrize("seed", range(4))
def test_half_steps_compose_and_reverse(seed):
    rng = np.random.default_rng(400 + seed)
    dt, c, eps0 = 1.2, 1.0, 0.9
    K, E, B, J, ro, rn = _mode(rng, c, eps0, dt)
    rmid = ro - dt / 2 * 1j * (K @ J)
    e1, b1 = _push1(K, E, B, J, ro, rmid, dt / 2, c, eps0)
    e2, b2 = _push1(K, e1, b1, J, rmid, rn, dt / 2, c, eps0)
    ef, bf = _push1(K, E, B, J, ro, rn, dt, c, eps0)
    s = np.abs(ef).max() + np.abs(bf).max()
    assert np.abs(e2 - ef).max() <= 1e-13 * s and np.abs(b2 - bf).max() <= 1e-13 * s
    # forward then backward in time with the same sources returns the start
    eb, bb = _push1(K, ef, bf, J, rn, ro, -dt, c, eps0)
    assert np.abs(eb - E).max() <= 1e-13 * s and np.abs(bb - B).max() <= 1e-13 * s


def test_push_is_first_order_consistent_with_maxwell():
    rng = np.random.default_rng(7)
    c, eps0 = 1.2, 0.6
    errs = []
    for h in (1e-2, 1e-3):
        K, E, B, J, ro, rn = _mode(np.random.default_rng(7), c, eps0, h)
        En, Bn = _push1(K, E, B, J, ro, rn, h, c, eps0)
        dE = 1j * c * c * np.cross(K, B) - J / eps0
        dB = -1j * np.cross(K, E)
        errs.append(max(np.abs((En - E) / h - dE).max(), np.abs((Bn - B) / h - dB).max()))
    assert 5 < errs[0] / errs[1] < 20  # error is O(h)
    del rng
