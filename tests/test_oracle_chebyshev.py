"""Pins of the oracle's Chebyshev polynomial and filter (CPU only).

Each check compares the oracle with something other than its own formula:
trigonometric / hyperbolic identities, the explicit power-sum expansion of
T_n, the growth bound of Lemma cheb-est (section 3.1), and the spectral
closed form rho(A) U = Q diag(rho(lambda)) Q^T U (section 2.1, first
paragraph) on planted and diagonal matrices.
"""
from fractions import Fraction
from math import factorial

import numpy as np
import pytest

import oracle
from paper_1904_10585_amd import workloads as wl


def explicit_T(n, x):
    """T_n(x) from the explicit sum n/2 * sum_k (-1)^k (n-k-1)!/(k!(n-2k)!) (2x)^(n-2k)
    evaluated in exact rational arithmetic."""
    if n == 0:
        return Fraction(1)
    x = Fraction(x)
    s = Fraction(0)
    for k in range(n // 2 + 1):
        s += Fraction((-1) ** k * factorial(n - k - 1), factorial(k) * factorial(n - 2 * k)) * (2 * x) ** (n - 2 * k)
    return Fraction(n, 2) * s


@pytest.mark.parametrize("d", range(0, 16))
def test_cos_identity(d):
    th = np.linspace(0.0, np.pi, 1001)
    np.testing.assert_allclose(oracle.cheb_T(d, np.cos(th)), np.cos(d * th), atol=1e-12)


@pytest.mark.parametrize("d", range(0, 16))
def test_cosh_identity_and_parity(d):
    x = np.linspace(1e-3, 3.0, 500)
    t = np.cosh(x)
    np.testing.assert_allclose(oracle.cheb_T(d, t), np.cosh(d * x), rtol=1e-11)
    np.testing.assert_allclose(oracle.cheb_T(d, -t), (-1) ** d * np.cosh(d * x), rtol=1e-11)


@pytest.mark.parametrize("d", [1, 2, 3, 5, 8, 10, 12])
def test_explicit_power_sum(d):
    pts = [Fraction(k, 7) for k in range(-21, 22)]
    ref = np.array([float(explicit_T(d, x)) for x in pts])
    got = oracle.cheb_T(d, np.array([float(x) for x in pts]))
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("d", [1, 2, 4, 8, 10, 12, 20])
def test_lemma_cheb_est(d):
    # |T_d(+-(1+eps))| >= 2^(d min(sqrt(eps),1) - 1)   (section 3.1, Lemma cheb-est)
    eps = np.logspace(-6, 2, 400)
    bound = 2.0 ** (d * np.minimum(np.sqrt(eps), 1.0) - 1.0)
    for s in (1.0, -1.0):
        assert np.all(np.abs(oracle.cheb_T(d, s * (1.0 + eps))) >= bound * (1 - 1e-14))


def test_interval_map_endpoints():
    a, b = -5.0, 0.8
    np.testing.assert_allclose(oracle.interval_map([a, b, (a + b) / 2], a, b), [-1.0, 1.0, 0.0], atol=1e-15)


@pytest.mark.parametrize("d,q", [(1, 1), (2, 1), (8, 1), (10, 1), (3, 2), (0, 1)])
def test_filter_planted_closed_form(d, q):
    n, p = 96, 7
    X, lam, Q = wl.planted(n, 8, (2.0, 10.0), (-1.0, 0.5), config=99, index=d)
    U = wl.start_block(n, p, config=99, index=d)
    a, b = -1.0, 0.5
    Y = oracle.chebyshev_filter(lambda B: X @ B, U, d, a, b, q)
    # spectral definition of rho(X)^q U
    ref = Q @ ((oracle.rho(lam, d, a, b) ** q)[:, None] * (Q.T @ U))
    err = np.linalg.norm(Y - ref, axis=0) / np.linalg.norm(ref, axis=0)
    assert err.max() < 1e-11, err.max()


def test_filter_diagonal_entrywise():
    x = np.linspace(-3.0, 4.0, 57)
    U = np.random.default_rng(3).standard_normal((57, 3))
    a, b, d = -1.5, 0.75, 9
    Y = oracle.chebyshev_filter(lambda B: x[:, None] * B, U, d, a, b)
    s = (x - (a + b) / 2) / ((b - a) / 2)
    ref = np.array([float(explicit_T(d, Fraction(v))) for v in s])[:, None] * U
    np.testing.assert_allclose(Y, ref, rtol=1e-10, atol=1e-12)


def test_filter_longdouble_bound():
    # the FP64 recurrence against the same recurrence in 80-bit long double:
    # bounds the oracle's own rounding (relative error well below 1e-13)
    n, p, d, a, b = 64, 4, 10, -1.0, 0.5
    X, _, _ = wl.planted(n, 6, (2.0, 10.0), (-1.0, 0.5), config=98)
    U = wl.start_block(n, p, config=98)
    Y = oracle.chebyshev_filter(lambda B: X @ B, U, d, a, b)
    XL = X.astype(np.longdouble)
    c, e = np.longdouble(a + b) / 2, np.longdouble(b - a) / 2
    Y0 = U.astype(np.longdouble)
    Y1 = (XL @ Y0 - c * Y0) / e
    for _ in range(1, d):
        Y0, Y1 = Y1, 2 * (XL @ Y1 - c * Y1) / e - Y0
    rel = np.linalg.norm((Y - Y1).astype(np.float64), axis=0) / np.linalg.norm(Y, axis=0)
    assert rel.max() < 1e-13
