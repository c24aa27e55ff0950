"""Pins of the oracle's Lanczos estimate and interval / block-size rules
(section 4.1, 4.2) against facts other than its own formulas."""
import numpy as np
import pytest

import oracle


def sym(n, seed, spec=None):
    g = np.random.default_rng(seed)
    Q, R = np.linalg.qr(g.standard_normal((n, n)))
    Q = Q * np.sign(np.diag(R))
    lam = g.standard_normal(n) if spec is None else np.asarray(spec, dtype=np.float64)
    return (Q * lam) @ Q.T, np.sort(lam)


def test_whole_space_gives_the_eigenvalues():
    """K_3(X, V0) with 16-column blocks spans R^48: Rayleigh-Ritz on it is
    the full eigendecomposition."""
    X, lam = sym(48, 1)
    V0 = np.random.default_rng(2).standard_normal((48, 16))
    theta, Y, res = oracle.block_krylov_ritz(X, V0, 3)
    np.testing.assert_allclose(theta, lam, atol=1e-12)
    assert np.max(res) < 1e-12
    assert np.abs(Y.T @ Y - np.eye(48)).max() < 1e-12


@pytest.mark.parametrize("n,steps", [(200, 3), (500, 6)])
def test_interlacing_and_residual_bracket(n, steps):
    """Cauchy interlacing: lambda_min <= theta_min and theta_max <= lambda_max;
    every Ritz value has an eigenvalue within its residual norm."""
    X, lam = sym(n, n)
    V0 = np.random.default_rng(n + 1).standard_normal((n, 16))
    theta, _, res = oracle.block_krylov_ritz(X, V0, steps)
    assert theta[0] >= lam[0] - 1e-12 and theta[-1] <= lam[-1] + 1e-12
    gap = np.min(np.abs(lam[None, :] - theta[:, None]), axis=1)
    assert np.all(gap <= res + 1e-12)
    lo, hi, rlo, rhi = oracle.lanczos_bounds(X, V0, steps)
    assert (lo, hi, rlo, rhi) == (theta[0], theta[-1], res[0], res[-1])


def test_invariant_start_block():
    """V0 spanning 16 eigenvectors: Ritz values are those eigenvalues with
    zero residuals after one step."""
    n = 120
    X, lam = sym(n, 7)
    w, U = np.linalg.eigh(X)
    V0 = U[:, 10:26] @ np.random.default_rng(8).standard_normal((16, 16))
    theta, _, res = oracle.block_krylov_ritz(X, V0, 1)
    np.testing.assert_allclose(theta, w[10:26], atol=1e-12)
    assert np.max(res) < 1e-12


def test_isolated_smallest_eigenvalue_converges():
    """A planted spectrum with lambda_min = -7 well below a bulk in [-2, 1]:
    eight block steps pin lambda_min to high relative accuracy."""
    g = np.random.default_rng(3)
    spec = np.concatenate([[-7.0], g.uniform(-2.0, 1.0, 1999)])
    X, lam = sym(2000, 4, spec)
    V0 = g.standard_normal((2000, 16))
    lo, hi, rlo, _ = oracle.lanczos_bounds(X, V0, 8)
    assert abs(lo - lam[0]) <= 1e-8 * 7.0
    assert rlo <= 1e-3


def test_interval_rules_worked_examples():
    """Section 4.1 with numbers: all positive, a = -5, eta = 0.1 gives
    b = -0.5; the r largest with theta_r = 2, eta = 0.2, a = -5 - 0.5 gives
    b = 0.8 * 2 + 0.2 * (-5.5) = 0.5."""
    assert oracle.interval_policy(-5.0, 0.0, 0.1) == (-5.0, -0.5)
    a, b = oracle.interval_policy(-5.0, 0.5, 0.2, top_r=40, theta_r=2.0)
    assert a == -5.5 and abs(b - 0.5) < 1e-15
    with pytest.raises(ValueError):
        oracle.interval_policy(1.0, 0.0, 0.1)          # PSD: all-positive rule has no interval
    with pytest.raises(ValueError):
        oracle.interval_policy(-1.0, 0.0, 0.1, top_r=3, theta_r=-2.0)


def test_block_size_rules_worked_examples():
    """Section 4.2 with numbers: r = 40, q = 1.5 gives 5 + 60 = 65; all
    positive with 37 positive Ritz values and 8 guards gives 45; clamped to
    the 128-column limit."""
    assert oracle.block_size_policy(40, 1.5) == 65
    assert oracle.block_size_policy(3, 2.2) == 12          # ceil(5 + 6.6)
    assert oracle.block_size_policy(0, n_pos=37, guards=8) == 45
    assert oracle.block_size_policy(100, 2.0) == 128
    with pytest.raises(ValueError):
        oracle.block_size_policy(10, 1.0)


@pytest.mark.parametrize("theta_r,a,b,q,eps", [(1.0, -5.0, 0.8, 1, 1e-6), (1.0, -2.0, 0.8, 2, 1e-8),
                                               (5.0, -1.0, 0.5, 1, 1e-3), (1.2, -5.0, 0.8, 3, 1e-2)])
def test_degree_rule_is_the_smallest_sufficient_degree(theta_r, a, b, q, eps):
    """Lemma ctr1's requirement T_d(1 + l)^q >= 1/eps, checked with the
    oracle's Chebyshev polynomial (pinned on its own): the rule's degree
    meets it and one less does not."""
    d = oracle.degree_policy(theta_r, a, b, q, eps, d_min=1, d_max=10_000)
    x = 1.0 + 2.0 * (theta_r - b) / (b - a)
    assert oracle.cheb_T(d, x) ** q >= (1.0 - 1e-12) / eps
    assert oracle.cheb_T(d - 1, x) ** q < 1.0 / eps
    assert oracle.interval_map(theta_r, a, b) == pytest.approx(x)


def test_degree_schedule_grows_like_log_k():
    """Theorem conv1: eps_k = eps_0 / k gives d_k = O(log k): nondecreasing,
    and d_k - d_1 stays within log(k) / acosh(1 + l) + 1."""
    a, b, th = -5.0, 0.8, 1.5
    x = 1.0 + 2.0 * (th - b) / (b - a)
    ds = [oracle.degree_policy(th, a, b, 1, 1e-2 / k, d_min=1, d_max=10_000) for k in range(1, 2001)]
    assert all(d1 <= d2 for d1, d2 in zip(ds, ds[1:]))
    for k in (10, 100, 1000, 2000):
        assert ds[k - 1] - ds[0] <= np.log(k) / np.arccosh(x) + 1
