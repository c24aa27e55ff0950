"""Pins of the oracle's optional outputs: the Ritz residual norms (the
convergence measure of eq. RR) and the singular-value shrinkage of
section 5.2.1, against hand-computed values, constructed factorisations and
their defining properties."""
import numpy as np

import oracle


def _orthogonal(rng, n, k):
    Q, R = np.linalg.qr(rng.standard_normal((n, k)))
    return Q * np.sign(np.diag(R))


def test_ritz_residuals_hand_values():
    # X e_1 - X_11 e_1 is the off-diagonal part of X's first column
    X = np.array([[2.0, 3.0, 0.0], [3.0, 1.0, 4.0], [0.0, 4.0, 5.0]])
    V = np.eye(3)[:, :2]
    theta = np.array([2.0, 1.0])
    r = oracle.ritz_residuals(lambda B: X @ B, V, theta)
    assert np.allclose(r, [3.0, 5.0], rtol=0, atol=1e-15)
    # a wrong Ritz value moves the residual by exactly |delta| along v
    r2 = oracle.ritz_residuals(lambda B: X @ B, V[:, :1], np.array([2.5]))
    assert abs(r2[0] - np.hypot(3.0, 0.5)) < 1e-15


def test_ritz_residuals_vanish_on_eigenpairs():
    rng = np.random.default_rng(3)
    Q = _orthogonal(rng, 40, 40)
    lam = np.linspace(-3, 7, 40)
    X = (Q * lam) @ Q.T
    r = oracle.ritz_residuals(lambda B: X @ B, Q[:, :6], lam[:6])
    assert r.max() < 1e-13
    # a rotated pair of eigenvectors with a clustered-free spectrum is not
    # an eigenpair: the residual is the exact norm of the mixing
    c, s = np.cos(0.3), np.sin(0.3)
    v = c * Q[:, 0] + s * Q[:, 1]
    th = c * c * lam[0] + s * s * lam[1]
    want = np.hypot(c * (lam[0] - th), s * (lam[1] - th))
    got = oracle.ritz_residuals(lambda B: X @ B, v[:, None], np.array([th]))[0]
    assert abs(got - want) < 1e-13


def test_svd_shrink_hand_values():
    M = np.array([[3.0, 0.0], [0.0, 1.0], [0.0, 0.0]])
    assert np.allclose(oracle.svd_shrink(M, 2.0), [[1.0, 0.0], [0.0, 0.0], [0.0, 0.0]], atol=1e-15)
    assert np.allclose(oracle.svd_shrink(M, 0.0), M, atol=1e-15)
    assert np.allclose(oracle.svd_shrink(M, 5.0), 0.0, atol=1e-15)


def test_svd_shrink_constructed_factorisation():
    # M = U diag(s) V^T built from known factors: the shrinkage is
    # U diag((s - tau)_+) V^T, the nuclear-norm proximal point
    rng = np.random.default_rng(5)
    U = _orthogonal(rng, 30, 8)
    V = _orthogonal(rng, 20, 8)
    s = np.array([9.0, 7.5, 6.0, 4.0, 3.0, 2.0, 1.0, 0.5])
    M = (U * s) @ V.T
    tau = 2.5
    want = (U * np.maximum(s - tau, 0.0)) @ V.T
    assert np.abs(oracle.svd_shrink(M, tau) - want).max() < 1e-13
    # the proximal point minimises tau ||Y||_* + 1/2 ||Y - M||_F^2: no
    # random perturbation does better
    def obj(Y):
        return tau * np.linalg.svd(Y, compute_uv=False).sum() + 0.5 * np.sum((Y - M) ** 2)
    f0 = obj(want)
    for _ in range(20):
        assert obj(want + 1e-3 * rng.standard_normal(M.shape)) > f0


def test_svd_shrink_factor_on_exact_subspace():
    # with V the top-p right singular vectors and theta = s^2, L V^T is the
    # full shrinkage as soon as tau >= s_{p+1} (the rest is shrunk to zero)
    rng = np.random.default_rng(7)
    U = _orthogonal(rng, 25, 10)
    V = _orthogonal(rng, 18, 10)
    s = np.array([12.0, 10.0, 8.0, 6.5, 5.0, 2.0, 1.5, 1.0, 0.4, 0.1])
    M = (U * s) @ V.T
    p = 5
    for tau in (2.0, 3.0, 5.5):
        L = oracle.svd_shrink_factor(M, V[:, :p], s[:p] ** 2, tau)
        want = (U * np.maximum(s - tau, 0.0)) @ V.T
        assert np.abs(L @ V[:, :p].T - want).max() < 1e-12, tau
        # the nonzero singular values of the result are (s_i - tau)_+
        sv = np.linalg.svd(L @ V[:, :p].T, compute_uv=False)
        assert np.allclose(sv[:p], np.sort(np.maximum(s[:p] - tau, 0.0))[::-1], atol=1e-12)
    # tau = 0 gives the projection M V V^T; sigma = 0 columns are zero
    L0 = oracle.svd_shrink_factor(M, V[:, :p], s[:p] ** 2, 0.0)
    assert np.abs(L0 @ V[:, :p].T - M @ V[:, :p] @ V[:, :p].T).max() < 1e-12
    Lz = oracle.svd_shrink_factor(np.zeros((4, 3)), np.eye(3)[:, :2], np.zeros(2), 0.0)
    assert np.all(Lz == 0.0)
