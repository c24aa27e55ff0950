"""Pins of the extended-precision extraction (CPU).

It is the reference where the FP64 oracle's own rounding is too large for
the FP64 tolerance (a cold random start), so it is pinned at better than
FP64 accuracy: exact rational Chebyshev values, an exactly invariant start
block on a diagonal matrix, and the Jacobi solver's residual and
orthogonality measured in extended precision.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle.extended import chebyshev_filter_ld, mgs2, LD
from paper_1904_10585_amd import workloads as wl
from test_oracle_chebyshev import explicit_T

pytestmark = pytest.mark.skipif(np.finfo(np.longdouble).eps > 1e-18,
                                reason="numpy.longdouble is not 80-bit extended here")


def test_filter_exact_rational_diagonal():
    # diagonal X with entries exact in binary: T_d of the mapped entries in
    # exact rationals times U; extended precision gets ~1e-18, FP64 ~1e-15
    x = np.arange(-24, 33) / 8.0
    U = np.random.default_rng(5).standard_normal((x.size, 3))
    a, b, d = -1.5, 0.75, 9
    c, e = Fraction(a + b) / 2, Fraction(b - a) / 2
    t = np.array([float(explicit_T(d, (Fraction(v) - c) / e)) for v in x])
    exact = [[explicit_T(d, (Fraction(v) - c) / e) * Fraction(u) for u in row] for v, row in zip(x, U)]
    Y = chebyshev_filter_ld(np.diag(x), U, d, a, b)
    err = max(abs(Fraction(float(Y[i, j])) + Fraction(float(Y[i, j] - LD(float(Y[i, j])))) - exact[i][j])
              / abs(exact[i][j]) for i in range(x.size) for j in range(3) if exact[i][j] != 0)
    assert err < 1e-17, float(err)
    assert np.allclose(Y.astype(np.float64), t[:, None] * U, rtol=1e-14)


def test_invariant_block_gives_diagonal_eigenvalues():
    # span(U) = span(e_S) exactly, so theta = x_S to extended precision
    g = np.random.default_rng(6)
    x = g.permutation(np.arange(1, 101)) / 16.0 - 2.0
    S = np.argsort(-x)[:6]
    U = np.zeros((100, 6))
    U[S, :] = g.standard_normal((6, 6))
    out = oracle.extract_longdouble(np.diag(x), U, 5, -2.0, 2.5)
    theta, V = out["theta"], out["V"]
    ref = np.sort(x[S])[::-1].astype(LD)
    assert np.max(np.abs(theta - ref) / np.abs(ref)) < 1e-17
    off = np.ones(100, bool)
    off[S] = False
    assert np.max(np.abs(V[off])) == 0.0
    assert np.max(np.abs(V.T @ V - np.eye(6, dtype=LD))) < 1e-17


def test_jacobi_ld_residual_and_orthogonality():
    g = np.random.default_rng(7)
    A = g.standard_normal((24, 24))
    H = (A + A.T) / 2
    theta, Z = oracle.jacobi_eigh_ld(H)
    HL = H.astype(LD)
    res = np.max(np.abs(HL @ Z - Z * theta))
    assert res < 1e-17 * np.max(np.abs(np.linalg.eigvalsh(H)))
    assert np.max(np.abs(Z.T @ Z - np.eye(24, dtype=LD))) < 1e-17
    np.testing.assert_allclose(theta.astype(np.float64), np.sort(np.linalg.eigvalsh(H))[::-1], atol=1e-13)


def test_mgs2_basis_of_an_ill_conditioned_block():
    g = np.random.default_rng(8)
    Y = g.standard_normal((120, 8)) @ np.diag(np.logspace(0, 9, 8))
    Q = mgs2(Y)
    assert np.max(np.abs(Q.T @ Q - np.eye(8, dtype=LD))) < 1e-17
    Us, _, _ = np.linalg.svd(Y, full_matrices=False)
    assert oracle.sin_theta(Q.astype(np.float64), Us) < 1e-12


def test_agrees_with_fp64_oracle_on_a_warm_step():
    n, p, r, d, a, b = 400, 12, 6, 8, -1.0, 0.5
    X, _, _ = wl.planted(n, r, (2.0, 10.0), (-1.0, 0.5), config=99)
    U = oracle.extract(X, X, wl.start_block(n, p, config=99), d, a, b)["V"]
    ref = oracle.extract(X, X, U, d, a, b)
    out = oracle.extract_longdouble(X, U, d, a, b)
    theta, V = out["theta"], out["V"]
    assert oracle.ritz_rel_err(ref["theta"], theta.astype(np.float64), r) < 1e-14
    assert oracle.sin_theta(np.linalg.qr(V[:, :r].astype(np.float64))[0], ref["V"][:, :r]) < 1e-13
