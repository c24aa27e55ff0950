"""Pins of the oracle's nearest-correlation dual, exact gradient method,
extrapolation and PFPG loop (section 5.1, section 4.3) against facts other
than their own formulas."""
import numpy as np
import pytest

import oracle
from paper_1904_10585_amd import workloads as wl


def test_gradient_matches_finite_differences():
    """grad F of eq. NCE-gradient against central differences of F of eq.
    NCE-dual-equiv (F is continuously differentiable: f(l) = 1/2 max(l,0)^2)."""
    n = 40
    G = wl.nce_matrix(n, 6, config=150, index=1)
    x = np.random.default_rng(1).uniform(-3.0, 3.0, n)
    _, g, _ = oracle.nce_dual(G, x)
    h = 1e-6
    fd = np.empty(n)
    for i in range(n):
        e = np.zeros(n)
        e[i] = h
        fd[i] = (oracle.nce_dual(G, x + e)[0] - oracle.nce_dual(G, x - e)[0]) / (2 * h)
    np.testing.assert_allclose(g, fd, atol=1e-6)


def test_correlation_matrix_is_its_own_solution():
    """G PSD with unit diagonal: x0 = 1 - diag(G) = 0 has zero gradient and
    the primal point is G itself."""
    g = np.random.default_rng(2)
    A = g.standard_normal((50, 8))
    C = A @ A.T
    d = np.sqrt(np.diag(C))
    C = C / d[:, None] / d[None, :]
    _, grad, _ = oracle.nce_dual(C, np.zeros(50))
    assert np.abs(grad).max() < 1e-12
    r = oracle.nce_grad(C, max_iter=5)                # the relative stop test needs g0 > 0
    assert np.abs(r["x"]).max() < 1e-12
    np.testing.assert_allclose(oracle.nce_primal(C, r["x"]), C, atol=1e-12)


def alternating_projections(G, iters):
    """Nearest correlation matrix by alternating projections with Dykstra's
    correction (Higham 2002): an algorithm independent of the dual."""
    Y = G.copy()
    dS = np.zeros_like(G)
    for _ in range(iters):
        R = Y - dS
        w, Q = np.linalg.eigh(R)
        X = (Q * np.maximum(w, 0.0)) @ Q.T
        dS = X - R
        Y = X.copy()
        np.fill_diagonal(Y, 1.0)
    return Y


@pytest.mark.parametrize("example", [6, 7])
def test_solution_kkt_duality_and_independent_solver(example):
    """At the exact method's solution: X = P_+(G + Diag(x)) is PSD with unit
    diagonal, complementary to the dual slack, its primal value equals
    1/2 ||G||^2 - F(x) (strong duality), and it is the matrix alternating
    projections converge to."""
    n = 30
    G = wl.nce_matrix(n, example, config=151, index=example)
    r = oracle.nce_grad(G, tol=1e-12, max_iter=5000)
    X = oracle.nce_primal(G, r["x"])
    S = X - (G + np.diag(r["x"]))                   # the negative part: PSD, X S = 0
    assert np.abs(np.diag(X) - 1.0).max() < 1e-9
    assert np.linalg.eigvalsh(X).min() > -1e-10 and np.linalg.eigvalsh(S).min() > -1e-10
    assert np.abs(X @ S).max() < 1e-9
    primal = 0.5 * np.linalg.norm(G - X) ** 2
    assert abs(primal - (0.5 * np.linalg.norm(G) ** 2 - r["F"])) <= 1e-9 * primal
    Xap = alternating_projections(G, 3000)
    assert np.abs(Xap - X).max() < 1e-6


@pytest.mark.parametrize("example,n,printed", [(6, 500, 8.9e3), (6, 1000, 2.6e4), (7, 500, 1.3e5)])
def test_objective_matches_the_paper_table(example, n, printed):
    """Table ncm prints F at the solution for random instances of the same
    examples (two digits); the value concentrates as n grows, so a fresh
    draw lands within a few percent."""
    G = wl.nce_matrix(n, example, config=152, index=n)
    r = oracle.nce_grad(G)
    assert r["gnorm"] <= 1e-7 * r["g0"]
    assert abs(r["F"] - printed) <= 0.05 * printed, r["F"]


def test_extrapolation_is_exact_on_a_linear_iteration():
    """x_{k+1} = A x_k + c in R^5: five differences span the error space, so
    the extrapolation of section 4.3 (lambda -> 0) returns the fixed point."""
    g = np.random.default_rng(3)
    Q, _ = np.linalg.qr(g.standard_normal((5, 5)))
    A = (Q * np.array([0.9, 0.7, -0.5, 0.3, 0.1])) @ Q.T
    c = g.standard_normal(5)
    xs = [g.standard_normal(5)]
    for _ in range(6):
        xs.append(A @ xs[-1] + c)
    fixed = np.linalg.solve(np.eye(5) - A, c)
    assert np.abs(oracle.rna_extrapolate(xs, 1e-14) - fixed).max() < 1e-6
    assert np.abs(xs[-1] - fixed).max() > 1e-2                 # the plain iterate is far from it
    # equal differences: U^T U has equal entries, the weights are equal and
    # sum to one, so the result is the mean of the first l + 1 points (the
    # Gram is rank one: the regularised solve leaves ~cond * eps = 1e-8)
    v = g.standard_normal(5)
    np.testing.assert_allclose(oracle.rna_extrapolate([c, c + v, c + 2 * v, c + 3 * v], 1e-8), c + v, atol=1e-6)


@pytest.mark.parametrize("example,n", [(6, 300), (7, 400)])
def test_pfpg_reaches_the_exact_solution(example, n):
    """PFPG's filtered gradients converge to the exact method's point: the
    same F to 1e-9 relative and x within the stopping tolerance; the block
    shrinks from 128 to the positive count plus guards."""
    G = wl.nce_matrix(n, example, config=153, index=n)
    e = oracle.nce_grad(G)
    f = oracle.nce_pfpg(G, wl.start_block(n, 128, config=153, index=n), wl.start_block(n, 16, config=154, index=n))
    assert f["gnorm"] <= 1e-7 * f["g0"]
    assert abs(f["F"] - e["F"]) <= 1e-9 * abs(e["F"])
    assert np.abs(f["x"] - e["x"]).max() <= 1e-3
    assert f["n_pos"] == e["n_pos"] and f["p"] < 128 and f["p"] >= f["n_pos"]


@pytest.mark.parametrize("example,n", [(6, 40), (7, 30)])
def test_primal_drs_reaches_the_dual_solution(example, n):
    """DRS on the primal (PSD projection, entrywise prox of the affine part)
    and the dual gradient method are different algorithms on the same
    problem: the same nearest correlation matrix, unit diagonal, PSD."""
    G = wl.nce_matrix(n, example, config=155, index=n)
    Xd = oracle.nce_primal(G, oracle.nce_grad(G, tol=1e-12, max_iter=5000)["x"])
    r = oracle.nce_drs(G, tol=1e-12, max_iter=20000)
    assert np.abs(r["X"] - Xd).max() < 1e-8
    assert np.abs(np.diag(r["X"]) - 1.0).max() < 1e-8 and np.linalg.eigvalsh(r["X"]).min() > -1e-10


def test_pfam_reaches_the_nearest_correlation_matrix():
    """PFAM's projections from the extracted subspace converge to the dual
    method's nearest correlation matrix (the block starts truncated: about
    n / 2 positive eigenvalues against 128 columns)."""
    n = 300
    G = wl.nce_matrix(n, 6, config=156, index=n)
    Xd = oracle.nce_primal(G, oracle.nce_grad(G, tol=1e-10)["x"])
    f = oracle.nce_pfam(G, wl.start_block(n, 128, config=156, index=n), wl.start_block(n, 16, config=157, index=n))
    assert f["converged"] and f["p"] < 128
    assert np.abs(f["X"] - Xd).max() < 1e-5
    h = np.array(f["history"])
    assert h[-1, 6] < 1e-5                              # unit diagonal at the end
