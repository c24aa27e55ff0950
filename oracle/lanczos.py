"""Spectrum estimate, interval / block-size rules (section 4.1, 4.2) and
the filter-degree rule (section 3, Lemma ctr1 and Theorem conv1).

Test infrastructure (see ``oracle/__init__``).

Section 4.1 places the left end a of the damping interval at the smallest
eigenvalue lambda_n of the input matrix and names the Lanczos method as the
way to estimate it; b then follows one of two rules (all positive
eigenvalues wanted, or the r largest).  Section 4.2 sizes the block: 5 + q r
columns for the r largest, or the positive count of the previous iterate
plus guard columns.

``block_krylov_ritz`` is the estimate by its definition: the Rayleigh-Ritz
values of X on the block Krylov space
    K_s(X, V0) = span{V0, X V0, ..., X^(s-1) V0},
with an orthonormal basis built in FP64 (each new block X V_j orthogonalised
against all earlier blocks twice, then by numpy's QR).  Parity is pinned by
tests/test_oracle_lanczos.py: when K is the whole space the Ritz values are
the eigenvalues; Cauchy interlacing (theta_min >= lambda_min,
theta_max <= lambda_max); every Ritz value has an eigenvalue within its
residual norm; the residual equals ||X y - theta y|| formed directly.
"""
import numpy as np


def block_krylov_ritz(X, V0, steps):
    """Ritz values (ascending), Ritz vectors and residual norms of symmetric
    X on K_steps(X, V0) (section 4.1: the Lanczos estimate of lambda_n).

    V0 is n x s; the basis has s * steps columns (requires s * steps <= n
    and a Krylov space of full dimension)."""
    X = np.asarray(X, dtype=np.float64)
    n, s = V0.shape
    blocks = [np.linalg.qr(np.asarray(V0, dtype=np.float64))[0]]
    for j in range(1, steps):
        B = np.hstack(blocks)
        W = X @ blocks[-1]
        for _ in range(2):
            W = W - B @ (B.T @ W)
        blocks.append(np.linalg.qr(W)[0])
    V = np.hstack(blocks)
    H = V.T @ X @ V
    H = 0.5 * (H + H.T)
    theta, Z = np.linalg.eigh(H)
    Y = V @ Z
    res = np.linalg.norm(X @ Y - Y * theta, axis=0)
    return theta, Y, res


def lanczos_bounds(X, V0, steps):
    """(theta_min, theta_max, res_min, res_max) of ``block_krylov_ritz``."""
    theta, _, res = block_krylov_ritz(X, V0, steps)
    return theta[0], theta[-1], res[0], res[-1]


def interval_policy(lam_min, margin, eta, top_r=0, theta_r=0.0):
    """Damping interval of section 4.1: a = lam_min - margin; all positive
    eigenvalues wanted (top_r <= 0): b = eta a; the r largest:
    b = (1 - eta) theta_r + eta a.  Returns (a, b); raises ValueError
    unless a < b."""
    a = lam_min - margin
    b = eta * a if top_r <= 0 else (1.0 - eta) * theta_r + eta * a
    if not a < b:
        raise ValueError("interval rule gives a >= b")
    return a, b


def block_size_policy(top_r, q=2.0, n_pos=0, guards=0):
    """Block size of section 4.2: 5 + q r (rounded up) for the r largest,
    n_pos + guards for all positive eigenvalues; clamped to [1, 128]."""
    if top_r > 0:
        if not q > 1.0:
            raise ValueError("q must exceed 1")
        p = int(np.ceil(5.0 + q * top_r))
    else:
        p = n_pos + guards
    return int(min(128, max(1, p)))


def degree_policy(theta_r, a, b, q=1, eps=1e-6, d_min=1, d_max=64):
    """Degree for sin <= eps after one filtered step (Lemma ctr1): theta_r
    maps to 1 + l, l = 2 (theta_r - b) / (b - a), the unwanted spectrum into
    [-1, 1]; the error after one step is bounded by a start-angle factor over
    T_d(1 + l)^q (the step of the proof before Lemma cheb-est bounds T_d from
    below), so the smallest d with T_d(1 + l)^q >= 1 / eps, from
    T_d(x) = cosh(d acosh x) for x >= 1.  Clamped to [d_min, d_max]."""
    if not (a < b < theta_r) or not (0.0 < eps < 1.0) or q < 1 or not (1 <= d_min <= d_max):
        raise ValueError("need a < b < theta_r, 0 < eps < 1, q >= 1, 1 <= d_min <= d_max")
    x = 1.0 + 2.0 * (theta_r - b) / (b - a)
    d = int(np.ceil(np.arccosh(eps ** (-1.0 / q)) / np.arccosh(x)))
    return int(min(d_max, max(d_min, d)))
