"""One subspace extraction: filter, orthonormalise, Rayleigh-Ritz.

Test infrastructure (see ``oracle/__init__``).  FP64 throughout.  The steps
follow the paper's filtered-subspace-extraction order (section 2.1: filter,
then one QR; section 2.2, eq. RR: H = V^T X V, H = Y Lambda Y^T, Ritz
vectors V Y), with the outputs PFPG and PFAM consume (section 2.2, the
projection P_S(X) = S S^T X S S^T; section 2.3, P_+(P_U(Z)) in eq. PFAM1)
and the SVD route of section 5.2.1 (subspace extraction on A^T A).
"""
import numpy as np

from .chebyshev import chebyshev_filter

RANK_TOL = 1e-13


def orthonormalize(Y):
    """Orthonormal basis of range(Y) by one Householder QR (section 2.1).

    Columns are scaled to unit norm first (this changes R, not the range).
    Returns (Q, rank_deficient) where rank_deficient flags
    min|R_ii| / max|R_ii| < 1e-13, the case in which trailing columns of Q
    are an arbitrary orthonormal completion.
    """
    Y = np.asarray(Y, dtype=np.float64)
    norms = np.linalg.norm(Y, axis=0)
    norms[norms == 0.0] = 1.0
    Q, R = np.linalg.qr(Y / norms, mode="reduced")
    dR = np.abs(np.diag(R))
    rank_deficient = bool(dR.min() < RANK_TOL * dR.max())
    return Q, rank_deficient


def rayleigh_ritz(apply_X, Q):
    """Rayleigh-Ritz on range(Q) (section 2.2, eq. RR).

    H = Q^T (X Q), symmetrised; H = Z diag(theta) Z^T with theta sorted in
    descending order (the paper's eigenvalue order, section 1 notation);
    Ritz vectors V = Q Z.  Returns (theta, V, H).
    """
    W = apply_X(Q)
    H = Q.T @ W
    H = 0.5 * (H + H.T)
    theta, Z = np.linalg.eigh(H)
    order = np.argsort(-theta, kind="stable")
    theta = theta[order]
    Z = Z[:, order]
    return theta, Q @ Z, H


def ritz_residuals(apply_X, V, theta):
    """Column residual norms ||X v_i - theta_i v_i||_2."""
    R = apply_X(V) - V * theta
    return np.linalg.norm(R, axis=0)


def extract(X_filter, X_rr, U, d, a, b, q=1):
    """One polynomial-filtered subspace extraction on a symmetric matrix.

    Follows section 2.1 (U+ = orth(rho(A) U), eq. subspace-update) and
    section 2.2 (eq. RR).  ``X_filter`` is the matrix the filter is applied
    with (the dequantised low-precision copy in the precision forms),
    ``X_rr`` the one Rayleigh-Ritz projects (the full-precision matrix).
    Returns a dict with theta (descending), V (n-by-p Ritz vectors, the
    warm start of the next call), Q, H, n_pos = #{theta_i > 0} and the
    rank-deficiency flag.
    """
    Xf = np.asarray(X_filter, dtype=np.float64)
    Xr = np.asarray(X_rr, dtype=np.float64)
    Y = chebyshev_filter(lambda B: Xf @ B, U, d, a, b, q)
    Q, deficient = orthonormalize(Y)
    theta, V, H = rayleigh_ritz(lambda B: Xr @ B, Q)
    return {
        "theta": theta,
        "V": V,
        "Q": Q,
        "H": H,
        "Y": Y,
        "n_pos": int(np.count_nonzero(theta > 0)),
        "rank_deficient": deficient,
    }


def extract_gram(M_filter, M_rr, U, d, a, b, q=1):
    """Subspace extraction for the singular pairs of a rectangular M.

    Section 5.2.1: the SVD of M is obtained from an eigen-subspace of
    A = M^T M.  The filter applies A as M^T (M Y).  Rayleigh-Ritz on
    A = M^T M is done as the SVD of B = M Q, which is the same p-by-p
    problem (B^T B = Q^T A Q) without squaring its condition.  Returns
    sigma (descending singular values), theta = sigma^2, V = Q Z (right
    Ritz vectors, n-by-p) and the left Ritz vectors B Z / sigma.
    """
    Mf = np.asarray(M_filter, dtype=np.float64)
    Mr = np.asarray(M_rr, dtype=np.float64)
    Y = chebyshev_filter(lambda B: Mf.T @ (Mf @ B), U, d, a, b, q)
    Q, deficient = orthonormalize(Y)
    B = Mr @ Q
    P, s, Zt = np.linalg.svd(B, full_matrices=False)
    Z = Zt.T
    return {
        "sigma": s,
        "theta": s * s,
        "V": Q @ Z,
        "U_left": P,
        "Q": Q,
        "Y": Y,
        "rank_deficient": deficient,
    }


def svd_shrink(M, tau):
    """Singular-value shrinkage shrink_tau(M) = U diag(max(s_i - tau, 0)) V^T
    (section 5.2.1: the proximal map of tau times the nuclear norm), from
    the full SVD of M."""
    M = np.asarray(M, dtype=np.float64)
    Uf, s, Vt = np.linalg.svd(M, full_matrices=False)
    return (Uf * np.maximum(s - tau, 0.0)) @ Vt


def svd_shrink_factor(M, V, theta, tau):
    """Left factor L of the shrinkage of M restricted to the Ritz subspace.

    With V the right Ritz vectors of Rayleigh-Ritz on M^T M (section 5.2.1)
    and theta their Ritz values, B = M V has orthogonal columns of norms
    sigma_i = sqrt(theta_i), so M P_V = B V^T is an SVD up to normalising
    the columns of B, and shrink_tau(M P_V) = L V^T with
    L = B diag(max(sigma_i - tau, 0) / sigma_i) (zero where sigma_i = 0).
    """
    M = np.asarray(M, dtype=np.float64)
    B = M @ np.asarray(V, dtype=np.float64)
    sigma = np.sqrt(np.maximum(np.asarray(theta, dtype=np.float64), 0.0))
    f = np.zeros_like(sigma)
    keep = sigma > tau
    f[keep] = (sigma[keep] - tau) / sigma[keep]
    return B * f


def lowrank_projection(V, theta):
    """P_V(X) = V diag(theta) V^T for Ritz pairs (section 2.2, eq. RR)."""
    return (V * theta) @ V.T


def psd_projection(V, theta):
    """P_+(P_V(X)): keep only the Ritz pairs with theta > 0 (eq. PFAM1).

    By eq. RR, P_V(X) = V diag(theta) V^T with V orthonormal, so its
    projection onto the PSD cone zeroes the negative theta.
    """
    keep = theta > 0
    Vp = V[:, keep]
    return (Vp * theta[keep]) @ Vp.T
