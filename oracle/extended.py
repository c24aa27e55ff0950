"""One extraction in 80-bit extended precision (numpy.longdouble).

Test infrastructure (see ``oracle/__init__``).  The same steps as
``extract.extract`` (section 2.1: the Chebyshev recurrence, then one
orthonormalisation; section 2.2, eq. RR: H = Q^T X Q, H = Z Theta Z^T,
V = Q Z), carried out with a 64-bit significand.  It bounds the FP64
oracle's own rounding where an input makes the FP64 result sensitive (a
cold random start, whose filtered block is ill-conditioned): there the
FP64 oracle is not accurate to the FP64 parity tolerance, and this is the
reference the tolerance is checked against.

numpy.linalg has no extended-precision factorisations, so the
orthonormalisation is modified Gram-Schmidt applied twice and the p-by-p
eigenproblem is cyclic Jacobi, both written out here.  Plain loops over
columns and rotation planes: meant for p <= ~64.

Pins (tests/test_oracle_extended.py): the filter against exact rational
Chebyshev values on a diagonal matrix; an exactly invariant start block
gives the diagonal's eigenvalues to extended precision; the Jacobi solver's
residual and orthogonality measured in extended precision, and its
eigenvalues against LAPACK; agreement with the FP64 oracle on
well-conditioned warm steps.
"""
import numpy as np

LD = np.longdouble


def chebyshev_filter_ld(X, U, d, a, b, q=1):
    """T_d(L(X))^q U by the three-term recurrence of section 2.1 in extended
    precision, L(X) = (X - cI)/e with c = (a+b)/2, e = (b-a)/2; the power q
    (eq. pfpg2) applies the whole polynomial q times."""
    XL = np.asarray(X).astype(LD)
    c = (LD(a) + LD(b)) / 2
    e = (LD(b) - LD(a)) / 2
    Y = np.asarray(U).astype(LD)
    for _ in range(q):
        if d == 0:
            continue
        Y_prev = Y
        Y_cur = (XL @ Y_prev - c * Y_prev) / e
        for _k in range(1, d):
            Y_next = 2 * (XL @ Y_cur - c * Y_cur) / e - Y_prev
            Y_prev, Y_cur = Y_cur, Y_next
        Y = Y_cur
    return Y


def mgs2(Y):
    """Orthonormal basis of range(Y): modified Gram-Schmidt, twice."""
    Q = np.array(Y, dtype=LD)
    Q /= np.sqrt(np.sum(Q * Q, axis=0))
    for _pass in range(2):
        for j in range(Q.shape[1]):
            v = Q[:, j].copy()
            for i in range(j):
                v -= (Q[:, i] @ v) * Q[:, i]
            Q[:, j] = v / np.sqrt(v @ v)
    return Q


def jacobi_eigh_ld(H, max_sweeps=40):
    """Cyclic Jacobi on a symmetric H in extended precision.

    Each rotation in plane (i, j) zeroes the (i, j) entry of the current
    matrix; sweeps stop once the off-diagonal norm is below 1e-19 ||H||_F.
    Returns (theta descending, Z) with H = Z diag(theta) Z^T.
    """
    A = np.array(H, dtype=LD)
    p = A.shape[0]
    Z = np.eye(p, dtype=LD)
    fro = np.sqrt(np.sum(A * A))
    offdiag = ~np.eye(p, dtype=bool)
    for _sweep in range(max_sweeps):
        off = np.sqrt(np.sum(A[offdiag] ** 2))
        if off <= LD(1e-19) * fro:
            break
        for i in range(p - 1):
            for j in range(i + 1, p):
                aij = A[i, j]
                if aij == 0:
                    continue
                tau = (A[j, j] - A[i, i]) / (2 * aij)
                t = (LD(1) if tau >= 0 else LD(-1)) / (abs(tau) + np.sqrt(1 + tau * tau))
                c = 1 / np.sqrt(1 + t * t)
                s = t * c
                ci, cj = A[:, i].copy(), A[:, j].copy()
                A[:, i], A[:, j] = c * ci - s * cj, s * ci + c * cj
                ri, rj = A[i, :].copy(), A[j, :].copy()
                A[i, :], A[j, :] = c * ri - s * rj, s * ri + c * rj
                zi, zj = Z[:, i].copy(), Z[:, j].copy()
                Z[:, i], Z[:, j] = c * zi - s * zj, s * zi + c * zj
    theta = np.diag(A).copy()
    order = np.argsort(-theta.astype(np.float64), kind="stable")
    return theta[order], Z[:, order]


def extract_longdouble(X, U, d, a, b, q=1):
    """Filter, orthonormalise and Rayleigh-Ritz in extended precision.

    Returns a dict of numpy.longdouble arrays: theta (descending), the Ritz
    vectors V = Q Z and the filtered block Y; the caller rounds them to FP64
    for comparisons.
    """
    Y = chebyshev_filter_ld(X, U, d, a, b, q)
    Q = mgs2(Y)
    H = Q.T @ (np.asarray(X).astype(LD) @ Q)
    H = (H + H.T) / 2
    theta, Z = jacobi_eigh_ld(H)
    return {"theta": theta, "V": Q @ Z, "Y": Y}
