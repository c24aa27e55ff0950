"""Cyclic Jacobi eigensolver for small symmetric matrices (pure Python).

Test infrastructure (see ``oracle/__init__``).  An algorithm independent of
LAPACK's ``eigh`` (which ``rayleigh_ritz`` uses), so that the p-by-p
eigensolve of the Rayleigh-Ritz step (section 2.2, eq. RR: H = Y Lambda Y^T)
is pinned by two unrelated methods.  Pure-Python loops: meant for p <= ~32.
"""
import math

import numpy as np


def _rotation(app, aqq, apq):
    """(c, s) of the plane rotation that zeroes the (p, q) entry."""
    if apq == 0.0:
        return 1.0, 0.0
    tau = (aqq - app) / (2.0 * apq)
    if tau >= 0.0:
        t = 1.0 / (tau + math.sqrt(1.0 + tau * tau))
    else:
        t = -1.0 / (-tau + math.sqrt(1.0 + tau * tau))
    c = 1.0 / math.sqrt(1.0 + t * t)
    return c, t * c


def jacobi_eigh(H, tol=1e-15, max_sweeps=60):
    """Eigen-decomposition of a symmetric H by cyclic-by-row Jacobi sweeps.

    Each rotation J in plane (p, q) is chosen so that (J^T A J)_{pq} = 0;
    sweeps repeat until the off-diagonal Frobenius norm is below
    tol * ||H||_F.  Returns (theta descending, Z) with H = Z diag(theta) Z^T.
    """
    A = [list(map(float, row)) for row in np.asarray(H, dtype=np.float64)]
    n = len(A)
    V = [[1.0 if i == j else 0.0 for j in range(n)] for i in range(n)]
    fro = math.sqrt(sum(A[i][j] ** 2 for i in range(n) for j in range(n)))
    for _sweep in range(max_sweeps):
        off = math.sqrt(sum(A[i][j] ** 2 for i in range(n) for j in range(n) if i != j))
        if off <= tol * fro:
            break
        for p in range(n - 1):
            for q in range(p + 1, n):
                c, s = _rotation(A[p][p], A[q][q], A[p][q])
                if s == 0.0:
                    continue
                # A <- A J (columns p, q)
                for k in range(n):
                    akp, akq = A[k][p], A[k][q]
                    A[k][p] = c * akp - s * akq
                    A[k][q] = s * akp + c * akq
                # A <- J^T A (rows p, q)
                for k in range(n):
                    apk, aqk = A[p][k], A[q][k]
                    A[p][k] = c * apk - s * aqk
                    A[q][k] = s * apk + c * aqk
                # V <- V J
                for k in range(n):
                    vkp, vkq = V[k][p], V[k][q]
                    V[k][p] = c * vkp - s * vkq
                    V[k][q] = s * vkp + c * vkq
    theta = np.array([A[i][i] for i in range(n)])
    Z = np.array(V)
    order = np.argsort(-theta, kind="stable")
    return theta[order], Z[:, order]
