"""Chebyshev polynomials and the filter rho(A) U (paper section 2.1).

Test infrastructure (see ``oracle/__init__``).  FP64 throughout.
"""
import numpy as np


def cheb_T(d, t):
    """T_d(t), Chebyshev polynomial of the first kind of degree d.

    Section 2.1, eq. cheb: cos(d arccos t) on [-1, 1]; outside it, half the
    sum of the d-th powers of t - sqrt(t^2 - 1) and t + sqrt(t^2 - 1).
    Pinned by cos(k theta), cosh(k x), parity and the explicit power-sum
    coefficients in tests/test_oracle_chebyshev.py.
    """
    t = np.asarray(t, dtype=np.float64)
    out = np.empty_like(t)
    inside = np.abs(t) <= 1.0
    out[inside] = np.cos(d * np.arccos(t[inside]))
    to = t[~inside]
    r = np.sqrt(to * to - 1.0)
    out[~inside] = 0.5 * ((to - r) ** d + (to + r) ** d)
    return out


def interval_map(t, a, b):
    """Affine map sending the damping interval [a, b] onto [-1, 1].

    Section 2.1, eq. cheb-linear-map: (t - (b + a)/2) / ((b - a)/2).
    """
    return (np.asarray(t, dtype=np.float64) - (b + a) / 2.0) / ((b - a) / 2.0)


def rho(t, d, a, b):
    """The filter polynomial rho(t) = T_d(interval_map(t)) (eq. cheb-linear-map)."""
    return cheb_T(d, interval_map(t, a, b))


def chebyshev_filter(apply_A, U, d, a, b, q=1):
    """rho(A)^q U through the three-term Chebyshev recurrence.

    Section 2.1 (eq. cheb-linear-map, eq. subspace-update) and the recurrence
    noted in section 4 (eq. cheby-recursion-map, whose coefficient names are
    swapped in the text).  With c = (a+b)/2, e = (b-a)/2 and
    L(A) = (A - cI)/e:

        Y_0 = U,  Y_1 = L(A) Y_0,  Y_{k+1} = 2 L(A) Y_k - Y_{k-1},

    so that Y_d = T_d(L(A)) U.  ``apply_A`` maps an n-by-p block to A times
    it (A = X for a symmetric X, A = M^T M for the SVD route).  The power q
    (eq. pfpg2) applies the whole polynomial q times.  No scaling: FP64 holds
    every magnitude the tested workloads reach.
    """
    if d < 0 or q < 0:
        raise ValueError("degree and power must be non-negative")
    c = (a + b) / 2.0
    e = (b - a) / 2.0
    Y = np.asarray(U, dtype=np.float64)
    for _ in range(q):
        if d == 0:
            continue
        Y_prev = Y
        Y_cur = (apply_A(Y) - c * Y) / e
        for _k in range(1, d):
            Y_next = 2.0 * (apply_A(Y_cur) - c * Y_cur) / e - Y_prev
            Y_prev, Y_cur = Y_cur, Y_next
        Y = Y_cur
    return Y
