"""Nearest correlation estimation by the dual gradient method, exact and
polynomial-filtered (section 5.1 with section 2.2 and section 4), and by
DRS on the primal, exact and polynomial-filtered (PFAM, eq. PFAM1-PFAM2).

Test infrastructure (see ``oracle/__init__``).

Section 5.1 solves min 1/2 ||G - X||_F^2 subject to diag(X) = 1 and X PSD
through its dual (eq. NCE-dual):
    F(x) = 1/2 sum_i max(lambda_i(G + Diag(x)), 0)^2 - 1^T x,
    grad F(x) = diag(P_+(G + Diag(x))) - 1            (eq. NCE-gradient),
the spectral function of eq. mat-opt with B(x) = G + Diag(x).  The paper
compares a gradient method on F with a fixed step (every iteration a full
eigendecomposition) against PFPG (eq. pfpg1-pfpg2 with R = 0), whose
gradient takes P_+ in the subspace extracted by the polynomial filter:
    x^{k+1} = x^k - tau (diag(P_+(P_{U^k}(B(x^k)))) - 1),
    U^{k+1} = orth(rho(B(x^{k+1})) U^k).
Both are accelerated by the regularised extrapolation of section 4.3.

``nce_dual`` is the definition (numpy's full ``eigh``), ``nce_grad`` the
exact gradient method, ``nce_pfpg`` the filtered one built on
``oracle.extract`` (the FP64 extraction) and ``oracle.lanczos_bounds`` (the
interval rule of section 4.1).  Readings where the paper leaves a choice:
  * the extrapolation combines the l + 1 points x^{k-l}..x^k with the
    coefficients of section 4.3 over their l + 1 successive differences, its
    regularisation lambda taken relative to ||U^T U||_F; it runs after every
    l + 1 gradient steps and restarts the history from its result;
  * the block size is the previous step's positive count plus the guard
    columns (section 4.2), rounded up to a multiple of 16 and clamped to
    [16, p_max]; while more than p_max eigenvalues are positive the
    gradient uses the p_max largest Ritz pairs (the count falls below the
    limit as the dual iterate moves down); columns added when the block
    grows are the next columns of the caller's start block U0;
  * the damping interval is a = theta_min - res_min of the block Lanczos
    bound, b = eta a (all positive eigenvalues wanted), refreshed every
    ``lanczos_every`` iterations from the same Lanczos start block.
Pinned by tests/test_oracle_nce.py: the gradient against finite differences
of F, the fixed point of a correlation matrix, the KKT conditions and
strong duality at the solution, agreement with an independent solver
(alternating projections with Dykstra's correction), the objective values
printed in the paper's NCE table, the extrapolation's exactness on a linear
iteration, PFPG reaching the exact method's solution, and the primal DRS
and PFAM reaching the dual method's nearest correlation matrix.
"""
import numpy as np

from .extract import extract
from .lanczos import lanczos_bounds


def nce_dual(G, x):
    """(F(x), grad F(x), #positive eigenvalues) of eq. NCE-dual-equiv /
    eq. NCE-gradient by the full eigendecomposition of G + Diag(x)."""
    w, Q = np.linalg.eigh(np.asarray(G, dtype=np.float64) + np.diag(x))
    wp = np.maximum(w, 0.0)
    F = 0.5 * float(np.sum(wp * wp)) - float(np.sum(x))
    g = (Q * Q) @ wp - 1.0
    return F, g, int(np.count_nonzero(w > 0))


def nce_primal(G, x):
    """X = P_+(G + Diag(x)), the primal point of a dual x."""
    w, Q = np.linalg.eigh(np.asarray(G, dtype=np.float64) + np.diag(x))
    return (Q * np.maximum(w, 0.0)) @ Q.T


def rna_extrapolate(points, lam):
    """Section 4.3: points x^{k-l}..x^{k+1} (l + 2 of them); U holds their
    l + 1 successive differences; c = argmin_{1^T c = 1} c^T (U^T U +
    lambda I) c, i.e. c proportional to (U^T U + lambda I)^{-1} 1 (lambda
    relative to ||U^T U||_F); returns sum_i c_i x^{k-l+i}."""
    P = np.column_stack([np.asarray(v, dtype=np.float64) for v in points])
    U = P[:, 1:] - P[:, :-1]
    M = U.T @ U
    scale = np.linalg.norm(M)
    if scale == 0.0:
        return P[:, -1].copy()
    z = np.linalg.solve(M / scale + lam * np.eye(M.shape[0]), np.ones(M.shape[0]))
    c = z / np.sum(z)
    return P[:, :-1] @ c


def _history_step(hist, x, l, lam):
    """Append x to the extrapolation history; extrapolate when it holds l + 2
    points.  Returns the next iterate."""
    if l <= 0:
        return x
    hist.append(x.copy())
    if len(hist) == l + 2:
        x = rna_extrapolate(hist, lam)
        hist[:] = [x.copy()]
    return x


def nce_grad(G, x0=None, tau=1.6, tol=1e-7, max_iter=500, rna_l=3, rna_lam=1e-8):
    """The gradient method on F with a fixed step (the paper's Grad): every
    iteration a full eigendecomposition.  Stops when ||grad F(x)|| <=
    tol ||grad F(x0)||.  Returns dict(x, F, gnorm, iters, n_pos, history)
    with history rows (F, ||g||, n_pos) per evaluated iterate."""
    G = np.asarray(G, dtype=np.float64)
    x = (1.0 - np.diag(G)) if x0 is None else np.array(x0, dtype=np.float64)
    hist, rows, g0 = [x.copy()], [], None
    for k in range(max_iter):
        F, g, npos = nce_dual(G, x)
        gn = float(np.linalg.norm(g))
        g0 = gn if g0 is None else g0
        rows.append((F, gn, npos))
        if gn <= tol * g0:
            return {"x": x, "F": F, "gnorm": gn, "g0": g0, "iters": k, "n_pos": npos, "history": rows}
        x = _history_step(hist, x - tau * g, rna_l, rna_lam)
    return {"x": x, "F": F, "gnorm": gn, "g0": g0, "iters": max_iter, "n_pos": npos, "history": rows}


def nce_pfpg(G, U0, V0, x0=None, tau=1.6, degree=10, guards=8, p_max=128, eta=0.1, tol=1e-7,
             max_iter=500, rna_l=3, rna_lam=1e-8, lanczos_steps=4, lanczos_every=10):
    """PFPG on the NCE dual (eq. pfpg1-pfpg2, R = 0) with the readings of
    the module docstring.  U0: n x p_max start block; V0: n x 16 Lanczos
    start block.  Returns dict(x, F, gnorm, iters, n_pos, p, history) with
    history rows (F, ||g||, n_pos, p, a, b) per evaluated iterate, F and g
    from the Ritz pairs (the values the method itself sees).  x is the last
    evaluated iterate (no step after the last evaluation)."""
    G = np.asarray(G, dtype=np.float64)
    n = G.shape[0]
    U0 = np.asarray(U0, dtype=np.float64)
    p_max = min(p_max, n, U0.shape[1])
    x = (1.0 - np.diag(G)) if x0 is None else np.array(x0, dtype=np.float64)

    def interval(B):
        lo, _, res, _ = lanczos_bounds(B, V0, lanczos_steps)
        a = lo - res
        if not a < 0.0:
            raise ValueError("the all-positive interval rule needs a negative smallest eigenvalue")
        return a, eta * a

    B = G + np.diag(x)
    a, b = interval(B)
    p = p_max
    U = U0[:, :p]
    hist, rows, g0 = [x.copy()], [], None
    for k in range(max_iter):
        r = extract(B, B, U, degree, a, b)
        theta, V = r["theta"], r["V"]
        tp = np.maximum(theta, 0.0)
        g = (V * V) @ tp - 1.0                     # diag(P_+(P_U(B)))- 1
        F = 0.5 * float(np.sum(tp * tp)) - float(np.sum(x))
        gn = float(np.linalg.norm(g))
        g0 = gn if g0 is None else g0
        npos = r["n_pos"]
        rows.append((F, gn, npos, p, a, b))
        if gn <= tol * g0 or k + 1 == max_iter:
            return {"x": x, "F": F, "gnorm": gn, "g0": g0, "iters": k, "n_pos": npos, "p": p, "history": rows,
                    "converged": gn <= tol * g0}
        x = _history_step(hist, x - tau * g, rna_l, rna_lam)
        B = G + np.diag(x)
        p_new = int(min(p_max, max(16, -(-(npos + guards) // 16) * 16)))
        U = V[:, :p_new] if p_new <= p else np.hstack([V, U0[:, p:p_new]])
        p = p_new
        if lanczos_every > 0 and (k + 1) % lanczos_every == 0:
            a, b = interval(B)


def _drs_update(Z, P, G, t):
    """One step of the DRS map of the PFAM section on the NCE primal with
    F the indicator of the PSD cone (prox_tF = P_+) and G(X) = 1/2 ||X -
    G||_F^2 plus the indicator of diag(X) = 1, whose prox is entrywise:
    (t G_ij + Y_ij) / (1 + t) off the diagonal, 1 on it.  Returns dZ with
    Z^{k+1} = prox_tG(2 P - Z) - P + Z = Z + dZ (eq. PFAM1, P the PSD
    projection of Z or of its projection onto the subspace)."""
    prox = (t * G + (2.0 * P - Z)) / (1.0 + t)
    np.fill_diagonal(prox, 1.0)
    return prox - P


def nce_drs(G, Z0=None, t=0.5, tol=1e-7, max_iter=5000):
    """The DRS iteration with the exact P_+ (full eigendecomposition of Z
    each step).  Stops when ||dZ||_F <= tol ||dZ_0||_F.  Returns dict(Z, X,
    iters, residual, residual0) with X = P_+(Z) of the last evaluated
    iterate."""
    G = np.asarray(G, dtype=np.float64)
    Z = G.copy() if Z0 is None else np.array(Z0, dtype=np.float64)
    r0 = None
    for k in range(max_iter):
        w, Q = np.linalg.eigh(Z)
        P = (Q * np.maximum(w, 0.0)) @ Q.T
        dZ = _drs_update(Z, P, G, t)
        r = float(np.linalg.norm(dZ))
        r0 = r if r0 is None else r0
        Z = Z + dZ
        if r <= tol * r0:
            break
    return {"Z": Z, "X": P, "iters": k, "residual": r, "residual0": r0}


def nce_pfam(G, U0, V0, Z0=None, t=0.5, degree=10, guards=8, p_max=128, eta=0.1, tol=1e-7, max_iter=500,
             lanczos_steps=4, lanczos_every=10):
    """PFAM (eq. PFAM1-PFAM2) on the NCE primal: the DRS step above with
    P = P_+(P_U(Z)) = V_+ Theta_+ V_+^T from one extraction on Z per step,
    warm-started; interval, block size and U0 columns as in ``nce_pfpg``.
    Every step: P from the extraction on Z, dZ, then Z += dZ; stops when
    ||dZ|| <= tol ||dZ_0|| or at max_iter (Z then holds the step taken, X =
    P the projection it was taken from).  History rows: (||dZ||,
    1/2 ||G - P||_F^2, n_pos, p, a, b, max |diag(P) - 1|)."""
    G = np.asarray(G, dtype=np.float64)
    n = G.shape[0]
    U0 = np.asarray(U0, dtype=np.float64)
    p_max = min(p_max, n, U0.shape[1])
    Z = G.copy() if Z0 is None else np.array(Z0, dtype=np.float64)

    def interval(M):
        lo, _, res, _ = lanczos_bounds(M, V0, lanczos_steps)
        a = lo - res
        if not a < 0.0:
            raise ValueError("the all-positive interval rule needs a negative smallest eigenvalue")
        return a, eta * a

    a, b = interval(Z)
    p = p_max
    U = U0[:, :p]
    rows, r0 = [], None
    for k in range(max_iter):
        r = extract(Z, Z, U, degree, a, b)
        theta, V = r["theta"], r["V"]
        P = (V * np.maximum(theta, 0.0)) @ V.T
        dZ = _drs_update(Z, P, G, t)
        res = float(np.linalg.norm(dZ))
        r0 = res if r0 is None else r0
        npos = r["n_pos"]
        rows.append((res, 0.5 * float(np.linalg.norm(G - P) ** 2), npos, p, a, b,
                     float(np.abs(np.diag(P) - 1.0).max())))
        Z = Z + dZ
        if res <= tol * r0 or k + 1 == max_iter:
            return {"Z": Z, "X": P, "iters": k, "residual": res, "residual0": r0, "n_pos": npos, "p": p,
                    "history": rows, "converged": res <= tol * r0}
        p_new = int(min(p_max, max(16, -(-(npos + guards) // 16) * 16)))
        U = V[:, :p_new] if p_new <= p else np.hstack([V, U0[:, p:p_new]])
        p = p_new
        if lanczos_every > 0 and (k + 1) % lanczos_every == 0:
            a, b = interval(Z)
