"""Distances between subspaces and Ritz values (paper section 3.1).

Test infrastructure (see ``oracle/__init__``).
"""
import numpy as np


def sin_theta(Vg, Vr):
    """Largest principal-angle sine between range(Vg) and range(Vr).

    Definition in section 3.1 (principal angles from the singular values of
    Vg^T Vr).  Computed as ||Vg - Vr (Vr^T Vg)||_2 for orthonormal inputs,
    which keeps full FP64 resolution for tiny angles (the
    sqrt(1 - sigma_min^2) form cannot resolve angles below ~1e-8).
    """
    Vg = np.asarray(Vg, dtype=np.float64)
    Vr = np.asarray(Vr, dtype=np.float64)
    R = Vg - Vr @ (Vr.T @ Vg)
    return float(np.linalg.norm(R, 2))


def projector_distance(Vg, Vr):
    """||Vg Vg^T - Vr Vr^T||_2, equal to the largest principal-angle sine
    for equal dimensions (the identity quoted in the proof of Lemma ctr1)."""
    Pg = Vg @ Vg.T
    Pr = Vr @ Vr.T
    return float(np.linalg.norm(Pg - Pr, 2))


def ritz_rel_err(theta_g, theta_r, r=None):
    """max_i |theta_g[i] - theta_r[i]| / |theta_r[i]| over the first r,
    both sorted in descending order."""
    tg = np.asarray(theta_g, dtype=np.float64)
    tr = np.asarray(theta_r, dtype=np.float64)
    if r is None:
        r = len(tr)
    return float(np.max(np.abs(tg[:r] - tr[:r]) / np.abs(tr[:r])))


def orth_error(Q):
    """||Q^T Q - I||_2."""
    Q = np.asarray(Q, dtype=np.float64)
    return float(np.linalg.norm(Q.T @ Q - np.eye(Q.shape[1]), 2))
