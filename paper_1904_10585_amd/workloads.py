"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

Holds none of the extraction's arithmetic: only random draws and the
workload table.  The paper measures on datasets that are not available here
(NCE matrices, completion data, images, SDP instances); planted-spectrum
symmetric matrices X = Q diag(lambda) Q^T with a few large eigenvalues on
top of a bulk stand in for its low-rank iterates, and a rank-r-plus-noise M
stands in for the SVD route.

Seeds: numpy PCG64 keyed by SeedSequence([10585, config, stream, index]);
streams 0 = Q, 1 = lambda, 2 = U0, 3 = perturbation E_k (index k),
4 = session parameters, 5 = arrivals, 6 = factors of M, 7 = noise of M,
8 = off-diagonal entries of an NCE matrix G.
"""
from dataclasses import dataclass, field

import numpy as np

SEED_ROOT = 10585
S_Q, S_LAMBDA, S_U0, S_PERTURB, S_SESSION, S_ARRIVAL, S_MFACT, S_MNOISE, S_NCE = range(9)


def rng(config, stream, index=0):
    return np.random.Generator(np.random.PCG64(
        np.random.SeedSequence([SEED_ROOT, int(config), int(stream), int(index)])))


@dataclass(frozen=True)
class Workload:
    """One synthetic workload: planted spectrum + filter settings."""
    name: str
    config: int
    n: int
    p: int
    degree: int
    a: float
    b: float
    n_top: int
    top: tuple
    rest: tuple
    steps: int
    perturb: float = 1e-3
    extra: dict = field(default_factory=dict)


# Damping intervals: the paper's rule puts a at the smallest eigenvalue and b
# at the top of the unwanted part (section 4.1).  For single-precision
# filters a is pushed below the spectrum until the growth ratio between the
# largest and the smallest wanted eigenvalue stays below ~2e10.
WORKLOADS = {
    "tiny_fp64": Workload("tiny_fp64", 1, 512, 16, 8, -1.0, 0.5, 12, (2.0, 10.0), (-1.0, 0.5), 11),
    "planted_8192": Workload("planted_8192", 2, 8192, 64, 10, -5.0, 0.8, 64, (1.0, 20.0), (-2.0, 0.8), 50),
    "planted_8192_tight": Workload("planted_8192_tight", 2, 8192, 64, 10, -2.0, 0.8, 64, (1.0, 20.0), (-2.0, 0.8), 50),
    "planted_16384_bf16": Workload("planted_16384_bf16", 3, 16384, 128, 12, -10.0, 0.8, 64, (1.0, 20.0), (-2.0, 0.8), 50),
    "gram_12000x6000_fp8": Workload("gram_12000x6000_fp8", 5, 6000, 48, 8, 0.0, 4.0, 40, (), (), 30,
                                    extra={"m": 12000, "rank": 40, "noise": 0.01}),
}

SERVING = {
    "n_choices": (1024, 2048, 4096, 8192, 12288),
    "p_choices": (8, 16, 32, 64, 96),
    "degree_choices": (6, 8, 10),
    "sessions": 2000,
    "steps": 30,
    "top": (1.0, 20.0),
    "rest": (-2.0, 0.8),
}


def serving_interval(degree):
    """Damping interval of a serving session (same widening rule)."""
    return (-5.0, 0.8) if degree >= 10 else (-2.1, 0.8)


def haar_orthogonal(n, g):
    """Haar-distributed orthogonal matrix: QR of an N(0,1) matrix with the
    signs of diag(R) moved into Q."""
    G = g.standard_normal((n, n))
    Q, R = np.linalg.qr(G)
    return Q * np.sign(np.diag(R))


def planted_eigenvalues(n, n_top, top, rest, g):
    """n_top draws uniform in ``top`` followed by n - n_top uniform in ``rest``."""
    lam = np.empty(n)
    lam[:n_top] = g.uniform(top[0], top[1], n_top)
    lam[n_top:] = g.uniform(rest[0], rest[1], n - n_top)
    return lam


def planted_matrix(Q, lam):
    """X = Q diag(lam) Q^T, symmetrised to the last bit."""
    X = (Q * lam) @ Q.T
    return 0.5 * (X + X.T)


def planted(n, n_top, top, rest, config, index=0):
    """(X, lam, Q) for a planted-spectrum symmetric matrix in FP64."""
    Q = haar_orthogonal(n, rng(config, S_Q, index))
    lam = planted_eigenvalues(n, n_top, top, rest, rng(config, S_LAMBDA, index))
    return planted_matrix(Q, lam), lam, Q


def perturbation(n, config, k, scale=1e-3, index=0):
    """E_k = scale * (G + G^T)/2 / sqrt(n), G i.i.d. N(0,1) (||E||_2 ~ 1.4 scale)."""
    g = rng(config, S_PERTURB, (index << 20) + k)
    G = g.standard_normal((n, n))
    return scale * 0.5 * (G + G.T) / np.sqrt(n)


def start_block(n, p, config, index=0):
    """Cold-start block U0 with i.i.d. N(0,1) entries."""
    return rng(config, S_U0, index).standard_normal((n, p))


def lowrank_plus_noise(m, n, r, noise, config, index=0):
    """M = A B^T + noise * N(0,1), A m-by-r and B n-by-r with N(0,1) entries."""
    gf = rng(config, S_MFACT, index)
    A = gf.standard_normal((m, r))
    B = gf.standard_normal((n, r))
    N = rng(config, S_MNOISE, index).standard_normal((m, n))
    return A @ B.T + noise * N


def nce_matrix(n, example, config, index=0):
    """Symmetric G of the nearest correlation examples of section 5.1: unit
    diagonal, off-diagonal entries i.i.d. uniform in [-1, 1] (example 6) or
    [0, 2] (example 7); the upper triangle is drawn and mirrored."""
    lo, hi = {6: (-1.0, 1.0), 7: (0.0, 2.0)}[int(example)]
    T = rng(config, S_NCE, index).uniform(lo, hi, (n, n))
    G = np.triu(T, 1)
    G = G + G.T
    np.fill_diagonal(G, 1.0)
    return G


def workload_matrices(w, index=0):
    """Base matrix of a symmetric workload (FP64) with its spectrum."""
    return planted(w.n, w.n_top, w.top, w.rest, w.config, index)
