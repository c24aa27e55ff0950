"""The p x p eigensolve of Rayleigh-Ritz (section 2.2, eq. RR) on its own,
through pf_eigh: the direct dense solver that extractions fall back to.

Each matrix is checked against the oracle's Rayleigh-Ritz step with Q = I
(LAPACK eigh in FP64) on the eigenvalues, and against the definition on the vectors:
orthonormal columns and small residuals ||H z_i - theta_i z_i||, which pin
the eigenvectors wherever they are unique and accept any orthonormal basis
of an eigenspace with repeated eigenvalues.  Bounds: eigenvalues within
1e-13 ||H||_2, residuals 1e-12 ||H||_2, orthogonality 1e-12."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import pf_module

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pf_module()


def with_spectrum(lam, seed):
    p = len(lam)
    Q, R = np.linalg.qr(np.random.default_rng(seed).standard_normal((p, p)))
    Q = Q * np.sign(np.diag(R))
    return (Q * lam) @ Q.T


def gpu_eigh(H, ld_pad=0):
    pf = pf_module()
    p = H.shape[0]
    ld = p + ld_pad
    Hd = torch.zeros((p, ld), dtype=torch.float64, device="cuda").t()[:p]
    Hd.copy_(torch.from_numpy(H))
    Zd = torch.full((p, ld), 7.0, dtype=torch.float64, device="cuda").t()[:p]
    th = torch.zeros(p, dtype=torch.float64, device="cuda")
    pf.pf_eigh(Hd, th, Zd)
    torch.cuda.synchronize()
    return th.cpu().numpy(), Zd.cpu().numpy()


def check(H, name, ld_pad=0):
    th, Z = gpu_eigh(H, ld_pad)
    Hs = 0.5 * (H + H.T)
    ref, _, _ = oracle.rayleigh_ritz(lambda B: Hs @ B, np.eye(len(th)))
    nrm = max(np.linalg.norm(Hs, 2), 1e-300)
    ev = np.max(np.abs(th - ref)) / nrm
    orth = np.abs(Z.T @ Z - np.eye(len(th))).max()
    res = np.max(np.linalg.norm(Hs @ Z - Z * th, axis=0)) / nrm
    print(f"{name}: p={len(th)} eig {ev:.1e} orth {orth:.1e} res {res:.1e}")
    assert np.all(np.diff(th) <= 0), "theta not descending"
    assert ev <= 1e-13, ev
    assert orth <= 1e-12, orth
    assert res <= 1e-12, res


@pytest.mark.parametrize("p", [1, 2, 3, 5, 16, 31, 32, 33, 48, 64, 65, 96, 127, 128])
def test_random_symmetric(p):
    G = np.random.default_rng(1000 + p).standard_normal((p, p))
    check(G + G.T, "goe", ld_pad=3 if p % 2 else 0)


def test_unsymmetric_input_uses_symmetric_part():
    G = np.random.default_rng(7).standard_normal((40, 40))
    check(G, "unsymmetric")


SPECTRA = {
    # planted top block over a dense unwanted part (guard columns)
    "top_and_bulk": lambda r: np.concatenate([r.uniform(1, 20, 64), r.uniform(-2, 0.8, 64)]),
    # squared singular values of a rank-40 M over a noise cluster
    "gram_large_range": lambda r: np.concatenate([r.uniform(3e7, 1.5e8, 40), r.uniform(0, 3.5, 8)]),
    "two_values": lambda r: np.repeat([5.0, -1.0], [3, 125]),
    "graded": lambda r: 10.0 ** r.uniform(-12, 3, 96),
    "tight_cluster": lambda r: 1.0 + 1e-9 * r.standard_normal(80),
    "cluster_steps": lambda r: np.concatenate([1.0 + 1e-6 * np.arange(40), r.uniform(-1, 0.5, 88)]),
    "tiny_scale": lambda r: 1e-200 * r.uniform(-1, 1, 64),
    # Rayleigh-Ritz matrix with guard columns: the guard Ritz values crowd
    # within ~0.1 (a loose cluster) or ~1e-5 / 1e-8 (tight) below the top block
    "guard_cluster": lambda r: np.concatenate([r.uniform(1, 20, 64), -0.6 + 0.1 * r.standard_normal(64)]),
    "guard_cluster_1e-5": lambda r: np.concatenate([r.uniform(1, 20, 64), -0.6 + 1e-5 * r.standard_normal(64)]),
    "guard_cluster_1e-8": lambda r: np.concatenate([r.uniform(1, 20, 64), -0.6 + 1e-8 * r.standard_normal(64)]),
    "huge_scale": lambda r: 1e150 * r.uniform(-1, 1, 64),
}


@pytest.mark.parametrize("name", sorted(SPECTRA))
def test_hard_spectra(name):
    r = np.random.default_rng(hash(name) % 1000)
    check(with_spectrum(SPECTRA[name](r), 11), name)


def test_structured_matrices():
    r = np.random.default_rng(3)
    check(np.eye(128), "identity")
    check(np.diag(np.repeat([1.0, 2.0, 3.0, 4.0], 32)), "repeated diagonal")
    v = r.standard_normal(100)
    check(np.outer(v, v), "rank one")
    off = r.uniform(0, 1, 127)
    T = np.diag(r.uniform(-1, 1, 128)) + np.diag(off, 1) + np.diag(off, -1)
    T[64, 63] = T[63, 64] = 0.0
    check(T, "split tridiagonal")
    W = np.diag(np.abs(np.arange(-50, 51)).astype(float)) + np.diag(np.ones(100), 1) + np.diag(np.ones(100), -1)
    check(W, "Wilkinson W101")


@pytest.mark.parametrize("name", ["rank2", "rank5", "rank10_p64", "rank40", "two_degenerate",
                                  "identity_plus_rank3", "zero_block_half"])
def test_rank_deficient(name):
    """Eigenspaces of rank-deficient and low-rank-plus-identity H: clusters
    whose spread is rounding noise (the null space of a low-rank X seen
    through the subspace)."""
    r = np.random.default_rng(500)
    if name.startswith("rank"):
        k = int(name[4:].split("_")[0])
        p = 64 if "p64" in name else 128
        B = r.standard_normal((p, k))
        H = B @ B.T
    elif name == "two_degenerate":
        H = with_spectrum(np.concatenate([np.ones(30), np.zeros(60), r.uniform(-3, 3, 38)]), 12)
    elif name == "identity_plus_rank3":
        B = r.standard_normal((96, 3))
        H = np.eye(96) + B @ B.T
    else:
        G = r.standard_normal((64, 64))
        H = np.zeros((128, 128))
        H[:64, :64] = G + G.T
    check(H, name)


def test_zero_and_nonfinite():
    th, Z = gpu_eigh(np.zeros((24, 24)))
    assert np.all(th == 0) and np.array_equal(Z, np.eye(24))
    H = np.eye(24)
    H[3, 5] = np.nan
    th, Z = gpu_eigh(H)
    assert np.all(np.isnan(th)) and np.array_equal(Z, np.eye(24))
