"""FP64 CPU oracle for polynomial-filtered subspace extraction.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, deliberately
unoptimised reference of what one extraction computes (Li, Liu, Wen, Yuan,
"Polynomial-filtered methods for matrix optimization", arXiv 1904.10585):

  * the Chebyshev filter rho(A) U evaluated by its three-term recurrence
    (section 2.1, eq. cheb, eq. cheb-linear-map, eq. subspace-update),
  * orthonormalisation of the filtered block by one QR (section 2.1),
  * the Rayleigh-Ritz step H = Q^T X Q, H = Z Theta Z^T, V = Q Z
    (section 2.2, eq. RR), with the low-rank projection P_V(X) and the PSD
    projection P_+(P_V(X)) used by PFPG/PFAM (section 2.2-2.3),
  * the SVD route through A^T A (section 5.2.1) and its singular-value
    shrinkage, the residual norms of the Ritz pairs,
  * the same extraction in 80-bit extended precision, which bounds the
    FP64 oracle's own rounding on ill-conditioned (cold-start) inputs,
  * the BF16 / FP8-E4M3 quantisers that define the low-precision copies
    of X the GPU filter reads.
  * the Lanczos estimate of the smallest eigenvalue and the damping
    interval / block size rules of sections 4.1-4.2.
  * the nearest correlation dual of section 5.1 by the exact gradient
    method and by PFPG, with the extrapolation of section 4.3, and its
    primal by DRS with the exact PSD projection and by PFAM.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it.  It shares no code with the HIP path (no common
kernels, headers, helpers or constants) and never imports it; the product
path fails loudly when its HIP library is missing instead of falling back
here.

Parity status of each function is stated in its docstring; every function
here is pinned by ``tests/test_oracle_*.py`` against closed forms,
invariants, brute force or an independent algorithm.
"""

from .chebyshev import cheb_T, interval_map, rho, chebyshev_filter
from .extract import (orthonormalize, rayleigh_ritz, extract, extract_gram,
                      psd_projection, lowrank_projection, ritz_residuals, svd_shrink, svd_shrink_factor)
from .metrics import sin_theta, projector_distance, ritz_rel_err, orth_error
from .jacobi import jacobi_eigh
from .extended import extract_longdouble, jacobi_eigh_ld
from .lanczos import block_krylov_ritz, lanczos_bounds, interval_policy, block_size_policy, degree_policy
from .nce import nce_dual, nce_primal, rna_extrapolate, nce_grad, nce_pfpg, nce_drs, nce_pfam
from .quantize import (bf16_round, fp8_e4m3_round, fp8_tile_quantize,
                       fp8_tile_dequantize)

__all__ = [
    "cheb_T", "interval_map", "rho", "chebyshev_filter",
    "orthonormalize", "rayleigh_ritz", "extract", "extract_gram",
    "psd_projection", "lowrank_projection", "ritz_residuals", "svd_shrink", "svd_shrink_factor",
    "sin_theta", "projector_distance", "ritz_rel_err", "orth_error",
    "block_krylov_ritz", "lanczos_bounds", "interval_policy", "block_size_policy", "degree_policy",
    "jacobi_eigh", "extract_longdouble", "jacobi_eigh_ld",
    "nce_dual", "nce_primal", "rna_extrapolate", "nce_grad", "nce_pfpg", "nce_drs", "nce_pfam",
    "bf16_round", "fp8_e4m3_round", "fp8_tile_quantize", "fp8_tile_dequantize",
]
