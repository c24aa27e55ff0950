// Small dense p x p kernels of an extraction, one workgroup per matrix, in LDS.
//
//  * chol_rinv: CholeskyQR factor of a Gram matrix G = Y^T Y (the QR of
//    section 2.1 done as G = R^T R, Q = Y R^{-1}): column equilibration
//    D = diag(G)^{-1/2}, Cholesky D G D = L L^T, and R^{-1} = D L^{-T}.
//    A pivot below tol marks the column rank-deficient: it is left out of
//    the elimination and the caller replaces it (see k_block.hip).
//  * jacobi: symmetric eigendecomposition H = Z diag(theta) Z^T (section
//    2.2, eq. RR) by cyclic Jacobi in parallel (round-robin) order: each
//    round rotates p/2 disjoint planes, p-1 rounds make a sweep, sweeps run
//    until no off-diagonal entry is above the threshold.  Output sorted by
//    descending theta (the paper's eigenvalue order).
#include "pf_internal.h"

#include <cmath>

namespace pfx {
namespace {

__device__ inline void set_status(pf_info* info, int code) {
  if (info) atomicCAS(&info->status, 0, code);
}

// ---------------------------------------------------------------------------
// Cholesky + triangular inverse.  LDS: A (p*p doubles, row-major): lower
// triangle holds the elimination, strict upper triangle later holds the
// strictly lower part of L^{-1} transposed; plus D, pivots, L^{-1} diagonal.
__global__ __launch_bounds__(256) void chol_rinv_kernel(const double* __restrict__ G, int ldg, int p,
                                                        double* __restrict__ Rinv, int ldr,
                                                        int* __restrict__ deficient,
                                                        pf_info* info, int pass, double tol) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* A = reinterpret_cast<double*>(smem_raw);
  double* D = A + p * p;
  double* piv = D + p;
  double* xd = piv + p;
  int* def = reinterpret_cast<int*>(xd + p);
  __shared__ int bad_nonfinite;
  const int t = threadIdx.x, nt = blockDim.x;
  if (t == 0) bad_nonfinite = 0;
  __syncthreads();

  for (int i = t; i < p; i += nt) {
    const double gii = G[i + (int64_t)i * ldg];
    if (!isfinite(gii)) bad_nonfinite = 1;
    D[i] = gii > 0.0 ? 1.0 / sqrt(gii) : 0.0;
    def[i] = 0;
  }
  __syncthreads();
  for (int idx = t; idx < p * p; idx += nt) {
    const int i = idx / p, j = idx % p;
    const double gij = G[i + (int64_t)j * ldg];
    if (!isfinite(gij)) bad_nonfinite = 1;
    A[idx] = (i >= j) ? gij * D[i] * D[j] : 0.0;
  }
  __syncthreads();
  if (bad_nonfinite) {
    if (t == 0) set_status(info, PF_ERR_NONFINITE);
    for (int idx = t; idx < ldr * ldr; idx += nt) Rinv[idx] = 0.0;
    return;
  }

  // Right-looking elimination in the L D L^T form: column k stays
  // unscaled, so each step needs one barrier; scaling happens at the end.
  for (int k = 0; k < p; ++k) {
    const double pk = A[k * p + k];
    const bool ok = pk > tol && D[k] > 0.0;
    if (t == 0) { piv[k] = ok ? pk : 1.0; def[k] = ok ? 0 : 1; }
    if (ok) {
      const double inv = 1.0 / pk;
      const int m = p - k - 1;                 // trailing order
      const int cnt = m * (m + 1) / 2;
      for (int e = t; e < cnt; e += nt) {
        // e -> (i, j) with k < j <= i < p, row-major over the lower triangle
        int i = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
        while ((i + 1) * (i + 2) / 2 <= e) ++i;
        while (i * (i + 1) / 2 > e) --i;
        const int j = e - i * (i + 1) / 2;
        const int ii = k + 1 + i, jj = k + 1 + j;
        A[ii * p + jj] -= A[ii * p + k] * A[jj * p + k] * inv;
      }
    }
    __syncthreads();
  }
  // L[i][k] = A[i][k] / sqrt(piv_k); deficient columns become e_k.
  for (int idx = t; idx < p * p; idx += nt) {
    const int i = idx / p, k = idx % p;
    if (i < k) continue;
    if (def[k]) A[idx] = (i == k) ? 1.0 : 0.0;
    else A[idx] = (i == k) ? sqrt(piv[k]) : A[idx] / sqrt(piv[k]);
  }
  __syncthreads();

  // X = L^{-1} by right-looking substitution on L X = I, rows left unscaled
  // (Xu) until the end: X[i][j] -= L[i][k] * Xu[k][j] / L[k][k].
  // Strictly lower X[i][j] (i > j) lives at A[j*p + i].
  for (int i = t; i < p; i += nt) xd[i] = 1.0;
  for (int idx = t; idx < p * p; idx += nt) {
    const int i = idx / p, j = idx % p;
    if (i < j) A[idx] = 0.0;
  }
  __syncthreads();
  for (int k = 0; k < p - 1; ++k) {
    const double invk = 1.0 / A[k * p + k];
    const int rows = p - k - 1, cols = k + 1;
    for (int e = t; e < rows * cols; e += nt) {
      const int i = k + 1 + e / cols, j = e % cols;
      const double xkj = (j == k) ? xd[k] : A[j * p + k];
      const double lik = A[i * p + k];
      if (lik != 0.0) A[j * p + i] -= lik * xkj * invk;
    }
    __syncthreads();
  }
  // Rinv = D L^{-T}: Rinv[i][j] = D_i X[j][i] (j >= i), X[j][i] = Xu[j][i] / L[j][j]
  for (int idx = t; idx < ldr * ldr; idx += nt) {
    const int i = idx % ldr, j = idx / ldr;   // column-major output
    double v = 0.0;
    if (i < p && j < p && j >= i) {
      const double ljj = A[j * p + j];
      const double xji = (i == j) ? xd[j] : A[i * p + j];
      const double di = def[i] ? 1.0 : D[i];
      v = di * xji / ljj;
    }
    Rinv[idx] = v;
  }
  int ndef = 0;
  for (int i = 0; i < p; ++i) ndef += def[i];
  for (int i = t; i < ldr; i += nt) deficient[i] = (i < p) ? def[i] : 0;
  if (t == 0 && info) {
    info->deficient += ndef;
    if (pass >= 2 && ndef > 0) set_status(info, PF_ERR_BREAKDOWN);
  }
}

// ---------------------------------------------------------------------------
// Jacobi.  LDS: A (pe*pe), V (pe*pe, or global when it does not fit),
// rotation parameters per pair.
struct Rot {
  int i, j;
  double c, s, t;
  int active;
};

__global__ __launch_bounds__(256) void jacobi_kernel(const double* __restrict__ H, int ldh, int p,
                                                     double* __restrict__ theta, double* __restrict__ Z,
                                                     int ldz, double* __restrict__ Vglob, pf_info* info,
                                                     int which, int max_sweeps, double tol_rel,
                                                     int v_in_lds) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int pe = (p + 1) & ~1;
  const int half = pe / 2;
  double* A = reinterpret_cast<double*>(smem_raw);
  Rot* rot = reinterpret_cast<Rot*>(A + pe * pe);
  double* V = v_in_lds ? reinterpret_cast<double*>(rot + half) : Vglob;
  __shared__ double partial[256];
  __shared__ double fro2;
  __shared__ int sweeps_done;
  const int t = threadIdx.x, nt = blockDim.x;

  double local = 0.0;
  for (int idx = t; idx < pe * pe; idx += nt) {
    const int i = idx / pe, j = idx % pe;
    double v = 0.0;
    if (i < p && j < p) {
      // symmetrise: H is symmetric up to rounding of its two halves
      v = 0.5 * (H[i + (int64_t)j * ldh] + H[j + (int64_t)i * ldh]);
    }
    A[idx] = v;
    V[idx] = (i == j) ? 1.0 : 0.0;
    local += v * v;
  }
  partial[t] = local;
  __syncthreads();
  if (t == 0) {               // fixed summation order: reproducible threshold
    double f = 0.0;
    for (int i = 0; i < nt; ++i) f += partial[i];
    fro2 = f;
  }
  __syncthreads();
  const double tol_abs = 1e-18 * sqrt(fro2);

  int sweep = 0;
  bool converged = false;
  for (; sweep < max_sweeps; ++sweep) {
    int any_in_sweep = 0;
    for (int r = 0; r < pe - 1; ++r) {
      int act = 0;
      if (t < half) {
        int i, j;
        if (t == 0) { i = r; j = pe - 1; }
        else { i = (r + t) % (pe - 1); j = (r - t + (pe - 1)) % (pe - 1); }
        if (i > j) { const int tmp = i; i = j; j = tmp; }
        const double aii = A[i * pe + i], ajj = A[j * pe + j], aij = A[i * pe + j];
        const double thr = fmax(tol_rel * sqrt(fabs(aii) * fabs(ajj)), tol_abs);
        Rot R;
        R.i = i; R.j = j; R.c = 1.0; R.s = 0.0; R.t = 0.0; R.active = 0;
        if (fabs(aij) > thr) {
          const double tau = (ajj - aii) / (2.0 * aij);
          const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          const double cc = 1.0 / sqrt(1.0 + tt * tt);
          R.c = cc; R.s = tt * cc; R.t = tt; R.active = 1;
          act = 1;
        }
        rot[t] = R;
      }
      act = __syncthreads_or(act);
      if (!act) continue;
      any_in_sweep = 1;
      // A <- J^T A J on 2x2 blocks of pairs (P <= Q), mirrored.
      const int nblk = half * half;
      for (int b = t; b < nblk; b += nt) {
        const int P = b / half, Q = b % half;
        if (P > Q) continue;
        const Rot r1 = rot[P], r2 = rot[Q];
        if (!r1.active && !r2.active) continue;
        const int i1 = r1.i, j1 = r1.j, i2 = r2.i, j2 = r2.j;
        if (P == Q) {
          const double aij = A[i1 * pe + j1];
          A[i1 * pe + i1] -= r1.t * aij;
          A[j1 * pe + j1] += r1.t * aij;
          A[i1 * pe + j1] = 0.0;
          A[j1 * pe + i1] = 0.0;
          continue;
        }
        const double a11 = A[i1 * pe + i2], a12 = A[i1 * pe + j2];
        const double a21 = A[j1 * pe + i2], a22 = A[j1 * pe + j2];
        // right: columns (i2, j2)
        const double b11 = r2.c * a11 - r2.s * a12, b12 = r2.s * a11 + r2.c * a12;
        const double b21 = r2.c * a21 - r2.s * a22, b22 = r2.s * a21 + r2.c * a22;
        // left: rows (i1, j1)
        const double z11 = r1.c * b11 - r1.s * b21, z21 = r1.s * b11 + r1.c * b21;
        const double z12 = r1.c * b12 - r1.s * b22, z22 = r1.s * b12 + r1.c * b22;
        A[i1 * pe + i2] = z11; A[i1 * pe + j2] = z12;
        A[j1 * pe + i2] = z21; A[j1 * pe + j2] = z22;
        A[i2 * pe + i1] = z11; A[j2 * pe + i1] = z12;
        A[i2 * pe + j1] = z21; A[j2 * pe + j1] = z22;
      }
      // V <- V J
      for (int e = t; e < pe * half; e += nt) {
        const int row = e / half, P = e % half;
        const Rot r1 = rot[P];
        if (!r1.active) continue;
        const double vi = V[row * pe + r1.i], vj = V[row * pe + r1.j];
        V[row * pe + r1.i] = r1.c * vi - r1.s * vj;
        V[row * pe + r1.j] = r1.s * vi + r1.c * vj;
      }
      __syncthreads();
    }
    if (!any_in_sweep) { converged = true; break; }
  }
  if (t == 0) sweeps_done = sweep;
  __syncthreads();

  // Sort by descending theta (ties by index) and write out.
  for (int i = t; i < p; i += nt) {
    const double ti = A[i * pe + i];
    int rank = 0;
    for (int j = 0; j < p; ++j) {
      const double tj = A[j * pe + j];
      rank += (tj > ti) || (tj == ti && j < i);
    }
    theta[rank] = ti;
    for (int row = 0; row < p; ++row) Z[row + (int64_t)rank * ldz] = V[row * pe + i];
  }
  // zero padding of Z
  for (int idx = t; idx < ldz * ldz; idx += nt) {
    const int row = idx % ldz, col = idx / ldz;
    if (row >= p || col >= p) Z[idx] = (row == col) ? 1.0 : 0.0;
  }
  if (t == 0 && info) {
    if (which == 1) {
      int npos = 0;
      for (int i = 0; i < p; ++i) npos += A[i * pe + i] > 0.0;
      info->n_pos = npos;
      info->sweeps_rr = sweeps_done;
      if (!converged) set_status(info, PF_ERR_NOCONV);
    } else {
      info->sweeps_pre = sweeps_done;
    }
  }
}

}  // namespace

void launch_chol_rinv(const double* G, int ldg, int p, double* Rinv, int ldr, int* deficient,
                      pf_info* info, int pass, hipStream_t st) {
  const size_t lds = (size_t)p * p * 8 + 3 * (size_t)p * 8 + (size_t)p * 4 + 16;
  static size_t cur = 0;
  ensure_lds((const void*)chol_rinv_kernel, lds, cur);
  const double tol = 1e-14;
  chol_rinv_kernel<<<1, 256, lds, st>>>(G, ldg, p, Rinv, ldr, deficient, info, pass, tol);
  PFX_HIP(hipGetLastError());
}

size_t jacobi_lds_bytes(int p) {
  const int pe = (p + 1) & ~1;
  const size_t base = (size_t)pe * pe * 8 + (size_t)(pe / 2) * sizeof(Rot);
  const size_t withv = base + (size_t)pe * pe * 8;
  return withv <= 160 * 1024 - 4096 ? withv : base;   // static LDS: 2 KiB of partial sums
}

void launch_jacobi(const double* H, int ldh, int p, double* theta, double* Z, int ldz,
                   double* Zwork, pf_info* info, int which, int max_sweeps, hipStream_t st) {
  const int pe = (p + 1) & ~1;
  const size_t base = (size_t)pe * pe * 8 + (size_t)(pe / 2) * sizeof(Rot);
  const size_t lds = jacobi_lds_bytes(p);
  const int v_in_lds = lds > base;
  static size_t cur = 0;
  ensure_lds((const void*)jacobi_kernel, lds, cur);
  const double tol_rel = which == 1 ? 1e-15 : 1e-12;
  jacobi_kernel<<<1, 256, lds, st>>>(H, ldh, p, theta, Z, ldz, Zwork, info, which, max_sweeps,
                                     tol_rel, v_in_lds);
  PFX_HIP(hipGetLastError());
}

}  // namespace pfx
