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
template <int PMAX>
__global__ __launch_bounds__(256) void chol_rinv_kernel(const double* __restrict__ G, int ldg, int p,
                                                        double* __restrict__ Rinv, int ldr,
                                                        int* __restrict__ deficient,
                                                        pf_info* info, int pass, double tol) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int lda = p + 1;                        // odd stride: rows spread over banks
  double* A = reinterpret_cast<double*>(smem_raw);
  double* D = A + p * lda;
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
    const int j = idx / p, i = idx - j * p;            // coalesced over i
    const double gij = G[i + (int64_t)j * ldg];
    if (!isfinite(gij)) bad_nonfinite = 1;
    A[i * lda + j] = (i >= j) ? gij * D[i] * D[j] : 0.0;
  }
  __syncthreads();
  if (bad_nonfinite) {
    if (t == 0) set_status(info, PF_ERR_NONFINITE);
    for (int idx = t; idx < ldr * ldr; idx += nt) Rinv[idx] = 0.0;
    return;
  }

  // Right-looking elimination in the L D L^T form: column k stays
  // unscaled, so each step needs one barrier; scaling happens at the end.
  // Thread t updates rows k+1 + (t>>2) + 64m, columns k+1 + (t&3) + 4u.
  const int tr = t >> 2, tc = t & 3;
  for (int k = 0; k < p; ++k) {
    const double pk = A[k * lda + k];
    const bool ok = pk > tol && D[k] > 0.0;
    if (t == 0) { piv[k] = ok ? pk : 1.0; def[k] = ok ? 0 : 1; }
    if (ok) {
      const double inv = 1.0 / pk;
      for (int i = k + 1 + tr; i < p; i += 64) {
        const double lik = A[i * lda + k] * inv;
        // all loads of the row segment first, then the stores (one LDS
        // round trip instead of one per element)
        // loads are unconditional (indices clamped into the matrix) so that
        // they issue back to back; only the stores are predicated
        double cj[PMAX / 4], aj[PMAX / 4];
#pragma unroll
        for (int u = 0; u < PMAX / 4; ++u) {
          const int j = min(k + 1 + tc + 4 * u, i);
          cj[u] = A[j * lda + k];
          aj[u] = A[i * lda + j];
        }
#pragma unroll
        for (int u = 0; u < PMAX / 4; ++u) {
          const int j = k + 1 + tc + 4 * u;
          if (j <= i) A[i * lda + j] = aj[u] - lik * cj[u];
        }
      }
    }
    __syncthreads();
  }
  // L[i][k] = A[i][k] / sqrt(piv_k); deficient columns become e_k.
  for (int i = tr; i < p; i += 64) {
    for (int k = tc; k <= i; k += 4) {
      const int idx = i * lda + k;
      if (def[k]) A[idx] = (i == k) ? 1.0 : 0.0;
      else A[idx] = (i == k) ? sqrt(piv[k]) : A[idx] / sqrt(piv[k]);
    }
    for (int j = i + 1 + tc; j < p; j += 4) A[i * lda + j] = 0.0;   // upper part: L^{-1} storage
  }
  for (int i = t; i < p; i += nt) xd[i] = 1.0;
  __syncthreads();

  // X = L^{-1} by right-looking substitution on L X = I, rows left unscaled
  // (Xu) until the end: X[i][j] -= L[i][k] * Xu[k][j] / L[k][k].
  // Strictly lower X[i][j] (i > j) lives at A[j*p + i].
  for (int k = 0; k < p - 1; ++k) {
    const double invk = 1.0 / A[k * lda + k];
    for (int i = k + 1 + tr; i < p; i += 64) {
      const double lik = A[i * lda + k] * invk;
      if (lik == 0.0) continue;
      double xk[PMAX / 4], xi[PMAX / 4];
#pragma unroll
      for (int u = 0; u < PMAX / 4; ++u) {
        const int j = min(tc + 4 * u, k);
        xk[u] = A[j * lda + k];                 // position (k, k) is L[k][k]: replaced below
        xi[u] = A[j * lda + i];
        if (tc + 4 * u == k) xk[u] = xd[k];
      }
#pragma unroll
      for (int u = 0; u < PMAX / 4; ++u) {
        const int j = tc + 4 * u;
        if (j <= k) A[j * lda + i] = xi[u] - lik * xk[u];
      }
    }
    __syncthreads();
  }
  // Rinv = D L^{-T}: Rinv[i][j] = D_i X[j][i] (j >= i), X[j][i] = Xu[j][i] / L[j][j]
  for (int idx = t; idx < ldr * ldr; idx += nt) {
    const int i = idx % ldr, j = idx / ldr;   // column-major output
    double v = 0.0;
    if (i < p && j < p && j >= i) {
      const double ljj = A[j * lda + j];
      const double xji = (i == j) ? xd[j] : A[i * lda + j];
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
// Jacobi.  LDS: A (pe x pe, row stride pe+1 so rows spread over banks),
// V^T (row i = column i of V, so the plane rotations of V <- V J touch two
// contiguous rows), rotation parameters per pair (structure of arrays) and
// the list of 2x2 blocks (P, Q), P <= Q, each updated by one thread.
//
// first_order: when every off-diagonal entry is at most 1% of the gap of its
// two diagonal entries (the pre-rotation of a warm step, where H is the
// previous Ritz basis projected on a slightly perturbed matrix), the
// eigenvectors to first order, Z = I + K with K_ij = h_ij / (h_jj - h_ii),
// replace the sweeps; the pre-rotation needs only that each column is
// dominated by one eigen-direction, and any invertible Z keeps the span.
__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

template <int PMAX>
__global__ __launch_bounds__(256) void jacobi_kernel(const double* __restrict__ H, int ldh, int p,
                                                     double* __restrict__ theta, double* __restrict__ Z,
                                                     int ldz, double* __restrict__ Vglob, pf_info* info,
                                                     int which, int max_sweeps, double tol_rel,
                                                     int v_in_lds, int first_order) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int pe = (p + 1) & ~1;
  const int half = pe / 2;
  const int nblk = half * (half + 1) / 2;
  const int lda = pe + 1;
  const int ldv = v_in_lds ? pe + 2 : pe;
  double* A = reinterpret_cast<double*>(smem_raw);
  double* rc = A + pe * lda;
  double* rs = rc + half;
  double* rt = rs + half;
  double* dg = rt + half;                        // pe values: first-order eigenvalues
  int* ri = reinterpret_cast<int*>(dg + pe);
  int* rj = ri + half;
  unsigned* blk = reinterpret_cast<unsigned*>(rj + half);
  double* VT = v_in_lds ? reinterpret_cast<double*>(blk + ((nblk + 1) & ~1)) : Vglob;
  __shared__ double wsum[4];
  __shared__ int sweeps_done, not_diag;
  const int t = threadIdx.x, nt = blockDim.x;

  double local = 0.0;
  if (t == 0) not_diag = 0;
  for (int idx = t; idx < pe * pe; idx += nt) {
    const int j = idx / pe, i = idx - j * pe;    // coalesced over i
    double v = 0.0;
    if (i < p && j < p) v = 0.5 * (H[i + (int64_t)j * ldh] + H[j + (int64_t)i * ldh]);   // symmetrise
    A[i * lda + j] = v;
    VT[j * ldv + i] = (i == j) ? 1.0 : 0.0;
    local += v * v;
  }
  for (int b = t; b < half * half; b += nt) {
    const int P = b / half, Q = b - P * half;
    if (P <= Q) blk[P * half - P * (P - 1) / 2 + (Q - P)] = ((unsigned)P << 16) | (unsigned)Q;
  }
  local = wave_sum(local);
  if ((t & 63) == 0) wsum[t >> 6] = local;
  __syncthreads();
  const double fro = sqrt(wsum[0] + wsum[1] + wsum[2] + wsum[3]);   // fixed order
  // below this an off-diagonal entry is rounding noise of the rotations
  const double tol_abs = 2.220446049250313e-16 * fro;

  bool converged = false;
  int sweep = 0;
  if (first_order) {
    for (int idx = t; idx < p * p; idx += nt) {
      const int i = idx / p, j = idx - i * p;
      if (i == j) continue;
      const double aij = A[i * lda + j];
      if (fabs(aij) > tol_abs && !(fabs(aij) <= 0.01 * fabs(A[j * lda + j] - A[i * lda + i]))) not_diag = 1;
    }
    __syncthreads();
    if (!not_diag) {
      for (int idx = t; idx < p * p; idx += nt) {
        const int j = idx / p, i = idx - j * p;
        if (i == j) continue;
        const double aij = A[i * lda + j];
        VT[j * ldv + i] = fabs(aij) > tol_abs ? aij / (A[j * lda + j] - A[i * lda + i]) : 0.0;
      }
      for (int j = t; j < p; j += nt) {
        double d = A[j * lda + j];
        for (int i = 0; i < p; ++i) {
          const double aij = A[i * lda + j];
          if (i != j && fabs(aij) > tol_abs) d += aij * aij / (A[j * lda + j] - A[i * lda + i]);
        }
        dg[j] = d;
      }
      __syncthreads();
      for (int j = t; j < p; j += nt) A[j * lda + j] = dg[j];
      converged = true;
      __syncthreads();
    }
  }

  for (; !converged && sweep < max_sweeps; ++sweep) {
    int any_in_sweep = 0;
    for (int r = 0; r < pe - 1; ++r) {
      int act = 0;
      if (t < half) {
        int i, j;
        if (t == 0) { i = r; j = pe - 1; }
        else { i = r + t; if (i >= pe - 1) i -= pe - 1; j = r - t; if (j < 0) j += pe - 1; }
        if (i > j) { const int tmp = i; i = j; j = tmp; }
        const double aii = A[i * lda + i], ajj = A[j * lda + j], aij = A[i * lda + j];
        const double thr = fmax(tol_rel * sqrt(fabs(aii) * fabs(ajj)), tol_abs);
        double c = 1.0, s = 0.0, tt = 0.0;
        if (fabs(aij) > thr) {
          const double tau = (ajj - aii) / (2.0 * aij);
          tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + tt * tt);
          s = tt * c;
          act = 1;
        }
        rc[t] = c; rs[t] = s; rt[t] = act ? tt : 0.0; ri[t] = i; rj[t] = j;
      }
      act = __syncthreads_or(act);
      if (!act) continue;
      any_in_sweep = 1;
      // A <- J^T A J on 2x2 blocks of pairs, upper blocks mirrored.  A thread
      // owns up to BMAX blocks: all loads, then all stores.
      {
        // blocks per thread: ceil((PMAX/2)(PMAX/2 + 1)/2 / 256)
        constexpr int BMAX = ((PMAX / 2) * (PMAX / 2 + 1) / 2 + 255) / 256;
        double a11[BMAX], a12[BMAX], a21[BMAX], a22[BMAX];
        int bi1[BMAX], bj1[BMAX], bi2[BMAX], bj2[BMAX], kind[BMAX];
#pragma unroll
        for (int u = 0; u < BMAX; ++u) {
          const int b = min(t + u * nt, nblk - 1);   // clamped: loads stay unconditional
          const unsigned pq = blk[b];
          const int P = pq >> 16, Q = pq & 0xFFFF;
          bi1[u] = ri[P]; bj1[u] = rj[P]; bi2[u] = ri[Q]; bj2[u] = rj[Q];
          const double tP = rt[P], tQ = rt[Q];
          kind[u] = (t + u * nt >= nblk || (tP == 0.0 && tQ == 0.0)) ? 0 : (P == Q ? 1 : 2);
          a11[u] = A[bi1[u] * lda + bi2[u]]; a12[u] = A[bi1[u] * lda + bj2[u]];
          a21[u] = A[bj1[u] * lda + bi2[u]]; a22[u] = A[bj1[u] * lda + bj2[u]];
          const double c1 = rc[P], s1 = rs[P], c2 = rc[Q], s2 = rs[Q];
          if (kind[u] == 1) {
            a21[u] = tP;                                 // keep t of the pair
          } else {
            const double b11 = c2 * a11[u] - s2 * a12[u], b12 = s2 * a11[u] + c2 * a12[u];
            const double b21 = c2 * a21[u] - s2 * a22[u], b22 = s2 * a21[u] + c2 * a22[u];
            a11[u] = c1 * b11 - s1 * b21; a21[u] = s1 * b11 + c1 * b21;
            a12[u] = c1 * b12 - s1 * b22; a22[u] = s1 * b12 + c1 * b22;
          }
        }
#pragma unroll
        for (int u = 0; u < BMAX; ++u) {
          if (kind[u] == 0) continue;
          const int i1 = bi1[u], j1 = bj1[u], i2 = bi2[u], j2 = bj2[u];
          if (kind[u] == 1) {
            // diagonal block of pair (i1, j1): a11, a22 the diagonal entries,
            // a12 = a_{i1 j1}, a21 = t; the rotation zeroes a_{i1 j1}
            A[i1 * lda + i1] = a11[u] - a21[u] * a12[u];
            A[j1 * lda + j1] = a22[u] + a21[u] * a12[u];
            A[i1 * lda + j1] = 0.0;
            A[j1 * lda + i1] = 0.0;
          } else {
            A[i1 * lda + i2] = a11[u]; A[i1 * lda + j2] = a12[u];
            A[j1 * lda + i2] = a21[u]; A[j1 * lda + j2] = a22[u];
            A[i2 * lda + i1] = a11[u]; A[j2 * lda + i1] = a12[u];
            A[i2 * lda + j1] = a21[u]; A[j2 * lda + j1] = a22[u];
          }
        }
      }
      // V <- V J: thread (k = t/8, part t%8) rotates a contiguous run of
      // rows i_k, j_k of V^T; all loads issue before the stores.
      {
        const int part = t & 7;
        const int chunk = (pe + 7) >> 3;
        const int x0 = part * chunk;
        const int xe = min(pe, x0 + chunk);
        for (int k = t >> 3; k < half; k += nt >> 3) {
          if (rt[k] == 0.0) continue;
          const double c = rc[k], s = rs[k];
          double* __restrict__ vi = VT + ri[k] * ldv;
          double* __restrict__ vj = VT + rj[k] * ldv;
          double va[16], vb[16];
#pragma unroll
          for (int u = 0; u < 16; ++u)
            if (x0 + u < xe) { va[u] = vi[x0 + u]; vb[u] = vj[x0 + u]; }
#pragma unroll
          for (int u = 0; u < 16; ++u)
            if (x0 + u < xe) { vi[x0 + u] = c * va[u] - s * vb[u]; vj[x0 + u] = s * va[u] + c * vb[u]; }
        }
      }
      __syncthreads();
    }
    if (!any_in_sweep) { converged = true; break; }
  }
  if (t == 0) sweeps_done = first_order && !not_diag ? 0 : sweep;
  __syncthreads();

  // Sort by descending theta (ties by index) and write out.
  for (int i = t; i < p; i += nt) {
    const double ti = A[i * lda + i];
    int rank = 0;
    for (int j = 0; j < p; ++j) {
      const double tj = A[j * lda + j];
      rank += (tj > ti) || (tj == ti && j < i);
    }
    theta[rank] = ti;
    for (int row = 0; row < p; ++row) Z[row + (int64_t)rank * ldz] = VT[i * ldv + row];
  }
  for (int idx = t; idx < ldz * ldz; idx += nt) {
    const int row = idx % ldz, col = idx / ldz;
    if (row >= p || col >= p) Z[idx] = (row == col) ? 1.0 : 0.0;
  }
  if (t == 0 && info) {
    if (which == 1) {
      int npos = 0;
      for (int i = 0; i < p; ++i) npos += A[i * lda + i] > 0.0;
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
  const size_t lds = (size_t)p * (p + 1) * 8 + 3 * (size_t)p * 8 + (size_t)p * 4 + 16;
  // Pivots of the equilibrated Gram are squared sines of the angle between a
  // column and the span of the previous ones.  Below 1e-10 (angle < 1e-5)
  // the column is treated as dependent: CholeskyQR2 reaches working
  // orthogonality only while cond(Y) stays well below 1/sqrt(eps).
  const double tol = 1e-10;
  if (p <= 32) {
    chol_rinv_kernel<32><<<1, 256, lds, st>>>(G, ldg, p, Rinv, ldr, deficient, info, pass, tol);
  } else if (p <= 64) {
    chol_rinv_kernel<64><<<1, 256, lds, st>>>(G, ldg, p, Rinv, ldr, deficient, info, pass, tol);
  } else {
    static size_t cur = 0;
    ensure_lds((const void*)chol_rinv_kernel<128>, lds, cur);
    chol_rinv_kernel<128><<<1, 256, lds, st>>>(G, ldg, p, Rinv, ldr, deficient, info, pass, tol);
  }
  PFX_HIP(hipGetLastError());
}

static size_t jacobi_base_bytes(int p) {
  const int pe = (p + 1) & ~1;
  const int half = pe / 2;
  const int nblk = half * (half + 1) / 2;
  return (size_t)pe * (pe + 1) * 8 + (size_t)half * (3 * 8 + 2 * 4) + (size_t)pe * 8 +
         (size_t)((nblk + 1) & ~1) * 4;
}

size_t jacobi_lds_bytes(int p) {
  const int pe = (p + 1) & ~1;
  const size_t base = jacobi_base_bytes(p);
  const size_t withv = base + (size_t)pe * (pe + 2) * 8;
  return withv <= 160 * 1024 - 256 ? withv : base;   // static LDS: 36 bytes
}

void launch_jacobi(const double* H, int ldh, int p, double* theta, double* Z, int ldz,
                   double* Zwork, pf_info* info, int which, int max_sweeps, hipStream_t st) {
  const size_t base = jacobi_base_bytes(p);
  const size_t lds = jacobi_lds_bytes(p);
  const int v_in_lds = lds > base;
  static size_t cur32 = 0, cur64 = 0, cur128 = 0;
  // Rayleigh-Ritz: converge to FP64 resolution; pre-rotation: a rotation
  // accurate to 1e-10 keeps every FP32 recurrence column on its direction.
  const double tol_rel = which == 1 ? 1e-15 : 1e-10;
  const int fo = which == 0 ? 1 : 0;
  if (p <= 32) {
    ensure_lds((const void*)jacobi_kernel<32>, lds, cur32);
    jacobi_kernel<32><<<1, 256, lds, st>>>(H, ldh, p, theta, Z, ldz, Zwork, info, which, max_sweeps, tol_rel,
                                           v_in_lds, fo);
  } else if (p <= 64) {
    ensure_lds((const void*)jacobi_kernel<64>, lds, cur64);
    jacobi_kernel<64><<<1, 256, lds, st>>>(H, ldh, p, theta, Z, ldz, Zwork, info, which, max_sweeps, tol_rel,
                                           v_in_lds, fo);
  } else {
    ensure_lds((const void*)jacobi_kernel<128>, lds, cur128);
    jacobi_kernel<128><<<1, 256, lds, st>>>(H, ldh, p, theta, Z, ldz, Zwork, info, which, max_sweeps, tol_rel,
                                            v_in_lds, fo);
  }
  PFX_HIP(hipGetLastError());
}

}  // namespace pfx
