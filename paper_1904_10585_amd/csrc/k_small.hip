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
// Cholesky + triangular inverse, register resident.  Thread (bi, bj) of a
// (PMAX/4)^2 grid holds the 4x4 blocks (bi, bj) of the equilibrated Gram
// matrix G and of W, which starts as I.  Step k of the right-looking
// elimination in L D L^T form broadcasts column k of G and row k of W
// through LDS (double-buffered: one barrier per step) and applies
//     G[i][j] -= G[i][k] G[k][j] / d_k   (i, j > k)
//     W[i][:] -= G[i][k] / d_k * W[k][:] (i > k),
// the same row operations on W as on G, so that at the end
// G = L_1 D L_1^T with L_1 unit lower triangular and W = L_1^{-1}.  Then
// R = D^{1/2} L_1^T (of the equilibrated matrix) and
//     R^{-1}[i][j] = s_i W[j][i] / sqrt(d_j),   i <= j,
// with s = diag(G)^{-1/2} the equilibration.
template <int PMAX>
__global__ __launch_bounds__((PMAX / 4) * (PMAX / 4)) void chol_rinv_kernel(
    const double* __restrict__ G, int ldg, int p, double* __restrict__ Rinv, int ldr,
    int* __restrict__ deficient, pf_info* info, int pass, double tol, double near_tol) {
  constexpr int NBK = PMAX / 4;
  constexpr int NT = NBK * NBK;
  __shared__ __align__(16) double s_eq[PMAX], s_piv[PMAX], s_col[2][PMAX], s_row[2][PMAX];
  __shared__ int s_def[PMAX];
  __shared__ int s_bad, s_far;
  const int t = threadIdx.x;
  const int bi = t / NBK, bj = t % NBK;
  const int i0 = 4 * bi, j0 = 4 * bj;
  if (t == 0) { s_bad = 0; s_far = 0; }
  __syncthreads();

  double g[4][4], w[4][4];
  bool bad = false;
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int i = i0 + r, j = j0 + c;
      double v = i == j ? 1.0 : 0.0;                 // identity padding past p
      if (i < p && j < p) {
        v = G[i + (int64_t)j * ldg];
        bad |= !isfinite(v);
      }
      g[r][c] = v;
      w[r][c] = i == j ? 1.0 : 0.0;
    }
  if (bad) s_bad = 1;
  if (bi == bj) {
#pragma unroll
    for (int r = 0; r < 4; ++r) s_eq[i0 + r] = g[r][r] > 0.0 ? 1.0 / sqrt(g[r][r]) : 0.0;
  }
  __syncthreads();
  if (s_bad) {
    if (t == 0) set_status(info, PF_ERR_NONFINITE);
    for (int idx = t; idx < ldr * ldr; idx += NT) Rinv[idx] = 0.0;
    return;
  }
  double si[4], sj[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) { si[u] = s_eq[i0 + u]; sj[u] = s_eq[j0 + u]; }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (i0 + r < p && j0 + c < p) g[r][c] *= si[r] * sj[c];

  // Second CholeskyQR pass: the equilibrated Gram matrix of an already
  // orthonormalised block is I + E with E small.  To first order
  // chol(I + E) = I + U (U: strict upper part of E, diagonal E_ii / 2) and
  // (I + U)^{-1} = I - U; the neglected terms are O(|E|^2), below the
  // working precision when |E| <= near_tol.
  if (near_tol > 0.0) {
    double dev = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (i0 + r < p && j0 + c < p) dev = fmax(dev, fabs(g[r][c] - (i0 + r == j0 + c ? 1.0 : 0.0)));
    if (!(dev <= near_tol)) s_far = 1;
    __syncthreads();
    if (!s_far) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int i = i0 + r, j = j0 + c;
          if (i < p && j < p && i < ldr && j < ldr) {
            const double u = i == j ? 0.5 * (g[r][c] - 1.0) : (i < j ? g[r][c] : 0.0);
            Rinv[i + (int64_t)j * ldr] = si[r] * ((i == j ? 1.0 : 0.0) - u);
          }
        }
      for (int idx = t; idx < ldr * ldr; idx += NT) {
        const int i = idx % ldr, j = idx / ldr;
        if (i >= p || j >= p) Rinv[idx] = 0.0;
      }
      for (int i = t; i < ldr; i += NT) deficient[i] = 0;
      return;
    }
  }

  for (int k = 0; k < p; ++k) {
    const int buf = k & 1, kb = k >> 2, kr = k & 3;
    // owners publish column k of G and row k of W (kr is uniform: a scalar
    // branch picks the registers)
    if (bj == kb) {
      switch (kr) {
        case 0: for (int r = 0; r < 4; ++r) s_col[buf][i0 + r] = g[r][0]; break;
        case 1: for (int r = 0; r < 4; ++r) s_col[buf][i0 + r] = g[r][1]; break;
        case 2: for (int r = 0; r < 4; ++r) s_col[buf][i0 + r] = g[r][2]; break;
        default: for (int r = 0; r < 4; ++r) s_col[buf][i0 + r] = g[r][3]; break;
      }
    }
    if (bi == kb) {
      switch (kr) {
        case 0: for (int c = 0; c < 4; ++c) s_row[buf][j0 + c] = w[0][c]; break;
        case 1: for (int c = 0; c < 4; ++c) s_row[buf][j0 + c] = w[1][c]; break;
        case 2: for (int c = 0; c < 4; ++c) s_row[buf][j0 + c] = w[2][c]; break;
        default: for (int c = 0; c < 4; ++c) s_row[buf][j0 + c] = w[3][c]; break;
      }
    }
    __syncthreads();
    const double pk = s_col[buf][k];
    double ci[4], cj[4], wk[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      ci[u] = s_col[buf][i0 + u];
      cj[u] = s_col[buf][j0 + u];
      wk[u] = s_row[buf][j0 + u];
    }
    // a dependent column (equilibrated pivot <= tol; a zero column has pivot
    // 0) is left out of the elimination
    const bool ok = pk > tol;
    if (t == 0) { s_piv[k] = ok ? pk : 1.0; s_def[k] = ok ? 0 : 1; }
    const double inv = ok ? 1.0 / pk : 0.0;
    double li[4], gj[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      li[u] = (i0 + u > k) ? ci[u] * inv : 0.0;
      gj[u] = (j0 + u > k) ? cj[u] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        g[r][c] -= li[r] * gj[c];
        w[r][c] -= li[r] * wk[c];
      }
  }
  __syncthreads();

  // R^{-1}[i][j] = s_i W[j][i] / sqrt(d_j) for i <= j: this thread's W block
  // (rows i0.., columns j0..) lands transposed at rows j0.., columns i0..
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int wr = i0 + r, wc = j0 + c;          // W[wr][wc] -> Rinv[wc][wr]
      if (wr < p && wc < p && wc < ldr && wr < ldr) {
        double v = 0.0;
        if (wc <= wr) {
          const double s = s_def[wc] ? 1.0 : s_eq[wc];
          v = s * w[r][c] / sqrt(s_piv[wr]);
        }
        Rinv[wc + (int64_t)wr * ldr] = v;
      }
    }
  for (int idx = t; idx < ldr * ldr; idx += NT) {
    const int i = idx % ldr, j = idx / ldr;
    if (i >= p || j >= p) Rinv[idx] = 0.0;
  }
  for (int i = t; i < ldr; i += NT) deficient[i] = (i < p) ? s_def[i] : 0;
  if (t == 0) {
    int ndef = 0;
    for (int i = 0; i < p; ++i) ndef += s_def[i];
    if (info) {
      info->deficient += ndef;
      if (pass >= 2 && ndef > 0) set_status(info, PF_ERR_BREAKDOWN);
    }
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

__device__ inline double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// Pair k of round r of the round-robin order over pe (even) indices: index
// pe-1 stays, the others rotate; every pair meets once in pe-1 rounds.
__device__ inline void rr_pair(int r, int k, int pe, int& i, int& j) {
  if (k == 0) {
    i = r;
    j = pe - 1;
  } else {
    i = r + k;
    if (i >= pe - 1) i -= pe - 1;
    j = r - k;
    if (j < 0) j += pe - 1;
  }
  if (i > j) { const int x = i; i = j; j = x; }
}

// VLDS: V^T lives in LDS (p <= 98); otherwise in the global work buffer.
// Separate instantiations keep every LDS access a ds_* instruction (a
// pointer that may be either would make them all flat accesses).
template <int PMAX, bool VLDS>
__global__ __launch_bounds__(256) void jacobi_kernel(const double* __restrict__ H, int ldh, int p,
                                                     double* __restrict__ theta, double* __restrict__ Z,
                                                     int ldz, double* __restrict__ Vglob, pf_info* info,
                                                     int which, int max_sweeps, double tol_rel,
                                                     int first_order, const int* skip) {
  if (skip && *skip) return;                     // the refinement solved this matrix
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int pe = (p + 1) & ~1;
  const int half = pe / 2;
  const int nblk = half * (half + 1) / 2;
  const int lda = pe + 1;
  const int ldv = VLDS ? pe + 2 : pe;
  double* A = reinterpret_cast<double*>(smem_raw);
  double* rc = A + pe * lda;
  double* rs = rc + half;
  double* rt = rs + half;
  double* dg = rt + half;                        // pe values
  int* perm = reinterpret_cast<int*>(dg + pe);   // pe values
  unsigned* blk = reinterpret_cast<unsigned*>(perm + pe);
  double* VT;
  if constexpr (VLDS) VT = reinterpret_cast<double*>(blk + ((nblk + 1) & ~1));
  else VT = Vglob;
  __shared__ double wsum[4];
  __shared__ int not_diag;
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

  // the 2x2 blocks (P, Q), P <= Q, of pair space this thread updates
  constexpr int BMAX = ((PMAX / 2) * (PMAX / 2 + 1) / 2 + 255) / 256;
  int bP[BMAX], bQ[BMAX];
#pragma unroll
  for (int u = 0; u < BMAX; ++u) {
    const int b = t + u * nt;
    const unsigned pq = blk[min(b, nblk - 1)];
    bP[u] = b < nblk ? (int)(pq >> 16) : -1;
    bQ[u] = (int)(pq & 0xFFFF);
  }

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

  while (!converged) {
    // a sweep runs only while some off-diagonal entry is above its threshold
    int above = 0;
    for (int idx = t; idx < p * p; idx += nt) {
      const int i = idx / p, j = idx - i * p;
      if (i < j) {
        const double thr = fmax(tol_rel * sqrt(fabs(A[i * lda + i]) * fabs(A[j * lda + j])), tol_abs);
        above |= fabs(A[i * lda + j]) > thr;
      }
    }
    above = __syncthreads_or(above);
    if (!above) { converged = true; break; }
    if (sweep >= max_sweeps) break;
    ++sweep;
    for (int r = 0; r < pe - 1; ++r) {
      // rotation of each pair (one lane per pair, first wave only)
      if (t < half) {
        int i, j;
        rr_pair(r, t, pe, i, j);
        const double aii = A[i * lda + i], ajj = A[j * lda + j], aij = A[i * lda + j];
        const double thr = fmax(tol_rel * sqrt(fabs(aii) * fabs(ajj)), tol_abs);
        double c = 1.0, sn = 0.0, tt = 0.0;
        if (fabs(aij) > thr) {
          // tan of the rotation angle, smaller root: t = sign(d) x / (|d| + hypot(d, x))
          const double d = ajj - aii, x = 2.0 * aij;
          const double tq = x / (fabs(d) + sqrt(d * d + x * x));
          tt = d >= 0.0 ? tq : -tq;
          c = 1.0 / sqrt(1.0 + tt * tt);
          sn = tt * c;
        }
        rc[t] = c; rs[t] = sn; rt[t] = tt;
      }
      __syncthreads();
      // A <- J^T A J on the 2x2 blocks of pairs (upper blocks mirrored): all
      // loads of this thread's blocks, then the stores
      {
        double a11[BMAX], a12[BMAX], a21[BMAX], a22[BMAX];
        int i1[BMAX], j1[BMAX], i2[BMAX], j2[BMAX], kind[BMAX];
#pragma unroll
        for (int u = 0; u < BMAX; ++u) {
          const int P = max(bP[u], 0), Q = bQ[u];
          rr_pair(r, P, pe, i1[u], j1[u]);
          rr_pair(r, Q, pe, i2[u], j2[u]);
          const double tP = rt[P], tQ = rt[Q];
          const double c1 = rc[P], s1 = rs[P], c2 = rc[Q], s2 = rs[Q];
          a11[u] = A[i1[u] * lda + i2[u]]; a12[u] = A[i1[u] * lda + j2[u]];
          a21[u] = A[j1[u] * lda + i2[u]]; a22[u] = A[j1[u] * lda + j2[u]];
          kind[u] = (bP[u] < 0 || (tP == 0.0 && tQ == 0.0)) ? 0 : (P == Q ? 1 : 2);
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
          const int x1 = i1[u], y1 = j1[u], x2 = i2[u], y2 = j2[u];
          if (kind[u] == 1) {
            // diagonal block of the pair: the rotation zeroes a_{x1 y1}
            A[x1 * lda + x1] = a11[u] - a21[u] * a12[u];
            A[y1 * lda + y1] = a22[u] + a21[u] * a12[u];
            A[x1 * lda + y1] = 0.0;
            A[y1 * lda + x1] = 0.0;
          } else {
            A[x1 * lda + x2] = a11[u]; A[x1 * lda + y2] = a12[u];
            A[y1 * lda + x2] = a21[u]; A[y1 * lda + y2] = a22[u];
            A[x2 * lda + x1] = a11[u]; A[y2 * lda + x1] = a12[u];
            A[x2 * lda + y1] = a21[u]; A[y2 * lda + y1] = a22[u];
          }
        }
      }
      // V <- V J: eight threads per pair rotate a run of the two rows of V^T
      {
        constexpr int CH = PMAX / 8;                 // entries per thread and row
        const int part = t & 7;
        const int x0 = part * CH;
        for (int k = t >> 3; k < half; k += nt >> 3) {
          if (rt[k] == 0.0) continue;
          int i, j;
          rr_pair(r, k, pe, i, j);
          const double c = rc[k], sn = rs[k];
          double* __restrict__ vi = VT + i * ldv;
          double* __restrict__ vj = VT + j * ldv;
          double va[CH], vb[CH];
#pragma unroll
          for (int u = 0; u < CH; ++u) {            // clamped loads, predicated stores
            const int x = min(x0 + u, pe - 1);
            va[u] = vi[x];
            vb[u] = vj[x];
          }
#pragma unroll
          for (int u = 0; u < CH; ++u)
            if (x0 + u < pe) { vi[x0 + u] = c * va[u] - sn * vb[u]; vj[x0 + u] = sn * va[u] + c * vb[u]; }
        }
      }
      __syncthreads();
    }
  }
  const int sweeps_done = first_order && !not_diag ? 0 : sweep;

  // Sort by descending theta, ties by index.  The key orders NaN below every
  // number, so (key, index) is a strict total order even for non-finite
  // input and the ranks are a permutation of 0..p-1.
  for (int i = t; i < p; i += nt) {
    const double ti = A[i * lda + i];
    const double ki = isnan(ti) ? -INFINITY : ti;
    int rank = 0;
    for (int j = 0; j < p; ++j) {
      const double tj = A[j * lda + j];
      const double kj = isnan(tj) ? -INFINITY : tj;
      rank += (kj > ki) || (kj == ki && j < i);
    }
    theta[rank] = ti;
    perm[rank] = i;
  }
  __syncthreads();
  for (int idx = t; idx < ldz * ldz; idx += nt) {
    const int row = idx % ldz, col = idx / ldz;
    const int src = min(max(col < p ? perm[col] : 0, 0), p - 1);
    Z[idx] = (row < p && col < p) ? VT[src * ldv + row] : (row == col ? 1.0 : 0.0);
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

// ---------------------------------------------------------------------------
// Eigen-refinement for a nearly diagonal H (the Rayleigh-Ritz matrix of a
// warm step, the pre-rotation matrix).  Z starts at I and each iteration
//   A = Z^T H Z,  K_ij = a_ij / (a_jj - a_ii)  (i != j; antisymmetric),
//   Z <- Z (I + K + K^2 / 2),  Z <- Z (3 I - Z^T Z) / 2,
// i.e. all plane rotations of a Jacobi sweep at once to first order (the
// truncated exponential of K), followed by a Newton-Schulz step that
// restores orthonormality.  Off-diagonal entries go from eps to
// O(eps^2 / gap): the convergence is quadratic while every |a_ij| is small
// against its gap.  When some |K_ij| exceeds 0.01 (eigenvalues close
// against their coupling, or a cold start) the kernel reports failure and
// the Jacobi kernel that follows solves H from scratch.  Every product is a
// PP x PP FP64 MFMA contraction (v_mfma_f64_16x16x4f64) on LDS-resident
// matrices (global scratch for PP = 128).
typedef double d4v __attribute__((ext_vector_type(4)));

// C = op(A) B for PP x PP column-major matrices (leading dimension LD),
// op(A) = A^T when TA.  Wave w computes the output column blocks w, w+4, ...
// with all PP/16 row tiles of a block at once: independent accumulators
// hide the MFMA latency and share one B fragment per K step.
// Lane l of a 16x16x4 FP64 MFMA holds A[l%16][l/16] and B[l/16][l%16];
// accumulator j holds D[4j + l/16][l%16].
template <int PP, int LD, bool TA>
__device__ inline void gemm_pp(double* __restrict__ C, const double* __restrict__ A, const double* __restrict__ B,
                               int wave, int lane) {
  constexpr int NTL = PP / 16;
  const int r = lane & 15, kq = lane >> 4;
  for (int tj = wave; tj < NTL; tj += 4) {
    const int jc = tj * 16 + r;
    d4v acc[NTL];
#pragma unroll
    for (int ti = 0; ti < NTL; ++ti) acc[ti] = d4v{0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
    for (int kk = 0; kk < PP; kk += 4) {
      const int k = kk + kq;
      const double b = B[k + jc * LD];
      double a[NTL];
#pragma unroll
      for (int ti = 0; ti < NTL; ++ti) {
        const int i = ti * 16 + r;
        a[ti] = TA ? A[k + i * LD] : A[i + k * LD];
      }
#pragma unroll
      for (int ti = 0; ti < NTL; ++ti) acc[ti] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ti], b, acc[ti], 0, 0, 0);
    }
#pragma unroll
    for (int ti = 0; ti < NTL; ++ti)
#pragma unroll
      for (int j = 0; j < 4; ++j) C[(ti * 16 + 4 * j + kq) + jc * LD] = acc[ti][j];
  }
}

template <int PMAX, bool SH>
__global__ __launch_bounds__(256) void eig_refine_kernel(const double* __restrict__ H, int ldh, int p,
                                                         double* __restrict__ theta, double* __restrict__ Z,
                                                         int ldz, double* __restrict__ gscratch, int* refined,
                                                         pf_info* info, int which, int max_iter) {
  constexpr int PP = PMAX, LD = PP + 1, MS = PP * LD;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* buf;
  if constexpr (SH) buf = reinterpret_cast<double*>(smem_raw);
  else buf = gscratch;
  double* Hs = buf;
  double* Zc = buf + MS;
  double* T1 = buf + 2 * MS;
  double* T2 = buf + 3 * MS;
  __shared__ double wsum[4];
  __shared__ int s_rank[PMAX];
  __shared__ double s_th[PMAX];
  const int t = threadIdx.x, nt = blockDim.x;
  const int lane = t & 63, wave = t >> 6;

  double local = 0.0;
  for (int idx = t; idx < PP * PP; idx += nt) {
    const int i = idx % PP, j = idx / PP;
    double v = 0.0;
    if (i < p && j < p) v = 0.5 * (H[i + (int64_t)j * ldh] + H[j + (int64_t)i * ldh]);   // symmetrise
    Hs[i + j * LD] = v;
    Zc[i + j * LD] = i == j ? 1.0 : 0.0;
    local += v * v;
  }
  local = wave_sum(local);
  if (lane == 0) wsum[wave] = local;
  __syncthreads();
  const double fro = sqrt(wsum[0] + wsum[1] + wsum[2] + wsum[3]);
  // Rayleigh-Ritz: off-diagonal entries below this are at the rounding
  // level of the PP-term FP64 products that form A; the pre-rotation needs
  // each column on its eigen-direction to 1e-10 only
  const double tol = which == 1 ? 64.0 * 2.220446049250313e-16 * fro : 1e-10 * fro;

  __shared__ double s_kmax[4];
  bool converged = false;
  int it = 0;
  for (;; ++it) {
    if (it == 0) {
      // Z = I: A = H
      for (int idx = t; idx < PP * PP; idx += nt) {
        const int i = idx % PP, j = idx / PP;
        T2[i + j * LD] = Hs[i + j * LD];
      }
    } else {
      gemm_pp<PP, LD, false>(T1, Hs, Zc, wave, lane);     // T1 = H Z
      __syncthreads();
      gemm_pp<PP, LD, true>(T2, Zc, T1, wave, lane);      // T2 = A = Z^T H Z
    }
    __syncthreads();
    int above = 0, far = 0;
    double kmax = 0.0;
    for (int idx = t; idx < PP * PP; idx += nt) {
      const int i = idx % PP, j = idx / PP;
      double k = 0.0;
      if (i != j && i < p && j < p) {
        const double aij = 0.5 * (T2[i + j * LD] + T2[j + i * LD]);
        if (fabs(aij) > tol) {
          above = 1;
          const double gap = T2[j + j * LD] - T2[i + i * LD];
          if (!(fabs(aij) <= 0.01 * fabs(gap))) far = 1;
          else k = aij / gap;
        }
      }
      kmax = fmax(kmax, fabs(k));
      T1[i + j * LD] = k;                                  // K (antisymmetric)
    }
    kmax = wave_max(kmax);
    if (lane == 0) s_kmax[wave] = kmax;
    above = __syncthreads_or(above);
    far = __syncthreads_or(far);
    kmax = fmax(fmax(s_kmax[0], s_kmax[1]), fmax(s_kmax[2], s_kmax[3]));
    if (!above) { converged = true; break; }
    if (far || it >= max_iter) break;
    if (which == 0) {
      // pre-rotation: the first-order eigenvectors Z = I + K (invertible, so
      // the span is kept; each column on one eigen-direction to O(K^2)) and
      // second-order eigenvalues theta_i = a_ii + sum_j a_ij K_ji
      for (int idx = t; idx < PP * PP; idx += nt) {
        const int i = idx % PP, j = idx / PP;
        Zc[i + j * LD] = (i == j ? 1.0 : 0.0) + T1[i + j * LD];
      }
      for (int i = t; i < p; i += nt) {
        double th = T2[i + i * LD];
        for (int j = 0; j < p; ++j) th += T2[j + i * LD] * T1[j + i * LD];
        T2[i + i * LD] = th;
      }
      __syncthreads();
      converged = true;
      break;
    }
    const bool small_k = kmax < 1e-4;
    gemm_pp<PP, LD, false>(T2, T1, T1, wave, lane);       // T2 = K^2
    __syncthreads();
    for (int idx = t; idx < PP * PP; idx += nt) {
      const int i = idx % PP, j = idx / PP;
      T1[i + j * LD] = (i == j ? 1.0 : 0.0) + T1[i + j * LD] + 0.5 * T2[i + j * LD];   // M = I + K + K^2/2
    }
    __syncthreads();
    if (it == 0) {
      // Z = I: Z M = M
      for (int idx = t; idx < PP * PP; idx += nt) {
        const int i = idx % PP, j = idx / PP;
        T2[i + j * LD] = T1[i + j * LD];
      }
    } else {
      gemm_pp<PP, LD, false>(T2, Zc, T1, wave, lane);     // T2 = Z M
    }
    __syncthreads();
    if (small_k) {
      // M is orthogonal to O(|K|^4) (M^T M = I + K^4 / 4): no re-orthonormalisation
      for (int idx = t; idx < PP * PP; idx += nt) {
        const int i = idx % PP, j = idx / PP;
        Zc[i + j * LD] = T2[i + j * LD];
      }
      __syncthreads();
      continue;
    }
    gemm_pp<PP, LD, true>(T1, T2, T2, wave, lane);        // T1 = (Z M)^T (Z M)
    __syncthreads();
    for (int idx = t; idx < PP * PP; idx += nt) {
      const int i = idx % PP, j = idx / PP;
      T1[i + j * LD] = 0.5 * ((i == j ? 3.0 : 0.0) - T1[i + j * LD]);   // (3 I - Z^T Z) / 2
    }
    __syncthreads();
    gemm_pp<PP, LD, false>(Zc, T2, T1, wave, lane);       // Z <- Z M (3 I - ...) / 2
    __syncthreads();
  }
  if (!converged) {
    if (t == 0) *refined = 0;
    return;
  }
  // theta = diag(A) (Rayleigh quotients of the orthonormal columns of Z),
  // sorted descending (NaN lowest, ties by index), Z columns permuted alike
  for (int i = t; i < p; i += nt) s_th[i] = T2[i + i * LD];
  __syncthreads();
  for (int i = t; i < p; i += nt) {
    const double ti = s_th[i];
    const double ki = isnan(ti) ? -INFINITY : ti;
    int rank = 0;
    for (int j = 0; j < p; ++j) {
      const double kj = isnan(s_th[j]) ? -INFINITY : s_th[j];
      rank += (kj > ki) || (kj == ki && j < i);
    }
    theta[rank] = ti;
    s_rank[rank] = i;
  }
  __syncthreads();
  for (int idx = t; idx < ldz * ldz; idx += nt) {
    const int row = idx % ldz, col = idx / ldz;
    const int src = min(max(col < p ? s_rank[col] : 0, 0), p - 1);
    Z[idx] = (row < p && col < p) ? Zc[row + src * LD] : (row == col ? 1.0 : 0.0);
  }
  if (t == 0) {
    *refined = 1;
    if (info) {
      if (which == 1) {
        int npos = 0;
        for (int i = 0; i < p; ++i) npos += s_th[i] > 0.0;
        info->n_pos = npos;
        info->sweeps_rr = 0;
        info->refine_rr = it;
      } else {
        info->sweeps_pre = 0;
        info->refine_pre = it;
      }
    }
  }
}

}  // namespace

void launch_chol_rinv(const double* G, int ldg, int p, double* Rinv, int ldr, int* deficient,
                      pf_info* info, int pass, hipStream_t st, double near_tol) {
  // Pivots of the equilibrated Gram are squared sines of the angle between a
  // column and the span of the previous ones.  Below 1e-10 (angle < 1e-5)
  // the column is treated as dependent: CholeskyQR2 reaches working
  // orthogonality only while cond(Y) stays well below 1/sqrt(eps).
  const double tol = 1e-10;
  if (p <= 32) {
    chol_rinv_kernel<32><<<1, 64, 0, st>>>(G, ldg, p, Rinv, ldr, deficient, info, pass, tol, near_tol);
  } else if (p <= 64) {
    chol_rinv_kernel<64><<<1, 256, 0, st>>>(G, ldg, p, Rinv, ldr, deficient, info, pass, tol, near_tol);
  } else {
    chol_rinv_kernel<128><<<1, 1024, 0, st>>>(G, ldg, p, Rinv, ldr, deficient, info, pass, tol, near_tol);
  }
  PFX_HIP(hipGetLastError());
}

static size_t jacobi_base_bytes(int p) {
  const int pe = (p + 1) & ~1;
  const int half = pe / 2;
  const int nblk = half * (half + 1) / 2;
  return (size_t)pe * (pe + 1) * 8 + (size_t)half * 3 * 8 + (size_t)pe * (8 + 4) +
         (size_t)((nblk + 1) & ~1) * 4;
}

size_t jacobi_lds_bytes(int p) {
  const int pe = (p + 1) & ~1;
  const size_t base = jacobi_base_bytes(p);
  const size_t withv = base + (size_t)pe * (pe + 2) * 8;
  return withv <= 160 * 1024 - 256 ? withv : base;   // static LDS: 36 bytes
}

size_t eig_scratch_bytes(int p) {
  return p > 64 ? (size_t)4 * 128 * 129 * sizeof(double) + 256 : 256;
}

void launch_jacobi(const double* H, int ldh, int p, double* theta, double* Z, int ldz,
                   double* Zwork, pf_info* info, int which, int max_sweeps, hipStream_t st, double* escratch,
                   int* refined) {
  const size_t base = jacobi_base_bytes(p);
  const size_t lds = jacobi_lds_bytes(p);
  const bool v_in_lds = lds > base;
  static size_t cur32 = 0, cur64 = 0, cur128 = 0, cur128g = 0, ecur32 = 0, ecur64 = 0;
  // Rayleigh-Ritz: converge to FP64 resolution; pre-rotation: a rotation
  // accurate to 1e-10 keeps every FP32 recurrence column on its direction.
  const double tol_rel = which == 1 ? 1e-15 : 1e-10;
  const int fo = which == 0 ? 1 : 0;
  const int* skip = nullptr;
  if (refined) {
    // quadratically convergent refinement first; the Jacobi kernel below
    // returns at once when it succeeded
    const int iters = 6;
    if (p <= 32) {
      const size_t e = (size_t)4 * 32 * 33 * 8;
      ensure_lds((const void*)eig_refine_kernel<32, true>, e, ecur32);
      eig_refine_kernel<32, true><<<1, 256, e, st>>>(H, ldh, p, theta, Z, ldz, escratch, refined, info, which,
                                                     iters);
    } else if (p <= 64) {
      const size_t e = (size_t)4 * 64 * 65 * 8;
      ensure_lds((const void*)eig_refine_kernel<64, true>, e, ecur64);
      eig_refine_kernel<64, true><<<1, 256, e, st>>>(H, ldh, p, theta, Z, ldz, escratch, refined, info, which,
                                                     iters);
    } else {
      eig_refine_kernel<128, false><<<1, 256, 0, st>>>(H, ldh, p, theta, Z, ldz, escratch, refined, info, which,
                                                       iters);
    }
    PFX_HIP(hipGetLastError());
    skip = refined;
  }
  if (p <= 32) {
    ensure_lds((const void*)jacobi_kernel<32, true>, lds, cur32);
    jacobi_kernel<32, true><<<1, 256, lds, st>>>(H, ldh, p, theta, Z, ldz, Zwork, info, which, max_sweeps,
                                                 tol_rel, fo, skip);
  } else if (p <= 64) {
    ensure_lds((const void*)jacobi_kernel<64, true>, lds, cur64);
    jacobi_kernel<64, true><<<1, 256, lds, st>>>(H, ldh, p, theta, Z, ldz, Zwork, info, which, max_sweeps,
                                                 tol_rel, fo, skip);
  } else if (v_in_lds) {
    ensure_lds((const void*)jacobi_kernel<128, true>, lds, cur128);
    jacobi_kernel<128, true><<<1, 256, lds, st>>>(H, ldh, p, theta, Z, ldz, Zwork, info, which, max_sweeps,
                                                  tol_rel, fo, skip);
  } else {
    ensure_lds((const void*)jacobi_kernel<128, false>, lds, cur128g);
    jacobi_kernel<128, false><<<1, 256, lds, st>>>(H, ldh, p, theta, Z, ldz, Zwork, info, which, max_sweeps,
                                                   tol_rel, fo, skip);
  }
  PFX_HIP(hipGetLastError());
}

}  // namespace pfx
