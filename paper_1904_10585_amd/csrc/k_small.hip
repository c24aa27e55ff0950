// Small dense p x p kernels of an extraction, one workgroup per matrix, in LDS.
//
//  * chol_rinv: CholeskyQR factor of a Gram matrix G = Y^T Y (the QR of
//    section 2.1 done as G = R^T R, Q = Y R^{-1}): column equilibration
//    D = diag(G)^{-1/2}, Cholesky D G D = L L^T, and R^{-1} = D L^{-T}.
//    A pivot below tol marks the column rank-deficient: it is left out of
//    the elimination and the caller replaces it (see k_block.hip).
//  * eig_refine + syev: symmetric eigendecomposition H = Z diag(theta) Z^T
//    (section 2.2, eq. RR), output sorted by descending theta (the paper's
//    eigenvalue order).  A quadratically convergent refinement solves the
//    nearly diagonal matrices of warm steps; a direct dense solver
//    (tridiagonal reduction, bisection, inverse iteration) takes the rest.
#include "pf_internal.h"
#include "group.h"

#include <cmath>
#include <stdexcept>

namespace pfx {
namespace {

__device__ inline void set_status(pf_info* info, int code) {
  if (info) atomicCAS(&info->status, 0, code);
}

// 1/q for q in a normal range: the hardware estimate refined by two Newton
// steps r += r (1 - q r), each squaring the relative error.
__device__ inline double rcp_nr2(double q) {
  double r = __builtin_amdgcn_rcp(q);
  r = fma(fma(-q, r, 1.0), r, r);
  return fma(fma(-q, r, 1.0), r, r);
}

template <int V>
struct IntC {
  static constexpr int value = V;
};

// f(IntC<K>{}) for K = B .. E - 1 in order.
template <int B, int E, typename F>
__device__ __attribute__((always_inline)) inline void static_for(F& f) {
  if constexpr (B < E) {
    f(IntC<B>{});
    static_for<B + 1, E>(f);
  }
}

// ---------------------------------------------------------------------------
// Cholesky + triangular inverse, register resident.  Thread (bi, bj) of a
// (PMAX/BR) x (PMAX/BC) grid holds the BR x BC blocks (bi, bj) of the equilibrated Gram
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
template <int PMAX, int BR, int BC, bool UNROLL>
__device__ __attribute__((always_inline)) inline void chol_rinv_impl(
    const double* __restrict__ G, int ldg, int p, double* __restrict__ Rinv, int ldr,
    int* __restrict__ deficient, pf_info* info, int pass, double tol, double near_tol) {
  static_assert(BC % BR == 0 && BC % 2 == 0, "a step block spans whole row blocks");
  constexpr int NBR = PMAX / BR, NBC = PMAX / BC;
  constexpr int NT = NBR * NBC;
  __shared__ __align__(16) double s_eq[PMAX], s_piv[PMAX], s_col[2][PMAX], s_row[2][PMAX];
  __shared__ int s_def[PMAX];
  __shared__ int s_bad, s_far;
  const int t = threadIdx.x;
  const int bi = t / NBC, bj = t % NBC;
  const int i0 = BR * bi, j0 = BC * bj;
  if (t == 0) { s_bad = 0; s_far = 0; }
  __syncthreads();

  double g[BR][BC], w[BR][BC];
  bool bad = false;
#pragma unroll
  for (int r = 0; r < BR; ++r)
#pragma unroll
    for (int c = 0; c < BC; ++c) {
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
#pragma unroll
  for (int r = 0; r < BR; ++r)
#pragma unroll
    for (int c = 0; c < BC; ++c)
      if (i0 + r == j0 + c) s_eq[i0 + r] = g[r][c] > 0.0 ? 1.0 / sqrt(g[r][c]) : 0.0;
  __syncthreads();
  if (s_bad) {
    if (t == 0) set_status(info, PF_ERR_NONFINITE);
    for (int idx = t; idx < ldr * ldr; idx += NT) Rinv[idx] = 0.0;
    return;
  }
  double si[BR], sj[BC];
#pragma unroll
  for (int u = 0; u < BR; ++u) si[u] = s_eq[i0 + u];
#pragma unroll
  for (int u = 0; u < BC; ++u) sj[u] = s_eq[j0 + u];
#pragma unroll
  for (int r = 0; r < BR; ++r)
#pragma unroll
    for (int c = 0; c < BC; ++c)
      if (i0 + r < p && j0 + c < p) g[r][c] *= si[r] * sj[c];

  // Second CholeskyQR pass: the equilibrated Gram matrix of an already
  // orthonormalised block is I + E with E small.  To first order
  // chol(I + E) = I + U (U: strict upper part of E, diagonal E_ii / 2) and
  // (I + U)^{-1} = I - U; the neglected terms are O(|E|^2), below the
  // working precision when |E| <= near_tol.
  if (near_tol > 0.0) {
    double dev = 0.0;
#pragma unroll
    for (int r = 0; r < BR; ++r)
#pragma unroll
      for (int c = 0; c < BC; ++c)
        if (i0 + r < p && j0 + c < p) dev = fmax(dev, fabs(g[r][c] - (i0 + r == j0 + c ? 1.0 : 0.0)));
    if (!(dev <= near_tol)) s_far = 1;
    __syncthreads();
    if (!s_far) {
#pragma unroll
      for (int r = 0; r < BR; ++r)
#pragma unroll
        for (int c = 0; c < BC; ++c) {
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

  if constexpr (UNROLL) {
    // Steps k = BC kb + kr, the BC steps of a column block unrolled so that
    // the published register column is a compile-time choice.  Steps past p
    // (fewer than BC) meet the identity padding: unit pivot, zero
    // multipliers, no change.
    const int nkb = (p + BC - 1) / BC;
    for (int kb = 0; kb < nkb; ++kb) {
      const auto step = [&](auto krc) __attribute__((always_inline)) {
        constexpr int kr = decltype(krc)::value;
        constexpr int buf = kr & 1;
        const int k = BC * kb + kr;
        // owners publish column k of G and row k of W
        if (bj == kb) {
#pragma unroll
          for (int r = 0; r < BR; ++r) s_col[buf][i0 + r] = g[r][kr];
        }
        if (bi == k / BR) {
#pragma unroll
          for (int c = 0; c < BC; ++c) s_row[buf][j0 + c] = w[kr % BR][c];
        }
        __syncthreads();
        const double pk = s_col[buf][k];
        double ci[BR], cj[BC], wk[BC];
#pragma unroll
        for (int u = 0; u < BR; ++u) ci[u] = s_col[buf][i0 + u];
#pragma unroll
        for (int u = 0; u < BC; ++u) {
          cj[u] = s_col[buf][j0 + u];
          wk[u] = s_row[buf][j0 + u];
        }
        // a dependent column (equilibrated pivot <= tol; a zero column has
        // pivot 0) is left out of the elimination
        const bool ok = pk > tol;
        if (t == 0) { s_piv[k] = ok ? pk : 1.0; s_def[k] = ok ? 0 : 1; }
        const double inv = ok ? rcp_nr2(pk) : 0.0;
        double li[BR], gj[BC];
#pragma unroll
        for (int u = 0; u < BR; ++u) li[u] = (i0 + u > k) ? ci[u] * inv : 0.0;
#pragma unroll
        for (int u = 0; u < BC; ++u) gj[u] = (j0 + u > k) ? cj[u] : 0.0;
#pragma unroll
        for (int r = 0; r < BR; ++r)
#pragma unroll
          for (int c = 0; c < BC; ++c) {
            g[r][c] -= li[r] * gj[c];
            w[r][c] -= li[r] * wk[c];
          }
        // keep each step's updates inside the step: sunk past the next
        // barrier they keep several steps' multipliers live
        __builtin_amdgcn_sched_barrier(0);
      };
      static_for<0, BC>(step);
    }
  } else {
    // One step per iteration (the unrolled form spills inside the loop at
    // the larger sizes).  k's position in its blocks is uniform: scalar
    // branches pick the published registers.
    for (int k = 0; k < p; ++k) {
      const int buf = k & 1, kbc = k / BC, kc = k % BC, kbr = k / BR, kr = k % BR;
      if (bj == kbc) {
#pragma unroll
        for (int c = 0; c < BC; ++c)
          if (c == kc) {
#pragma unroll
            for (int r = 0; r < BR; ++r) s_col[buf][i0 + r] = g[r][c];
          }
      }
      if (bi == kbr) {
#pragma unroll
        for (int r = 0; r < BR; ++r)
          if (r == kr) {
#pragma unroll
            for (int c = 0; c < BC; ++c) s_row[buf][j0 + c] = w[r][c];
          }
      }
      __syncthreads();
      const double pk = s_col[buf][k];
      double ci[BR], cj[BC], wk[BC];
#pragma unroll
      for (int u = 0; u < BR; ++u) ci[u] = s_col[buf][i0 + u];
#pragma unroll
      for (int u = 0; u < BC; ++u) {
        cj[u] = s_col[buf][j0 + u];
        wk[u] = s_row[buf][j0 + u];
      }
      const bool ok = pk > tol;
      if (t == 0) { s_piv[k] = ok ? pk : 1.0; s_def[k] = ok ? 0 : 1; }
      const double inv = ok ? 1.0 / pk : 0.0;
      double li[BR], gj[BC];
#pragma unroll
      for (int u = 0; u < BR; ++u) li[u] = (i0 + u > k) ? ci[u] * inv : 0.0;
#pragma unroll
      for (int u = 0; u < BC; ++u) gj[u] = (j0 + u > k) ? cj[u] : 0.0;
      // rows of this block all at or above k: nothing left to eliminate
      if (i0 + BR - 1 > k) {
#pragma unroll
        for (int r = 0; r < BR; ++r)
#pragma unroll
          for (int c = 0; c < BC; ++c) {
            g[r][c] -= li[r] * gj[c];
            w[r][c] -= li[r] * wk[c];
          }
      }
    }
  }
  __syncthreads();
  for (int k = t; k < p; k += NT) s_piv[k] = 1.0 / sqrt(s_piv[k]);   // now 1 / sqrt(d_k)
  __syncthreads();

  // R^{-1}[i][j] = s_i W[j][i] / sqrt(d_j) for i <= j: this thread's W block
  // (rows i0.., columns j0..) lands transposed at rows j0.., columns i0..
#pragma unroll
  for (int r = 0; r < BR; ++r)
#pragma unroll
    for (int c = 0; c < BC; ++c) {
      const int wr = i0 + r, wc = j0 + c;          // W[wr][wc] -> Rinv[wc][wr]
      if (wr < p && wc < p && wc < ldr && wr < ldr) {
        double v = 0.0;
        if (wc <= wr) {
          const double s = s_def[wc] ? 1.0 : s_eq[wc];
          v = s * w[r][c] * s_piv[wr];
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
// Dense symmetric eigensolver H = Z diag(theta) Z^T for the p x p matrices of
// an extraction (p <= PMAX <= 128), steps 1-4 below in one workgroup of
// 8 * PMAX threads (p <= 64; at p > 64 step 1 alone, the rest run as the
// kernel chain after RefineK).  It runs where the refinement below cannot
// (cold steps, guard columns whose Ritz values crowd together), so its cost
// does not depend on how far H is from diagonal:
//  1. Householder reduction to tridiagonal T = Q^T H Q (H scaled by a power
//     of two so that max |h_ij| is in [0.5, 1)).  Step k reflects column k
//     with P = I - beta v v^T; the trailing block is updated as
//     A <- A - v w^T - w v^T, y = beta A v, w = y - (beta/2)(v^T y) v.
//     The matrix lives in registers (R8 entries of one row per lane); the
//     reflectors are kept in LDS (in global scratch when SPLIT).
//  2. Eigenvalues of T by bisection on Sturm counts (the number of negative
//     pivots of the LDL^T factorisation of T - x I, pivots kept away from
//     zero by pivmin): one count per thread at 8 PMAX points of the
//     Gershgorin interval brackets every eigenvalue, then eight-way
//     bisection (the eight lanes of a team count at the seven interior
//     points of the bracket, three bits per round).
//  3. Eigenvectors of T by inverse iteration (three solves with the
//     row-pivoted LU of T - lambda I from a fixed pseudo-random start).
//     Eigenvalues closer than 1e-3 ||T|| form a cluster that one team
//     takes in order, orthogonalising each iterate against the cluster's
//     earlier vectors (modified Gram-Schmidt), shifts of coincident
//     eigenvalues separated by 10 eps |lambda|.  A cluster that is an
//     eigenspace to working accuracy (spread <= 1e-13 ||T||, e.g. the null
//     space of a rank-deficient H) shares one shift just above it and is
//     orthogonalised twice per step.
//  4. Z = Q Z_T by applying the reflectors in reverse order.
// Output: theta descending (the paper's order), Z's columns alike; Z holds
// T's eigenvectors between steps 3 and 4, and its rows and columns p..pad-1
// (pad >= p, pad <= ldz) are set to the identity.
__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ inline double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

__device__ inline double wave_min(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}

// Lane moves inside rows of 16 lanes through DPP (a VALU operand modifier,
// no LDS round trip): quad_perm [1,0,3,2] = 0xB1, [2,3,0,1] = 0x4E,
// row_half_mirror = 0x141, row_mirror = 0x140, row_shr:1 = 0x111 (lane i
// takes lane i-1; the first lane of a row gets 0), row_shl:1 = 0x101.
template <int CTRL>
__device__ inline double dpp_mov(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int CTRL>
__device__ inline int dpp_mov_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

// Sums over aligned groups of 8 / 16 lanes and over the wave; every lane of
// the group gets the same value (each step adds commuting pairs).
__device__ inline double sum8(double v) {
  v += dpp_mov<0xB1>(v);
  v += dpp_mov<0x4E>(v);
  v += dpp_mov<0x141>(v);
  return v;
}

__device__ inline double sum16(double v) {
  v = sum8(v);
  v += dpp_mov<0x140>(v);
  return v;
}

template <int LANE>
__device__ inline double read_lane(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), LANE);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), LANE);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ inline double lane0(double v) { return read_lane<0>(v); }

// Sum over the wave (all lanes active): row sums, then row_bcast:15 adds
// row 0 into row 1 and row 2 into row 3 (row mask 0xA), row_bcast:31 adds
// rows 0-1 into rows 2-3 (row mask 0xC); lane 63 holds the total, read
// into a uniform value.
template <int CTRL, int ROWS>
__device__ inline double dpp_rows(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ inline double sum64(double v) {
  v = sum16(v);
  v += dpp_rows<0x142, 0xA>(v);
  v += dpp_rows<0x143, 0xC>(v);
  return read_lane<63>(v);
}

// 1/q: the hardware estimate and one Newton step (r += r (1 - q r)).
__device__ inline double rcp_nr(double q) {
  double r = __builtin_amdgcn_rcp(q);
  return fma(fma(-q, r, 1.0), r, r);
}

// Number of eigenvalues of T below x (Sturm count on the pivots of T - x I).
// The loads of four steps are issued ahead of their recurrence steps.
__device__ inline int sturm_count(const double* d, const double* e2, int p, double x, double pivmin) {
  double q = d[0] - x;
  if (fabs(q) <= pivmin) q = -pivmin;
  int c = q < 0.0;
  int i = 1;
  for (; i + 3 < p; i += 4) {
    double dx[4], f[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      dx[u] = d[i + u] - x;
      f[u] = e2[i + u - 1];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      q = dx[u] - f[u] * rcp_nr(q);
      if (fabs(q) <= pivmin) q = -pivmin;
      c += q < 0.0;
    }
  }
  for (; i < p; ++i) {
    q = (d[i] - x) - e2[i - 1] * rcp_nr(q);
    if (fabs(q) <= pivmin) q = -pivmin;
    c += q < 0.0;
  }
  return c;
}

// Start vector of inverse iteration: entry i of vector j, uniform in (-1, 1)
// from an integer mix of (i, j).
__device__ inline double start_entry(int i, int j) {
  uint32_t h = (uint32_t)i * 0x9E3779B1u + (uint32_t)j * 0x85EBCA77u + 0x165667B1u;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  h *= 0x297A2D39u;
  h ^= h >> 15;
  return (double)h * (2.0 / 4294967296.0) - 1.0;
}

// Cluster of eigenvalue jj of the ascending list lam[0..p): [cs, ce) chained
// by gaps <= 1e-3 ||T||; kind 0 = alone, 1 = loose (every gap >= 1e-11
// ||T||), 2 = tight, 3 = an eigenspace to working accuracy (spread <= 1e-13
// ||T||).
__device__ inline int cluster_kind(const double* lam, int p, double tnorm, int jj, int& cs, int& ce) {
  const double ortol = 1e-3 * tnorm;
  cs = jj;
  while (cs > 0 && !(lam[cs] - lam[cs - 1] > ortol)) --cs;
  ce = jj + 1;
  while (ce < p && !(lam[ce] - lam[ce - 1] > ortol)) ++ce;
  if (ce - cs == 1) return 0;
  if (lam[ce - 1] - lam[cs] <= 1e-13 * tnorm) return 3;
  for (int q = cs + 1; q < ce; ++q)
    if (lam[q] - lam[q - 1] < 1e-11 * tnorm) return 2;
  return 1;
}

// Eigenvector j of the tridiagonal T (diagonal d, off-diagonal e, ascending
// eigenvalues lam) by inverse iteration, for one 16-lane team (PMAX/16 rows
// per lane): two solves with the row-pivoted LU of T - lam_j I from a fixed
// pseudo-random start when lam_j is alone or in a loose cluster (the loose
// flag is raised for the latter); a tight cluster is taken in order by the
// team of its first member, each iterate orthogonalised against the
// cluster's earlier vectors.  The vector goes to column j of Zt (ld ldt).
template <int PMAX>
__device__ __attribute__((always_inline)) inline void invit_team(int j, int p, const double* __restrict__ d,
                                                                const double* __restrict__ e,
                                                                const double* __restrict__ lam, double tnorm,
                                                                double* __restrict__ Zt, int ldt, int* loose) {
  constexpr int R16 = PMAX / 16;
  constexpr double EPS = 2.220446049250313e-16;
  const int part16 = threadIdx.x & 15, r0 = part16 * R16;
  const double tiny = EPS * tnorm;
  double ur[R16], lm[R16], zr[R16];
  unsigned pv = 0;
  double sig = 0.0;
  // row-pivoted LU of T - sig I, rows r0..r0+R16-1 on this lane:
  // ur = 1/u_ii, lm = multiplier, pv = rows i, i+1 swapped.  The rest of U
  // follows from these: u_{i,i+1} = d_{i+1} - sig after a swap, else the
  // running super-diagonal (e_i, or -l_{i-1} e_i after a swap at i-1);
  // u_{i,i+2} = e_{i+1} after a swap, else 0.
  auto factor = [&]() {
    pv = 0;
    double ca = 0.0, cb = 0.0;
#pragma unroll 1
    for (int s = 0; s < 16; ++s) {
      if (part16 == s) {
        double a = s == 0 ? d[0] - sig : ca;
        double b = s == 0 ? (p > 1 ? e[0] : 0.0) : cb;
#pragma unroll
        for (int u = 0; u < R16; ++u) {
          const int i = r0 + u;
          ur[u] = 0.0;
          lm[u] = 0.0;
          if (i < p - 1) {
            const double c = e[i], an = d[i + 1] - sig;
            const double bn = i + 1 < p - 1 ? e[i + 1] : 0.0;
            if (fabs(a) >= fabs(c)) {
              if (fabs(a) <= tiny) a = a >= 0.0 ? tiny : -tiny;
              const double r = rcp_nr(a);
              const double l = c * r;
              ur[u] = r;
              lm[u] = l;
              a = an - l * b;
              b = bn;
            } else {
              const double r = rcp_nr(c);
              const double l = a * r;
              ur[u] = r;
              lm[u] = l;
              pv |= 1u << u;
              a = b - l * an;
              b = -l * bn;
            }
          } else if (i == p - 1) {
            if (fabs(a) <= tiny) a = a >= 0.0 ? tiny : -tiny;
            ur[u] = rcp_nr(a);
          }
        }
        ca = a;
        cb = b;
      }
      ca = dpp_mov<0x111>(ca);                 // lane s+1 receives lane s's state
      cb = dpp_mov<0x111>(cb);
    }
  };
  // zr <- (T - sig I)^{-1} zr with the factors above
  auto solve = [&]() {
    // forward: y = L^{-1} P z (carry w = the running value of z_i)
    const double znext = dpp_mov<0x101>(zr[0]);  // first row of the next lane
    double w = 0.0;
#pragma unroll 1
    for (int s = 0; s < 16; ++s) {
      if (part16 == s) {
        double wi = s == 0 ? zr[0] : w;
#pragma unroll
        for (int u = 0; u < R16; ++u) {
          const int i = r0 + u;
          if (i < p - 1) {
            double zn = u + 1 < R16 ? zr[u + 1] : znext;
            double zi = wi;
            if (pv & (1u << u)) {
              const double tmp = zi;
              zi = zn;
              zn = tmp;
            }
            zr[u] = zi;
            wi = zn - lm[u] * zi;
          } else if (i == p - 1) {
            zr[u] = wi;
          }
        }
        w = wi;
      }
      w = dpp_mov<0x111>(w);
    }
    // back: x_i = (y_i - u2_i x_{i+1} - u3_i x_{i+2}) / u_ii
    const double lprev = dpp_mov<0x111>(lm[R16 - 1]);   // last row of the previous lane
    const unsigned pprev = ((unsigned)dpp_mov_i<0x111>((int)pv) >> (R16 - 1)) & 1u;
    double x1 = 0.0, x2 = 0.0;
#pragma unroll 1
    for (int s = 15; s >= 0; --s) {
      if (part16 == s) {
        double a1 = x1, a2 = x2;
#pragma unroll
        for (int u = R16 - 1; u >= 0; --u) {
          const int i = r0 + u;
          if (i < p) {
            const bool sw = (pv >> u) & 1u;
            const bool swp = u > 0 ? ((pv >> (u - 1)) & 1u) : (i > 0 && pprev);
            const double lp = u > 0 ? lm[u > 0 ? u - 1 : 0] : lprev;
            double u2 = 0.0, u3 = 0.0;
            if (i < p - 1) {
              u2 = sw ? d[i + 1] - sig : (swp ? -lp * e[i] : e[i]);
              if (sw && i + 1 < p - 1) u3 = e[i + 1];
            }
            const double xi = (zr[u] - u2 * a1 - u3 * a2) * ur[u];
            zr[u] = xi;
            a2 = a1;
            a1 = xi;
          }
        }
        x1 = a1;
        x2 = a2;
      }
      x1 = dpp_mov<0x101>(x1);                 // lane s-1 receives lane s's rows
      x2 = dpp_mov<0x101>(x2);
    }
  };
  auto start = [&](int mm, int salt) {
#pragma unroll
    for (int u = 0; u < R16; ++u) zr[u] = r0 + u < p ? start_entry(r0 + u, mm + salt) : 0.0;
  };
  // orthogonalise zr against columns j..mm-1 (modified Gram-Schmidt,
  // `passes` times), then normalise
  auto orthonormalise = [&](int j, int mm, int passes, int it) {
    for (int ps = 0; ps < passes; ++ps) {
      for (int q = j; q < mm; ++q) {
        const double* col = Zt + (int64_t)q * ldt;
        double dot = 0.0;
#pragma unroll
        for (int u = 0; u < R16; ++u)
          if (r0 + u < p) dot += col[r0 + u] * zr[u];
        dot = sum16(dot);
#pragma unroll
        for (int u = 0; u < R16; ++u)
          if (r0 + u < p) zr[u] -= dot * col[r0 + u];
      }
    }
    double ss = 0.0;
#pragma unroll
    for (int u = 0; u < R16; ++u) ss += zr[u] * zr[u];
    ss = sum16(ss);
    if (ss > 0.0 && ss < INFINITY) {
      const double inv = 1.0 / sqrt(ss);
#pragma unroll
      for (int u = 0; u < R16; ++u) zr[u] *= inv;
    } else {
      start(mm, 7919 * (it + 1));
    }
  };
  int cs, ce;
  const int kind = cluster_kind(lam, p, tnorm, j, cs, ce);
  if (kind <= 1) {
    // alone or in a loose cluster: two solves from the exact shift (the
    // loose clusters are orthonormalised together after step 4)
    if (kind == 1) *loose = 1;
    sig = lam[j];
    factor();
    start(j, 0);
    for (int it = 0; it < 2; ++it) {
      solve();
      orthonormalise(j, j, 0, it);
    }
#pragma unroll
    for (int u = 0; u < R16; ++u)
      if (r0 + u < p) Zt[r0 + u + (int64_t)j * ldt] = zr[u];
    return;
  }
  if (j != cs) return;                       // the cluster's first team takes it in order
  // An eigenspace to working accuracy shares one shift just above it:
  // it amplifies the whole eigenspace alike (so successive iterates do
  // not collapse onto one direction) and damps the rest by >= 1e-9 per
  // solve.  A tight cluster uses separated shifts and Gram-Schmidt.
  const bool degen = kind == 3;
  const double spread = lam[ce - 1] - lam[cs];
  double sprev = 0.0;
  for (int mm = cs; mm < ce; ++mm) {
    if (!degen || mm == cs) {
      sig = lam[mm];
      if (degen) sig = lam[ce - 1] + 1e3 * fmax(spread, EPS * tnorm);
      else if (mm > cs && sig - sprev < 10.0 * EPS * fabs(sig)) sig = sprev + 10.0 * EPS * fabs(sig);
      sprev = sig;
      factor();
    }
    start(mm, 0);
    const int nit = degen ? 2 : 3;
    for (int it = 0; it < nit; ++it) {
      solve();
      orthonormalise(cs, mm, degen ? 2 : 1, it);
    }
#pragma unroll
    for (int u = 0; u < R16; ++u)
      if (r0 + u < p) Zt[r0 + u + (int64_t)mm * ldt] = zr[u];
  }
}

// Z <- Q Z for two vectors held by a 16-lane team (rows part16 + 16 u),
// Q = P_0 ... P_{p-3} from the Householder vectors (entry (r, k) of v_k at
// V[r * rs + k * ks], rows k+1..p-1) and their beta.
template <int PMAX>
__device__ __attribute__((always_inline)) inline void reflect_back(double (&z0)[PMAX / 16], double (&z1)[PMAX / 16],
                                                                  int p, const double* __restrict__ V, int rs,
                                                                  int ks, const double* __restrict__ beta) {
  constexpr int R16 = PMAX / 16;
  const int part16 = threadIdx.x & 15;
  // the loads of step k-1 are issued before the arithmetic of step k, and
  // each dot product runs as two interleaved chains
  auto load = [&](int k, double (&av)[R16]) {
#pragma unroll
    for (int u = 0; u < R16; ++u) {
      const int r = part16 + 16 * u;
      av[u] = k >= 0 && r > k && r < p ? V[r * rs + k * ks] : 0.0;
    }
  };
  double av[R16];
  load(p - 3, av);
  for (int k = p - 3; k >= 0; --k) {
    double an[R16];
    load(k - 1, an);
    const double b = beta[k];
    if (b != 0.0) {
      double d0a = 0.0, d0b = 0.0, d1a = 0.0, d1b = 0.0;
#pragma unroll
      for (int u = 0; u < R16; u += 2) {
        d0a = fma(av[u], z0[u], d0a);
        d1a = fma(av[u], z1[u], d1a);
        if (u + 1 < R16) {
          d0b = fma(av[u + 1], z0[u + 1], d0b);
          d1b = fma(av[u + 1], z1[u + 1], d1b);
        }
      }
      const double d0 = b * sum16(d0a + d0b);
      const double d1 = b * sum16(d1a + d1b);
#pragma unroll
      for (int u = 0; u < R16; ++u) {
        z0[u] -= d0 * av[u];
        z1[u] -= d1 * av[u];
      }
    }
#pragma unroll
    for (int u = 0; u < R16; ++u) av[u] = an[u];
  }
}

// Global state of the dense solver when its phases run as separate kernels
// (PMAX = 128): the tridiagonal T, the Householder vectors (column k of V
// holds v_k, ld PMAX), the eigenvalues, T's eigenvectors and a copy for the
// Newton-Schulz steps.
template <int PMAX>
struct SyevScratch {
  double *d, *e, *e2, *beta, *lam, *par, *V, *Zt, *Zp;
  int *done, *loose;
  __device__ explicit SyevScratch(double* g) {
    d = g;
    e = d + PMAX;
    e2 = e + PMAX;
    beta = e2 + PMAX;
    lam = beta + PMAX;
    par = lam + PMAX;                            // Gershgorin lo, hi, pivmin, ||T||, scale
    V = par + 8;
    Zt = V + PMAX * PMAX;
    Zp = Zt + PMAX * PMAX;
    done = reinterpret_cast<int*>(Zp + PMAX * PMAX);
    loose = done + 1;
  }
};
template <int PMAX>
constexpr size_t syev_scratch_bytes() {
  return (size_t)(5 * PMAX + 8 + 3 * PMAX * PMAX) * sizeof(double) + 2 * sizeof(int);
}

// SPLIT: run the load and step 1 only and leave T, the Householder vectors
// and the Gershgorin bracket in the global state at gsc (SyevScratch); the
// other steps then run as separate kernels over many workgroups.
template <int PMAX, bool SPLIT = false>
__device__ __attribute__((always_inline)) inline void syev_impl(const double* __restrict__ H, int ldh, int p,
                                                               double* __restrict__ theta, double* __restrict__ Z,
                                                               int ldz, int pad, pf_info* info, int which,
                                                               const int* skip, double* gsc = nullptr) {
  if (skip && *skip) return;                     // the refinement solved this matrix
  constexpr int NT = 8 * PMAX;
  constexpr int NW = NT / 64;
  constexpr int LDA = PMAX + 1;
  constexpr int R8 = PMAX / 8;                   // rows per lane of an 8-lane team
  constexpr int R16 = PMAX / 16;                 // rows per lane of a 16-lane team
  constexpr double EPS = 2.220446049250313e-16;
  constexpr double SAFMIN = 2.2250738585072014e-308;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* A = reinterpret_cast<double*>(smem_raw);   // Householder vectors: v_k in column k
  // entry `row` of v_k: LDS column k, or column k of the global V
  auto vstore = [&](int row, int k, double v) {
    if constexpr (SPLIT) SyevScratch<PMAX>(gsc).V[k * PMAX + row] = v;
    else A[row * LDA + k] = v;
  };
  __shared__ double s_d[PMAX], s_e[PMAX], s_e2[PMAX], s_beta[PMAX], s_v[PMAX], s_y[PMAX], s_lam[PMAX], s_x[PMAX];
  __shared__ int s_cnt[NT];
  __shared__ double s_red[NW];
  __shared__ double s_par[4];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int team = t >> 3, part = t & 7, base8 = lane & ~7;

  // ---- load sym(H) into registers: lane (row team, part) holds row `team`,
  // columns part, part+8, part+16, ... (interleaved, so that the eight
  // lanes of a team read eight adjacent doubles of v and y, free of LDS
  // bank conflicts); find max |h_ij| and non-finite entries
  auto colj = [&](int u) { return part + 8 * u; };
  double a[R8];
  double amax = 0.0;
  int bad = 0;
#pragma unroll
  for (int u = 0; u < R8; ++u) {
    const int j = colj(u);
    double v = 0.0;
    if (team < p && j < p) {
      v = 0.5 * (H[team + (int64_t)j * ldh] + H[j + (int64_t)team * ldh]);
      bad |= !isfinite(v);
    }
    a[u] = v;
    amax = fmax(amax, fabs(v));
  }
  amax = wave_max(amax);
  if (lane == 0) s_red[wave] = amax;
  bad = __syncthreads_or(bad);
  amax = 0.0;
  for (int w = 0; w < NW; ++w) amax = fmax(amax, s_red[w]);
  if (bad || amax == 0.0) {
    // non-finite input: NaN Ritz values and a reported status; H = 0: zero
    // eigenvalues with the identity as eigenvectors
    for (int idx = t; idx < pad * pad; idx += NT) {
      const int row = idx % pad, col = idx / pad;
      Z[row + (int64_t)col * ldz] = row == col ? 1.0 : 0.0;
    }
    for (int i = t; i < p; i += NT) theta[i] = bad ? __builtin_nan("") : 0.0;
    if (t == 0 && info) {
      if (bad) set_status(info, PF_ERR_NONFINITE);
      if (which == 1) {
        info->n_pos = 0;
        info->dense_rr = 1;
      } else {
        info->dense_pre = 1;
      }
    }
    if constexpr (SPLIT) {
      if (t == 0) *SyevScratch<PMAX>(gsc).done = 1;   // the later kernels return at once
    }
    return;
  }
  int ex;
  (void)frexp(amax, &ex);
  const double scale = ldexp(1.0, ex);           // exact power-of-two scaling
  const double sinv = ldexp(1.0, -ex);
#pragma unroll
  for (int u = 0; u < R8; ++u) a[u] *= sinv;
  // entry (team, col) of this lane's registers, 0 if it holds other columns
  auto entry = [&](int col) {
    double v = 0.0;
#pragma unroll
    for (int u = 0; u < R8; ++u)
      if (colj(u) == col) v = a[u];
    return v;
  };
  if (part == 0 && team < p) s_x[team] = a[0];  // column 0
  __syncthreads();

  // ---- 1. Householder tridiagonalisation ----------------------------------
  // The trailing matrix stays in registers; a step publishes v (s_v), y
  // (s_y) and the next column (s_x) through LDS.  v also goes to column k of
  // the reflector store (vstore), kept for the back-transform.
  for (int k = 0; k + 2 < p; ++k) {
    const int m = p - k - 1;                     // trailing size
    if (wave == 0) {
      const double xa = lane < m ? s_x[k + 1 + lane] : 0.0;
      const double xb = lane + 64 < m ? s_x[k + 1 + lane + 64] : 0.0;
      const double x0 = lane0(xa);
      const double tail = sum64((lane == 0 ? 0.0 : xa * xa) + xb * xb);
      double alpha = x0, beta = 0.0, v0 = x0;
      if (tail != 0.0) {
        const double nrm = sqrt(x0 * x0 + tail);
        alpha = x0 >= 0.0 ? -nrm : nrm;
        beta = 1.0 / (nrm * (nrm + fabs(x0)));
        v0 = x0 - alpha;
      }
      if (lane < m) {
        const double vv = lane == 0 ? v0 : xa;
        s_v[k + 1 + lane] = vv;
        vstore(k + 1 + lane, k, vv);
      }
      if (lane + 64 < m) {
        s_v[k + 65 + lane] = xb;
        vstore(k + 65 + lane, k, xb);
      }
      if (lane == 0) {
        s_d[k] = s_x[k];
        s_e[k] = alpha;
        s_beta[k] = beta;
      }
    }
    __syncthreads();
    const double beta = s_beta[k];
    const bool row_on = team > k && team < p;
    if (beta != 0.0) {
      double vj[R8];
#pragma unroll
      for (int u = 0; u < R8; ++u) {
        const int j = colj(u);
        vj[u] = j > k && j < p ? s_v[j] : 0.0;
      }
      if (row_on) {
        double acc4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int u = 0; u < R8; ++u) acc4[u & 3] += a[u] * vj[u];
        double acc = sum8((acc4[0] + acc4[1]) + (acc4[2] + acc4[3]));
        if (part == 0) s_y[team] = beta * acc;
      }
      __syncthreads();
      double kv = (lane < m ? s_v[k + 1 + lane] * s_y[k + 1 + lane] : 0.0) +
                  (lane + 64 < m ? s_v[k + 65 + lane] * s_y[k + 65 + lane] : 0.0);
      kv = 0.5 * beta * sum64(kv);               // same value in every wave
      if (row_on) {
        // v_i w_j + w_i v_j = v_i y_j + (y_i - 2 kv v_i) v_j
        const double vi = s_v[team], ci = s_y[team] - 2.0 * kv * vi;
#pragma unroll
        for (int u = 0; u < R8; ++u) {
          const int j = colj(u);
          if (j > k && j < p) a[u] -= vi * s_y[j] + ci * vj[u];
        }
      }
    }
    // publish column k+1 (rows k+1.., the diagonal included)
    if (team > k && team < p && ((k + 1) & 7) == part) s_x[team] = entry(k + 1);
    __syncthreads();
  }
  if (team == p - 1 && ((p - 1) & 7) == part) s_d[p - 1] = entry(p - 1);
  if (t == 0) {
    if (p >= 2) {
      s_d[p - 2] = s_x[p - 2];
      s_e[p - 2] = s_x[p - 1];
      s_beta[p - 2] = 0.0;
    }
    s_beta[p - 1] = 0.0;
  }
  __syncthreads();

  // ---- 2. eigenvalues: Gershgorin bracket, coarse counts, 8-way bisection -
  if (wave == 0) {
    double lo = INFINITY, hi = -INFINITY, e2max = 0.0;
    for (int i = lane; i < p; i += 64) {
      const double ea = i > 0 ? fabs(s_e[i - 1]) : 0.0;
      const double eb = i < p - 1 ? fabs(s_e[i]) : 0.0;
      lo = fmin(lo, s_d[i] - ea - eb);
      hi = fmax(hi, s_d[i] + ea + eb);
      if (i < p - 1) {
        const double e2 = s_e[i] * s_e[i];
        s_e2[i] = e2;
        e2max = fmax(e2max, e2);
      }
    }
    lo = wave_min(lo);
    hi = wave_max(hi);
    e2max = wave_max(e2max);
    if (lane == 0) {
      const double tnorm = fmax(fabs(lo), fabs(hi));
      const double pivmin = SAFMIN * fmax(1.0, e2max);
      const double widen = 2.1 * tnorm * EPS * p + 4.2 * pivmin;
      s_par[0] = lo - widen;
      s_par[1] = hi + widen;
      s_par[2] = pivmin;
      s_par[3] = tnorm;
    }
  }
  __syncthreads();
  if constexpr (SPLIT) {
    const SyevScratch<PMAX> sc(gsc);
    for (int i = t; i < p; i += NT) {
      sc.d[i] = s_d[i];
      sc.e[i] = s_e[i];
      sc.e2[i] = s_e2[i];
      sc.beta[i] = s_beta[i];
    }
    if (t < 4) sc.par[t] = s_par[t];
    if (t == 0) {
      sc.par[4] = scale;
      *sc.done = 0;
      *sc.loose = 0;
    }
    return;
  }
  const double pivmin = s_par[2], tnorm = s_par[3];
  // coarse pass: every thread counts at one of NT points splitting the
  // Gershgorin interval into NT + 1 parts
  const double glo = s_par[0], gw = (s_par[1] - s_par[0]) / (double)(NT + 1);
  s_cnt[t] = sturm_count(s_d, s_e2, p, glo + gw * (double)(t + 1), pivmin);
  __syncthreads();
  if (team < p) {
    // the first point with more than `team` eigenvalues below it brackets
    // eigenvalue `team` (counts rise with x)
    int lo_i = 0, hi_i = NT;                     // search [lo_i, hi_i) for that point
    while (lo_i < hi_i) {
      const int mid = (lo_i + hi_i) >> 1;
      if (s_cnt[mid] > team) hi_i = mid;
      else lo_i = mid + 1;
    }
    double lo = lo_i == 0 ? s_par[0] : glo + gw * (double)lo_i;
    double hi = lo_i == NT ? s_par[1] : glo + gw * (double)(lo_i + 1);
    // eight-way bisection: the lanes of a team count at the seven interior
    // points of the bracket
    for (int it = 0; it < 40; ++it) {
      if (hi - lo <= fmax(2.0 * EPS * fmax(fabs(lo), fabs(hi)), EPS * tnorm)) break;
      const double w8 = (hi - lo) * 0.125;
      const int cnt = part < 7 ? sturm_count(s_d, s_e2, p, lo + w8 * (double)(part + 1), pivmin) : p;
      const unsigned bits = (unsigned)(__ballot(cnt > team) >> base8) & 0x7Fu;
      const int first = bits ? __builtin_ctz(bits) : 7;   // point first+1 is the first above
      const double nlo = first == 0 ? lo : lo + w8 * (double)first;
      const double nhi = first == 7 ? hi : lo + w8 * (double)(first + 1);
      lo = nlo;
      hi = nhi;
    }
    if (part == 0) s_lam[team] = 0.5 * (lo + hi);   // ascending
  }
  __syncthreads();

  __shared__ int s_loose;
  if (t == 0) s_loose = 0;
  __syncthreads();

  // ---- 3. inverse iteration: 16-lane teams, two eigenvalues each --------
  for (int pass = 0; pass < 2; ++pass) {
    const int j = (t >> 4) + pass * (PMAX / 2);
    if (j < p) invit_team<PMAX>(j, p, s_d, s_e, s_lam, tnorm, Z, ldz, &s_loose);   // T's eigenvectors go to Z first
  }
  __syncthreads();

  // ---- 4. back-transform Z = Q Z_T, columns in descending order ----------
  // 16-lane teams, columns j0 and j0 + PMAX/2 together; rows r = part16 + 16 u
  {
    const int part16 = t & 15;
    const int j0 = t >> 4, j1 = j0 + PMAX / 2;
    double z0[R16], z1[R16];
#pragma unroll
    for (int u = 0; u < R16; ++u) {
      const int r = part16 + 16 * u;
      z0[u] = j0 < p && r < p ? Z[r + (int64_t)j0 * ldz] : 0.0;
      z1[u] = j1 < p && r < p ? Z[r + (int64_t)j1 * ldz] : 0.0;
    }
    __syncthreads();                             // every column read before any is rewritten
    if (j0 < p) {
      reflect_back<PMAX>(z0, z1, p, A, LDA, 1, s_beta);
#pragma unroll
      for (int u = 0; u < R16; ++u) {
        const int r = part16 + 16 * u;
        if (r < p) {
          Z[r + (int64_t)(p - 1 - j0) * ldz] = z0[u];
          if (j1 < p) Z[r + (int64_t)(p - 1 - j1) * ldz] = z1[u];
        }
      }
      if (part16 == 0) {
        theta[p - 1 - j0] = s_lam[j0] * scale;
        if (j1 < p) theta[p - 1 - j1] = s_lam[j1] * scale;
      }
    }
  }
  // ---- loose clusters: independent inverse iteration leaves inner products
  // of order eps ||T|| / gap between members; two Newton-Schulz steps
  // Z_c <- Z_c (3 I - Z_c^T Z_c) / 2 on the final vectors (Q is orthogonal,
  // so this equals orthonormalising Z_T) make the block orthonormal, the
  // mixing being of the same order, so residuals stay at eps ||T||.  Each
  // step stages Z in the LDS array the reflectors no longer need.
  __syncthreads();
  if (s_loose) {
    const int part16 = t & 15, r0 = part16 * R16;
    for (int ns = 0; ns < 2; ++ns) {
      for (int idx = t; idx < p * p; idx += NT) {
        const int r = idx % p, c = idx / p;
        A[c * LDA + r] = Z[r + (int64_t)c * ldz];
      }
      __syncthreads();
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int j = (t >> 4) + h * (PMAX / 2);
        int cs = 0, ce = 0;
        if (j >= p || cluster_kind(s_lam, p, tnorm, j, cs, ce) != 1) continue;
        const int cj = p - 1 - j;                // final column of eigenvalue j
        double zj[R16], acc[R16];
#pragma unroll
        for (int u = 0; u < R16; ++u) {
          zj[u] = r0 + u < p ? A[cj * LDA + r0 + u] : 0.0;
          acc[u] = 0.0;
        }
        for (int q = p - ce; q < p - cs; ++q) {  // the cluster's final columns
          double zq[R16];
          double dot = 0.0;
#pragma unroll
          for (int u = 0; u < R16; ++u) {
            zq[u] = r0 + u < p ? A[q * LDA + r0 + u] : 0.0;
            dot += zq[u] * zj[u];
          }
          dot = sum16(dot);
#pragma unroll
          for (int u = 0; u < R16; ++u) acc[u] += dot * zq[u];
        }
#pragma unroll
        for (int u = 0; u < R16; ++u)
          if (r0 + u < p) Z[r0 + u + (int64_t)cj * ldz] = 1.5 * zj[u] - 0.5 * acc[u];
      }
      __syncthreads();
    }
  }
  for (int idx = t; idx < pad * pad; idx += NT) {
    const int row = idx % pad, col = idx / pad;
    if (row >= p || col >= p) Z[row + (int64_t)col * ldz] = row == col ? 1.0 : 0.0;
  }
  if (t == 0 && info) {
    if (which == 1) {
      int npos = 0;
      for (int i = 0; i < p; ++i) npos += s_lam[i] > 0.0;
      info->n_pos = npos;
      info->dense_rr = 1;
    } else {
      info->dense_pre = 1;
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
// the dense solver that follows solves H from scratch.  The pre-rotation
// leaves such a pair coupled instead when its two diagonal entries lie
// within 1e-3 ||H||_F: columns with nearly equal Ritz values are amplified
// alike by the filter, so mixing them costs no conditioning, and guard
// columns in the dense unwanted part of the spectrum do crowd together.
// Every product is a
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

// Scratch of a Rayleigh-Ritz eigensolve that the refinement leaves with
// clusters (see eig_refine_impl): the refined basis Zr, the clusters' block
// B (their rows and columns of Zr^T H Zr, entries across clusters zeroed),
// its eigenvectors W and eigenvalues, the Rayleigh quotients of all
// columns, the clustered column indices, a membership flag per column, the
// cluster row count and the refinement's iteration count.  Placed after the
// refinement's own working matrices when those live in global scratch.
template <int PP>
struct ClusterScratch {
  double *Zr, *B, *W, *thc, *diag;
  int *idx, *member, *k, *iters;
  __device__ explicit ClusterScratch(double* g) {
    double* b = g + (PP > 64 ? 4 * PP * (PP + 1) : 0);
    Zr = b;
    B = Zr + PP * PP;
    W = B + PP * PP;
    thc = W + PP * PP;
    diag = thc + PP;
    idx = reinterpret_cast<int*>(diag + PP);
    member = idx + PP;
    k = member + PP;
    iters = k + 1;
  }
};
template <int PP>
constexpr size_t cluster_scratch_bytes() {
  return (PP > 64 ? (size_t)4 * PP * (PP + 1) * sizeof(double) : 0) + (size_t)(3 * PP * PP + 2 * PP) * sizeof(double) +
         (size_t)(2 * PP + 2) * sizeof(int);
}

// The refinement's block size, and its loops over all PP x PP entries with
// the trip count known at compile time, unrolled so that the loads of several
// entries are in flight together (at PP = 128 the matrices live in global
// scratch, where a rolled loop waits for each load in turn).
constexpr int kRefineThreads = 256;
template <int N, int NT, typename F>
__device__ __attribute__((always_inline)) inline void pp_loop(int t, F&& f) {
  static_assert(N % NT == 0, "whole rounds");
#pragma unroll 8
  for (int r = 0; r < N / NT; ++r) f(t + NT * r);
}

template <int PMAX, bool SH>
__device__ __attribute__((always_inline)) inline void eig_refine_impl(const double* __restrict__ H, int ldh, int p,
                                                                     double* __restrict__ theta,
                                                                     double* __restrict__ Z, int ldz,
                                                                     double* __restrict__ gscratch, int* refined,
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
  const int t = threadIdx.x, nt = kRefineThreads;
  const int lane = t & 63, wave = t >> 6;

  double local = 0.0;
  pp_loop<PP * PP, kRefineThreads>(t, [&](int idx) {
    const int i = idx % PP, j = idx / PP;
    double v = 0.0;
    if (i < p && j < p) v = 0.5 * (H[i + (int64_t)j * ldh] + H[j + (int64_t)i * ldh]);   // symmetrise
    Hs[i + j * LD] = v;
    Zc[i + j * LD] = i == j ? 1.0 : 0.0;
    local += v * v;
  });
  local = wave_sum(local);
  if (lane == 0) wsum[wave] = local;
  __syncthreads();
  const double fro = sqrt(wsum[0] + wsum[1] + wsum[2] + wsum[3]);
  // Rayleigh-Ritz: off-diagonal entries below this are at the rounding
  // level of the PP-term FP64 products that form A; the pre-rotation needs
  // each column on its eigen-direction to 1e-10 only
  const double tol = which == 1 ? 64.0 * 2.220446049250313e-16 * fro : 1e-10 * fro;

  __shared__ double s_kmax[4], s_ncp[4];
  __shared__ int s_lab[PMAX], s_cnt[PMAX];
  bool converged = false, clustered = false;
  // Clusters of coupled Ritz values are left to an exact solve of their
  // block where the iterations are cheap (the LDS-resident sizes, p <= 64):
  // at p = 128 the products run from global scratch and the extra
  // iterations cost more than the smaller dense solve saves (measured: the
  // n = 16384, p = 128 precision-form step 5.86 -> 6.49 ms).
  constexpr bool kClusters = PMAX <= 64;
  int it = 0;
  for (;; ++it) {
    if (it == 0) {
      // Z = I: A = H
      pp_loop<PP * PP, kRefineThreads>(t, [&](int idx) {
        const int i = idx % PP, j = idx / PP;
        T2[i + j * LD] = Hs[i + j * LD];
      });
    } else {
      gemm_pp<PP, LD, false>(T1, Hs, Zc, wave, lane);     // T1 = H Z
      __syncthreads();
      gemm_pp<PP, LD, true>(T2, Zc, T1, wave, lane);      // T2 = A = Z^T H Z
    }
    __syncthreads();
    int above = 0, far = 0, coupled = 0;
    double kmax = 0.0;
    if (which == 1 && kClusters) {
      // Rayleigh-Ritz: a pair coupled beyond the first-order range
      // (|a_ij| > 0.01 |a_jj - a_ii|, close Ritz values of guard columns)
      // joins its columns into a cluster (connected components of such
      // pairs); pairs inside a cluster are not rotated, pairs across
      // clusters take the first-order step.  A cluster's block is solved
      // exactly once the rest has converged.
      int ncoupled = 0;
      for (int i = t; i < PMAX; i += nt) s_lab[i] = i;
      __syncthreads();
      for (int idx = t; idx < p * p; idx += nt) {
        const int i = idx % p, j = idx / p;
        if (i == j) continue;
        const double aij = 0.5 * (T2[i + j * LD] + T2[j + i * LD]);
        const double gap = T2[j + j * LD] - T2[i + i * LD];
        if (fabs(aij) > tol && fabs(aij) > 0.01 * fabs(gap)) {
          coupled = 1;
          ++ncoupled;
        }
      }
      coupled = __syncthreads_or(coupled);
      if (coupled) {
        // a Rayleigh-Ritz matrix far from diagonal (a cold step) goes
        // straight to the dense solver rather than to clusters
        if (it == 0) {
          const double nc = wave_sum((double)ncoupled);
          if (lane == 0) s_ncp[wave] = nc;
          __syncthreads();
          far = s_ncp[0] + s_ncp[1] + s_ncp[2] + s_ncp[3] > 0.25 * p * p;
          __syncthreads();
        }
        for (;;) {
          int changed = 0;
          for (int idx = t; idx < p * p; idx += nt) {
            const int i = idx % p, j = idx / p;
            if (i == j) continue;
            const double aij = 0.5 * (T2[i + j * LD] + T2[j + i * LD]);
            const double gap = T2[j + j * LD] - T2[i + i * LD];
            if (fabs(aij) > tol && fabs(aij) > 0.01 * fabs(gap)) {
              const int lj = s_lab[j];
              if (lj < s_lab[i]) {
                atomicMin(&s_lab[i], lj);
                changed = 1;
              }
            }
          }
          if (!__syncthreads_or(changed)) break;
        }
      }
      pp_loop<PP * PP, kRefineThreads>(t, [&](int idx) {
        const int i = idx % PP, j = idx / PP;
        double k = 0.0;
        if (i != j && i < p && j < p && s_lab[i] != s_lab[j]) {
          const double aij = 0.5 * (T2[i + j * LD] + T2[j + i * LD]);
          if (fabs(aij) > tol) {
            k = aij / (T2[j + j * LD] - T2[i + i * LD]);
            above = 1;
          }
        }
        kmax = fmax(kmax, fabs(k));
        T1[i + j * LD] = k;                                // K (antisymmetric)
      });
    } else {
      pp_loop<PP * PP, kRefineThreads>(t, [&](int idx) {
        const int i = idx % PP, j = idx / PP;
        double k = 0.0;
        if (i != j && i < p && j < p) {
          const double aij = 0.5 * (T2[i + j * LD] + T2[j + i * LD]);
          if (fabs(aij) > tol) {
            above = 1;
            const double gap = T2[j + j * LD] - T2[i + i * LD];
            if (fabs(aij) <= 0.01 * fabs(gap)) k = aij / gap;
            else if (!(which == 0 && fabs(gap) <= 1e-3 * fro)) far = 1;   // else: left coupled
          }
        }
        kmax = fmax(kmax, fabs(k));
        T1[i + j * LD] = k;                                // K (antisymmetric)
      });
    }
    kmax = wave_max(kmax);
    if (lane == 0) s_kmax[wave] = kmax;
    above = __syncthreads_or(above);
    far = __syncthreads_or(far);
    kmax = fmax(fmax(s_kmax[0], s_kmax[1]), fmax(s_kmax[2], s_kmax[3]));
    if (far) break;
    if (!above) {
      converged = true;
      clustered = coupled != 0;
      break;
    }
    if (it >= max_iter) break;
    if (which == 0) {
      // pre-rotation: the first-order eigenvectors Z = I + K (invertible, so
      // the span is kept; each column on one eigen-direction to O(K^2)) and
      // second-order eigenvalues theta_i = a_ii + sum_j a_ij K_ji
      pp_loop<PP * PP, kRefineThreads>(t, [&](int idx) {
        const int i = idx % PP, j = idx / PP;
        Zc[i + j * LD] = (i == j ? 1.0 : 0.0) + T1[i + j * LD];
      });
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
    pp_loop<PP * PP, kRefineThreads>(t, [&](int idx) {
      const int i = idx % PP, j = idx / PP;
      T1[i + j * LD] = (i == j ? 1.0 : 0.0) + T1[i + j * LD] + 0.5 * T2[i + j * LD];   // M = I + K + K^2/2
    });
    __syncthreads();
    if (it == 0) {
      // Z = I: Z M = M
      pp_loop<PP * PP, kRefineThreads>(t, [&](int idx) {
        const int i = idx % PP, j = idx / PP;
        T2[i + j * LD] = T1[i + j * LD];
      });
    } else {
      gemm_pp<PP, LD, false>(T2, Zc, T1, wave, lane);     // T2 = Z M
    }
    __syncthreads();
    if (small_k) {
      // M is orthogonal to O(|K|^4) (M^T M = I + K^4 / 4): no re-orthonormalisation
      pp_loop<PP * PP, kRefineThreads>(t, [&](int idx) {
        const int i = idx % PP, j = idx / PP;
        Zc[i + j * LD] = T2[i + j * LD];
      });
      __syncthreads();
      continue;
    }
    gemm_pp<PP, LD, true>(T1, T2, T2, wave, lane);        // T1 = (Z M)^T (Z M)
    __syncthreads();
    pp_loop<PP * PP, kRefineThreads>(t, [&](int idx) {
      const int i = idx % PP, j = idx / PP;
      T1[i + j * LD] = 0.5 * ((i == j ? 3.0 : 0.0) - T1[i + j * LD]);   // (3 I - Z^T Z) / 2
    });
    __syncthreads();
    gemm_pp<PP, LD, false>(Zc, T2, T1, wave, lane);       // Z <- Z M (3 I - ...) / 2
    __syncthreads();
  }
  if (!converged) {
    if (t == 0) *refined = 0;
    return;
  }
  if (clustered) {
    // Columns still coupled above tol form clusters (connected components
    // of the coupled pairs; every other pair of A is below tol).  Their
    // block of A is solved exactly by the dense solver that follows, which
    // then combines: Z = Zr on the other columns, Zr W on the clusters.
    // the clusters are those of the last iteration's classification
    ClusterScratch<PMAX> cs(gscratch);
    for (int i = t; i < PMAX; i += nt) s_cnt[i] = 0;
    __syncthreads();
    for (int i = t; i < p; i += nt) atomicAdd(&s_cnt[s_lab[i]], 1);
    __syncthreads();
    if (t == 0) {
      int k = 0;
      for (int i = 0; i < p; ++i) {
        const int m = s_cnt[s_lab[i]] >= 2;
        cs.member[i] = m;
        if (m) cs.idx[k++] = i;
      }
      *cs.k = k;
      *cs.iters = it;
      s_cnt[0] = k;
    }
    __syncthreads();
    const int k = s_cnt[0];
    for (int idx = t; idx < PMAX * PMAX; idx += nt) {
      const int i = idx % PMAX, j = idx / PMAX;
      cs.Zr[idx] = (i < p && j < p) ? Zc[i + j * LD] : 0.0;
      double b = 0.0;
      if (i < k && j < k) {
        const int r = cs.idx[i], c = cs.idx[j];
        if (s_lab[r] == s_lab[c]) b = i == j ? T2[r + r * LD] : 0.5 * (T2[r + c * LD] + T2[c + r * LD]);
      }
      cs.B[idx] = b;
    }
    for (int i = t; i < p; i += nt) cs.diag[i] = T2[i + i * LD];
    __syncthreads();
    if (t == 0) *refined = 2;
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
        info->dense_rr = 0;
        info->refine_rr = it;
      } else {
        info->dense_pre = 0;
        info->refine_pre = it;
      }
    }
  }
}

struct CholArgs {
  const double* G; int ldg; int p; double* Rinv; int ldr; int* deficient; pf_info* info; int pass;
  double tol, near_tol;
};
template <int PMAX, int BR, int BC, bool UNROLL>
struct CholK {
  using Args = CholArgs;
  static constexpr int kThreads = (PMAX / BR) * (PMAX / BC), kMinWaves = 1;
  static __device__ __attribute__((always_inline)) void body(const Args& a, uint3) {
    chol_rinv_impl<PMAX, BR, BC, UNROLL>(a.G, a.ldg, a.p, a.Rinv, a.ldr, a.deficient, a.info, a.pass, a.tol,
                                         a.near_tol);
  }
};

struct EigArgs {
  const double* H; int ldh; int p; double* theta; double* Z; int ldz; int pad; double* gscratch; int* refined;
  pf_info* info; int which; int max_iter; const int* skip;
};
// After the dense solve of the clusters' block B = W diag(thc) W^T: the
// Ritz pairs are (diag_i, Zr e_i) for the columns outside the clusters and
// (thc_c, Zr[:, idx] W e_c) for the clustered ones, sorted by descending
// value (NaN lowest, ties by position) as the refinement sorts them.
template <int PMAX>
__device__ __attribute__((always_inline)) inline void cluster_combine(const EigArgs& a, const ClusterScratch<PMAX>& cs,
                                                                      int k) {
  const int t = threadIdx.x, nt = blockDim.x;
  const int p = a.p;
  __shared__ double s_eth[PMAX];
  __shared__ int s_src[PMAX], s_rk[PMAX];
  if (t == 0) {
    int e = 0;
    for (int i = 0; i < p; ++i)
      if (!cs.member[i]) {
        s_eth[e] = cs.diag[i];
        s_src[e++] = i;
      }
    for (int c = 0; c < k; ++c) {
      s_eth[e] = cs.thc[c];
      s_src[e++] = -1 - c;
    }
  }
  __syncthreads();
  for (int e = t; e < p; e += nt) {
    const double ke = isnan(s_eth[e]) ? -INFINITY : s_eth[e];
    int rank = 0;
    for (int f = 0; f < p; ++f) {
      const double kf = isnan(s_eth[f]) ? -INFINITY : s_eth[f];
      rank += (kf > ke) || (kf == ke && f < e);
    }
    a.theta[rank] = s_eth[e];
    s_rk[rank] = e;
  }
  __syncthreads();
  for (int idx = t; idx < a.ldz * a.ldz; idx += nt) {
    const int row = idx % a.ldz, col = idx / a.ldz;
    double v = row == col ? 1.0 : 0.0;
    if (row < p && col < p) {
      const int src = s_src[s_rk[col]];
      if (src >= 0) {
        v = cs.Zr[row + src * PMAX];
      } else {
        const int c = -1 - src;
        v = 0.0;
        for (int m = 0; m < k; ++m) v = fma(cs.Zr[row + cs.idx[m] * PMAX], cs.W[m + c * PMAX], v);
      }
    }
    a.Z[idx] = v;
  }
  if (t == 0 && a.info) {
    int npos = 0;
    for (int e = 0; e < p; ++e) npos += s_eth[e] > 0.0;
    a.info->n_pos = npos;
    a.info->dense_rr = 1;
    a.info->refine_rr = *cs.iters;
    a.info->dense_rows = k;
  }
}

template <int PMAX>
struct SyevK {
  using Args = EigArgs;
  static constexpr int kThreads = 8 * PMAX, kMinWaves = 1;
  static __device__ __attribute__((always_inline)) void body(const Args& a, uint3) {
    // skip: the refinement's outcome (1: solved; 2: solved but for clusters
    // of coupled columns, whose block this kernel solves; 0 or no
    // refinement: the whole matrix)
    const int state = a.skip ? *a.skip : 0;
    if (state == 1) return;
    const bool cl = state == 2;
    const ClusterScratch<PMAX> cs(a.gscratch);
    const int k = cl ? *cs.k : a.p;
    syev_impl<PMAX>(cl ? cs.B : a.H, cl ? PMAX : a.ldh, k, cl ? cs.thc : a.theta, cl ? cs.W : a.Z,
                    cl ? PMAX : a.ldz, cl ? k : a.pad, cl ? nullptr : a.info, a.which, nullptr);
    if (cl) {
      __syncthreads();
      cluster_combine<PMAX>(a, cs, k);
    }
  }
};

// The dense solver at PMAX = 128 as a chain of kernels.  The reduction to
// tridiagonal form is sequential and stays in one workgroup (SyevTriK);
// everything after it is independent per eigenvalue or per column and runs
// over many workgroups, at the latency of one eigenvalue rather than of all
// of them: the eigenvalues by 65-way multisection (one workgroup each,
// SyevBisK), T's eigenvectors (four 16-lane teams per workgroup, SyevInvK),
// the back-transform (32 columns per workgroup, SyevBackK) and the two
// Newton-Schulz steps of loose clusters (one column per workgroup, from Z
// to a copy and back, SyevNsK), whose second launch also pads Z and fills
// pf_info.  The global state sits after the refinement's scratch.
template <int PMAX>
__device__ inline double* syev_gsc(const EigArgs& a) {
  return a.gscratch + (cluster_scratch_bytes<PMAX>() + 255) / 256 * 256 / sizeof(double);
}
__device__ inline bool syev_skip(const EigArgs& a) { return a.skip && *a.skip; }

template <int PMAX>
struct SyevTriK {
  using Args = EigArgs;
  static constexpr int kThreads = 8 * PMAX, kMinWaves = 1;
  static __device__ __attribute__((always_inline)) void body(const Args& a, uint3) {
    if (syev_skip(a)) return;
    syev_impl<PMAX, true>(a.H, a.ldh, a.p, a.theta, a.Z, a.ldz, a.pad, a.info, a.which, nullptr,
                          syev_gsc<PMAX>(a));
  }
};
template <int PMAX>
struct SyevBisK {
  using Args = EigArgs;
  static constexpr int kThreads = 64, kMinWaves = 1;
  static __device__ __attribute__((always_inline)) void body(const Args& a, uint3 bid) {
    constexpr double EPS = 2.220446049250313e-16;
    if (syev_skip(a)) return;
    const SyevScratch<PMAX> sc(syev_gsc<PMAX>(a));
    const int p = a.p, b = (int)bid.x, t = threadIdx.x;
    if (*sc.done || b >= p) return;
    __shared__ double s_d[PMAX], s_e2[PMAX];
    for (int i = t; i < p; i += 64) {
      s_d[i] = sc.d[i];
      s_e2[i] = sc.e2[i];
    }
    __syncthreads();
    // eigenvalue b (ascending): the 64 lanes count at the 64 interior points
    // of the bracket, which shrinks 65-fold a round from the Gershgorin
    // interval
    double lo = sc.par[0], hi = sc.par[1];
    const double pivmin = sc.par[2], tnorm = sc.par[3];
    for (int it = 0; it < 32; ++it) {
      if (hi - lo <= fmax(2.0 * EPS * fmax(fabs(lo), fabs(hi)), EPS * tnorm)) break;
      const double wq = (hi - lo) * (1.0 / 65.0);
      const int cnt = sturm_count(s_d, s_e2, p, lo + wq * (double)(t + 1), pivmin);
      const unsigned long long bits = __ballot(cnt > b);
      const int first = bits ? __builtin_ctzll(bits) : 64;   // point `first` is the first above
      const double nlo = first == 0 ? lo : lo + wq * (double)first;
      const double nhi = first == 64 ? hi : lo + wq * (double)(first + 1);
      lo = nlo;
      hi = nhi;
    }
    if (t == 0) sc.lam[b] = 0.5 * (lo + hi);
  }
};
template <int PMAX>
struct SyevInvK {
  using Args = EigArgs;
  static constexpr int kThreads = 64, kMinWaves = 1;
  static __device__ __attribute__((always_inline)) void body(const Args& a, uint3 bid) {
    if (syev_skip(a)) return;
    const SyevScratch<PMAX> sc(syev_gsc<PMAX>(a));
    const int p = a.p, t = threadIdx.x;
    if (*sc.done) return;
    __shared__ double s_d[PMAX], s_e[PMAX], s_lam[PMAX];
    for (int i = t; i < p; i += 64) {
      s_d[i] = sc.d[i];
      s_e[i] = sc.e[i];
      s_lam[i] = sc.lam[i];
    }
    __syncthreads();
    const int j = (int)bid.x * 4 + (t >> 4);
    if (j < p) invit_team<PMAX>(j, p, s_d, s_e, s_lam, sc.par[3], sc.Zt, PMAX, sc.loose);
  }
};
template <int PMAX>
struct SyevBackK {
  using Args = EigArgs;
  static constexpr int kThreads = 256, kMinWaves = 1;
  static __device__ __attribute__((always_inline)) void body(const Args& a, uint3 bid) {
    constexpr int R16 = PMAX / 16;
    if (syev_skip(a)) return;
    const SyevScratch<PMAX> sc(syev_gsc<PMAX>(a));
    const int p = a.p, t = threadIdx.x;
    if (*sc.done) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* V = reinterpret_cast<double*>(smem_raw);   // v_k in column k, ld PMAX
    __shared__ double s_beta[PMAX];
    {
      // columns 0..p-3 of V, 16 bytes a lane, eight loads in flight
      const int n2 = (p - 2) * PMAX / 2;
      const double2* src = reinterpret_cast<const double2*>(sc.V);
      double2* dst = reinterpret_cast<double2*>(V);
      for (int i0 = t; i0 < n2; i0 += 8 * kThreads) {
        double2 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int i = i0 + u * kThreads;
          if (i < n2) v[u] = src[i];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int i = i0 + u * kThreads;
          if (i < n2) dst[i] = v[u];
        }
      }
    }
    for (int i = t; i < p; i += kThreads) s_beta[i] = sc.beta[i];
    __syncthreads();
    const int part16 = t & 15;
    const int j0 = (int)bid.x * 32 + (t >> 4), j1 = j0 + 16;
    if (j0 >= p) return;
    double z0[R16], z1[R16];
#pragma unroll
    for (int u = 0; u < R16; ++u) {
      const int r = part16 + 16 * u;
      z0[u] = r < p ? sc.Zt[r + j0 * PMAX] : 0.0;
      z1[u] = j1 < p && r < p ? sc.Zt[r + j1 * PMAX] : 0.0;
    }
    reflect_back<PMAX>(z0, z1, p, V, 1, PMAX, s_beta);
    // columns in descending order of the eigenvalues
#pragma unroll
    for (int u = 0; u < R16; ++u) {
      const int r = part16 + 16 * u;
      if (r < p) {
        a.Z[r + (int64_t)(p - 1 - j0) * a.ldz] = z0[u];
        if (j1 < p) a.Z[r + (int64_t)(p - 1 - j1) * a.ldz] = z1[u];
      }
    }
    if (part16 == 0) {
      const double scale = sc.par[4];
      a.theta[p - 1 - j0] = sc.lam[j0] * scale;
      if (j1 < p) a.theta[p - 1 - j1] = sc.lam[j1] * scale;
    }
  }
};
// One Newton-Schulz step z_j <- (3 z_j - sum_q (z_q . z_j) z_q) / 2 over the
// final columns q of a loose cluster (STEP 0: Z to the copy, 1: back).
template <int PMAX, int STEP>
struct SyevNsK {
  using Args = EigArgs;
  static constexpr int kThreads = 64, kMinWaves = 1;
  static __device__ __attribute__((always_inline)) void body(const Args& a, uint3 bid) {
    constexpr int XR = (PMAX + 63) / 64;
    if (syev_skip(a)) return;
    const SyevScratch<PMAX> sc(syev_gsc<PMAX>(a));
    const int p = a.p, t = threadIdx.x, j = (int)bid.x;
    if (*sc.done) return;
    __shared__ double s_lam[PMAX];
    if (*sc.loose && j < p) {
      for (int i = t; i < p; i += 64) s_lam[i] = sc.lam[i];
      __syncthreads();
      int cs, ce;
      if (cluster_kind(s_lam, p, sc.par[3], j, cs, ce) == 1) {
        const double* src = STEP == 0 ? a.Z : sc.Zp;
        double* dst = STEP == 0 ? sc.Zp : a.Z;
        const int ls = STEP == 0 ? a.ldz : PMAX, ld = STEP == 0 ? PMAX : a.ldz;
        const int cj = p - 1 - j;
        double zj[XR], acc[XR];
#pragma unroll
        for (int x = 0; x < XR; ++x) {
          const int r = t + 64 * x;
          zj[x] = r < p ? src[r + (int64_t)cj * ls] : 0.0;
          acc[x] = 0.0;
        }
        // four cluster columns a round: their loads and sums overlap
        for (int q0 = p - ce; q0 < p - cs; q0 += 4) {
          double zq[4][XR], dot[4];
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const int q = q0 + c;
            dot[c] = 0.0;
#pragma unroll
            for (int x = 0; x < XR; ++x) {
              const int r = t + 64 * x;
              zq[c][x] = q < p - cs && r < p ? src[r + (int64_t)q * ls] : 0.0;
              dot[c] += zq[c][x] * zj[x];
            }
          }
#pragma unroll
          for (int c = 0; c < 4; ++c) dot[c] = sum64(dot[c]);
#pragma unroll
          for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int x = 0; x < XR; ++x) acc[x] += dot[c] * zq[c][x];
        }
#pragma unroll
        for (int x = 0; x < XR; ++x) {
          const int r = t + 64 * x;
          if (r < p) dst[r + (int64_t)cj * ld] = 1.5 * zj[x] - 0.5 * acc[x];
        }
      }
    }
    if (STEP == 1 && bid.x == 0) {
      for (int idx = t; idx < a.pad * a.pad; idx += 64) {
        const int row = idx % a.pad, col = idx / a.pad;
        if (row >= p || col >= p) a.Z[row + (int64_t)col * a.ldz] = row == col ? 1.0 : 0.0;
      }
      if (t == 0 && a.info) {
        if (a.which == 1) {
          int npos = 0;
          for (int i = 0; i < p; ++i) npos += sc.lam[i] > 0.0;
          a.info->n_pos = npos;
          a.info->dense_rr = 1;
        } else {
          a.info->dense_pre = 1;
        }
      }
    }
  }
};
template <int PMAX, bool SH>
struct RefineK {
  using Args = EigArgs;
  static constexpr int kThreads = kRefineThreads, kMinWaves = 1;
  static __device__ __attribute__((always_inline)) void body(const Args& a, uint3) {
    eig_refine_impl<PMAX, SH>(a.H, a.ldh, a.p, a.theta, a.Z, a.ldz, a.gscratch, a.refined, a.info, a.which,
                              a.max_iter);
  }
};

}  // namespace

void launch_chol_rinv(const double* G, int ldg, int p, double* Rinv, int ldr, int* deficient,
                      pf_info* info, int pass, hipStream_t st, double near_tol) {
  // Pivots of the equilibrated Gram are squared sines of the angle between a
  // column and the span of the previous ones.  Below 1e-10 (angle < 1e-5)
  // the column is treated as dependent: CholeskyQR2 reaches working
  // orthogonality only while cond(Y) stays well below 1/sqrt(eps).
  const double tol = 1e-10;
  const CholArgs a{G, ldg, p, Rinv, ldr, deficient, info, pass, tol, near_tol};
  if (p <= 32) {
    emit<CholK<32, 4, 4, true>>(a, dim3(1), 0, st);
  } else if (p <= 64) {
    emit<CholK<64, 4, 4, true>>(a, dim3(1), 0, st);
  } else {
    // 128 registers a lane at 1024 threads: the steps stay rolled (4 x 8
    // blocks on 512 threads were slower, 125 against 113 us, at p = 128)
    emit<CholK<128, 4, 4, false>>(a, dim3(1), 0, st);
  }
}

size_t eig_scratch_bytes(int p) {
  // the refinement's working matrices (p > 64) and the cluster scratch; for
  // p > 64 also the state of the dense solver's kernel chain
  if (p <= 64) return (p <= 32 ? cluster_scratch_bytes<32>() : cluster_scratch_bytes<64>()) + 256;
  return (cluster_scratch_bytes<128>() + 255) / 256 * 256 + syev_scratch_bytes<128>() + 256;
}

void launch_eigh(const double* H, int ldh, int p, double* theta, double* Z, int ldz, int pad, pf_info* info,
                 int which, hipStream_t st, double* escratch, int* refined) {
  EigArgs a{H, ldh, p, theta, Z, ldz, pad, escratch, refined, info, which, 6, nullptr};
  if (refined) {
    // quadratically convergent refinement first; the dense solver below
    // returns at once when it succeeded
    if (p <= 32) emit<RefineK<32, true>>(a, dim3(1), (size_t)4 * 32 * 33 * 8, st);
    else if (p <= 64) emit<RefineK<64, true>>(a, dim3(1), (size_t)4 * 64 * 65 * 8, st);
    else emit<RefineK<128, false>>(a, dim3(1), 0, st);
    a.skip = refined;
  }
  if (p <= 32) {
    emit<SyevK<32>>(a, dim3(1), (size_t)32 * 33 * 8, st);
  } else if (p <= 64) {
    emit<SyevK<64>>(a, dim3(1), (size_t)64 * 65 * 8, st);
  } else {
    if (!escratch) throw std::logic_error("launch_eigh: p > 64 needs the eigensolver scratch");
    emit<SyevTriK<128>>(a, dim3(1), 0, st);
    emit<SyevBisK<128>>(a, dim3(p), 0, st);
    emit<SyevInvK<128>>(a, dim3((p + 3) / 4), 0, st);
    emit<SyevBackK<128>>(a, dim3((p + 31) / 32), (size_t)128 * 128 * 8, st);
    emit<SyevNsK<128, 0>>(a, dim3(p), 0, st);
    emit<SyevNsK<128, 1>>(a, dim3(p), 0, st);
  }
}

}  // namespace pfx
