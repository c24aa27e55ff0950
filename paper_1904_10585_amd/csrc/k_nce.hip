// Kernels of the nearest-correlation PFPG loop (section 5.1): the dual
// gradient from the extracted Ritz pairs, the step on x with the diagonal of
// B(x) = G + Diag(x) rewritten in place, and the extrapolation of
// section 4.3 (Gram of successive differences, combination).  All in FP64;
// every reduction runs in a fixed order, so a run is reproducible.
#include <hip/hip_runtime.h>

#include "pf_internal.h"

namespace pfx {

namespace {

constexpr int kT = 256;

// sum of v over the block, in a fixed tree order; valid in thread 0
__device__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = kT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// g_i = sum_{j < p} max(theta_j, 0) V_ij^2 - 1  (diag(P_+(P_U(B))) - 1,
// eq. NCE-gradient in the extracted subspace); per-block partial sums of
// g_i^2 and x_i.  Skipped (g untouched, partials zero) when the extraction
// reported a numerical failure.
__global__ void nce_grad_kernel(const double* __restrict__ V, int64_t ldv, int p, const double* __restrict__ theta,
                                const double* __restrict__ x, double* __restrict__ g, int64_t n,
                                const pf_info* __restrict__ info, double* __restrict__ partial) {
  __shared__ double sth[128];
  __shared__ double sh[kT];
  const bool ok = info->status == 0;
  for (int j = threadIdx.x; j < p; j += kT) sth[j] = fmax(theta[j], 0.0);
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  double g2 = 0.0, xs = 0.0;
  if (ok && i < n) {
    double d = 0.0;
    for (int j = 0; j < p; ++j) {
      const double v = V[i + (int64_t)j * ldv];
      d = fma(sth[j] * v, v, d);
    }
    const double gi = d - 1.0;
    g[i] = gi;
    g2 = gi * gi;
    xs = x[i];
  }
  g2 = block_sum(g2, sh);
  xs = block_sum(xs, sh);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = g2;
    partial[2 * blockIdx.x + 1] = xs;
  }
}

// stats = (||g||^2, sum x, 1/2 sum max(theta, 0)^2, #{theta > 0}) from the
// block partials, summed in block order
__global__ void nce_stats_kernel(const double* __restrict__ partial, int blocks, const double* __restrict__ theta,
                                 int p, const pf_info* __restrict__ info, double* __restrict__ stats) {
  __shared__ double sh[kT];
  double g2 = 0.0, xs = 0.0, f = 0.0, np = 0.0;
  for (int b = threadIdx.x; b < blocks; b += kT) {
    g2 += partial[2 * b];
    xs += partial[2 * b + 1];
  }
  if (info->status == 0)
    for (int j = threadIdx.x; j < p; j += kT) {
      const double t = theta[j];
      if (t > 0.0) {
        f += 0.5 * t * t;
        np += 1.0;
      }
    }
  g2 = block_sum(g2, sh);
  xs = block_sum(xs, sh);
  f = block_sum(f, sh);
  np = block_sum(np, sh);
  if (threadIdx.x == 0) {
    stats[0] = g2;
    stats[1] = xs;
    stats[2] = f;
    stats[3] = np;
  }
}

// x_i -= tau g_i; B_ii = G_ii + x_i; the new x into column `slot` of the
// extrapolation history (when hist is given)
__global__ void nce_step_kernel(double* __restrict__ x, const double* __restrict__ g, double tau,
                                const double* __restrict__ gd, double* __restrict__ B, int64_t ldb, int64_t n,
                                double* __restrict__ hist, int64_t ldh, int slot) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i >= n) return;
  const double xn = x[i] - tau * g[i];
  x[i] = xn;
  B[i + i * ldb] = gd[i] + xn;
  if (hist) hist[i + (int64_t)slot * ldh] = xn;
}

// gd_i = G_ii; B_ii = G_ii + x_i; hist[:, 0] = x (B already holds G)
__global__ void nce_init_kernel(const double* __restrict__ x, double* __restrict__ gd, double* __restrict__ B,
                                int64_t ldb, int64_t n, double* __restrict__ hist) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i >= n) return;
  const double gi = B[i + i * ldb];
  gd[i] = gi;
  B[i + i * ldb] = gi + x[i];
  if (hist) hist[i] = x[i];
}

// M_ab = sum_i (h_{a+1} - h_a)_i (h_{b+1} - h_b)_i for a <= b < m (one block
// per entry, mirrored), h the history columns
__global__ void nce_diff_gram_kernel(const double* __restrict__ hist, int64_t ldh, int64_t n, int m,
                                     double* __restrict__ M) {
  __shared__ double sh[kT];
  const int a = blockIdx.x, b = blockIdx.y;
  if (a > b) return;                                   // uniform per block
  const double* ha = hist + (int64_t)a * ldh;
  const double* hb = hist + (int64_t)b * ldh;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kT) s = fma(ha[i + ldh] - ha[i], hb[i + ldh] - hb[i], s);
  s = block_sum(s, sh);
  if (threadIdx.x == 0) {
    M[a + b * m] = s;
    M[b + a * m] = s;
  }
}

struct Coef {
  double c[kNceMaxRna + 1];
};

// x = sum_a c_a h_a (a < m); B_ii = G_ii + x_i; hist[:, 0] = x
__global__ void nce_combine_kernel(Coef cf, int m, double* __restrict__ hist, int64_t ldh, double* __restrict__ x,
                                   const double* __restrict__ gd, double* __restrict__ B, int64_t ldb, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i >= n) return;
  double v = 0.0;
  for (int a = 0; a < m; ++a) v = fma(cf.c[a], hist[i + (int64_t)a * ldh], v);
  x[i] = v;
  B[i + i * ldb] = gd[i] + v;
  hist[i] = v;
}

// One DRS step of the PFAM section on the NCE primal, entrywise over the
// n x n matrices (thread i of block (bx, j) takes entry (i, j)):
//   y = 2 P - Z,  prox = (t G + y) / (1 + t) off the diagonal, 1 on it,
//   dZ = prox - P,  Z += dZ,
// P = P_+(P_U(Z)) from the extraction.  Per-block partials: sum dZ^2,
// sum (G - P)^2, max |P_ii - 1|.  Nothing is written when the extraction
// reported a numerical failure.
__global__ void drs_step_kernel(double* __restrict__ Z, int64_t ldz, const double* __restrict__ P, int64_t ldp,
                                const double* __restrict__ G, int64_t ldg, int64_t n, double t,
                                const pf_info* __restrict__ info, double* __restrict__ partial) {
  __shared__ double sh[kT];
  const bool ok = info->status == 0;
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  const int64_t j = blockIdx.y;
  double d2 = 0.0, o2 = 0.0, de = 0.0;
  if (ok && i < n) {
    const double pij = P[i + j * ldp];
    const double z = Z[i + j * ldz];
    const double gij = G[i + j * ldg];
    const double prox = (i == j) ? 1.0 : (t * gij + (2.0 * pij - z)) / (1.0 + t);
    const double dz = prox - pij;
    Z[i + j * ldz] = z + dz;
    d2 = dz * dz;
    o2 = (gij - pij) * (gij - pij);
    if (i == j) de = fabs(pij - 1.0);
  }
  d2 = block_sum(d2, sh);
  o2 = block_sum(o2, sh);
  // max over the block (fixed tree order)
  sh[threadIdx.x] = de;
  __syncthreads();
  for (int s = kT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int64_t b = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    partial[3 * b] = d2;
    partial[3 * b + 1] = o2;
    partial[3 * b + 2] = sh[0];
  }
}

// stats = (sum dZ^2, sum (G - P)^2, max |P_ii - 1|, #{theta > 0}) over the
// block partials, in block order
__global__ void drs_stats_kernel(const double* __restrict__ partial, int64_t blocks, const double* __restrict__ theta,
                                 int p, double* __restrict__ stats) {
  __shared__ double sh[kT];
  double d2 = 0.0, o2 = 0.0, de = 0.0, np = 0.0;
  for (int64_t b = threadIdx.x; b < blocks; b += kT) {
    d2 += partial[3 * b];
    o2 += partial[3 * b + 1];
    de = fmax(de, partial[3 * b + 2]);
  }
  for (int j = threadIdx.x; j < p; j += kT) np += theta[j] > 0.0 ? 1.0 : 0.0;
  d2 = block_sum(d2, sh);
  o2 = block_sum(o2, sh);
  np = block_sum(np, sh);
  sh[threadIdx.x] = de;
  __syncthreads();
  for (int s = kT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    stats[0] = d2;
    stats[1] = o2;
    stats[2] = sh[0];
    stats[3] = np;
  }
}

unsigned blocks_of(int64_t n) { return (unsigned)((n + kT - 1) / kT); }

}  // namespace

int64_t drs_partial_blocks(int64_t n) { return (int64_t)blocks_of(n) * n; }

void launch_drs_step(double* Z, int64_t ldz, const double* P, int64_t ldp, const double* G, int64_t ldg, int64_t n,
                     double t, const pf_info* info, const double* theta, int p, double* partial, double* stats,
                     hipStream_t st) {
  if (n > 65535) fail(PF_ERR_ARG, "drs: n exceeds the grid's y extent");
  drs_step_kernel<<<dim3(blocks_of(n), (unsigned)n), kT, 0, st>>>(Z, ldz, P, ldp, G, ldg, n, t, info, partial);
  PFX_HIP(hipGetLastError());
  drs_stats_kernel<<<1, kT, 0, st>>>(partial, drs_partial_blocks(n), theta, p, stats);
  PFX_HIP(hipGetLastError());
}

int nce_partial_blocks(int64_t n) { return (int)blocks_of(n); }

void launch_nce_init(const double* x, double* gd, double* B, int64_t ldb, int64_t n, double* hist, hipStream_t st) {
  nce_init_kernel<<<blocks_of(n), kT, 0, st>>>(x, gd, B, ldb, n, hist);
  PFX_HIP(hipGetLastError());
}

void launch_nce_grad(const double* V, int64_t ldv, int p, const double* theta, const double* x, double* g, int64_t n,
                     const pf_info* info, double* partial, double* stats, hipStream_t st) {
  if (p < 1 || p > 128) fail(PF_ERR_ARG, "nce: p out of range");
  nce_grad_kernel<<<blocks_of(n), kT, 0, st>>>(V, ldv, p, theta, x, g, n, info, partial);
  PFX_HIP(hipGetLastError());
  nce_stats_kernel<<<1, kT, 0, st>>>(partial, (int)blocks_of(n), theta, p, info, stats);
  PFX_HIP(hipGetLastError());
}

void launch_nce_step(double* x, const double* g, double tau, const double* gd, double* B, int64_t ldb, int64_t n,
                     double* hist, int64_t ldh, int slot, hipStream_t st) {
  nce_step_kernel<<<blocks_of(n), kT, 0, st>>>(x, g, tau, gd, B, ldb, n, hist, ldh, slot);
  PFX_HIP(hipGetLastError());
}

void launch_nce_diff_gram(const double* hist, int64_t ldh, int64_t n, int m, double* M, hipStream_t st) {
  if (m < 1 || m > kNceMaxRna + 1) fail(PF_ERR_ARG, "nce: extrapolation length out of range");
  nce_diff_gram_kernel<<<dim3((unsigned)m, (unsigned)m), kT, 0, st>>>(hist, ldh, n, m, M);
  PFX_HIP(hipGetLastError());
}

void launch_nce_combine(const double* c, int m, double* hist, int64_t ldh, double* x, const double* gd, double* B,
                        int64_t ldb, int64_t n, hipStream_t st) {
  if (m < 1 || m > kNceMaxRna + 1) fail(PF_ERR_ARG, "nce: extrapolation length out of range");
  Coef cf{};
  for (int a = 0; a < m; ++a) cf.c[a] = c[a];
  nce_combine_kernel<<<blocks_of(n), kT, 0, st>>>(cf, m, hist, ldh, x, gd, B, ldb, n);
  PFX_HIP(hipGetLastError());
}

}  // namespace pfx
