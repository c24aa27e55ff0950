// Tall-skinny block operations of an extraction and the quantisers.
//
//  * apply: C1 = A1 S and C2 = alpha (A2 S) + beta C1 for an n x p block
//    times a p x p FP64 matrix S held in LDS.  Used for the pre-rotation
//    (U W0, X U W0, and the first recurrence step in the same pass), for
//    Q = Y R^{-1} of CholeskyQR (section 2.1), and for the Ritz vectors
//    V = Q Z of eq. RR.  Products and sums in FP64.
//  * quantisers for the low-precision copies of X: BF16 (round to nearest
//    even) and OCP FP8-E4M3FN with one FP32 scale amax/448 per tile,
//    saturating at 448.
//  * psd_dense: P_+ = V_+ diag(theta_+) V_+^T (eq. PFAM1) as a dense matrix.
#include "pf_internal.h"
#include "group.h"

#include <cmath>

namespace pfx {
namespace {

__device__ inline uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// uniform in (0, 1) from 53 random bits
__device__ inline double u01(uint64_t h) { return ((double)(h >> 11) + 0.5) * (1.0 / 9007199254740992.0); }

typedef double d4v __attribute__((ext_vector_type(4)));

// One wave per 16 rows and one 16-column block jb of the result:
// C1[16 x 16] = A1[16 x p] S[:, 16 jb .. 16 jb + 15] with FP64 MFMA 16x16x4
// (lane l holds A1[row0 + l%16][k + l/16] and S[k + l/16][16 jb + l%16];
// the accumulator element r of lane l is row 4r + l/16, column l%16).
// Operands come straight from memory (S and the block are L2-resident);
// every load of a lane is issued before the first product, so one memory
// latency covers the kernel, and the K steps alternate between two
// accumulators to halve the dependent MFMA chain.  Workgroups of one row
// block read the same A rows and write disjoint columns: C must not alias A.
// S may be rectangular (p x q, q output columns), and with D the result is
// C1 = D - A1 S (D may be C1 itself: each element is read, then written, by
// one lane) -- a Gram-Schmidt update Y -= V C in one launch.
template <typename T>
struct ApplyDev {
  int64_t n; int p, q;
  const T* A1; int64_t lda1;
  const T* A2; int64_t lda2;
  const double* S; int lds_;
  T* C1; int64_t ldc1;
  T* C2; int64_t ldc2;
  double alpha, beta;
  const int* deficient;
  const pf_info* gate; pf_info* info_out;
  const double* theta; double* theta_out;
  const T* D; int64_t ldd;
};

template <typename T, int NB, bool TWO>
struct ApplyK {
  using Args = ApplyDev<T>;
  static constexpr int kThreads = 256, kMinWaves = 1;
  static __device__ __attribute__((always_inline)) void body(const Args& a, uint3 bid);
};

template <typename T, int NB, bool TWO>
__device__ void ApplyK<T, NB, TWO>::body(const ApplyDev<T>& a, uint3 bid) {
  const int64_t n = a.n, lda1 = a.lda1, lda2 = a.lda2, ldc1 = a.ldc1, ldc2 = a.ldc2, ldd = a.ldd;
  const int p = a.p, q = a.q, lds_ = a.lds_;
  const T* __restrict__ A1 = a.A1;
  const T* __restrict__ A2 = a.A2;
  const double* __restrict__ S = a.S;
  T* C1 = a.C1;
  T* C2 = a.C2;
  const double alpha = a.alpha, beta = a.beta;
  const int* __restrict__ deficient = a.deficient;
  const pf_info* gate = a.gate;
  pf_info* info_out = a.info_out;
  const double* __restrict__ theta = a.theta;
  double* theta_out = a.theta_out;
  const T* D = a.D;
  constexpr int KS = 4 * NB;                         // K steps of 4 cover the padded width 16 NB
  const int l = threadIdx.x & 63, c = l & 15, g = l >> 4;
  const int64_t row0 = (int64_t)bid.x * 64 + 16 * (threadIdx.x >> 6);
  const int j = 16 * (int)bid.y + c;                 // B column of this lane = its output column
  const int64_t arow = row0 + c;
  const bool rok = arow < n, jok = j < q;
  const int gst = gate ? gate->status : 0;
  const bool defj = deficient && jok && deficient[j];
  double a1[KS], a2[KS], b[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int k = 4 * ks + g;
    const bool kok = k < p;
    a1[ks] = (rok && kok) ? (double)A1[arow + k * lda1] : 0.0;
    if constexpr (TWO) a2[ks] = (rok && kok) ? (double)A2[arow + k * lda2] : 0.0;
    b[ks] = (kok && jok) ? S[k + (int64_t)j * lds_] : 0.0;
  }
  d4v acc1[2] = {d4v{0, 0, 0, 0}, d4v{0, 0, 0, 0}};
  d4v acc2[2] = {d4v{0, 0, 0, 0}, d4v{0, 0, 0, 0}};
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    acc1[ks & 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[ks], b[ks], acc1[ks & 1], 0, 0, 0);
    if constexpr (TWO) acc2[ks & 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2[ks], b[ks], acc2[ks & 1], 0, 0, 0);
  }
  if (gate && bid.x == 0 && bid.y == 0) {
    if (info_out && threadIdx.x == 0) *info_out = *gate;
    if (theta_out && gst == 0)
      for (int i = threadIdx.x; i < p; i += 256) theta_out[i] = theta[i];
  }
  if (gst != 0 || !jok) return;
  const d4v r1 = acc1[0] + acc1[1];
  const d4v r2 = acc2[0] + acc2[1];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t row = row0 + 4 * r + g;
    if (row >= n) continue;
    double v1 = r1[r];
    if (defj) {
      // rank-deficient column: a fixed pseudo-random direction, which the
      // next CholeskyQR pass orthogonalises against the others
      v1 = (2.0 * u01(mix64(((uint64_t)row << 8) ^ (uint64_t)j ^ 0x5DEECE66Dull)) - 1.0) / sqrt((double)n);
    }
    if (D) v1 = (double)D[row + j * ldd] - v1;
    C1[row + j * ldc1] = (T)v1;
    if constexpr (TWO) C2[row + j * ldc2] = (T)(alpha * r2[r] + beta * (double)(T)v1);
  }
}

template <typename T>
__global__ void copy_block_kernel(const T* __restrict__ src, int64_t lds_, T* __restrict__ dst, int64_t ldd,
                                  int64_t n, int p, int64_t n_pad, int p_pad) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= n_pad || j >= p_pad) return;
  dst[i + j * ldd] = (i < n && j < p) ? src[i + j * lds_] : T(0);
}

// out = alpha A + beta D1 + gamma D2 on rows < n (D1, D2 optional): the
// recurrence step around a caller-supplied product A = X Y.
template <typename T>
__global__ void combine_kernel(const T* __restrict__ A, const T* __restrict__ D1, const T* __restrict__ D2, T* out,
                               int64_t ld, int64_t n, int p, double alpha, double beta, double gamma) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= n || j >= p) return;
  const int64_t o = i + j * ld;
  double v = alpha * (double)A[o];
  if (D1) v += beta * (double)D1[o];
  if (D2) v += gamma * (double)D2[o];
  out[o] = (T)v;
}

template <typename T>
struct AxpbyArgs {
  const T* A; const T* B; T* dst; int64_t ld; int64_t n; int p; double alpha, beta;
};
template <typename T>
struct AxpbyK {
  using Args = AxpbyArgs<T>;
  static constexpr int kThreads = 256, kMinWaves = 1;
  static __device__ __attribute__((always_inline)) void body(const Args& a, uint3 bid) {
    const int64_t i = (int64_t)bid.x * 256 + threadIdx.x;
    const int j = bid.y;
    if (i >= a.n || j >= a.p) return;
    const int64_t o = i + j * a.ld;
    a.dst[o] = (T)(a.alpha * (double)a.A[o] + a.beta * (double)a.B[o]);
  }
};

__global__ void info_copy_kernel(const pf_info* src, pf_info* dst, const double* th, double* thd, int p) {
  const int t = threadIdx.x;
  if (dst && t == 0) *dst = *src;
  if (thd && src->status == 0)
    for (int i = t; i < p; i += blockDim.x) thd[i] = th[i];
}

// a step's pf_info to host-visible memory
struct InfoArgs {
  const pf_info* src; pf_info* dst;
};
struct InfoK {
  using Args = InfoArgs;
  static constexpr int kThreads = 64, kMinWaves = 1;
  static __device__ __attribute__((always_inline)) void body(const Args& a, uint3) {
    if (threadIdx.x == 0) *a.dst = *a.src;
  }
};

// Optional outputs of an extraction (residual norms, singular-value
// shrinkage).  Off the hot path: plain one-thread-per-element kernels.
//
// C = D - A S or C = A S for an n x q block C, A n x p (element TA), S p x q
// (FP64), D n x q (FP64, may be C itself: each thread reads and writes only
// its own element of D / C), accumulated in FP64.
template <typename TA, typename TC>
struct RectArgs {
  int64_t n; int p, q;
  const TA* A; int64_t lda;
  const double* S; int64_t lds_;
  const double* D; int64_t ldd;
  TC* C; int64_t ldc;
};
template <typename TA, typename TC>
struct RectK {
  using Args = RectArgs<TA, TC>;
  static constexpr int kThreads = 256, kMinWaves = 1;
  static __device__ __attribute__((always_inline)) void body(const Args& a, uint3 bid) {
    const int64_t i = (int64_t)bid.x * 256 + threadIdx.x;
    const int j = bid.y;
    if (i >= a.n || j >= a.q) return;
    double acc = 0.0;
    for (int k = 0; k < a.p; ++k) acc = fma((double)a.A[i + k * a.lda], a.S[k + j * a.lds_], acc);
    const double r = a.D ? a.D[i + j * a.ldd] - acc : acc;
    a.C[i + j * a.ldc] = (TC)r;
  }
};

// Per Ritz pair j < p: resid[j] = sqrt(z_j^T G z_j) (G = E^T E, so this is
// ||E z_j||), and the shrinkage weights of the Gram form:
// Zs[:, j] = Z[:, j] * max(sigma_j - tau, 0) / sigma_j, sigma_j =
// sqrt(max(theta_j, 0)) (zero when sigma_j = 0).  One workgroup.
struct ExtrasArgs {
  int p; int ld;                 // p x p matrices, leading dimension ld
  const double* Z; const double* G; const double* theta;
  double* resid;                 // may be null
  double tau; double* Zs;        // Zs may be null
};
struct ExtrasK {
  using Args = ExtrasArgs;
  static constexpr int kThreads = 128, kMinWaves = 1;
  static __device__ __attribute__((always_inline)) void body(const Args& a, uint3) {
    for (int j = threadIdx.x; j < a.p; j += 128) {
      const double* z = a.Z + (int64_t)j * a.ld;
      if (a.resid) {
        double s = 0.0;
        for (int c = 0; c < a.p; ++c) {
          double t = 0.0;
          for (int r = 0; r < a.p; ++r) t = fma(a.G[r + (int64_t)c * a.ld], z[r], t);
          s = fma(z[c], t, s);
        }
        a.resid[j] = sqrt(fmax(s, 0.0));
      }
      if (a.Zs) {
        const double sigma = sqrt(fmax(a.theta[j], 0.0));
        const double f = sigma > a.tau ? (sigma - a.tau) / sigma : 0.0;
        for (int r = 0; r < a.p; ++r) a.Zs[r + (int64_t)j * a.ld] = z[r] * f;
      }
    }
  }
};

template <typename T>
__global__ void normal_block_kernel(T* dst, int64_t ld, int64_t n, int p, uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= n) return;
  const uint64_t h1 = mix64(seed ^ mix64(((uint64_t)j << 40) ^ (uint64_t)i));
  const uint64_t h2 = mix64(h1);
  const double r = sqrt(-2.0 * log(u01(h1)));
  dst[i + j * ld] = (T)(r * cos(6.283185307179586 * u01(h2)));   // Box-Muller
}

__device__ inline uint16_t f32_to_bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((u >> 16) | 0x40);   // quiet NaN
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__global__ void quantize_bf16_kernel(const float* __restrict__ src, int64_t rows, int64_t cols, int64_t lds_,
                                     uint16_t* __restrict__ dst, int64_t ldd) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (i >= rows || j >= cols) return;
  dst[i + j * ldd] = f32_to_bf16_rne(src[i + j * lds_]);
}

// Eight consecutive rows of one column per thread: two 16-byte loads and
// one 16-byte store (src and dst 16-byte aligned, lds_ % 4 == 0 and
// ldd % 8 == 0; the last partial group of a column element by element).
typedef float q4v __attribute__((ext_vector_type(4)));
typedef unsigned q4u __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void quantize_bf16_vec_kernel(const float* __restrict__ src, int64_t rows,
                                                                int64_t cols, int64_t lds_,
                                                                uint16_t* __restrict__ dst, int64_t ldd) {
  const int64_t i = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 8;
  const int64_t j = blockIdx.y;
  if (i >= rows || j >= cols) return;
  const float* s = src + i + j * lds_;
  uint16_t* d = dst + i + j * ldd;
  if (i + 8 <= rows) {
    const q4v lo = *reinterpret_cast<const q4v*>(s);
    const q4v hi = *reinterpret_cast<const q4v*>(s + 4);
    q4u w;
    w[0] = f32_to_bf16_rne(lo[0]) | ((unsigned)f32_to_bf16_rne(lo[1]) << 16);
    w[1] = f32_to_bf16_rne(lo[2]) | ((unsigned)f32_to_bf16_rne(lo[3]) << 16);
    w[2] = f32_to_bf16_rne(hi[0]) | ((unsigned)f32_to_bf16_rne(hi[1]) << 16);
    w[3] = f32_to_bf16_rne(hi[2]) | ((unsigned)f32_to_bf16_rne(hi[3]) << 16);
    *reinterpret_cast<q4u*>(d) = w;
  } else {
    for (int64_t r = 0; r < rows - i; ++r) d[r] = f32_to_bf16_rne(s[r]);
  }
}

// E4M3FN code of v (round to nearest even, saturating at 448).
__device__ inline uint8_t f32_to_e4m3(float v) {
  const uint8_t sign = (__float_as_uint(v) >> 31) ? 0x80 : 0x00;
  const float a = fabsf(v);
  uint32_t code;
  if (!(a < 448.0f)) {
    code = 0x7E;                                  // +-448 (NaN inputs saturate too)
  } else if (a < 0.015625f) {                     // below 2^-6: multiples of 2^-9
    code = (uint32_t)rintf(a * 512.0f);           // 8 here is the smallest normal
  } else {
    int e;
    const float m = frexpf(a, &e);                // a = m 2^e, m in [0.5, 1)
    float q = rintf(m * 16.0f);                   // 4 significant bits
    if (q == 16.0f) { q = 8.0f; e += 1; }
    code = (uint32_t)((e + 6) << 3) | (uint32_t)(q - 8.0f);
    if (code > 0x7E) code = 0x7E;
  }
  return (uint8_t)(sign | code);
}

// One workgroup per tile: amax, scale = fp32(amax / 448), codes.
__global__ __launch_bounds__(256) void quantize_fp8_kernel(const float* __restrict__ src, int64_t rows,
                                                           int64_t cols, int64_t lds_, uint8_t* __restrict__ dst,
                                                           int64_t ldd, float* __restrict__ scales, int tile) {
  __shared__ float red[256];
  const int64_t I = blockIdx.x, J = blockIdx.y;
  const int64_t r0 = I * tile, c0 = J * tile;
  const int64_t rn = min((int64_t)tile, rows - r0), cn = min((int64_t)tile, cols - c0);
  float amax = 0.0f;
  for (int64_t e = threadIdx.x; e < rn * cn; e += 256) {
    const int64_t i = r0 + e % rn, j = c0 + e / rn;
    amax = fmaxf(amax, fabsf(src[i + j * lds_]));
  }
  red[threadIdx.x] = amax;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  amax = red[0];
  const float scale = amax > 0.0f ? amax / 448.0f : 1.0f;
  if (threadIdx.x == 0) scales[I + J * gridDim.x] = scale;
  for (int64_t e = threadIdx.x; e < rn * cn; e += 256) {
    const int64_t i = r0 + e % rn, j = c0 + e / rn;
    dst[i + j * ldd] = f32_to_e4m3(src[i + j * lds_] / scale);
  }
}

// out = V_+ diag(theta_+) V_+^T, 64 x 64 output tile per workgroup.
template <typename T>
__global__ __launch_bounds__(256) void psd_dense_kernel(const T* __restrict__ V, int64_t ldv,
                                                        const double* __restrict__ theta, int64_t n, int p,
                                                        T* __restrict__ out, int64_t ldo) {
  __shared__ double Vi[64][33], Vj[64][33];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t i0 = (int64_t)blockIdx.x * 64, j0 = (int64_t)blockIdx.y * 64;
  double acc[4][4] = {};
  for (int k0 = 0; k0 < p; k0 += 32) {
    for (int e = threadIdx.x; e < 64 * 32; e += 256) {
      const int rr = e % 64, kk = e / 64;
      const int k = k0 + kk;
      const double th = (k < p) ? fmax(theta[k], 0.0) : 0.0;
      Vi[rr][kk] = (k < p && i0 + rr < n) ? (double)V[i0 + rr + k * ldv] * th : 0.0;
      Vj[rr][kk] = (k < p && j0 + rr < n) ? (double)V[j0 + rr + k * ldv] : 0.0;
    }
    __syncthreads();
    for (int kk = 0; kk < 32; ++kk)
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) acc[a][b] += Vi[tx + 16 * a][kk] * Vj[ty + 16 * b][kk];
    __syncthreads();
  }
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      const int64_t i = i0 + tx + 16 * a, j = j0 + ty + 16 * b;
      if (i < n && j < n) out[i + j * ldo] = (T)acc[a][b];
    }
}

template <typename T, bool TWO>
void apply_t(const ApplyArgs& a, hipStream_t st) {
  const int nb = (a.p + 15) / 16;
  const int q = a.q > 0 ? a.q : a.p;
  const dim3 grid((unsigned)((a.n + 63) / 64), (unsigned)((q + 15) / 16));
  const T* D = static_cast<const T*>(a.D);
  const T* A1 = static_cast<const T*>(a.A1);
  const T* A2 = static_cast<const T*>(a.A2);
  T* C1 = static_cast<T*>(a.C1);
  T* C2 = static_cast<T*>(a.C2);
  const ApplyDev<T> dv{a.n, a.p, q, A1, a.lda1, A2, a.lda2, a.S, a.lds_, C1, a.ldc1, C2, a.ldc2, a.alpha, a.beta,
                       a.deficient, a.gate, a.info_out, a.theta, a.theta_out, D, a.ldd};
#define PFX_APPLY(NB) emit<ApplyK<T, NB, TWO>>(dv, grid, 0, st)
  switch (nb) {
    case 1: PFX_APPLY(1); break;
    case 2: PFX_APPLY(2); break;
    case 3: PFX_APPLY(3); break;
    case 4: PFX_APPLY(4); break;
    case 5: PFX_APPLY(5); break;
    case 6: PFX_APPLY(6); break;
    case 7: PFX_APPLY(7); break;
    default: PFX_APPLY(8); break;
  }
#undef PFX_APPLY
}

// dst = src^T for a rows x cols column-major matrix (element type T), in
// 64 x 64 tiles through LDS: reads and writes both run along columns.
template <typename T>
__global__ __launch_bounds__(256) void transpose_kernel(const T* __restrict__ src, int64_t lds_, int64_t rows,
                                                        int64_t cols, T* __restrict__ dst, int64_t ldd) {
  __shared__ T tile[64][65];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * 64, j0 = (int64_t)blockIdx.y * 64;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t i = i0 + tx, j = j0 + ty + 4 * r;
    if (i < rows && j < cols) tile[ty + 4 * r][tx] = src[i + j * lds_];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t j = j0 + tx, i = i0 + ty + 4 * r;      // dst row j, column i
    if (i < rows && j < cols) dst[j + i * ldd] = tile[tx][ty + 4 * r];
  }
}

// Block-upper H (m x m, column blocks of s filled in rows 0 .. (j+1)s-1)
// completed to the full symmetric matrix: entries below the diagonal
// blocks take their mirror images.
__global__ void sym_from_block_upper_kernel(double* H, int ldh, int m, int s) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  const int c = blockIdx.y;
  if (r >= m || r / s <= c / s) return;
  H[r + (int64_t)c * ldh] = H[c + (int64_t)r * ldh];
}

// Lanczos outputs from the Ritz values theta (descending, m of them), the
// eigenvectors Z (ld ldz) and the Gram G (s x s) of the residual block:
// the residual of Ritz vector i is ||Wr z_i|| with z_i its last s entries.
__global__ void lanczos_out_kernel(const double* theta, const double* Z, int ldz, int m, int s,
                                   const double* G, const pf_info* info, pf_bounds* out) {
  if (threadIdx.x != 0) return;
  double res[2];
  const int cols[2] = {m - 1, 0};
  for (int t = 0; t < 2; ++t) {
    const double* z = Z + (int64_t)cols[t] * ldz + (m - s);
    double q = 0.0;
    for (int a = 0; a < s; ++a)
      for (int b = 0; b < s; ++b) q += z[a] * G[a + b * s] * z[b];
    res[t] = sqrt(fmax(q, 0.0));
  }
  out->theta_min = theta[m - 1];
  out->theta_max = theta[0];
  out->res_min = res[0];
  out->res_max = res[1];
  out->status = info->status;
  out->replaced = info->deficient;
}

}  // namespace

void launch_apply(const ApplyArgs& a, hipStream_t st) {
  if (a.p <= 0 || a.p > 128) fail(PF_ERR_ARG, "apply: p out of range");
  if (a.ta1 != a.tc1 || (a.A2 && (a.ta2 != a.ta1 || a.tc2 != a.tc1)))
    fail(PF_ERR_UNSUPPORTED, "apply: mixed element types");
  const bool two = a.A2 != nullptr;
  if ((a.info_out || a.theta_out) && !a.gate) fail(PF_ERR_ARG, "apply: output copies need the gate");
  if (a.q < 0 || a.q > 128) fail(PF_ERR_ARG, "apply: q out of range");
  if (a.D && (a.D == a.A1 || a.D == a.A2 || two)) fail(PF_ERR_ARG, "apply: D must not alias an input, nor come with A2");
  // workgroups of one row block share A rows and write disjoint columns
  if (a.C1 == a.A1 || (two && (a.C1 == a.A2 || a.C2 == a.A1 || a.C2 == a.A2)))
    fail(PF_ERR_ARG, "apply: output aliases an input");
  if (a.ta1 == Elem::F64) { if (two) apply_t<double, true>(a, st); else apply_t<double, false>(a, st); }
  else { if (two) apply_t<float, true>(a, st); else apply_t<float, false>(a, st); }
}

void launch_copy_block(const void* src, int64_t lds_, Elem ts, void* dst, int64_t ldd, Elem td, int64_t n,
                       int p, int64_t n_pad, int p_pad, hipStream_t st) {
  if (ts != td) fail(PF_ERR_UNSUPPORTED, "copy_block: element types differ");
  dim3 grid((unsigned)((n_pad + 255) / 256), (unsigned)p_pad);
  if (ts == Elem::F64)
    copy_block_kernel<double><<<grid, 256, 0, st>>>(static_cast<const double*>(src), lds_,
                                                    static_cast<double*>(dst), ldd, n, p, n_pad, p_pad);
  else
    copy_block_kernel<float><<<grid, 256, 0, st>>>(static_cast<const float*>(src), lds_,
                                                   static_cast<float*>(dst), ldd, n, p, n_pad, p_pad);
  PFX_HIP(hipGetLastError());
}

void launch_axpby(const void* A, const void* B, void* dst, int64_t ld, Elem t, int64_t n, int p, double alpha,
                  double beta, hipStream_t st) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)p);
  if (t == Elem::F64) {
    const AxpbyArgs<double> a{static_cast<const double*>(A), static_cast<const double*>(B), static_cast<double*>(dst),
                              ld, n, p, alpha, beta};
    emit<AxpbyK<double>>(a, grid, 0, st);
  } else {
    const AxpbyArgs<float> a{static_cast<const float*>(A), static_cast<const float*>(B), static_cast<float*>(dst), ld,
                             n, p, alpha, beta};
    emit<AxpbyK<float>>(a, grid, 0, st);
  }
}

void launch_rect(int64_t n, int p, int q, const void* A, int64_t lda, Elem ta, const double* S, int64_t lds_,
                 const double* D, int64_t ldd, void* C, int64_t ldc, Elem tc, hipStream_t st) {
  if (n <= 0 || p <= 0 || q <= 0) return;
  const dim3 grid((unsigned)((n + 255) / 256), (unsigned)q);
  if (ta == Elem::F64 && tc == Elem::F64) {
    const RectArgs<double, double> a{n, p, q, static_cast<const double*>(A), lda, S, lds_, D, ldd,
                                     static_cast<double*>(C), ldc};
    emit<RectK<double, double>>(a, grid, 0, st);
  } else if (ta == Elem::F32 && tc == Elem::F64) {
    const RectArgs<float, double> a{n, p, q, static_cast<const float*>(A), lda, S, lds_, D, ldd,
                                    static_cast<double*>(C), ldc};
    emit<RectK<float, double>>(a, grid, 0, st);
  } else if (ta == Elem::F64 && tc == Elem::F32) {
    const RectArgs<double, float> a{n, p, q, static_cast<const double*>(A), lda, S, lds_, D, ldd,
                                    static_cast<float*>(C), ldc};
    emit<RectK<double, float>>(a, grid, 0, st);
  } else {
    fail(PF_ERR_UNSUPPORTED, "rect: element types");
  }
}

void launch_extras(int p, int ld, const double* Z, const double* G, const double* theta, double* resid, double tau,
                   double* Zs, hipStream_t st) {
  const ExtrasArgs a{p, ld, Z, G, theta, resid, tau, Zs};
  emit<ExtrasK>(a, dim3(1), 0, st);
}

void launch_info_to_host(const pf_info* src, pf_info* host_mapped, hipStream_t st) {
  const InfoArgs a{src, host_mapped};
  emit<InfoK>(a, dim3(1), 0, st);
}

void launch_normal_block(void* dst, int64_t ld, Elem t, int64_t n, int p, uint64_t seed, hipStream_t st) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)p);
  if (t == Elem::F64) normal_block_kernel<double><<<grid, 256, 0, st>>>(static_cast<double*>(dst), ld, n, p, seed);
  else normal_block_kernel<float><<<grid, 256, 0, st>>>(static_cast<float*>(dst), ld, n, p, seed);
  PFX_HIP(hipGetLastError());
}

void launch_quantize_bf16(const float* src, int64_t rows, int64_t cols, int64_t lds_, uint16_t* dst,
                          int64_t ldd, hipStream_t st) {
  const bool vec = reinterpret_cast<uintptr_t>(src) % 16 == 0 && reinterpret_cast<uintptr_t>(dst) % 16 == 0 &&
                   lds_ % 4 == 0 && ldd % 8 == 0;
  if (vec) {
    dim3 grid((unsigned)((rows + 2047) / 2048), (unsigned)cols);
    quantize_bf16_vec_kernel<<<grid, 256, 0, st>>>(src, rows, cols, lds_, dst, ldd);
  } else {
    dim3 grid((unsigned)((rows + 255) / 256), (unsigned)cols);
    quantize_bf16_kernel<<<grid, 256, 0, st>>>(src, rows, cols, lds_, dst, ldd);
  }
  PFX_HIP(hipGetLastError());
}

void launch_quantize_fp8(const float* src, int64_t rows, int64_t cols, int64_t lds_, uint8_t* dst,
                         int64_t ldd, float* scales, int tile, hipStream_t st) {
  dim3 grid((unsigned)((rows + tile - 1) / tile), (unsigned)((cols + tile - 1) / tile));
  quantize_fp8_kernel<<<grid, 256, 0, st>>>(src, rows, cols, lds_, dst, ldd, scales, tile);
  PFX_HIP(hipGetLastError());
}

void launch_psd_dense(const void* V, int64_t ldv, Elem t, const double* theta, int64_t n, int p, void* out,
                      int64_t ldo, hipStream_t st) {
  dim3 grid((unsigned)((n + 63) / 64), (unsigned)((n + 63) / 64));
  if (t == Elem::F64)
    psd_dense_kernel<double><<<grid, 256, 0, st>>>(static_cast<const double*>(V), ldv, theta, n, p,
                                                   static_cast<double*>(out), ldo);
  else
    psd_dense_kernel<float><<<grid, 256, 0, st>>>(static_cast<const float*>(V), ldv, theta, n, p,
                                                  static_cast<float*>(out), ldo);
  PFX_HIP(hipGetLastError());
}

void launch_transpose(const void* src, int64_t lds_, int64_t rows, int64_t cols, int esize, void* dst,
                      int64_t ldd, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return;
  dim3 grid((unsigned)((rows + 63) / 64), (unsigned)((cols + 63) / 64));
  switch (esize) {
    case 8:
      transpose_kernel<double><<<grid, 256, 0, st>>>(static_cast<const double*>(src), lds_, rows, cols,
                                                     static_cast<double*>(dst), ldd);
      break;
    case 4:
      transpose_kernel<float><<<grid, 256, 0, st>>>(static_cast<const float*>(src), lds_, rows, cols,
                                                    static_cast<float*>(dst), ldd);
      break;
    case 2:
      transpose_kernel<uint16_t><<<grid, 256, 0, st>>>(static_cast<const uint16_t*>(src), lds_, rows, cols,
                                                       static_cast<uint16_t*>(dst), ldd);
      break;
    default:
      transpose_kernel<uint8_t><<<grid, 256, 0, st>>>(static_cast<const uint8_t*>(src), lds_, rows, cols,
                                                      static_cast<uint8_t*>(dst), ldd);
      break;
  }
  PFX_HIP(hipGetLastError());
}

void launch_sym_from_block_upper(double* H, int ldh, int m, int s, hipStream_t st) {
  dim3 grid((unsigned)((m + 255) / 256), (unsigned)m);
  sym_from_block_upper_kernel<<<grid, 256, 0, st>>>(H, ldh, m, s);
  PFX_HIP(hipGetLastError());
}

void launch_lanczos_out(const double* theta, const double* Z, int ldz, int m, int s, const double* G,
                        const pf_info* info, pf_bounds* out, hipStream_t st) {
  lanczos_out_kernel<<<1, 64, 0, st>>>(theta, Z, ldz, m, s, G, info, out);
  PFX_HIP(hipGetLastError());
}

void launch_combine(const void* A, const void* D1, const void* D2, void* out, int64_t ld, Elem t, int64_t n, int p,
                    double alpha, double beta, double gamma, hipStream_t st) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)p);
  if (t == Elem::F64)
    combine_kernel<double><<<grid, 256, 0, st>>>(static_cast<const double*>(A), static_cast<const double*>(D1),
                                                 static_cast<const double*>(D2), static_cast<double*>(out), ld, n, p,
                                                 alpha, beta, gamma);
  else
    combine_kernel<float><<<grid, 256, 0, st>>>(static_cast<const float*>(A), static_cast<const float*>(D1),
                                                static_cast<const float*>(D2), static_cast<float*>(out), ld, n, p,
                                                alpha, beta, gamma);
  PFX_HIP(hipGetLastError());
}

}  // namespace pfx
