// Contractions C = alpha * A^T B + beta * D1 + gamma * D2 on gfx950 MFMA.
//
// Used for every product over the long dimension of an extraction:
//  * the Chebyshev filter step Y_{k+1} = (2/e) X Y_k - (2c/e) Y_k - Y_{k-1}
//    (section 2.1 / eq. cheby-recursion-map): A = X (symmetric, so X Y =
//    X^T Y and X is streamed along its contiguous columns), B = Y_k, with
//    the recurrence's axpy fused into the epilogue;
//  * Gram matrices Y^T Y of CholeskyQR and the projected matrix
//    H = Q^T (X Q) of Rayleigh-Ritz (section 2.2, eq. RR).
//
// Layout: A is K x M and B is K x N, column-major.  A workgroup of four
// waves owns a (16*MB) x (16*NB) output tile; the four waves split the
// workgroup's K range and are summed through LDS in a fixed tree order;
// workgroups along grid.z split K further and are summed by a second
// kernel in slab order.  No atomics: results are bitwise reproducible and
// independent of how many other problems share the device.
//
// Each lane loads VEC consecutive K elements of one column of A and of B
// (16-byte loads where both operands are 4-byte).  MFMA j of a step
// consumes element j of every lane, so lane group g (lanes 16g..16g+15)
// contributes K index k0 + VEC*g + j; the same permutation on both
// operands leaves the sum unchanged.
#include "pf_internal.h"
#include "group.h"

#include <algorithm>
#include <type_traits>

namespace pfx {
namespace {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef double d4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;

struct DevArgs {
  const void* A; int64_t lda;
  const void* B; int64_t ldb;
  int64_t K, M, N;
  int64_t kchunk;           // K range of one workgroup (multiple of 4*KSTEP)
  void* out; int64_t ldo;
  const void* D1; int64_t ld1;
  const void* D2; int64_t ld2;
  double alpha, beta, gamma;
  void* part; int64_t ldp;  // split-K slabs, ldp rows each
  int splitk;
  int lower;                // A symmetric, read as L + D/2 from its entries (k, m), k <= m
};

template <typename T, int VEC> struct VecLoad;
template <> struct VecLoad<float, 4> {
  static __device__ inline void go(const float* p, float (&o)[4]) {
    f4v v = *reinterpret_cast<const f4v*>(p);
    o[0] = v[0]; o[1] = v[1]; o[2] = v[2]; o[3] = v[3];
  }
};
template <> struct VecLoad<float, 2> {
  static __device__ inline void go(const float* p, float (&o)[2]) {
    f2v v = *reinterpret_cast<const f2v*>(p);
    o[0] = v[0]; o[1] = v[1];
  }
};
template <> struct VecLoad<double, 2> {
  static __device__ inline void go(const double* p, double (&o)[2]) {
    d2v v = *reinterpret_cast<const d2v*>(p);
    o[0] = v[0]; o[1] = v[1];
  }
};

// Load VEC elements of one column starting at K index kk (already including
// the lane-group offset).  CHECK masks columns past M and rows past K.
template <typename T, int VEC, bool CHECK>
__device__ inline void load_col(const T* col, int64_t kk, int64_t K, bool colok, T (&o)[VEC]) {
  if constexpr (!CHECK) {
    VecLoad<T, VEC>::go(col + kk, o);
  } else {
#pragma unroll
    for (int v = 0; v < VEC; ++v) o[v] = (colok && kk + v < K) ? col[kk + v] : T(0);
  }
}

template <typename TA, typename TB, bool F64, int MB, int NB>
struct Tile {
  static constexpr int VEC = (sizeof(TA) == 8 || sizeof(TB) == 8) ? 2 : 4;
  static constexpr int KSTEP = 4 * VEC;
  using TC = std::conditional_t<F64, double, float>;
  using AccV = std::conditional_t<F64, d4v, f4v>;

  TA ra[MB][VEC];
  TB rb[NB][VEC];

  template <bool CHECK>
  __device__ inline void load(const TA* const (&acol)[MB], const bool (&aok)[MB],
                              const TB* const (&bcol)[NB], int64_t kk, int64_t K) {
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) load_col<TA, VEC, CHECK>(acol[mb], kk, K, aok[mb], ra[mb]);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) load_col<TB, VEC, CHECK>(bcol[nb], kk, K, true, rb[nb]);
  }

  __device__ inline void mma(AccV (&acc)[MB][NB]) const {
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          if constexpr (F64) {
            acc[mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                (double)ra[mb][j], (double)rb[nb][j], acc[mb][nb], 0, 0, 0);
          } else {
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                (float)ra[mb][j], (float)rb[nb][j], acc[mb][nb], 0, 0, 0);
          }
        }
      }
    }
  }
};

// Row (inside a 16x16 block) of accumulator element r held by lane group g.
// f32 MFMA: rows 4g + r, four consecutive rows per lane; f64 MFMA: 4r + g.
template <bool F64>
__device__ inline int acc_row(int g, int r) { return F64 ? (4 * r + g) : (4 * g + r); }

template <typename TA, typename TB, typename TO, bool F64, int MB, int NB>
struct ContractK {
  using Args = DevArgs;
  static constexpr int kThreads = pfx::kThreads, kMinWaves = 1;
  static __device__ __attribute__((always_inline)) void body(const DevArgs& a, uint3 bid);
};

template <typename TA, typename TB, typename TO, bool F64, int MB, int NB>
__device__ void ContractK<TA, TB, TO, F64, MB, NB>::body(const DevArgs& a, uint3 bid) {
  using T = Tile<TA, TB, F64, MB, NB>;
  using TC = typename T::TC;
  using AccV = typename T::AccV;
  constexpr int VEC = T::VEC;
  constexpr int KSTEP = T::KSTEP;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  TC* red = reinterpret_cast<TC*>(smem_raw);   // 2 slots of MB*NB*4*64 values

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int c = lane & 15, g = lane >> 4;
  // a `lower` product's work grows with the row: its heaviest (bottom) row
  // tiles are dispatched first, the light ones fill the end
  const int64_t mtiles = (a.M + 16 * MB - 1) / (16 * MB);
  const int64_t m0 = (a.lower ? mtiles - 1 - (int64_t)bid.x : (int64_t)bid.x) * (16 * MB);
  const int64_t n0 = (int64_t)bid.y * (16 * NB);
  const int s = bid.z;

  // K range of this workgroup.  With `lower` the rows of this tile need K
  // up to the end of its diagonal block only, split evenly over the slabs
  // (the work per tile grows with its row; many tiles per CU even it out).
  int64_t kchunk = a.kchunk, kend_all = a.K;
  if (a.lower) {
    constexpr int64_t unit = (int64_t)kWaves * KSTEP;
    kend_all = min(a.M, m0 + 16 * MB);
    kchunk = ((kend_all + a.splitk - 1) / a.splitk + unit - 1) / unit * unit;
  }
  const int64_t kbeg_wg = (int64_t)s * kchunk;
  const int64_t kend_wg = min(kend_all, kbeg_wg + kchunk);
  const int64_t kw = kchunk / kWaves;
  const int64_t kb = kbeg_wg + (int64_t)wave * kw;
  const int64_t ke_all = min(kend_wg, kb + kw);
  // the diagonal block [m0, m0 + 16 MB) of a `lower` product is weighted
  // entry by entry after the plain steps
  const int64_t ke = a.lower ? min(ke_all, m0) : ke_all;

  const TA* A = static_cast<const TA*>(a.A);
  const TB* B = static_cast<const TB*>(a.B);
  const TA* acol[MB];
  bool aok[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
    const int64_t col = m0 + 16 * mb + c;
    aok[mb] = col < a.M;
    acol[mb] = A + (aok[mb] ? col : 0) * a.lda;
  }
  const TB* bcol[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) bcol[nb] = B + (n0 + 16 * nb + c) * a.ldb;

  AccV acc[MB][NB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = AccV{0, 0, 0, 0};

  const int64_t goff = (int64_t)VEC * g;
  if (kb < ke) {
    // Full steps need no masking when every A column of the tile exists.
    const bool cols_full = (m0 + 16 * MB) <= a.M;
    const int64_t nfull = cols_full ? (ke - kb) / KSTEP : 0;
    const int64_t kfull_end = kb + nfull * KSTEP;
    if (nfull > 0 && F64) {
      // FP64 MFMA (a 16x16x4 step is four times the work of the FP32 one):
      // three fragment sets, the loads of the next two steps in flight
      // during this step's MFMAs (0.115 -> 0.106 ms for the Rayleigh-Ritz
      // product at n = 8192, p = 64); no branch in the loop (loads past the
      // end repeat the last step, in range, and are not used)
      const int64_t klast = kfull_end - KSTEP;
      T t0, t1, t2;
      t0.template load<false>(acol, aok, bcol, kb + goff, a.K);
      t1.template load<false>(acol, aok, bcol, min(kb + KSTEP, klast) + goff, a.K);
      int64_t k = kb;
      for (; k + 3 * KSTEP <= kfull_end; k += 3 * KSTEP) {
        t2.template load<false>(acol, aok, bcol, min(k + 2 * KSTEP, klast) + goff, a.K);
        t0.mma(acc);
        t0.template load<false>(acol, aok, bcol, min(k + 3 * KSTEP, klast) + goff, a.K);
        t1.mma(acc);
        t1.template load<false>(acol, aok, bcol, min(k + 4 * KSTEP, klast) + goff, a.K);
        t2.mma(acc);
      }
      // t0 and t1 hold the (at most two) remaining steps
      if (k < kfull_end) t0.mma(acc);
      if (k + KSTEP < kfull_end) t1.mma(acc);
    } else if (nfull > 0) {
      // two fragment sets, next step's loads in flight during this step's
      // MFMAs (a third set made the FP32 products slower)
      T t0, t1;
      t0.template load<false>(acol, aok, bcol, kb + goff, a.K);
      int64_t k = kb;
      for (; k + 2 * KSTEP <= kfull_end; k += 2 * KSTEP) {
        t1.template load<false>(acol, aok, bcol, k + KSTEP + goff, a.K);
        t0.mma(acc);
        const int64_t k2 = min(k + 2 * KSTEP, kfull_end - KSTEP);
        t0.template load<false>(acol, aok, bcol, k2 + goff, a.K);
        t1.mma(acc);
      }
      if (k < kfull_end) t0.mma(acc);
    }
    for (int64_t k = kfull_end; k < ke; k += KSTEP) {
      T t;
      // mask rows past this wave's range as well as past K
      t.template load<true>(acol, aok, bcol, k + goff, ke);
      t.mma(acc);
    }
  }
  if (a.lower) {
    // entry (k, col) of the diagonal block: weight 1 for k < col, 1/2 on
    // the diagonal, 0 for k > col (exact scalings)
    for (int64_t k = max(kb, m0); k < ke_all; k += KSTEP) {
      T t;
      t.template load<true>(acol, aok, bcol, k + goff, ke_all);
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        const int64_t col = m0 + 16 * mb + c;
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          const int64_t kk = k + goff + v;
          t.ra[mb][v] = kk < col ? t.ra[mb][v] : (kk == col ? t.ra[mb][v] * (TA)0.5 : (TA)0);
        }
      }
      t.mma(acc);
    }
  }

  // Cross-wave sum, fixed order ((w0 + w1) + (w2 + w3)).
  constexpr int SLOT = MB * NB * 4 * 64;
  auto slot_idx = [&](int mb, int nb, int r) { return ((mb * NB + nb) * 4 + r) * 64 + lane; };
  if (wave & 1) {
    TC* dst = red + (wave >> 1) * SLOT;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) dst[slot_idx(mb, nb, r)] = acc[mb][nb][r];
  }
  __syncthreads();
  if (!(wave & 1)) {
    const TC* src = red + (wave >> 1) * SLOT;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[mb][nb][r] += src[slot_idx(mb, nb, r)];
  }
  __syncthreads();
  if (wave == 2) {
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[slot_idx(mb, nb, r)] = acc[mb][nb][r];
  }
  __syncthreads();
  if (wave != 0) return;
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[mb][nb][r] += red[slot_idx(mb, nb, r)];

  // Store: either the final epilogue (single K split) or a partial slab.
  if (a.splitk == 1) {
    TO* out = static_cast<TO*>(a.out);
    const TO* D1 = static_cast<const TO*>(a.D1);
    const TO* D2 = static_cast<const TO*>(a.D2);
    const TC al = (TC)a.alpha, be = (TC)a.beta, ga = (TC)a.gamma;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int64_t col = n0 + 16 * nb + c;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = m0 + 16 * mb + acc_row<F64>(g, r);
          if (row < a.M) {
            TC v = al * acc[mb][nb][r];
            if (D1) v += be * (TC)D1[row + col * a.ld1];
            if (D2) v += ga * (TC)D2[row + col * a.ld2];
            out[row + col * a.ldo] = (TO)v;
          }
        }
      }
  } else {
    TC* part = static_cast<TC*>(a.part) + (int64_t)s * a.ldp * a.N;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int64_t col = n0 + 16 * nb + c;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = m0 + 16 * mb + acc_row<F64>(g, r);
          part[row + col * a.ldp] = acc[mb][nb][r];
        }
      }
  }
}

// out = alpha * sum_s part[s] + beta * D1 + gamma * D2, slabs summed in order.
template <typename TC, typename TO>
struct SplitkReduceK {
  using Args = DevArgs;
  static constexpr int kThreads = 256, kMinWaves = 1;
  static __device__ __attribute__((always_inline)) void body(const DevArgs& a, uint3 bid);
};

template <typename TC, typename TO>
__device__ void SplitkReduceK<TC, TO>::body(const DevArgs& a, uint3 bid) {
  const int64_t i = (int64_t)bid.x * 256 + threadIdx.x;
  const int64_t j = bid.y;
  if (i >= a.M) return;
  const TC* part = static_cast<const TC*>(a.part) + i + j * a.ldp;
  const int64_t slab = a.ldp * a.N;
  // loads of 32 slabs in flight at a time, summed in slab order
  TC sum = TC(0);
  int s = 0;
  for (; s + 32 <= a.splitk; s += 32) {
    TC v[32];
#pragma unroll
    for (int u = 0; u < 32; ++u) v[u] = part[(int64_t)(s + u) * slab];
#pragma unroll
    for (int u = 0; u < 32; ++u) sum = (s + u == 0) ? v[u] : sum + v[u];
  }
  for (; s + 8 <= a.splitk; s += 8) {
    TC v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(s + u) * slab];
#pragma unroll
    for (int u = 0; u < 8; ++u) sum = (s + u == 0) ? v[u] : sum + v[u];
  }
  for (; s < a.splitk; ++s) sum = (s == 0) ? part[0] : sum + part[(int64_t)s * slab];
  TC v = (TC)a.alpha * sum;
  if (a.D1) v += (TC)a.beta * (TC) static_cast<const TO*>(a.D1)[i + j * a.ld1];
  if (a.D2) v += (TC)a.gamma * (TC) static_cast<const TO*>(a.D2)[i + j * a.ld2];
  static_cast<TO*>(a.out)[i + j * a.ldo] = (TO)v;
}

struct Choice {
  int MB, NB, VEC, KSTEP;
  bool f64;
};

Choice choose(Elem ta, Elem tb, bool f64_mfma, int64_t N) {
  Choice ch;
  ch.f64 = f64_mfma || ta == Elem::F64 || tb == Elem::F64;
  ch.NB = (int)(N / 16);
  // FP64 accumulators take twice the registers: half the rows per wave.
  // Wide blocks keep two 16-row blocks as well (one wave per SIMD, 16 MFMA
  // chains): with one, every 16 rows of A re-read the whole K x N block B
  if (ch.f64) ch.MB = 2;
  else ch.MB = ch.NB <= 4 ? 4 : 2;
  ch.VEC = (ta == Elem::F64 || tb == Elem::F64) ? 2 : 4;
  ch.KSTEP = 4 * ch.VEC;
  return ch;
}

struct Split {
  int S;
  int64_t kchunk;
  int64_t ldp;
  int64_t mtiles, ntiles;
};

Split plan_split(const Choice& ch, int64_t K, int64_t M, int64_t N, int requested) {
  Split sp;
  sp.mtiles = (M + 16 * ch.MB - 1) / (16 * ch.MB);
  sp.ntiles = (N + 16 * ch.NB - 1) / (16 * ch.NB);
  const int64_t tiles = sp.mtiles * sp.ntiles;
  const int64_t unit = (int64_t)kWaves * ch.KSTEP;          // kchunk granularity
  // >= 4 steps per wave for wide outputs; a few-tile output (a p x p Gram
  // product) needs many K slabs to occupy the GPU
  const int64_t min_chunk = tiles <= 4 ? unit : unit * 4;
  int64_t S = requested > 0 ? requested : std::max<int64_t>(1, 1024 / std::max<int64_t>(1, tiles));
  S = std::min<int64_t>(S, std::max<int64_t>(1, (K + min_chunk - 1) / min_chunk));
  S = std::max<int64_t>(1, std::min<int64_t>(S, 256));
  int64_t kchunk = round_up((K + S - 1) / S, unit);
  if (kchunk <= 0) kchunk = unit;
  S = std::max<int64_t>(1, (K + kchunk - 1) / kchunk);
  sp.S = (int)S;
  sp.kchunk = kchunk;
  sp.ldp = sp.mtiles * 16 * ch.MB;
  return sp;
}

template <typename TA, typename TB, typename TO, bool F64, int MB, int NB>
void launch_tile(const DevArgs& d, const Split& sp, int prof_main, int prof_reduce, hipStream_t st) {
  using TC = std::conditional_t<F64, double, float>;
  dim3 grid((unsigned)sp.mtiles, (unsigned)sp.ntiles, (unsigned)sp.S);
  const size_t lds = 2 * (size_t)MB * NB * 4 * 64 * sizeof(TC);
  const bool prof = prof_enabled();
  if (prof && prof_main >= 0) prof_begin(prof_main, st);
  emit<ContractK<TA, TB, TO, F64, MB, NB>>(d, grid, lds, st);
  if (prof && prof_main >= 0) prof_end(prof_main, st);
  if (sp.S > 1) {
    dim3 g2((unsigned)((d.M + 255) / 256), (unsigned)d.N);
    if (prof && prof_reduce >= 0) prof_begin(prof_reduce, st);
    emit<SplitkReduceK<TC, TO>>(d, g2, 0, st);
    if (prof && prof_reduce >= 0) prof_end(prof_reduce, st);
  }
}

template <typename TA, typename TB, typename TO, bool F64>
void dispatch_nb(const DevArgs& d, const Split& sp, int NB, int pm, int pr, hipStream_t st) {
  if constexpr (F64) {
    switch (NB) {
      case 1: launch_tile<TA, TB, TO, F64, 2, 1>(d, sp, pm, pr, st); break;
      case 2: launch_tile<TA, TB, TO, F64, 2, 2>(d, sp, pm, pr, st); break;
      case 3: launch_tile<TA, TB, TO, F64, 2, 3>(d, sp, pm, pr, st); break;
      case 4: launch_tile<TA, TB, TO, F64, 2, 4>(d, sp, pm, pr, st); break;
      case 5: launch_tile<TA, TB, TO, F64, 2, 5>(d, sp, pm, pr, st); break;
      case 6: launch_tile<TA, TB, TO, F64, 2, 6>(d, sp, pm, pr, st); break;
      case 7: launch_tile<TA, TB, TO, F64, 2, 7>(d, sp, pm, pr, st); break;
      case 8: launch_tile<TA, TB, TO, F64, 2, 8>(d, sp, pm, pr, st); break;
      default: fail(PF_ERR_UNSUPPORTED, "contract: block width above 128 columns");
    }
    return;
  }
  switch (NB) {
    case 1: launch_tile<TA, TB, TO, F64, 4, 1>(d, sp, pm, pr, st); break;
    case 2: launch_tile<TA, TB, TO, F64, 4, 2>(d, sp, pm, pr, st); break;
    case 3: launch_tile<TA, TB, TO, F64, 4, 3>(d, sp, pm, pr, st); break;
    case 4: launch_tile<TA, TB, TO, F64, 4, 4>(d, sp, pm, pr, st); break;
    case 5: launch_tile<TA, TB, TO, F64, 2, 5>(d, sp, pm, pr, st); break;
    case 6: launch_tile<TA, TB, TO, F64, 2, 6>(d, sp, pm, pr, st); break;
    case 7: launch_tile<TA, TB, TO, F64, 2, 7>(d, sp, pm, pr, st); break;
    case 8: launch_tile<TA, TB, TO, F64, 2, 8>(d, sp, pm, pr, st); break;
    default: fail(PF_ERR_UNSUPPORTED, "contract: block width above 128 columns");
  }
}

}  // namespace

size_t contract_part_bytes(int64_t K, int64_t M, int64_t N, Elem ta, Elem tb, bool f64_mfma, int splitk) {
  Choice ch = choose(ta, tb, f64_mfma, N);
  Split sp = plan_split(ch, K, M, N, splitk);
  if (sp.S <= 1) return 0;
  return (size_t)sp.S * sp.ldp * N * (ch.f64 ? 8 : 4);
}

int contract(const ContractArgs& x, hipStream_t st) {
  if (x.N % 16 != 0 || x.N <= 0 || x.N > 128) fail(PF_ERR_ARG, "contract: N must be 16..128, multiple of 16");
  Choice ch = choose(x.ta, x.tb, x.f64_mfma, x.N);
  Split sp = plan_split(ch, x.K, x.M, x.N, x.splitk);
  const size_t need = sp.S > 1 ? (size_t)sp.S * sp.ldp * x.N * (ch.f64 ? 8 : 4) : 0;
  if (need > x.part_bytes) {
    // fall back to fewer slabs rather than overrun the workspace
    int S = sp.S;
    while (S > 1 && (size_t)S * sp.ldp * x.N * (ch.f64 ? 8 : 4) > x.part_bytes) --S;
    sp = plan_split(ch, x.K, x.M, x.N, S);
  }
  DevArgs d;
  d.A = x.A; d.lda = x.lda; d.B = x.B; d.ldb = x.ldb;
  d.K = x.K; d.M = x.M; d.N = x.N; d.kchunk = sp.kchunk;
  d.out = x.out; d.ldo = x.ldo; d.D1 = x.D1; d.ld1 = x.ld1; d.D2 = x.D2; d.ld2 = x.ld2;
  d.alpha = x.alpha; d.beta = x.beta; d.gamma = x.gamma;
  d.part = x.part; d.ldp = sp.ldp; d.splitk = sp.S;
  d.lower = x.lower ? 1 : 0;
  if (x.lower && x.K != x.M) fail(PF_ERR_ARG, "contract: a lower-triangle product needs a square A");
  const bool of64 = x.to == Elem::F64;
  const int NB = ch.NB;
  if (!ch.f64) {
    if (x.ta != Elem::F32 || x.tb != Elem::F32 || of64) fail(PF_ERR_UNSUPPORTED, "contract: f32 MFMA needs f32 operands/output");
    dispatch_nb<float, float, float, false>(d, sp, NB, x.prof_main, x.prof_reduce, st);
  } else if (x.ta == Elem::F64 && x.tb == Elem::F64) {
    if (!of64) fail(PF_ERR_UNSUPPORTED, "contract: f64 operands need f64 output");
    dispatch_nb<double, double, double, true>(d, sp, NB, x.prof_main, x.prof_reduce, st);
  } else if (x.ta == Elem::F32 && x.tb == Elem::F32) {
    if (of64) {
      dispatch_nb<float, float, double, true>(d, sp, NB, x.prof_main, x.prof_reduce, st);
    } else {
      dispatch_nb<float, float, float, true>(d, sp, NB, x.prof_main, x.prof_reduce, st);
    }
  } else if (x.ta == Elem::F32 && x.tb == Elem::F64) {
    if (!of64) fail(PF_ERR_UNSUPPORTED, "contract: mixed operands need f64 output");
    dispatch_nb<float, double, double, true>(d, sp, NB, x.prof_main, x.prof_reduce, st);
  } else {
    fail(PF_ERR_UNSUPPORTED, "contract: unsupported operand types");
  }
  return sp.S;
}

}  // namespace pfx
