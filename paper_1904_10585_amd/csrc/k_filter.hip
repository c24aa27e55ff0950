// The FP32 filter product on BF16 matrix cores: Y_{k+1} = alpha X Y_k +
// beta Y_k + gamma Y_{k-1} (the Chebyshev recurrence step of section 2.1,
// eq. cheby-recursion-map) with products accurate to FP32.
//
// Every FP32 value splits exactly into three BF16 values by truncation:
// x = x1 + x2 + x3 with x1 the top 8 significand bits, x2 the next 8 and
// x3 the last 8.  X is streamed from HBM as FP32 and split in registers;
// Y_k is read as three BF16 planes written by the previous step.  The
// product keeps the six cross terms of order >= 2^-16,
//   x1 y1 + x1 y2 + x2 y1 + x1 y3 + x2 y2 + x3 y1,
// each exact in the FP32 accumulator of v_mfma_f32_16x16x32_bf16; the
// dropped terms are below 2^-24 relative, the rounding level of FP32.
// This moves the product from the FP32 MFMA rate (which bounds a native
// FP32 product at p = 64 below the HBM roof) to the BF16 rate, so the
// kernel is bound by the HBM stream of X.
//
// Layout: X is K x M column-major and used as X^T (X symmetric).  A
// workgroup of four waves owns 4 * 16 * MB output rows (16 * MB per wave)
// and all 16 * NB columns over a K range; grid.z splits K (summed in slab
// order by a second kernel).  The Y planes of each K step of 32 are staged
// once per workgroup in an LDS ring of four or five stages and shared by the
// four waves.  Lane l holds A[m = l%16][k = 8(l/16) .. +7] (eight consecutive K
// values of one X column: 32 bytes, one cache line per column and step) and
// B[k = 8(l/16) .. +7][n = l%16] (16 bytes of one Y plane column).
#include "pf_internal.h"
#include "group.h"

#include <algorithm>
#include <type_traits>

namespace pfx {
namespace {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));
typedef unsigned int uint2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int KSTEP = 32;

struct FArgs {
  const void* X; int64_t ldx;                          // K x M column-major, element type of XK
  const float* xscale; int64_t ldsc; int tile;         // FP8: one scale per tile x tile block
  const uint16_t* Yp; int64_t ldy; int64_t yplane;   // 3 planes of K x N
  int64_t K, M, N;
  int64_t kchunk;
  float* out; int64_t ldo;
  const float* D1; const float* D2; int64_t ldd;
  float alpha, beta, gamma;
  uint16_t* outp; int64_t ldop; int64_t oplane;       // planes of out (may be null)
  float* part; int64_t ldp;
  int splitk;
};

__device__ inline bf8v as_bf8(u4v v) { return __builtin_bit_cast(bf8v, v); }

// Exact three-way BF16 split of 8 FP32 values, packed two per dword.
__device__ inline void split8(const float (&x)[8], u4v& p1, u4v& p2, u4v& p3) {
  unsigned h[8], m[8], l[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const unsigned u = __float_as_uint(x[i]);
    const unsigned uh = u & 0xFFFF0000u;
    const float r = x[i] - __uint_as_float(uh);
    const unsigned ur = __float_as_uint(r);
    const unsigned um = ur & 0xFFFF0000u;
    const float rl = r - __uint_as_float(um);
    h[i] = uh;
    m[i] = um;
    l[i] = __float_as_uint(rl);
  }
  // v_perm_b32 with selector 0x07060302: low half = upper 16 bits of the
  // first value, high half = upper 16 bits of the second
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    p1[i] = __builtin_amdgcn_perm(h[2 * i + 1], h[2 * i], 0x07060302u);
    p2[i] = __builtin_amdgcn_perm(m[2 * i + 1], m[2 * i], 0x07060302u);
    p3[i] = __builtin_amdgcn_perm(l[2 * i + 1], l[2 * i], 0x07060302u);
  }
}

__device__ inline void split1(float x, uint16_t& a, uint16_t& b, uint16_t& c) {
  const unsigned u = __float_as_uint(x);
  const unsigned uh = u & 0xFFFF0000u;
  const float r = x - __uint_as_float(uh);
  const unsigned ur = __float_as_uint(r);
  const unsigned um = ur & 0xFFFF0000u;
  const float rl = r - __uint_as_float(um);
  a = (uint16_t)(uh >> 16);
  b = (uint16_t)(um >> 16);
  c = (uint16_t)(__float_as_uint(rl) >> 16);
}

__device__ inline void store_out(const FArgs& a, int64_t row, int64_t col, float v) {
  float r = a.alpha * v;
  if (a.D1) r += a.beta * a.D1[row + col * a.ldd];
  if (a.D2) r += a.gamma * a.D2[row + col * a.ldd];
  a.out[row + col * a.ldo] = r;
  if (a.outp) {
    uint16_t p1, p2, p3;
    split1(r, p1, p2, p3);
    uint16_t* o = a.outp + row + col * a.ldop;
    o[0] = p1;
    o[a.oplane] = p2;
    o[2 * a.oplane] = p3;
  }
}

// ---------------------------------------------------------------------------
// Main kernel: a four-stage LDS ring filled by direct global->LDS loads
// (global_load_lds_dwordx4: no VGPRs held by loads in flight, so three
// stages of X and Y stream while one is consumed).  One __shared__ array per
// stage keeps the compiler's LDS-DMA dependency tracking exact.
//
// X element kinds.  F32: split exactly into three BF16 pieces in registers
// (six MFMA cross terms).  BF16: used as stored, against the leading two Y
// planes (two MFMAs): Y is then carried to 16 significand bits (relative
// error below 2^-15), far finer than the 8 bits of X itself.  FP8 (OCP
// E4M3FN): decoded exactly to BF16 in registers, two MFMAs per tile as for
// BF16, then scaled by the FP32 scale of its tile x tile block.
constexpr int XK_F32 = 0, XK_BF16 = 1, XK_FP8 = 2;

// X stage: ROWS columns of X x 32 K values in 16-byte chunks, XCPC chunks
// per column; chunk (col, kc) at col * XCPC + (kc ^ swizzle(col)), the
// swizzle spreading the lanes of one LDS read over the banks.  Y stage:
// YPL planes x N columns x 32 K values, chunk (q, j, kc) at
// ((q * N + j) * 4) + (kc ^ ((j >> 1) & 3)).
template <int XK, int MB, int NB>
struct FCfg {
  static constexpr int ES = XK == XK_F32 ? 4 : XK == XK_BF16 ? 2 : 1;   // bytes per X element
  static constexpr int XCPC = KSTEP * ES / 16;    // X chunks per column and stage
  static constexpr int EPC = 16 / ES;             // X elements per chunk
  static constexpr int ROWS = kWaves * 16 * MB;   // output rows (X columns) per workgroup
  static constexpr int N16 = 16 * NB;
  // Y planes read per stage: all three for an FP32 X (the exact product);
  // the leading two for a BF16 or FP8 X, whose own rounding (2^-9 and
  // below) is far above the 2^-15 that dropping Y's third plane adds
  static constexpr int YPL = XK == XK_F32 ? 3 : 2;
  // LDS ring depth: four 40 KiB stages for an FP32 X, five 32 KiB stages
  // for the smaller two-plane stages of a BF16 or FP8 X (more bytes in
  // flight per CU against the load latency)
  static constexpr int NS = XK == XK_F32 ? 4 : 5;
  static constexpr int XCH = ROWS * XCPC;         // 16-byte X chunks per stage
  static constexpr int YCH = YPL * N16 * 4;       // 16-byte Y chunks per stage
  static constexpr int XOPS = XCH / kThreads;     // X wave-loads per wave per stage
  static_assert(XOPS * kThreads == XCH, "X stage must be a whole number of wave-loads");
  static constexpr int YINSTR = YCH / 64;         // Y wave-loads per workgroup per stage
  static constexpr int YMAX = (YINSTR + kWaves - 1) / kWaves;
  // every wave issues YMAX Y loads; those past YINSTR repeat a valid chunk
  // into padding after the Y chunks, so the issue code has no branch
  static constexpr int STAGE = XCH + kWaves * YMAX * 64;
  static constexpr int OPS = XOPS + YMAX;         // loads each wave issues per stage
  __device__ static int xswz(int col) {
    return XK == XK_F32 ? (col & 7) : XK == XK_BF16 ? ((col >> 1) & 3) : ((col >> 2) & 1);
  }
};

// The four stage buffers are file-scope LDS objects (sized for the largest
// tile): the compiler gives each its own alias scope, so the LDS reads of one
// stage wait only for the direct loads into that stage.
constexpr int kStageChunks = 2560;                 // 40 KiB per stage, 160 KiB for a 4-stage ring
__shared__ u4v g_st0[kStageChunks], g_st1[kStageChunks], g_st2[kStageChunks], g_st3[kStageChunks];
constexpr int kStage5Chunks = 2048;                // 32 KiB per stage, 160 KiB for a 5-stage ring
__shared__ u4v g_sf0[kStage5Chunks], g_sf1[kStage5Chunks], g_sf2[kStage5Chunks], g_sf3[kStage5Chunks],
    g_sf4[kStage5Chunks];

template <int B, int E, typename F>
__device__ __attribute__((always_inline)) inline void unroll_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    unroll_for<B + 1, E>(f);
  }
}

// One 16-byte direct global->LDS load per lane (global_load_lds_dwordx4).
// Kept out of the kernel templates: the builtin exists only for the device.
__device__ inline void dma16(const void* src, u4v* lds) {
  __builtin_amdgcn_global_load_lds(src, lds, 16, 0, 0);
}

// gfx9 s_waitcnt: vmcnt [3:0] + [15:14], expcnt [6:4] = 7 (no wait),
// lgkmcnt [11:8] (15 = no wait)
template <int N, int LGKM = 15>
__device__ inline void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | (0x7 << 4) | (LGKM << 8));
}

__device__ inline void wg_barrier() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

template <int XK, int MB, int NB>
struct FilterK {
  using Args = FArgs;
  static constexpr int kThreads = pfx::kThreads, kMinWaves = 1;
  static __device__ __attribute__((always_inline)) void body(const FArgs& a, uint3 bid);
};

template <int XK, int MB, int NB>
__device__ void FilterK<XK, MB, NB>::body(const FArgs& a, uint3 bid) {
  using C = FCfg<XK, MB, NB>;
  constexpr int NS = C::NS;
  static_assert(C::STAGE <= (NS == 4 ? kStageChunks : kStage5Chunks), "stage does not fit its LDS buffer");
  u4v* slot[NS];
  if constexpr (NS == 4) {
    slot[0] = g_st0; slot[1] = g_st1; slot[2] = g_st2; slot[3] = g_st3;
  } else {
    static_assert(NS == 5, "ring depth");
    slot[0] = g_sf0; slot[1] = g_sf1; slot[2] = g_sf2; slot[3] = g_sf3; slot[4] = g_sf4;
  }
  u4v* const st0 = slot[0];
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int c = lane & 15, g = lane >> 4;
  // XCD-aware tile order: workgroups are dispatched round-robin over the 8
  // XCDs, so the K range (slab) is the fast index and each XCD works on few
  // K ranges, keeping their Y rows in its L2.
  const int64_t L = bid.x;
  const int zslab = (int)(L % a.splitk);
  const int64_t mtile = L / a.splitk;
  const int64_t mt0 = mtile * C::ROWS;
  const int64_t kbeg = (int64_t)zslab * a.kchunk;
  const int64_t kend = min(a.K, kbeg + a.kchunk);

  // per-lane global bases of the stage loads (K offset added per stage)
  // (byte pointers; stage k0 adds k0 * ES)
  const unsigned char* xsrc[C::XOPS];
#pragma unroll
  for (int u = 0; u < C::XOPS; ++u) {
    const int pos = (wave * C::XOPS + u) * 64 + lane;
    const int col = pos / C::XCPC, kc = (pos % C::XCPC) ^ C::xswz(col);
    const int64_t gcol = min(mt0 + col, a.M - 1);          // columns past M: any valid column
    xsrc[u] = static_cast<const unsigned char*>(a.X) + (gcol * a.ldx + (int64_t)kc * C::EPC) * C::ES;
  }
  const uint16_t* ysrc[C::YMAX];
#pragma unroll
  for (int u = 0; u < C::YMAX; ++u) {
    const int instr = wave + kWaves * u;
    const int pos = (instr < C::YINSTR ? instr : 0) * 64 + lane;
    const int qj = pos >> 2, q = qj / C::N16, j = qj % C::N16;
    const int kc = (pos & 3) ^ ((j >> 1) & 3);
    ysrc[u] = a.Yp + q * a.yplane + (int64_t)j * a.ldy + 8 * kc;
  }
  auto issue = [&](u4v* xs, int64_t k0) {
    u4v* ys = xs + C::XCH;
#pragma unroll
    for (int u = 0; u < C::XOPS; ++u)
      dma16(xsrc[u] + k0 * C::ES, xs + (wave * C::XOPS + u) * 64);
#pragma unroll
    for (int u = 0; u < C::YMAX; ++u)
      dma16(ysrc[u] + k0, ys + (wave + kWaves * u) * 64);
  };

  f4v acc[MB][NB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f4v{0, 0, 0, 0};

  // per-stage scale of an FP8 tile: a wave's rows lie in one tile column
  // (tile is a multiple of 128 and a wave owns at most 64 aligned rows;
  // rows past M take the last column's) and a stage in one tile row
  auto xscale = [&](int64_t k0) -> float {
    if constexpr (XK == XK_FP8) return a.xscale[k0 / a.tile + (min(mt0 + (int64_t)wave * (16 * MB), a.M - 1) / a.tile) * a.ldsc];
    else return 1.0f;
  };
  // One stage's operands in registers: per 16-row block of the wave its X
  // chunk(s) (FP32: the two 16-byte halves of eight values; BF16: one chunk;
  // FP8: eight codes), per 16-column block its Y planes.  They are read from
  // LDS one stage ahead of the MFMAs that use them.
  struct Frags {
    u4v xa[MB], xb[MB];
    uint2v xq[MB];
    u4v y[NB][C::YPL];
  };
  auto load = [&](Frags& f, const u4v* xs, const u4v* ys) {
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      const int col = wave * (16 * MB) + 16 * mb + c;
      if constexpr (XK == XK_F32) {
        f.xa[mb] = xs[col * 8 + ((2 * g) ^ C::xswz(col))];
        f.xb[mb] = xs[col * 8 + ((2 * g + 1) ^ C::xswz(col))];
      } else if constexpr (XK == XK_BF16) {
        f.xa[mb] = xs[col * 4 + (g ^ C::xswz(col))];
      } else {
        const uint2v* xh = reinterpret_cast<const uint2v*>(xs);
        f.xq[mb] = xh[(col * 2 + ((g >> 1) ^ C::xswz(col))) * 2 + (g & 1)];
      }
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int j = 16 * nb + c;
      const int sw = g ^ ((j >> 1) & 3);
#pragma unroll
      for (int q = 0; q < C::YPL; ++q) f.y[nb][q] = ys[(q * C::N16 + j) * 4 + sw];
    }
  };
  auto mma = [&](const Frags& f, float sc) {
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      if constexpr (XK == XK_F32) {
        float xv[8];
#pragma unroll
        for (int i = 0; i < 4; ++i) { xv[i] = __uint_as_float(f.xa[mb][i]); xv[4 + i] = __uint_as_float(f.xb[mb][i]); }
        u4v x1, x2, x3;
        split8(xv, x1, x2, x3);
        const bf8v a1 = as_bf8(x1), a2 = as_bf8(x2), a3 = as_bf8(x3);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const bf8v b1 = as_bf8(f.y[nb][0]), b2 = as_bf8(f.y[nb][1]), b3 = as_bf8(f.y[nb][2]);
          f4v cc = acc[mb][nb];
          cc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a3, b1, cc, 0, 0, 0);   // smallest terms first
          cc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, b2, cc, 0, 0, 0);
          cc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b3, cc, 0, 0, 0);
          cc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, b1, cc, 0, 0, 0);
          cc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b2, cc, 0, 0, 0);
          cc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, cc, 0, 0, 0);
          acc[mb][nb] = cc;
        }
      } else {
        bf8v ax;
        if constexpr (XK == XK_BF16) {
          ax = as_bf8(f.xa[mb]);
        } else {
          // eight E4M3 codes -> exact BF16 via FP32
          const uint2v q = f.xq[mb];
          const f2v f0 = __builtin_amdgcn_cvt_pk_f32_fp8((int)q[0], false);
          const f2v f1 = __builtin_amdgcn_cvt_pk_f32_fp8((int)q[0], true);
          const f2v f2 = __builtin_amdgcn_cvt_pk_f32_fp8((int)q[1], false);
          const f2v f3 = __builtin_amdgcn_cvt_pk_f32_fp8((int)q[1], true);
          u4v w;
          w[0] = __builtin_amdgcn_perm(__float_as_uint(f0[1]), __float_as_uint(f0[0]), 0x07060302u);
          w[1] = __builtin_amdgcn_perm(__float_as_uint(f1[1]), __float_as_uint(f1[0]), 0x07060302u);
          w[2] = __builtin_amdgcn_perm(__float_as_uint(f2[1]), __float_as_uint(f2[0]), 0x07060302u);
          w[3] = __builtin_amdgcn_perm(__float_as_uint(f3[1]), __float_as_uint(f3[0]), 0x07060302u);
          ax = as_bf8(w);
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const bf8v b1 = as_bf8(f.y[nb][0]), b2 = as_bf8(f.y[nb][1]);
          if constexpr (XK == XK_BF16) {
            f4v cc = acc[mb][nb];
            cc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ax, b2, cc, 0, 0, 0);
            cc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ax, b1, cc, 0, 0, 0);
            acc[mb][nb] = cc;
          } else {
            f4v cc = f4v{0, 0, 0, 0};
            cc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ax, b2, cc, 0, 0, 0);
            cc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ax, b1, cc, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[mb][nb][r] = fmaf(sc, cc[r], acc[mb][nb][r]);
          }
        }
      }
    }
  };

  const int64_t nfull = (kend - kbeg) / KSTEP;
  // Past the last full stage the loads repeat the last one (an L2 hit, never
  // consumed), so the issue code and the wait counts are the same on every
  // stage.
  const int64_t klast = kbeg + (nfull - 1) * KSTEP;
  // Operands read from LDS one stage ahead of their MFMAs where that pays:
  // the tall BF16 tiles (p > 64) and the FP8 tiles up to p = 96 (wider ones
  // have no room for the second set of registers).  Measured one product at
  // a time: BF16 n = 16384, p = 128 261 -> 234 us; FP8 Gram products,
  // p = 48, 54.9 / 43.3 -> 50.7 / 41.0 us; the FP32 product (p = 64) and
  // the BF16 product at p = 64 gain nothing (72.7 -> 74.4, 36.2 -> 36.6 us).
  constexpr bool kAhead = (XK == XK_BF16 && MB == 4) || (XK == XK_FP8 && NB <= 6);
  if (nfull > 0 && kAhead) {
    // The ring holds NS stages; the loads of stage st + NS go into the slot
    // of stage st once stage st's operands are in registers.
    unroll_for<0, NS>([&](auto I) { issue(slot[decltype(I)::value], min(kbeg + decltype(I)::value * KSTEP, klast)); });
    wait_vmcnt<(NS - 1) * C::OPS, 0>();    // this wave's loads of stage 0 are done
    wg_barrier();                          // and every wave's
    Frags cur;
    load(cur, slot[0], slot[0] + C::XCH);
    // the slot index is a compile-time constant at every call, so each
    // stage's LDS object is known
    auto body = [&](auto SL, int64_t st) {
      constexpr int sl = decltype(SL)::value, nx = (sl + 1) % NS;
      // stage st + 1 has landed once only the loads of the NS - 2 stages
      // issued after it are outstanding; lgkmcnt 0: this wave's LDS reads
      // of stage st (into registers) are done.  After the barrier no wave
      // reads slot sl any more.
      wait_vmcnt<(NS - 2) * C::OPS, 0>();
      wg_barrier();
      issue(slot[sl], min(kbeg + (st + NS) * KSTEP, klast));
      Frags nxt;
      if (st + 1 < nfull) load(nxt, slot[nx], slot[nx] + C::XCH);
      mma(cur, xscale(kbeg + st * KSTEP));
      cur = nxt;
    };
    int64_t st = 0;
    for (; st + NS <= nfull; st += NS) unroll_for<0, NS>([&](auto I) { body(I, st + decltype(I)::value); });
    unroll_for<0, NS - 1>([&](auto I) {
      if (st + decltype(I)::value < nfull) body(I, st + decltype(I)::value);
    });
    wait_vmcnt<0>();                       // the repeated loads land before LDS is reused
  } else if (nfull > 0) {
    // Each stage issues the loads of the stage NS - 1 ahead into the slot
    // the previous stage used, then reads its own operands and multiplies.
    auto body = [&](auto SL, int64_t st) {
      constexpr int sl = decltype(SL)::value;
      // this wave's loads of stage st are done once only the loads of the
      // NS - 2 stages issued after it are outstanding, and its LDS reads of
      // stage st - 1 once lgkmcnt is 0; the barrier then makes every wave's
      // loads of stage st visible and frees the slot of stage st - 1
      wait_vmcnt<(NS - 2) * C::OPS, 0>();
      wg_barrier();
      issue(slot[(sl + NS - 1) % NS], min(kbeg + (st + NS - 1) * KSTEP, klast));
      Frags f;
      load(f, slot[sl], slot[sl] + C::XCH);
      mma(f, xscale(kbeg + st * KSTEP));
    };
    unroll_for<0, NS - 1>([&](auto I) { issue(slot[decltype(I)::value], min(kbeg + decltype(I)::value * KSTEP, klast)); });
    int64_t st = 0;
    for (; st + NS <= nfull; st += NS) unroll_for<0, NS>([&](auto I) { body(I, st + decltype(I)::value); });
    unroll_for<0, NS - 1>([&](auto I) {
      if (st + decltype(I)::value < nfull) body(I, st + decltype(I)::value);
    });
    wait_vmcnt<0>();
  }
  const int64_t ktail = kbeg + nfull * KSTEP;
  if (ktail < kend) {
    // ragged last step: masked register loads into stage 0
    wait_vmcnt<0>();
    __syncthreads();
#pragma unroll
    for (int u = 0; u < C::XOPS; ++u) {
      const int pos = (wave * C::XOPS + u) * 64 + lane;
      const int col = pos / C::XCPC, kc = (pos % C::XCPC) ^ C::xswz(col);
      unsigned char bytes[16];
#pragma unroll
      for (int e = 0; e < C::EPC; ++e) {
        const int64_t r = ktail + (int64_t)kc * C::EPC + e;   // K index of element e
#pragma unroll
        for (int bb = 0; bb < C::ES; ++bb)
          bytes[e * C::ES + bb] = r < kend ? xsrc[u][(ktail + e) * C::ES + bb] : 0;
      }
      u4v w;
#pragma unroll
      for (int i = 0; i < 4; ++i)
        w[i] = (unsigned)bytes[4 * i] | ((unsigned)bytes[4 * i + 1] << 8) | ((unsigned)bytes[4 * i + 2] << 16) |
               ((unsigned)bytes[4 * i + 3] << 24);
      st0[pos] = w;
    }
#pragma unroll
    for (int u = 0; u < C::YMAX; ++u) {
      const int instr = wave + kWaves * u;
      if (instr >= C::YINSTR) continue;
      const int pos = instr * 64 + lane;
      const int j = (pos >> 2) % C::N16;
      const int kc = (pos & 3) ^ ((j >> 1) & 3);
      unsigned w[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t r = ktail + 8 * kc + 2 * i;
        const unsigned lo = r < kend ? ysrc[u][ktail + 2 * i] : 0u;
        const unsigned hi = r + 1 < kend ? ysrc[u][ktail + 2 * i + 1] : 0u;
        w[i] = lo | (hi << 16);
      }
      st0[C::XCH + pos] = u4v{w[0], w[1], w[2], w[3]};
    }
    __syncthreads();
    Frags f;
    load(f, st0, st0 + C::XCH);
    mma(f, xscale(ktail));
  }
  const int64_t m0 = mt0 + (int64_t)wave * (16 * MB);

  // accumulator element r of lane (c, g): row 4g + r, column c of its block
  if (a.splitk == 1) {
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = m0 + 16 * mb + 4 * g + r;
          if (row < a.M) store_out(a, row, 16 * nb + c, acc[mb][nb][r]);
        }
  } else {
    float* part = a.part + (int64_t)zslab * a.ldp * a.N;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int64_t row = m0 + 16 * mb + 4 * g;
        *reinterpret_cast<f4v*>(part + row + (16 * nb + c) * a.ldp) = acc[mb][nb];
      }
  }
}

// Sum of the split-K slabs in slab order, then the epilogue.
struct FilterReduceK {
  using Args = FArgs;
  static constexpr int kThreads = 256, kMinWaves = 1;
  static __device__ __attribute__((always_inline)) void body(const FArgs& a, uint3 bid);
};

__device__ void FilterReduceK::body(const FArgs& a, uint3 bid) {
  const int64_t i = (int64_t)bid.x * 256 + threadIdx.x;
  const int64_t j = bid.y;
  if (i >= a.M) return;
  const float* part = a.part + i + j * a.ldp;
  const int64_t slab = a.ldp * a.N;
  float sum = 0.0f;
  int s = 0;
  for (; s + 8 <= a.splitk; s += 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(s + u) * slab];
#pragma unroll
    for (int u = 0; u < 8; ++u) sum = (s + u == 0) ? v[u] : sum + v[u];
  }
  for (; s < a.splitk; ++s) sum = (s == 0) ? part[0] : sum + part[(int64_t)s * slab];
  store_out(a, i, j, sum);
}

// Three BF16 planes of an n x p FP32 block (rows up to n_pad, columns up to
// p_pad; padding is zero).
struct SplitPlanesArgs {
  const float* src; int64_t lds_; int64_t n; int p;
  uint16_t* dst; int64_t ldd; int64_t plane; int64_t n_pad;
};
struct SplitPlanesK {
  using Args = SplitPlanesArgs;
  static constexpr int kThreads = 256, kMinWaves = 1;
  static __device__ __attribute__((always_inline)) void body(const Args& a, uint3 bid) {
    const float* __restrict__ src = a.src;
    uint16_t* __restrict__ dst = a.dst;
    const int64_t lds_ = a.lds_, n = a.n, ldd = a.ldd, plane = a.plane, n_pad = a.n_pad;
    const int p = a.p;
  const int64_t i = (int64_t)bid.x * 256 + threadIdx.x;
  const int j = bid.y;
  if (i >= n_pad) return;
  const float v = (i < n && j < p) ? src[i + j * lds_] : 0.0f;
  uint16_t p1, p2, p3;
  split1(v, p1, p2, p3);
  uint16_t* o = dst + i + j * ldd;
  o[0] = p1;
  o[plane] = p2;
  o[2 * plane] = p3;
  }
};

// Start of an extraction in one launch: the n x p start block copied into
// the padded work buffer (zero padding up to n_pad x p_pad), its three BF16
// planes when `planes` is set, and the step's pf_info cleared.
template <typename T>
struct BeginArgs {
  const T* src; int64_t lds_; T* dst; int64_t ldd;
  int64_t n; int p; int64_t n_pad; uint16_t* planes; int64_t plane; pf_info* info;
};
template <typename T>
struct BeginK {
  using Args = BeginArgs<T>;
  static constexpr int kThreads = 256, kMinWaves = 1;
  static __device__ __attribute__((always_inline)) void body(const Args& a, uint3 bid) {
    const T* __restrict__ src = a.src;
    T* __restrict__ dst = a.dst;
    uint16_t* __restrict__ planes = a.planes;
    const int64_t lds_ = a.lds_, ldd = a.ldd, n = a.n, n_pad = a.n_pad, plane = a.plane;
    const int p = a.p;
    pf_info* info = a.info;
  const int64_t i = (int64_t)bid.x * 256 + threadIdx.x;
  const int j = bid.y;
  if (info && i == 0 && j == 0) *info = pf_info{};
  if (i >= n_pad) return;
  const T v = (i < n && j < p) ? src[i + j * lds_] : T(0);
  dst[i + j * ldd] = v;
  if constexpr (std::is_same<T, float>::value) {
    if (planes) {
      uint16_t p1, p2, p3;
      split1(v, p1, p2, p3);
      uint16_t* o = planes + i + j * ldd;
      o[0] = p1;
      o[plane] = p2;
      o[2 * plane] = p3;
    }
  }
  }
};

struct FSplit {
  int S;
  int64_t kchunk, ldp, mtiles;
};

// Split-K so that the grid is about one resident workgroup per CU (the
// kernel's LDS ring fills most of a CU's LDS), each with a long K range.
FSplit fplan(int MB, int64_t K, int64_t M, int requested) {
  FSplit sp;
  const int64_t rows = (int64_t)kWaves * 16 * MB;
  sp.mtiles = (M + rows - 1) / rows;
  const int64_t unit = KSTEP;
  const int64_t min_chunk = unit * 8;
  int64_t S = requested > 0 ? requested : std::max<int64_t>(1, 256 / std::max<int64_t>(1, sp.mtiles));
  S = std::min<int64_t>(S, std::max<int64_t>(1, (K + min_chunk - 1) / min_chunk));
  S = std::max<int64_t>(1, std::min<int64_t>(S, 64));
  if (requested <= 0 && S >= 8) S = S / 8 * 8;        // a multiple of the XCD count
  (void)min_chunk;
  int64_t kchunk = round_up((K + S - 1) / S, unit);
  S = std::max<int64_t>(1, (K + kchunk - 1) / kchunk);
  sp.S = (int)S;
  sp.kchunk = kchunk;
  sp.ldp = sp.mtiles * rows;
  return sp;
}

template <int XK, int MB, int NB>
void launch_f(FArgs& a, const FSplit& sp, int pm, int pr, hipStream_t st) {
  dim3 grid((unsigned)(sp.mtiles * sp.S), 1, 1);
  const bool prof = prof_enabled();
  // the whole product (kernel and slab sum) is its own timing class
  const int pp = pm == PF_PROF_FILTER ? PF_PROF_FILTER_PRODUCT : -1;
  if (prof && pp >= 0) prof_begin(pp, st);
  if (prof && pm >= 0) prof_begin(pm, st);
  emit<FilterK<XK, MB, NB>>(a, grid, 0, st);
  if (prof && pm >= 0) prof_end(pm, st);
  if (sp.S > 1) {
    dim3 g2((unsigned)((a.M + 255) / 256), (unsigned)a.N);
    if (prof && pr >= 0) prof_begin(pr, st);
    emit<FilterReduceK>(a, g2, 0, st);
    if (prof && pr >= 0) prof_end(pr, st);
  }
  if (prof && pp >= 0) prof_end(pp, st);
}

// Rows per workgroup (16-row blocks per wave): every workgroup reloads the
// Y planes of its K slab, so wide blocks want tall tiles.  Four blocks per
// wave for a BF16 X with more than 64 columns (the stage then holds 16 KiB
// of X and 16 KiB of Y); two otherwise.  An FP32 X stage at p = 128 holds
// 16 KiB of X and 24 KiB of Y, the whole 40 KiB slot (one block per wave
// there, 8 KiB of X per 24 KiB of Y, was 10-20 % slower from n = 4096 up);
// An FP8 X with up to 64 columns and many rows takes four blocks per wave as
// well (each wave's 64 rows stay in one 128-row scale tile): measured on the
// Gram form's products, 50.7 -> 42.0 us with 12000 output rows, but 40.9 ->
// 41.6 us with 6000.
int mb_for(int xk, int NB, int64_t M) {
  if (xk == XK_BF16) return NB > 4 ? 4 : 2;
  if (xk == XK_FP8) return NB <= 4 && M >= 8192 ? 4 : 2;
  return 2;
}

int xk_of(pf_dtype t) {
  switch (t) {
    case PF_F32: return XK_F32;
    case PF_BF16: return XK_BF16;
    case PF_F8E4M3: return XK_FP8;
    default: fail(PF_ERR_UNSUPPORTED, "filter: X must be FP32, BF16 or FP8-E4M3 for FP32 work");
  }
  return XK_F32;
}

template <int XK>
void launch_xk(FArgs& a, const FSplit& sp, int MB, int NB, int pm, int pr, hipStream_t st) {
  if constexpr (XK == XK_F32) {
    switch (NB) {
      case 1: launch_f<XK, 2, 1>(a, sp, pm, pr, st); break;
      case 2: launch_f<XK, 2, 2>(a, sp, pm, pr, st); break;
      case 3: launch_f<XK, 2, 3>(a, sp, pm, pr, st); break;
      case 4: launch_f<XK, 2, 4>(a, sp, pm, pr, st); break;
      case 5: launch_f<XK, 2, 5>(a, sp, pm, pr, st); break;
      case 6: launch_f<XK, 2, 6>(a, sp, pm, pr, st); break;
      case 7: launch_f<XK, 2, 7>(a, sp, pm, pr, st); break;
      default: launch_f<XK, 2, 8>(a, sp, pm, pr, st); break;
    }
  } else {
    switch (NB) {
      case 1:
        if (XK == XK_FP8 && MB == 4) launch_f<XK, XK == XK_FP8 ? 4 : 2, 1>(a, sp, pm, pr, st);
        else launch_f<XK, 2, 1>(a, sp, pm, pr, st);
        break;
      case 2:
        if (XK == XK_FP8 && MB == 4) launch_f<XK, XK == XK_FP8 ? 4 : 2, 2>(a, sp, pm, pr, st);
        else launch_f<XK, 2, 2>(a, sp, pm, pr, st);
        break;
      case 3:
        if (XK == XK_FP8 && MB == 4) launch_f<XK, XK == XK_FP8 ? 4 : 2, 3>(a, sp, pm, pr, st);
        else launch_f<XK, 2, 3>(a, sp, pm, pr, st);
        break;
      case 4:
        if (XK == XK_FP8 && MB == 4) launch_f<XK, XK == XK_FP8 ? 4 : 2, 4>(a, sp, pm, pr, st);
        else launch_f<XK, 2, 4>(a, sp, pm, pr, st);
        break;
      case 5: launch_f<XK, XK == XK_BF16 ? 4 : 2, 5>(a, sp, pm, pr, st); break;
      case 6: launch_f<XK, XK == XK_BF16 ? 4 : 2, 6>(a, sp, pm, pr, st); break;
      case 7: launch_f<XK, XK == XK_BF16 ? 4 : 2, 7>(a, sp, pm, pr, st); break;
      default: launch_f<XK, XK == XK_BF16 ? 4 : 2, 8>(a, sp, pm, pr, st); break;
    }
  }
}

}  // namespace

size_t filter_bf16x6_part_bytes(pf_dtype xdt, int64_t K, int64_t M, int64_t N) {
  const int NB = (int)(N / 16);
  const FSplit sp = fplan(mb_for(xk_of(xdt), NB, M), K, M, 0);
  return sp.S > 1 ? (size_t)sp.S * sp.ldp * N * sizeof(float) : 0;
}

void filter_bf16x6(const FilterArgs& x, hipStream_t st) {
  if (x.N % 16 != 0 || x.N <= 0 || x.N > 128) fail(PF_ERR_ARG, "filter: N must be 16..128, multiple of 16");
  const int xk = xk_of(x.xdtype);
  if (xk == XK_FP8 && (x.xscale == nullptr || x.tile <= 0 || x.tile % 128 != 0))
    fail(PF_ERR_ARG, "filter: FP8 X needs tile scales with a tile that is a multiple of 128");
  const int NB = (int)(x.N / 16);
  const int MB = mb_for(xk, NB, x.M);
  FSplit sp = fplan(MB, x.K, x.M, x.splitk);
  while (sp.S > 1 && (size_t)sp.S * sp.ldp * x.N * sizeof(float) > x.part_bytes) sp = fplan(MB, x.K, x.M, sp.S - 1);
  FArgs a;
  a.X = x.X; a.ldx = x.ldx;
  a.xscale = x.xscale; a.ldsc = x.ldsc; a.tile = x.tile;
  a.Yp = x.Yp; a.ldy = x.ldy; a.yplane = x.yplane;
  a.K = x.K; a.M = x.M; a.N = x.N; a.kchunk = sp.kchunk;
  a.out = x.out; a.ldo = x.ldo; a.D1 = x.D1; a.D2 = x.D2; a.ldd = x.ldd;
  a.alpha = (float)x.alpha; a.beta = (float)x.beta; a.gamma = (float)x.gamma;
  a.outp = x.outp; a.ldop = x.ldop; a.oplane = x.oplane;
  a.part = static_cast<float*>(x.part); a.ldp = sp.ldp; a.splitk = sp.S;
  switch (xk) {
    case XK_F32: launch_xk<XK_F32>(a, sp, MB, NB, x.prof_main, x.prof_reduce, st); break;
    case XK_BF16: launch_xk<XK_BF16>(a, sp, MB, NB, x.prof_main, x.prof_reduce, st); break;
    default: launch_xk<XK_FP8>(a, sp, MB, NB, x.prof_main, x.prof_reduce, st); break;
  }
}

void launch_begin_block(const void* src, int64_t lds, Elem t, void* dst, int64_t ldd, int64_t n, int p,
                        int64_t n_pad, int p_pad, uint16_t* planes, int64_t plane, pf_info* info, hipStream_t st) {
  dim3 grid((unsigned)((n_pad + 255) / 256), (unsigned)p_pad);
  if (t == Elem::F64) {
    if (planes) fail(PF_ERR_ARG, "begin_block: BF16 planes need FP32 work");
    const BeginArgs<double> a{static_cast<const double*>(src), lds, static_cast<double*>(dst), ldd, n, p, n_pad,
                              nullptr, 0, info};
    emit<BeginK<double>>(a, grid, 0, st);
  } else {
    const BeginArgs<float> a{static_cast<const float*>(src), lds, static_cast<float*>(dst), ldd, n, p, n_pad,
                             planes, plane, info};
    emit<BeginK<float>>(a, grid, 0, st);
  }
}

void launch_split_planes(const float* src, int64_t lds, int64_t n, int p, uint16_t* dst, int64_t ldd,
                         int64_t plane, int64_t n_pad, int p_pad, hipStream_t st) {
  dim3 grid((unsigned)((n_pad + 255) / 256), (unsigned)p_pad);
  const SplitPlanesArgs a{src, lds, n, p, dst, ldd, plane, n_pad};
  emit<SplitPlanesK>(a, grid, 0, st);
}

}  // namespace pfx
