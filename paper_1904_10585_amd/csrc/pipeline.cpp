// The extraction pipeline: workspace plan and the launch sequence of one
// polynomial-filtered subspace extraction (section 2.1 then eq. RR).
//
//   Z = A U                                   first filter product
//   pre-rotation: H0 = U^T Z, H0 = W0 L0 W0^T, Y_0 = U W0,
//                 Y_1 = (Z W0 - c Y_0) / (e tau_1)
//   Y_{k+1} = (tau_k / tau_{k+1}) ((2/e) A Y_k - (2c/e) Y_k)
//             - (tau_{k-1} / tau_{k+1}) Y_{k-1}          k = 1 .. d-1
//   CholeskyQR2: G = Y^T Y, R = chol(G), Q = Y R^{-1}, twice
//   Rayleigh-Ritz: W = X_rr Q (FP64), H = Q^T W, H = Z Theta Z^T, V = Q Z
//
// For A = M^T M (PF_OP_GRAM, the SVD route of section 5.2.1) every product
// A Y is T = M Y followed by M^T T, and Rayleigh-Ritz runs on B = M Q:
// H = B^T B = Q^T A Q, theta = sigma^2.  The products contracting over the
// columns of M read a transposed copy of M (K contiguous for the MFMA).
//
// tau_k = T_k(s_ref) rescales the recurrence (PF_FLAG_SCALED); with tau = 1
// it is the plain three-term recurrence of eq. cheby-recursion-map.  The
// pre-rotation replaces U by its Ritz basis for the current matrix, which
// leaves span(rho(A) U) unchanged because the recurrence acts column by
// column (section 2.1: rho(A) (U W) = (rho(A) U) W).
#include "pf_internal.h"
#include "group.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace pfx {

struct Plan {
  pf_desc d;
  Elem work;
  int64_t n, n_pad;
  int p, p_pad;
  size_t esz;
  void* mem = nullptr;
  size_t bytes = 0;
  void* U;
  void* Z;
  void* Yb[3];
  uint16_t* Up;       // BF16 planes of U (split-BF16 filter)
  uint16_t* Ypl[3];   // BF16 planes of the recurrence ring
  int64_t plane;      // elements per plane
  void* Q1;
  void* Q;
  double* W;
  double* G;
  double* Rinv;
  double* Zeig;
  double* Ework;      // scratch of the eigen-refinement (p > 64)
  int* refined;       // set by the refinement when it converged
  double* theta;
  double* theta_pre;
  int* deficient;
  pf_info* info;
  void* part;
  size_t part_bytes;
  double* Xtra = nullptr;        // 2 p_pad x p_pad: E^T E and the scaled Z of the optional outputs
  // PF_OP_GRAM: M is m x n
  int64_t m = 0, m_pad = 0;
  void* T = nullptr;            // M Y (m x p, work dtype)
  uint16_t* Tpl = nullptr;      // its BF16 planes (split path)
  int64_t tplane = 0;
  double* B = nullptr;          // M Q (m x p, FP64) for Rayleigh-Ritz
  // transposed copies of the operators (n x m), allocated on first use
  struct Copy {
    void* data = nullptr; size_t bytes = 0; int64_t ld = 0;
    float* scale = nullptr; size_t scale_bytes = 0;
    const void* src = nullptr; pf_dtype dt = PF_F32; int64_t src_ld = 0; const float* src_scale = nullptr;
    int tile = 0;
  } mft, mrt;
};

namespace {

struct Layout {
  size_t off_Up, off_Ypl[3], off_T = 0, off_Tpl = 0, off_B = 0;
  size_t off_U, off_Z, off_Y[3], off_Q1, off_Q, off_W, off_G, off_Rinv, off_Zeig, off_theta,
      off_theta_pre, off_def, off_info, off_part, total, part_bytes, off_E, off_refined;
  size_t off_xtra = 0;
};

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

Layout layout_for(const pf_desc& d) {
  Layout L;
  const Elem work = d.work == PF_F64 ? Elem::F64 : Elem::F32;
  const size_t esz = work == Elem::F64 ? 8 : 4;
  const int64_t n_pad = round_up(d.n, 64);
  const int p_pad = (int)round_up(d.p, 16);
  const size_t blk = align256((size_t)n_pad * p_pad * esz);
  const size_t blk64 = align256((size_t)n_pad * p_pad * 8);
  const size_t sq = align256((size_t)p_pad * p_pad * 8);
  size_t o = 0;
  L.off_U = o; o += blk;
  L.off_Z = o; o += blk;
  for (int i = 0; i < 3; ++i) { L.off_Y[i] = o; o += blk; }
  L.off_Q1 = o; o += blk;
  L.off_Q = o; o += blk;
  L.off_W = o; o += blk64;
  L.off_G = o; o += sq;
  L.off_Rinv = o; o += sq;
  L.off_Zeig = o; o += sq;
  L.off_E = o; o += align256(eig_scratch_bytes(p_pad));
  L.off_refined = o; o += 256;
  L.off_theta = o; o += align256((size_t)p_pad * 8);
  L.off_theta_pre = o; o += align256((size_t)p_pad * 8);
  L.off_def = o; o += align256((size_t)p_pad * 4);
  L.off_info = o; o += align256(sizeof(pf_info));
  L.off_xtra = o; o += 2 * sq;
  const size_t planes = align256((size_t)3 * n_pad * p_pad * 2);
  L.off_Up = o; o += (work == Elem::F32) ? planes : 0;
  for (int i = 0; i < 3; ++i) { L.off_Ypl[i] = o; o += (work == Elem::F32) ? planes : 0; }
  const bool gram = d.op == PF_OP_GRAM;
  const int64_t m_pad = gram ? round_up(d.m, 64) : 0;
  if (gram) {
    L.off_T = o; o += align256((size_t)m_pad * p_pad * esz);
    L.off_Tpl = o; o += (work == Elem::F32) ? align256((size_t)3 * m_pad * p_pad * 2) : 0;
    L.off_B = o; o += align256((size_t)m_pad * p_pad * 8);
  }
  // split-K slabs: the largest any contraction of the sequence asks for
  const Elem xf = work;   // filter operand type (same as work in these forms)
  size_t part = 0;
  if (gram) {
    for (Elem ta : {work, Elem::F32, Elem::F64}) {
      part = std::max(part, contract_part_bytes(d.n, d.m, p_pad, ta, work, true, 0));
      part = std::max(part, contract_part_bytes(d.m, d.n, p_pad, ta, work, true, 0));
      part = std::max(part, contract_part_bytes(d.n, d.m, p_pad, ta, work, false, 0));
      part = std::max(part, contract_part_bytes(d.m, d.n, p_pad, ta, work, false, 0));
    }
    part = std::max(part, contract_part_bytes(d.m, p_pad, p_pad, Elem::F64, Elem::F64, true, 0));
    if (work == Elem::F32)
      for (pf_dtype xt : {PF_F32, PF_BF16, PF_F8E4M3}) {
        part = std::max(part, filter_bf16x6_part_bytes(xt, d.n, d.m, p_pad));
        part = std::max(part, filter_bf16x6_part_bytes(xt, d.m, d.n, p_pad));
      }
  }
  part = std::max(part, contract_part_bytes(d.n, d.n, p_pad, xf, work, work == Elem::F64, 0));
  part = std::max(part, contract_part_bytes(d.n, d.n, p_pad, Elem::F32, work, true, 0));
  part = std::max(part, contract_part_bytes(d.n, d.n, p_pad, Elem::F64, Elem::F64, true, 0));
  part = std::max(part, contract_part_bytes(d.n, p_pad, p_pad, work, work, true, 0));
  part = std::max(part, contract_part_bytes(d.n, p_pad, p_pad, work, Elem::F64, true, 0));
  if (work == Elem::F32)
    for (pf_dtype xt : {PF_F32, PF_BF16, PF_F8E4M3}) part = std::max(part, filter_bf16x6_part_bytes(xt, d.n, d.n, p_pad));
  L.part_bytes = align256(part);
  L.off_part = o; o += L.part_bytes;
  L.total = o;
  return L;
}

bool elem_ok_for_filter(const pf_desc& d, pf_dtype t) {
  if (d.work == PF_F64) return t == PF_F64;
  return t == PF_F32 || t == PF_BF16 || t == PF_F8E4M3;
}

void check_mat(const pf_mat* M, const char* name, int64_t rows) {
  if (!M) fail(PF_ERR_ARG, std::string(name) + " is NULL");
  if (!M->data) fail(PF_ERR_ARG, std::string(name) + ".data is NULL");
  if (M->ld < rows) fail(PF_ERR_ARG, std::string(name) + ".ld is smaller than the row count");
  size_t esz = M->dtype == PF_F64 ? 8 : M->dtype == PF_F32 ? 4 : M->dtype == PF_BF16 ? 2 : 1;
  if (((uintptr_t)M->data) % 16 != 0) fail(PF_ERR_ARG, std::string(name) + ".data must be 16-byte aligned");
  if (((size_t)M->ld * esz) % 16 != 0)
    fail(PF_ERR_ARG, std::string(name) + ".ld * element size must be a multiple of 16 bytes");
}

void host_coefficients(const pf_desc& d, std::vector<double>& tau) {
  const double c = 0.5 * (d.a + d.b), e = 0.5 * (d.b - d.a);
  tau.assign(d.degree + 2, 1.0);
  if (d.flags & PF_FLAG_SCALED) {
    const double s = (d.spec_ub - c) / e;
    if (s > 1.0) {
      tau[0] = 1.0;
      tau[1] = s;
      for (int k = 1; k <= d.degree; ++k) tau[k + 1] = 2.0 * s * tau[k] - tau[k - 1];
    }
  }
}

// pointers of a plan's buffers from its layout and base address P->mem
void carve(Plan* P, const Layout& L);

}  // namespace

void plan_validate(const pf_desc& d, const pf_mat* Xf, const pf_mat* Xr) {
  if (d.struct_size != sizeof(pf_desc)) fail(PF_ERR_ARG, "pf_desc.struct_size does not match this library");
  if (d.op != PF_OP_SYM && d.op != PF_OP_GRAM) fail(PF_ERR_ARG, "pf_desc.op is not a pf_op value");
  if (d.n < 1) fail(PF_ERR_ARG, "pf_desc.n must be >= 1");
  if (d.op == PF_OP_GRAM && d.m < 1) fail(PF_ERR_ARG, "pf_desc.m must be >= 1 for PF_OP_GRAM");
  if (d.p < 1 || d.p > 128 || d.p > d.n) fail(PF_ERR_ARG, "pf_desc.p must satisfy 1 <= p <= min(n, 128)");
  if (d.degree < 1) fail(PF_ERR_ARG, "pf_desc.degree must be >= 1");
  if (d.q < 1) fail(PF_ERR_ARG, "pf_desc.q must be >= 1");
  if (!std::isfinite(d.a) || !std::isfinite(d.b) || !(d.a < d.b))
    fail(PF_ERR_ARG, "damping interval must be finite with a < b");
  if (d.work != PF_F32 && d.work != PF_F64) fail(PF_ERR_ARG, "pf_desc.work must be PF_F32 or PF_F64");
  if ((d.flags & PF_FLAG_SCALED) && !(std::isfinite(d.spec_ub) && d.spec_ub > d.b))
    fail(PF_ERR_ARG, "PF_FLAG_SCALED needs a finite spec_ub > b");
  if (d.flags & ~(PF_FLAG_NO_PREROTATE | PF_FLAG_SCALED | PF_FLAG_COLD | PF_FLAG_NATIVE_F32 |
                  PF_FLAG_OPERATOR_UNCHANGED | PF_FLAG_REORTH))
    fail(PF_ERR_ARG, "unknown bits in pf_desc.flags");
  if (d.reserved != 0) fail(PF_ERR_ARG, "pf_desc.reserved must be 0");
  if (Xf || Xr) {
    const int64_t rows = d.op == PF_OP_GRAM ? d.m : d.n;
    check_mat(Xf, "X_filter", rows);
    check_mat(Xr, "X_rr", rows);
    if (!elem_ok_for_filter(d, Xf->dtype)) fail(PF_ERR_ARG, "X_filter dtype does not match pf_desc.work");
    if ((Xf->dtype == PF_BF16 || Xf->dtype == PF_F8E4M3) && (d.flags & PF_FLAG_NATIVE_F32))
      fail(PF_ERR_ARG, "PF_FLAG_NATIVE_F32 needs an FP32 X_filter");
    if (Xf->dtype == PF_F8E4M3 && (!Xf->tile_scale || Xf->tile <= 0 || Xf->tile % 128 != 0))
      fail(PF_ERR_ARG, "an FP8 X_filter needs tile_scale with a tile that is a positive multiple of 128");
    if (Xr->dtype == PF_BF16 || Xr->dtype == PF_F8E4M3)
      fail(PF_ERR_ARG, "X_rr must be F32 or F64 (Rayleigh-Ritz runs on the unquantised matrix)");
    if (d.work == PF_F64 && Xr->dtype != PF_F64) fail(PF_ERR_ARG, "work F64 needs an F64 X_rr");
    if (d.work == PF_F32 && Xr->dtype != PF_F32) fail(PF_ERR_ARG, "work F32 needs an F32 X_rr");
  }
}

size_t plan_bytes(const pf_desc& d) { return layout_for(d).total; }

Plan* plan_create(const pf_desc& d, hipStream_t zero_stream, bool async_zero) {
  plan_validate(d, nullptr, nullptr);
  Layout L = layout_for(d);
  Plan* P = new Plan();
  P->d = d;
  P->work = d.work == PF_F64 ? Elem::F64 : Elem::F32;
  P->esz = P->work == Elem::F64 ? 8 : 4;
  P->n = d.n;
  P->n_pad = round_up(d.n, 64);
  P->p = d.p;
  P->p_pad = (int)round_up(d.p, 16);
  P->bytes = L.total;
  hipError_t e = hipMalloc(&P->mem, L.total);
  if (e != hipSuccess) {
    delete P;
    (void)hipGetLastError();
    fail(PF_ERR_NOMEM, "hipMalloc of the extraction workspace failed");
  }
  // zero once: padding rows/columns of every block stay zero forever
  e = async_zero ? hipMemsetAsync(P->mem, 0, L.total, zero_stream) : hipMemset(P->mem, 0, L.total);
  if (e != hipSuccess) {
    (void)hipFree(P->mem);
    delete P;
    fail(PF_ERR_DEVICE, "hipMemset of the workspace failed");
  }
  carve(P, L);
  return P;
}

void enqueue_extraction_in(const pf_desc& d, void* base, const pf_mat& Xf, const pf_mat& Xr, void* U_inout,
                           int64_t ldu, double* theta_out, pf_info* info_out, hipStream_t st) {
  if (d.op != PF_OP_SYM) fail(PF_ERR_UNSUPPORTED, "a caller-placed workspace serves PF_OP_SYM only");
  Layout L = layout_for(d);
  Plan P;
  P.d = d;
  P.work = d.work == PF_F64 ? Elem::F64 : Elem::F32;
  P.esz = P.work == Elem::F64 ? 8 : 4;
  P.n = d.n;
  P.n_pad = round_up(d.n, 64);
  P.p = d.p;
  P.p_pad = (int)round_up(d.p, 16);
  P.bytes = L.total;
  P.mem = base;
  carve(&P, L);
  enqueue_extraction(&P, Xf, Xr, U_inout, ldu, U_inout, ldu, theta_out, info_out, st);
}

namespace {
void carve(Plan* P, const Layout& L) {
  const pf_desc& d = P->d;
  char* b = static_cast<char*>(P->mem);
  P->U = b + L.off_U;
  P->Z = b + L.off_Z;
  for (int i = 0; i < 3; ++i) P->Yb[i] = b + L.off_Y[i];
  P->Q1 = b + L.off_Q1;
  P->Q = b + L.off_Q;
  P->W = reinterpret_cast<double*>(b + L.off_W);
  P->G = reinterpret_cast<double*>(b + L.off_G);
  P->Rinv = reinterpret_cast<double*>(b + L.off_Rinv);
  P->Zeig = reinterpret_cast<double*>(b + L.off_Zeig);
  P->Ework = reinterpret_cast<double*>(b + L.off_E);
  P->refined = reinterpret_cast<int*>(b + L.off_refined);
  P->theta = reinterpret_cast<double*>(b + L.off_theta);
  P->theta_pre = reinterpret_cast<double*>(b + L.off_theta_pre);
  P->deficient = reinterpret_cast<int*>(b + L.off_def);
  P->info = reinterpret_cast<pf_info*>(b + L.off_info);
  P->Xtra = reinterpret_cast<double*>(b + L.off_xtra);
  P->part = b + L.off_part;
  P->plane = P->n_pad * P->p_pad;
  P->Up = P->work == Elem::F32 ? reinterpret_cast<uint16_t*>(b + L.off_Up) : nullptr;
  for (int i = 0; i < 3; ++i)
    P->Ypl[i] = P->work == Elem::F32 ? reinterpret_cast<uint16_t*>(b + L.off_Ypl[i]) : nullptr;
  P->part_bytes = L.part_bytes;
  if (d.op == PF_OP_GRAM) {
    P->m = d.m;
    P->m_pad = round_up(d.m, 64);
    P->T = b + L.off_T;
    P->Tpl = P->work == Elem::F32 ? reinterpret_cast<uint16_t*>(b + L.off_Tpl) : nullptr;
    P->tplane = P->m_pad * P->p_pad;
    P->B = reinterpret_cast<double*>(b + L.off_B);
  }
}
}  // namespace

void plan_destroy(Plan* P) {
  if (!P) return;
  if (P->mem) (void)hipFree(P->mem);
  for (Plan::Copy* c : {&P->mft, &P->mrt}) {
    if (c->data) (void)hipFree(c->data);
    if (c->scale) (void)hipFree(c->scale);
  }
  delete P;
}

void plan_set_desc(Plan* P, const pf_desc& d) { P->d = d; }

size_t plan_device_bytes(const Plan* P) {
  size_t b = P->bytes;
  for (const Plan::Copy* c : {&P->mft, &P->mrt}) b += c->bytes + c->scale_bytes;
  return b;
}

double* plan_theta(Plan* p) { return p->theta; }
pf_info* plan_info(Plan* p) { return p->info; }

namespace {

Elem elem_of(pf_dtype t) { return t == PF_F64 ? Elem::F64 : Elem::F32; }
void contract_into(Plan* P, const void* A, int64_t lda, Elem ta, const void* B, int64_t ldb, Elem tb,
                   int64_t K, int64_t M, void* out, int64_t ldo, Elem to, const void* D1,
                   const void* D2, int64_t ldd, double alpha, double beta, double gamma, bool f64,
                   hipStream_t st, int prof_main, int prof_reduce, bool lower = false);

void contract_into(Plan* P, const void* A, int64_t lda, Elem ta, const void* B, int64_t ldb, Elem tb,
                   int64_t K, int64_t M, void* out, int64_t ldo, Elem to, const void* D1,
                   const void* D2, int64_t ldd, double alpha, double beta, double gamma, bool f64,
                   hipStream_t st, int prof_main, int prof_reduce, bool lower) {
  ContractArgs c;
  c.lower = lower;
  c.A = A; c.lda = lda; c.ta = ta;
  c.B = B; c.ldb = ldb; c.tb = tb;
  c.K = K; c.M = M; c.N = P->p_pad;
  c.out = out; c.ldo = ldo; c.to = to;
  c.D1 = D1; c.ld1 = ldd; c.D2 = D2; c.ld2 = ldd;
  c.alpha = alpha; c.beta = beta; c.gamma = gamma;
  c.part = P->part; c.part_bytes = P->part_bytes;
  c.splitk = 0;
  c.f64_mfma = f64;
  c.prof_main = prof_main;
  c.prof_reduce = prof_reduce;
  contract(c, st);
}

uint16_t* planes_of(Plan* P, const void* y) {
  if (y == P->U) return P->Up;
  for (int i = 0; i < 3; ++i)
    if (y == P->Yb[i]) return P->Ypl[i];
  fail(PF_ERR_DEVICE, "internal: block without BF16 planes");
}

void refresh_planes(Plan* P, const void* y, hipStream_t st) {
  launch_split_planes(static_cast<const float*>(y), P->n_pad, P->n, P->p_pad, planes_of(P, y), P->n_pad, P->plane,
                      P->n_pad, P->p_pad, st);
}

size_t esize_of(pf_dtype t) { return t == PF_F64 ? 8 : t == PF_F32 ? 4 : t == PF_BF16 ? 2 : 1; }

// Transposed copy (n x m, ld = n rounded up to 64 elements) of an m x n operand,
// with the transposed tile-scale grid for FP8.  Rebuilt on every call unless
// PF_FLAG_OPERATOR_UNCHANGED is set and the same buffer was copied last time.
void ensure_copy(Plan* P, Plan::Copy& c, const pf_mat& M, hipStream_t st) {
  const bool same = c.data && c.src == M.data && c.dt == M.dtype && c.src_ld == M.ld &&
                    c.src_scale == M.tile_scale && c.tile == (M.dtype == PF_F8E4M3 ? M.tile : 0);
  if (same && (P->d.flags & PF_FLAG_OPERATOR_UNCHANGED)) return;
  const size_t es = esize_of(M.dtype);
  const int64_t ld = round_up(P->n, 64);          // the copy is n x m: n rows
  const size_t bytes = (size_t)ld * P->m * es;
  if (c.bytes < bytes) {
    if (c.data) (void)hipFree(c.data);
    c.data = nullptr;
    c.bytes = 0;
    if (hipMalloc(&c.data, bytes) != hipSuccess) {
      (void)hipGetLastError();
      fail(PF_ERR_NOMEM, "hipMalloc of the transposed operator copy failed");
    }
    c.bytes = bytes;
  }
  c.ld = ld;
  launch_transpose(M.data, M.ld, P->m, P->n, (int)es, c.data, ld, st);
  c.tile = 0;
  if (M.dtype == PF_F8E4M3) {
    const int64_t gm = (P->m + M.tile - 1) / M.tile, gn = (P->n + M.tile - 1) / M.tile;
    const size_t sb = (size_t)gm * gn * sizeof(float);
    if (c.scale_bytes < sb) {
      if (c.scale) (void)hipFree(c.scale);
      c.scale = nullptr;
      c.scale_bytes = 0;
      if (hipMalloc(&c.scale, sb) != hipSuccess) {
        (void)hipGetLastError();
        fail(PF_ERR_NOMEM, "hipMalloc of the transposed scale grid failed");
      }
      c.scale_bytes = sb;
    }
    launch_transpose(M.tile_scale, gm, gm, gn, 4, c.scale, gn, st);
    c.tile = M.tile;
  }
  c.src = M.data; c.dt = M.dtype; c.src_ld = M.ld; c.src_scale = M.tile_scale;
}

// One split-BF16 product out = alpha A^T Y + beta D1 + gamma D2 with A K x M
// (column-major, any filter dtype) and Y given by its planes.
void split_product(Plan* P, const void* A, int64_t lda, pf_dtype adt, const float* ascale, int tile, int64_t K,
                   int64_t M, const uint16_t* Yp, int64_t ldy, int64_t yplane, void* out, int64_t ldo,
                   const void* D1, const void* D2, double alpha, double beta, double gamma, uint16_t* outp,
                   int64_t oplane, hipStream_t st) {
  FilterArgs f;
  f.X = A; f.ldx = lda; f.xdtype = adt;
  if (adt == PF_F8E4M3) { f.xscale = ascale; f.tile = tile; f.ldsc = (K + tile - 1) / tile; }
  f.Yp = Yp; f.ldy = ldy; f.yplane = yplane;
  f.K = K; f.M = M; f.N = P->p_pad;
  f.out = static_cast<float*>(out); f.ldo = ldo;
  f.D1 = static_cast<const float*>(D1); f.D2 = static_cast<const float*>(D2); f.ldd = ldo;
  f.alpha = alpha; f.beta = beta; f.gamma = gamma;
  f.outp = outp; f.ldop = ldo; f.oplane = oplane;
  f.part = P->part; f.part_bytes = P->part_bytes;
  f.prof_main = PF_PROF_FILTER; f.prof_reduce = PF_PROF_FILTER_REDUCE;
  filter_bf16x6(f, st);
}

// One filter product out = alpha X Y + beta D1 + gamma D2 on the split-BF16
// path (FP32 work) or on the native MFMA path (FP32 with PF_FLAG_NATIVE_F32,
// or FP64).  want_planes: also write the planes of out for the next product.
// Caller-supplied product AY = A Y (pf_operator) into AY, checked.
void operator_product(Plan* P, const pf_operator* op, const void* Y, void* AY, hipStream_t st) {
  const pf_status s = op->apply(op->ctx, Y, P->n_pad, AY, P->n_pad, P->p_pad, st);
  if (s != PF_OK) fail(s, "the operator's apply callback returned an error");
}

void filter_product(Plan* P, const pf_mat& Xf, const void* y, void* out, const void* D1, const void* D2,
                    double alpha, double beta, double gamma, bool want_planes, hipStream_t st,
                    const pf_operator* op) {
  const int64_t ld = P->n_pad;
  if (op) {
    // the caller's product, then the recurrence step around it (W is free
    // until the Rayleigh-Ritz product)
    const bool plain = !D1 && !D2 && alpha == 1.0;
    void* AY = plain ? out : P->W;
    operator_product(P, op, y, AY, st);
    if (!plain) launch_combine(AY, D1, D2, out, ld, P->work, P->n, P->p_pad, alpha, beta, gamma, st);
    return;
  }
  const bool split = P->work == Elem::F32 && !(P->d.flags & PF_FLAG_NATIVE_F32);
  if (P->d.op == PF_OP_GRAM) {
    // T = M Y (contraction over the n columns of M: the transposed copy),
    // then out = alpha M^T T + beta D1 + gamma D2 (contraction over m)
    const Plan::Copy& c = P->mft;
    if (split) {
      split_product(P, c.data, c.ld, Xf.dtype, c.scale, c.tile, P->n, P->m, planes_of(P, y), ld, P->plane, P->T,
                    P->m_pad, nullptr, nullptr, 1.0, 0.0, 0.0, P->Tpl, P->tplane, st);
      split_product(P, Xf.data, Xf.ld, Xf.dtype, Xf.tile_scale, Xf.tile, P->m, P->n, P->Tpl, P->m_pad, P->tplane,
                    out, ld, D1, D2, alpha, beta, gamma, want_planes ? planes_of(P, out) : nullptr, P->plane, st);
    } else {
      contract_into(P, c.data, c.ld, elem_of(Xf.dtype), y, ld, P->work, P->n, P->m, P->T, P->m_pad, P->work,
                    nullptr, nullptr, P->m_pad, 1.0, 0.0, 0.0, P->work == Elem::F64, st, PF_PROF_FILTER,
                    PF_PROF_FILTER_REDUCE);
      contract_into(P, Xf.data, Xf.ld, elem_of(Xf.dtype), P->T, P->m_pad, P->work, P->m, P->n, out, ld, P->work,
                    D1, D2, ld, alpha, beta, gamma, P->work == Elem::F64, st, PF_PROF_FILTER,
                    PF_PROF_FILTER_REDUCE);
    }
    return;
  }
  if (split) {
    FilterArgs f;
    f.X = Xf.data; f.ldx = Xf.ld; f.xdtype = Xf.dtype;
    if (Xf.dtype == PF_F8E4M3) {
      f.xscale = Xf.tile_scale; f.tile = Xf.tile; f.ldsc = (P->n + Xf.tile - 1) / Xf.tile;
    }
    f.Yp = planes_of(P, y); f.ldy = ld; f.yplane = P->plane;
    f.K = P->n; f.M = P->n; f.N = P->p_pad;
    f.out = static_cast<float*>(out); f.ldo = ld;
    f.D1 = static_cast<const float*>(D1); f.D2 = static_cast<const float*>(D2); f.ldd = ld;
    f.alpha = alpha; f.beta = beta; f.gamma = gamma;
    f.outp = want_planes ? planes_of(P, out) : nullptr; f.ldop = ld; f.oplane = P->plane;
    f.part = P->part; f.part_bytes = P->part_bytes;
    f.prof_main = PF_PROF_FILTER; f.prof_reduce = PF_PROF_FILTER_REDUCE;
    filter_bf16x6(f, st);
  } else {
    contract_into(P, Xf.data, Xf.ld, elem_of(Xf.dtype), y, ld, P->work, P->n, P->n, out, ld, P->work, D1, D2, ld,
                  alpha, beta, gamma, P->work == Elem::F64, st, PF_PROF_FILTER, PF_PROF_FILTER_REDUCE);
  }
}

void gram(Plan* P, const void* A, Elem ta, const void* B, Elem tb, double* out, hipStream_t st) {
  contract_into(P, A, P->n_pad, ta, B, P->n_pad, tb, P->n, P->p_pad, out, P->p_pad, Elem::F64, nullptr,
                nullptr, 0, 1.0, 0.0, 0.0, true, st, -1, -1);
}

void apply(Plan* P, const void* A1, const void* A2, const double* S, void* C1, int64_t ldc1, void* C2,
           double alpha, double beta, const int* deficient, const pf_info* gate, hipStream_t st,
           pf_info* info_out = nullptr, double* theta_out = nullptr) {
  ApplyArgs a;
  a.n = P->n; a.p = P->p;
  a.A1 = A1; a.lda1 = P->n_pad; a.ta1 = P->work;
  a.A2 = A2; a.lda2 = P->n_pad; a.ta2 = P->work;
  a.S = S; a.lds_ = P->p_pad;
  a.C1 = C1; a.ldc1 = ldc1; a.tc1 = P->work;
  a.C2 = C2; a.ldc2 = P->n_pad; a.tc2 = P->work;
  a.alpha = alpha; a.beta = beta;
  a.deficient = deficient;
  a.gate = gate;
  a.info_out = info_out;
  a.theta = theta_out ? P->theta : nullptr;
  a.theta_out = theta_out;
  launch_apply(a, st);
}

// Phases of one extraction, in increasing order (grouped launches line up
// the same phase of many extractions).  Filter product t of the whole
// sequence (t = pass * degree + k) is phase kPhFilter + 10 t; the steps
// after the first product of a pass follow it at + 5 ..; orthonormalisation
// and Rayleigh-Ritz come after every product.
constexpr int64_t kPhBegin = 0, kPhFilter = 100, kPhOrth = 1 << 30, kPhRR = kPhOrth + 100;
int64_t ph_product(int64_t t) { return kPhFilter + 10 * t; }

}  // namespace

void enqueue_extraction(Plan* P, const pf_mat& Xf, const pf_mat& Xr, const void* U_in, int64_t ldu_in,
                        void* U_out, int64_t ldu_out, double* theta_out, pf_info* info_out, hipStream_t st,
                        const pf_operator* op, const pf_extras* ex) {
  const pf_desc& d = P->d;
  const double c = 0.5 * (d.a + d.b), e = 0.5 * (d.b - d.a);
  std::vector<double> tau;
  host_coefficients(d, tau);
  const Elem W = P->work;
  const Elem tr = elem_of(Xr.dtype);
  const int64_t ld = P->n_pad;

  if (current_recorder() && (d.op != PF_OP_SYM || op))
    fail(PF_ERR_UNSUPPORTED, "grouped extractions take PF_OP_SYM with a dense operator only");
  if ((int64_t)d.q * d.degree > 10000000) fail(PF_ERR_ARG, "degree * q is too large");
  const bool prof = prof_enabled();
  if (prof) prof_begin(PF_PROF_EXTRACT, st);
  const bool split = W == Elem::F32 && !(d.flags & PF_FLAG_NATIVE_F32) && !op;
  TraceRange trace_all("pf.extract");
  TraceRange trace("pf.begin");
  set_phase(kPhBegin);
  // U_in into the work buffer (with the planes of Y_0 = U for the split
  // filter) and pf_info cleared, in one launch
  launch_begin_block(U_in, ldu_in, W, P->U, ld, P->n, P->p, P->n_pad, P->p_pad, split ? planes_of(P, P->U) : nullptr,
                     P->plane, P->info, st);
  const Plan::Copy* rr_copy = nullptr;
  if (d.op == PF_OP_GRAM) {
    ensure_copy(P, P->mft, Xf, st);
    if (Xr.data == Xf.data && Xr.dtype == Xf.dtype && Xr.ld == Xf.ld) {
      rr_copy = &P->mft;                      // one operator for both: one copy
    } else {
      ensure_copy(P, P->mrt, Xr, st);
      rr_copy = &P->mrt;
    }
  }

  trace.next("pf.filter");
  void* cur = P->U;
  for (int pass = 0; pass < d.q; ++pass) {
    // the planes of Y_0 come with the copy of U; later passes start from
    // Y_d, whose planes the last step wrote
    // first product Z = A Y_0
    const int64_t ph0 = ph_product((int64_t)pass * d.degree);
    set_phase(ph0);
    filter_product(P, Xf, cur, P->Z, nullptr, nullptr, 1.0, 0.0, 0.0, false, st, op);
    const double a1 = 1.0 / (e * tau[1]), b1 = -c / (e * tau[1]);
    void* y_prev;
    void* y_cur;
    set_phase(ph0 + 5);
    if (pass == 0 && !(d.flags & PF_FLAG_NO_PREROTATE)) {
      gram(P, cur, W, P->Z, W, P->G, st);
      set_phase(ph0 + 6);
      launch_eigh(P->G, P->p_pad, P->p, P->theta_pre, P->Zeig, P->p_pad, P->p_pad, P->info, 0, st, P->Ework,
                  P->refined);
      set_phase(ph0 + 7);
      apply(P, cur, P->Z, P->Zeig, P->Yb[0], ld, P->Yb[1], a1, b1, nullptr, nullptr, st);
      y_prev = P->Yb[0];
      y_cur = P->Yb[1];
    } else {
      void* dst = (cur == P->Yb[1]) ? P->Yb[2] : P->Yb[1];
      launch_axpby(P->Z, cur, dst, ld, W, P->n, P->p_pad, a1, b1, st);
      y_prev = cur;
      y_cur = dst;
    }
    set_phase(ph0 + 8);
    if (split && (d.degree > 1 || pass + 1 < d.q)) refresh_planes(P, y_cur, st);
    // re-orthonormalisation of the recurrence pair every `every` products:
    // a cold start (every second one) or dynamic-range control on warm steps
    // (every max(4, ceil(d/2)): once in the middle of a degree-10 filter)
    const int every = ((d.flags & PF_FLAG_COLD) && pass == 0) ? 2
                      : (d.flags & PF_FLAG_REORTH)           ? std::max(4, (d.degree + 1) / 2)
                                                              : 0;
    const bool cold = every > 0;
    if (y_prev == P->U && cold) {
      // keep U intact for re-orthonormalisation: move Y_0 into the ring
      launch_axpby(y_prev, y_prev, P->Yb[0], ld, W, P->n, P->p_pad, 1.0, 0.0, st);
      y_prev = P->Yb[0];
    }
    for (int k = 1; k < d.degree; ++k) {
      void* y_next = nullptr;
      for (int i = 0; i < 3; ++i)
        if (P->Yb[i] != y_cur && P->Yb[i] != y_prev) { y_next = P->Yb[i]; break; }
      const double r = tau[k] / tau[k + 1];
      const double al = 2.0 * r / e, be = -2.0 * c * r / e, ga = -tau[k - 1] / tau[k + 1];
      const bool reorth = cold && (k + 1) % every == 0 && k + 1 < d.degree;
      // planes of Y_{k+1} feed the next product (or the next pass)
      const bool want = split && ((k + 1 < d.degree && !reorth) || (k + 1 == d.degree && pass + 1 < d.q));
      set_phase(ph_product((int64_t)pass * d.degree + k));
      filter_product(P, Xf, y_cur, y_next, y_cur, y_prev, al, be, ga, want, st, op);
      y_prev = y_cur;
      y_cur = y_next;
      if (reorth) {
        // (Y_{k+1}, Y_k) <- (Y_{k+1}, Y_k) R^{-1}, R from CholeskyQR2 of Y_{k+1}
        for (int pass2 = 0; pass2 < 2; ++pass2) {
          void* src_c = pass2 == 0 ? y_cur : P->Q1;
          void* src_p = pass2 == 0 ? y_prev : P->Q;
          void* dst_c = pass2 == 0 ? P->Q1 : y_cur;
          void* dst_p = pass2 == 0 ? P->Q : y_prev;
          gram(P, src_c, W, src_c, W, P->G, st);
          launch_chol_rinv(P->G, P->p_pad, P->p, P->Rinv, P->p_pad, P->deficient, P->info, 0, st);
          apply(P, src_c, src_p, P->Rinv, dst_c, ld, dst_p, 1.0, 0.0, P->deficient, nullptr, st);
        }
        if (split) refresh_planes(P, y_cur, st);
      }
    }
    cur = y_cur;
  }

  // CholeskyQR2 (section 2.1: orthonormalise the filtered block)
  trace.next("pf.orth");
  set_phase(kPhOrth);
  gram(P, cur, W, cur, W, P->G, st);
  set_phase(kPhOrth + 1);
  launch_chol_rinv(P->G, P->p_pad, P->p, P->Rinv, P->p_pad, P->deficient, P->info, 1, st);
  set_phase(kPhOrth + 2);
  apply(P, cur, nullptr, P->Rinv, P->Q1, ld, nullptr, 0.0, 0.0, P->deficient, nullptr, st);
  set_phase(kPhOrth + 3);
  gram(P, P->Q1, W, P->Q1, W, P->G, st);
  // the second pass sees I + E, |E| ~ cond(Y) * eps of the work precision:
  // first order suffices once |E|^2 is below that precision
  set_phase(kPhOrth + 4);
  launch_chol_rinv(P->G, P->p_pad, P->p, P->Rinv, P->p_pad, P->deficient, P->info, 2, st,
                   W == Elem::F64 ? 1e-8 : 3e-4);
  set_phase(kPhOrth + 5);
  apply(P, P->Q1, nullptr, P->Rinv, P->Q, ld, nullptr, 0.0, 0.0, P->deficient, nullptr, st);

  // Rayleigh-Ritz in FP64 (eq. RR)
  trace.next("pf.rayleigh_ritz");
  set_phase(kPhRR);
  if (d.op == PF_OP_GRAM) {
    // B = M Q (FP64), H = B^T B = Q^T (M^T M) Q: theta = sigma^2
    contract_into(P, rr_copy->data, rr_copy->ld, tr, P->Q, ld, W, P->n, P->m, P->B, P->m_pad, Elem::F64, nullptr,
                  nullptr, P->m_pad, 1.0, 0.0, 0.0, true, st, PF_PROF_RR, -1);
    contract_into(P, P->B, P->m_pad, Elem::F64, P->B, P->m_pad, Elem::F64, P->m, P->p_pad, P->G, P->p_pad,
                  Elem::F64, nullptr, nullptr, 0, 1.0, 0.0, 0.0, true, st, -1, -1);
  } else if (op) {
    // W = A Q by the caller's operator (work dtype), H = Q^T W in FP64
    operator_product(P, op, P->Q, P->W, st);
    gram(P, P->Q, W, P->W, W, P->G, st);
  } else {
    // X is symmetric: W = 2 (L + D/2) Q from one triangle (the entries on
    // and above the diagonal), half the products of X Q, and G = Q^T W has
    // the symmetric part Q^T X Q, the part the eigensolver reads.  The
    // residual norms need W = X Q itself.
    const bool half = !(ex && ex->resid);
    contract_into(P, Xr.data, Xr.ld, tr, P->Q, ld, W, P->n, P->n, P->W, ld, Elem::F64, nullptr, nullptr, ld,
                  half ? 2.0 : 1.0, 0.0, 0.0, true, st, PF_PROF_RR, -1, half);
    set_phase(kPhRR + 1);
    gram(P, P->Q, W, P->W, Elem::F64, P->G, st);
  }
  set_phase(kPhRR + 2);
  launch_eigh(P->G, P->p_pad, P->p, P->theta, P->Zeig, P->p_pad, P->p_pad, P->info, 1, st, P->Ework, P->refined);
  // Ritz vectors, with pf_info and theta copied out in the same launch
  set_phase(kPhRR + 3);
  apply(P, P->Q, nullptr, P->Zeig, U_out, ldu_out, nullptr, 0.0, 0.0, nullptr, P->info, st, info_out, theta_out);
  set_phase(kPhRR + 4);
  if (ex && (ex->resid || ex->shrink_left)) {
    if (current_recorder()) fail(PF_ERR_UNSUPPORTED, "grouped extractions have no optional outputs");
    trace.next("pf.outputs");
    double* Gres = P->Xtra;
    double* Zs = P->Xtra + (size_t)P->p_pad * P->p_pad;
    if (ex->resid) {
      if (op) fail(PF_ERR_UNSUPPORTED, "residual norms need a dense operator");
      // W = A Q (the Gram form: M^T B, B = M Q), then E = W - Q H in place;
      // the residual of Ritz pair j is ||E z_j|| (H z_j = theta_j z_j), from
      // the Gram matrix E^T E
      if (d.op == PF_OP_GRAM)
        contract_into(P, Xr.data, Xr.ld, tr, P->B, P->m_pad, Elem::F64, P->m, P->n, P->W, ld, Elem::F64, nullptr,
                      nullptr, ld, 1.0, 0.0, 0.0, true, st, -1, -1);
      launch_rect(P->n, P->p, P->p, P->Q, ld, W, P->G, P->p_pad, P->W, ld, P->W, ld, Elem::F64, st);
      gram(P, P->W, Elem::F64, P->W, Elem::F64, Gres, st);
    }
    launch_extras(P->p, P->p_pad, P->Zeig, Gres, P->theta, ex->resid, ex->shrink_tau,
                  ex->shrink_left ? Zs : nullptr, st);
    // shrink_tau(M P_V) = (B Zs) V^T
    if (ex->shrink_left)
      launch_rect(P->m, P->p, P->p, P->B, P->m_pad, Elem::F64, Zs, P->p_pad, nullptr, 0, ex->shrink_left,
                  ex->ld_shrink, W, st);
  }
  if (prof) prof_end(PF_PROF_EXTRACT, st);
}

void enqueue_extractions_grouped(int count, const ExtractionJob* jobs, hipStream_t st) {
  for (int i = 0; i < count; ++i) {
    if (jobs[i].desc.op != PF_OP_SYM) fail(PF_ERR_UNSUPPORTED, "grouped extractions take PF_OP_SYM only");
    for (int j = 0; j < i; ++j)
      if (jobs[j].plan == jobs[i].plan) fail(PF_ERR_ARG, "grouped extractions need a workspace each");
  }
  grouped_enqueue(
      count,
      [&](int i) {
        const ExtractionJob& j = jobs[i];
        plan_set_desc(j.plan, j.desc);
        enqueue_extraction(j.plan, j.Xf, j.Xr, j.U_in, j.ldu_in, j.U_out, j.ldu_out, j.theta_out, j.info_out, st);
        if (j.info_host) {
          set_phase(kPhRR + 10);
          launch_info_to_host(j.plan->info, j.info_host, st);
        }
      },
      st);
}

}  // namespace pfx
