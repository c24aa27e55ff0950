// Internal declarations of the pfx library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>
#include <string>

#include "../../include/pf.h"

namespace pfx {

// ---------------------------------------------------------------------------
// Errors.  Host code throws pfx::Error; the C-ABI layer converts it to a
// pf_status and a thread-local message.  Kernels never throw.
struct Error {
  pf_status status;
  std::string msg;
};
[[noreturn]] void fail(pf_status s, const std::string& msg);
void check_hip(hipError_t e, const char* what);
#define PFX_HIP(call) ::pfx::check_hip((call), #call)

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Raise a kernel's dynamic-LDS limit to `bytes` when it needs more than the
// 64 KiB default (tracked per kernel in `cur`; the kernel's static LDS plus
// `bytes` must stay within the 160 KiB of a CU).
inline void ensure_lds(const void* kernel, size_t bytes, size_t& cur) {
  if (bytes > 65536 && bytes > cur) {
    PFX_HIP(hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    cur = bytes;
  }
}

// ---------------------------------------------------------------------------
// Contractions C = A^T B over the long dimension K (the hot kernels).
//
// A is K x M and B is K x N, both column-major, so both operands are read
// along K, the contiguous direction: for the symmetric filter product
// X Y = X^T Y the A operand is X itself (section 2.1), for Gram matrices
// Y^T Y and Rayleigh-Ritz H = Q^T W it is the tall block.
enum class Elem : int { F32 = 0, F64 = 1 };

struct ContractArgs {
  const void* A; int64_t lda; Elem ta;
  const void* B; int64_t ldb; Elem tb;
  int64_t K, M, N;          // N is a multiple of 16 (padded block width)
  // epilogue: out = alpha * (A^T B) + beta * D1 + gamma * D2  (D1/D2 optional)
  void* out; int64_t ldo; Elem to;
  const void* D1; int64_t ld1;   // same type as out
  const void* D2; int64_t ld2;
  double alpha, beta, gamma;
  // split-K workspace (S slabs of round_up(M,64) x N in the MFMA type)
  void* part; size_t part_bytes;
  int splitk;               // 0 = choose automatically
  bool f64_mfma;            // contract in FP64 (products and sums) even for F32 operands
  int prof_main = -1;       // profiling class of the product kernel (-1: none)
  int prof_reduce = -1;     // profiling class of the split-K sum
  // A symmetric (K == M) and read on and above its diagonal only (entries
  // (k, m) with k <= m of the column-major A, which by symmetry hold the
  // lower triangle's values): the product is (L + D/2) B with L the strict
  // lower triangle and D the diagonal of A, so that Q^T (L + D/2) Q plus
  // its transpose is Q^T A Q at half the work
  bool lower = false;
};
// Enqueue; returns the split-K factor used.
int contract(const ContractArgs& a, hipStream_t st);
// Partial-workspace bytes contract() needs for these shapes and types.
size_t contract_part_bytes(int64_t K, int64_t M, int64_t N, Elem ta, Elem tb, bool f64_mfma, int splitk);

// ---------------------------------------------------------------------------
// FP32 filter product on BF16 matrix cores (exact three-way split of X in
// registers, Y as three BF16 planes, six cross terms):
// out = alpha X^T Y + beta D1 + gamma D2, optionally also the planes of out.
struct FilterArgs {
  const void* X; int64_t ldx; pf_dtype xdtype = PF_F32;   // F32, BF16 or F8E4M3 (K x M column-major)
  const float* xscale = nullptr; int64_t ldsc = 0; int tile = 0;   // FP8 tile scales
  const uint16_t* Yp; int64_t ldy; int64_t yplane;
  int64_t K, M, N;
  float* out; int64_t ldo;
  const float* D1; const float* D2; int64_t ldd;
  double alpha, beta, gamma;
  uint16_t* outp; int64_t ldop; int64_t oplane;
  void* part; size_t part_bytes;
  int splitk = 0;
  int prof_main = -1, prof_reduce = -1;
};
void filter_bf16x6(const FilterArgs& a, hipStream_t st);
size_t filter_bf16x6_part_bytes(pf_dtype xdt, int64_t K, int64_t M, int64_t N);
// Start of an extraction: copy the start block into the padded work buffer
// (element type t), write its BF16 planes if planes is set (FP32 only) and
// clear *info, in one launch.
void launch_begin_block(const void* src, int64_t lds, Elem t, void* dst, int64_t ldd, int64_t n, int p,
                        int64_t n_pad, int p_pad, uint16_t* planes, int64_t plane, pf_info* info, hipStream_t st);
void launch_split_planes(const float* src, int64_t lds, int64_t n, int p, uint16_t* dst, int64_t ldd,
                         int64_t plane, int64_t n_pad, int p_pad, hipStream_t st);

// ---------------------------------------------------------------------------
// Small dense kernels on p x p matrices (one workgroup each).
// near_tol > 0: when the equilibrated G is within near_tol of I (a second
// CholeskyQR pass), R^{-1} is written from the first-order factor directly.
void launch_chol_rinv(const double* G, int ldg, int p, double* Rinv, int ldr,
                      int* deficient, pf_info* info, int pass, hipStream_t st, double near_tol = 0.0);
// Symmetric eigendecomposition of a p x p FP64 matrix (p <= 128), theta
// descending, Z (ldz >= pad >= p) its eigenvectors, rows and columns
// p..pad-1 of Z set to the identity.  escratch / refined: scratch of
// eig_scratch_bytes(p) and one int; when given, a quadratically convergent
// refinement runs first and the dense solver only where it reports failure.
// which: 1 = Rayleigh-Ritz, 0 = pre-rotation (info fields and tolerances).
void launch_eigh(const double* H, int ldh, int p, double* theta, double* Z, int ldz, int pad, pf_info* info,
                 int which, hipStream_t st, double* escratch = nullptr, int* refined = nullptr);
size_t eig_scratch_bytes(int p);
// H (m x m) whose column blocks of s hold rows 0 .. (j+1)s-1 completed to the
// symmetric matrix (entries below the diagonal blocks mirrored).
void launch_sym_from_block_upper(double* H, int ldh, int m, int s, hipStream_t st);
// Lanczos outputs (extreme Ritz values, residual norms from the residual
// block's Gram G (s x s), status and replaced-column count of *info).
void launch_lanczos_out(const double* theta, const double* Z, int ldz, int m, int s, const double* G,
                        const pf_info* info, pf_bounds* out, hipStream_t st);
// Block Lanczos bounds (pf_lanczos_bounds), stream-ordered on st; scratch
// allocated and freed stream-ordered.
void enqueue_lanczos(const pf_mat& X, int64_t n, const double* V0, int64_t ldv0, int steps, pf_bounds* out,
                     hipStream_t st);

// ---------------------------------------------------------------------------
// Tall-skinny block operations (n x p blocks, p <= 128).
// C1 = A1 * S;  if A2: C2 = alpha * (A2 * S) + beta * C1.
// S is p x p FP64 column-major (ld lds_).  Elem of A1/A2/C1/C2 given.
struct ApplyArgs {
  int64_t n; int p;
  const void* A1; int64_t lda1; Elem ta1;
  const void* A2; int64_t lda2; Elem ta2;
  const double* S; int lds_;
  void* C1; int64_t ldc1; Elem tc1;
  void* C2; int64_t ldc2; Elem tc2;
  double alpha, beta;
  const int* deficient;      // replace flagged columns of C1 (CholQR)
  const pf_info* gate;       // if non-null: skip writes unless gate->status == 0
  // with gate: *info_out = *gate, and theta_out[0..p) = theta when the
  // status is 0 (the step's outputs, in the same launch)
  pf_info* info_out = nullptr;
  const double* theta = nullptr;
  double* theta_out = nullptr;
  // q output columns (0: p), S then p x q; with D (element type of C1,
  // ld ldd, may be C1 itself): C1 = D - A1 S
  int q = 0;
  const void* D = nullptr;
  int64_t ldd = 0;
};
void launch_apply(const ApplyArgs& a, hipStream_t st);

// Copy an n x p block (column-major, ld) into a padded buffer (ld_dst,
// p_pad columns, zero fill of padding columns and rows up to n_pad).
void launch_copy_block(const void* src, int64_t lds, Elem ts, void* dst, int64_t ldd, Elem td,
                       int64_t n, int p, int64_t n_pad, int p_pad, hipStream_t st);
// out = alpha * A + beta * D1 + gamma * D2 on rows < n (D1, D2 optional;
// n x p blocks of one ld and element type)
void launch_combine(const void* A, const void* D1, const void* D2, void* out, int64_t ld, Elem t, int64_t n, int p,
                    double alpha, double beta, double gamma, hipStream_t st);
// dst = alpha * A + beta * B (n x p blocks, same element type)
void launch_axpby(const void* A, const void* B, void* dst, int64_t ld, Elem t, int64_t n, int p,
                  double alpha, double beta, hipStream_t st);
void launch_normal_block(void* dst, int64_t ld, Elem t, int64_t n, int p, uint64_t seed,
                         hipStream_t st);

// quantisers
void launch_quantize_bf16(const float* src, int64_t rows, int64_t cols, int64_t lds,
                          uint16_t* dst, int64_t ldd, hipStream_t st);
void launch_quantize_fp8(const float* src, int64_t rows, int64_t cols, int64_t lds,
                         uint8_t* dst, int64_t ldd, float* scales, int tile, hipStream_t st);
// dst (cols x rows, ld ldd) = src^T (src rows x cols, ld lds), esize 1/2/4/8.
void launch_transpose(const void* src, int64_t lds, int64_t rows, int64_t cols, int esize, void* dst,
                      int64_t ldd, hipStream_t st);
void launch_psd_dense(const void* V, int64_t ldv, Elem t, const double* theta, int64_t n, int p,
                      void* out, int64_t ldo, hipStream_t st);

// ---------------------------------------------------------------------------
// Kernel timing hooks (pf_profile_*): event pairs around launches of a class.
constexpr int kProfClasses = 5;
bool prof_enabled();
void prof_begin(int cls, hipStream_t st);
void prof_end(int cls, hipStream_t st);

// Named host-side ranges for a tracing profiler (roctx; no-ops unless
// PF_ROCTX=1).  TraceRange: one range for a scope; next() closes the
// current range and opens another.
void trace_push(const char* name);
void trace_pop();
struct TraceRange {
  explicit TraceRange(const char* name) { trace_push(name); }
  void next(const char* name) {
    trace_pop();
    trace_push(name);
  }
  ~TraceRange() { trace_pop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

// ---------------------------------------------------------------------------
// Nearest-correlation PFPG loop (k_nce.hip, nce.cpp).
constexpr int kNceMaxRna = 7;   // longest extrapolation window l
int nce_partial_blocks(int64_t n);
void launch_nce_init(const double* x, double* gd, double* B, int64_t ldb, int64_t n, double* hist, hipStream_t st);
// g, per-block partials (2 doubles per block) and stats[4] =
// (||g||^2, sum x, 1/2 sum max(theta,0)^2, #{theta > 0})
void launch_nce_grad(const double* V, int64_t ldv, int p, const double* theta, const double* x, double* g, int64_t n,
                     const pf_info* info, double* partial, double* stats, hipStream_t st);
void launch_nce_step(double* x, const double* g, double tau, const double* gd, double* B, int64_t ldb, int64_t n,
                     double* hist, int64_t ldh, int slot, hipStream_t st);
void launch_nce_diff_gram(const double* hist, int64_t ldh, int64_t n, int m, double* M, hipStream_t st);
void launch_nce_combine(const double* c, int m, double* hist, int64_t ldh, double* x, const double* gd, double* B,
                        int64_t ldb, int64_t n, hipStream_t st);
int64_t drs_partial_blocks(int64_t n);
// one DRS step on the NCE primal (Z += prox(2P - Z) - P, entrywise) and
// stats[4] = (||dZ||^2, ||G - P||^2, max |diag(P) - 1|, #{theta > 0})
void launch_drs_step(double* Z, int64_t ldz, const double* P, int64_t ldp, const double* G, int64_t ldg, int64_t n,
                     double t, const pf_info* info, const double* theta, int p, double* partial, double* stats,
                     hipStream_t st);
void run_nce_pfam(const pf_pfam_opts& o, int64_t n, const double* G, int64_t ldg, double* Z, int64_t ldz, double* X,
                  int64_t ldx, const double* U0, int64_t ldu0, const double* V0, int64_t ldv0, pf_pfam_result* out,
                  double* history, hipStream_t st);
void run_nce_pfpg(const pf_nce_opts& o, int64_t n, const double* G, int64_t ldg, double* x, const double* U0,
                  int64_t ldu0, const double* V0, int64_t ldv0, pf_nce_result* out, double* history, hipStream_t st);

// ---------------------------------------------------------------------------
// The extraction pipeline.
struct Plan;
// zero_stream: clear the workspace with hipMemsetAsync on that stream (the
// stream the plan is first used on) instead of a synchronous hipMemset.
Plan* plan_create(const pf_desc& d, hipStream_t zero_stream = nullptr, bool async_zero = false);
void plan_destroy(Plan* p);
size_t plan_bytes(const pf_desc& d);
void plan_validate(const pf_desc& d, const pf_mat* Xf, const pf_mat* Xr);
// Enqueue one extraction.  U_in (ld ldu_in) may alias U_out.
// With op, the caller's operator takes the place of Xf and Xr (PF_OP_SYM;
// no BF16 split).
// ex: optional outputs (residual norms, the Gram form's shrinkage), or null.
void enqueue_extraction(Plan* plan, const pf_mat& Xf, const pf_mat& Xr, const void* U_in,
                        int64_t ldu_in, void* U_out, int64_t ldu_out, double* theta_out,
                        pf_info* info_out, hipStream_t st, const pf_operator* op = nullptr,
                        const pf_extras* ex = nullptr);
// One PF_OP_SYM extraction whose workspace (plan_bytes(d) bytes, cleared by
// the caller, 256-byte aligned) starts at base: no allocation.  U_inout is
// both the start block and the output.
void enqueue_extraction_in(const pf_desc& d, void* base, const pf_mat& Xf, const pf_mat& Xr, void* U_inout,
                           int64_t ldu, double* theta_out, pf_info* info_out, hipStream_t st);
// Many independent PF_OP_SYM extractions with dense operators, enqueued on
// st as grouped launches (each phase of every job in as few launches as its
// kernel instances allow).  Jobs must use distinct plans.  Each job's
// results are bitwise those of enqueue_extraction alone.  info_host, when
// set, receives the job's pf_info (a mapped pinned address) at the end.
struct ExtractionJob {
  Plan* plan;
  pf_desc desc;
  pf_mat Xf, Xr;
  const void* U_in; int64_t ldu_in;
  void* U_out; int64_t ldu_out;
  double* theta_out;
  pf_info* info_out;
  pf_info* info_host = nullptr;
};
void enqueue_extractions_grouped(int count, const ExtractionJob* jobs, hipStream_t st);
// refresh the numeric fields (interval, flags) of a cached plan
void plan_set_desc(Plan* P, const pf_desc& d);
// device bytes a plan holds (workspace and operator copies)
size_t plan_device_bytes(const Plan* P);
// plan-owned buffers (for sessions)
double* plan_theta(Plan* p);
pf_info* plan_info(Plan* p);

// ---------------------------------------------------------------------------
// Session state shared by pf_session_* and the server: the warm-start block
// V (updated in place by every step), theta, the device info record, and
// the workspace plan.
struct SessionCore {
  Plan* plan = nullptr;
  pf_desc desc{};
  void* U = nullptr;        // n_pad x p, work dtype
  int64_t ldu = 0;
  double* theta = nullptr;
  pf_info* info = nullptr;
  int64_t steps = 0;
  int device = 0;
};
// Device bytes a session holds (workspace, block, theta, info).
size_t session_bytes(const pf_desc& d);
// Allocate and initialise (U0 copied, or N(0,1) from seed when U0 is NULL),
// stream-ordered on st; sync: wait for the initialisation on the host.
SessionCore* session_create(const pf_desc& d, const void* U0, int64_t ldu0, uint64_t seed, hipStream_t st,
                            bool sync);
void session_destroy(SessionCore* s);
// Enqueue one step on st (the first step of a session runs as a cold start).
void session_enqueue_step(SessionCore* s, const pf_mat& Xf, const pf_mat& Xr, hipStream_t st,
                          const pf_operator* op = nullptr, const pf_extras* ex = nullptr);
// Copy the info record of the last step to host-visible memory (a mapped
// pinned buffer), stream-ordered: the host reads it once the step is done.
void launch_info_to_host(const pf_info* src, pf_info* host_mapped, hipStream_t st);
// C (n x q, ld ldc) = D - A S (D FP64 n x q, may be C) or A S (D null);
// A n x p, S p x q FP64; element types (ta, tc): (F64, F64), (F32, F64),
// (F64, F32).  FP64 accumulation.
void launch_rect(int64_t n, int p, int q, const void* A, int64_t lda, Elem ta, const double* S, int64_t lds_,
                 const double* D, int64_t ldd, void* C, int64_t ldc, Elem tc, hipStream_t st);
// resid[j] = sqrt(z_j^T G z_j) (resid may be null); Zs[:, j] = z_j *
// max(sqrt(theta_j) - tau, 0) / sqrt(theta_j) (Zs may be null); j < p.
void launch_extras(int p, int ld, const double* Z, const double* G, const double* theta, double* resid, double tau,
                   double* Zs, hipStream_t st);

}  // namespace pfx
