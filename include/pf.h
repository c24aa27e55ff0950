/*
 * pf.h -- polynomial-filtered subspace extraction on one MI355X (gfx950).
 *
 * One *extraction* is the step PFPG and PFAM call each iteration in place of
 * a full eigendecomposition (Li, Liu, Wen, Yuan, arXiv 1904.10585):
 *
 *   1. Chebyshev filter  Y = rho(A)^q U,  rho(t) = T_d((t - c)/e),
 *      c = (a+b)/2, e = (b-a)/2 (section 2.1, eq. cheb, eq. cheb-linear-map),
 *      evaluated by the three-term recurrence
 *          Y_1 = (A Y_0 - c Y_0)/e,  Y_{k+1} = 2 (A Y_k - c Y_k)/e - Y_{k-1}
 *      (section 4, eq. cheby-recursion-map, read with the t-coefficient
 *      2/(b-a));
 *   2. orthonormalisation of Y (section 2.1, eq. subspace-update: U+ =
 *      orth(rho(A) U)), done on the device by CholeskyQR2;
 *   3. Rayleigh-Ritz (section 2.2, eq. RR): H = Q^T X Q, H = Z Theta Z^T,
 *      Ritz vectors V = Q Z, which give the low-rank projection
 *      P_V(X) = V Theta V^T and the PSD projection P_+(P_V(X)) of
 *      eq. PFAM1 (keep theta_i > 0).
 *
 * A is either a dense symmetric X (PF_OP_SYM) or A = M^T M for a
 * rectangular M (PF_OP_GRAM, the SVD route of section 5.2.1; the Ritz
 * values are then sigma^2 and Rayleigh-Ritz runs on B = M Q).
 *
 * Conventions
 *  - Every matrix is column-major with a leading dimension (BLAS style).
 *  - Every data pointer passed to the library is DEVICE memory on the
 *    current HIP device unless the argument says "host".
 *  - Calls are stream-ordered on the given hipStream_t (passed as void*;
 *    NULL = the default stream).  They return as soon as the work is
 *    enqueued; argument errors are detected synchronously before any work
 *    is enqueued and leave every output untouched.
 *  - Numerical outcomes (Cholesky breakdown,
 *    non-finite data) are written by the device into a pf_info record
 *    once the stream reaches the end of the extraction.
 *  - No C++ exception crosses this boundary.  pf_last_error() returns a
 *    thread-local message for the last non-PF_OK status of this thread.
 *  - The library is not re-entrant per session; distinct sessions and
 *    distinct pf_extract calls on distinct streams may run concurrently.
 */
#ifndef PF_H
#define PF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PF_ABI_VERSION 3

typedef enum pf_status {
  PF_OK = 0,
  PF_ERR_ARG = 1,         /* invalid argument (see pf_last_error) */
  PF_ERR_NOMEM = 2,       /* device or host allocation failed */
  PF_ERR_DEVICE = 3,      /* a HIP runtime call failed */
  PF_ERR_BREAKDOWN = 4,   /* Cholesky of the Gram matrix broke down */
  PF_ERR_NOCONV = 5,      /* reserved: the eigensolver is direct and always ends */
  PF_ERR_NONFINITE = 6,   /* Inf/NaN met in the filtered block */
  PF_ERR_BUSY = 7,        /* session has work in flight */
  PF_ERR_UNSUPPORTED = 8  /* valid request the library does not implement */
} pf_status;

typedef enum pf_dtype {
  PF_F64 = 0,
  PF_F32 = 1,
  PF_BF16 = 2,
  PF_F8E4M3 = 3  /* OCP E4M3FN, with one FP32 scale per tile x tile block */
} pf_dtype;

typedef enum pf_op {
  PF_OP_SYM = 0,  /* A = X, X n-by-n symmetric */
  PF_OP_GRAM = 1  /* A = M^T M, M m-by-n */
} pf_op;

/* Flags of pf_desc.flags. */
#define PF_FLAG_NO_PREROTATE 0x1u /* skip the Ritz rotation of U by X U before
                                     the recurrence (on by default: it keeps
                                     every column of the recurrence dominated
                                     by one eigen-direction, which the FP32
                                     forms need; the span is unchanged) */
#define PF_FLAG_SCALED 0x2u       /* divide step k of the recurrence by
                                     T_k(s_ref), s_ref = mapped spec_ub: the
                                     same span, no overflow for large |A| */
#define PF_FLAG_NATIVE_F32 0x8u   /* F32 filter products on the FP32 MFMA
                                     pipe instead of the default exact
                                     three-way BF16 split (six BF16 MFMA
                                     cross terms, FP32 accumulation) */
#define PF_FLAG_OPERATOR_UNCHANGED 0x10u /* PF_OP_GRAM: X_filter / X_rr hold the
                                     same values as in the previous call on
                                     this stream (or session) with the same
                                     buffers, so the library may reuse its
                                     transposed copies of M instead of
                                     rebuilding them (a fixed M over a chain
                                     of extractions) */
#define PF_FLAG_REORTH 0x20u      /* dynamic-range control on warm steps: every
                                     max(4, ceil(degree / 2)) products (once,
                                     in the middle, for degree 10) the pair
                                     (Y_k, Y_{k-1}) is
                                     multiplied by the same R^{-1} from a
                                     CholeskyQR2 of Y_k (as on cold steps,
                                     where it happens every second product).
                                     With the columns ordered by descending
                                     Ritz value this removes from each column
                                     the components along the faster-growing
                                     directions before they swamp it: an FP32
                                     filter then keeps the smallest wanted
                                     directions when the growth ratio between
                                     the largest and the smallest wanted
                                     eigenvalue is far beyond single
                                     precision (a damping interval at the
                                     bulk's edge).  Same span; costs two Gram
                                     products, Cholesky factors and applies
                                     per re-orthonormalisation. */
#define PF_FLAG_COLD 0x4u         /* the start block is not a warm start:
                                     every second step the pair (Y_k, Y_{k-1})
                                     is multiplied by the same R^{-1} from a
                                     CholeskyQR2 of Y_k, which keeps the block
                                     well conditioned and (the recurrence
                                     acting column by column) leaves the span
                                     of the result unchanged.  Sessions set it
                                     on their first step. */

/* PF_OP_GRAM (section 5.2.1): X_filter and X_rr are M, m-by-n column-major.
 * Every filter product A Y is T = M Y followed by M^T T (the Chebyshev
 * epilogue fused into the second); the products over the n columns of M read
 * a transposed copy of M that the library builds in device memory it owns
 * (n x m in the dtype of the operand, allocated on first use, rebuilt on each
 * call unless PF_FLAG_OPERATOR_UNCHANGED).  Rayleigh-Ritz forms B = M Q and
 * H = B^T B in FP64: theta_i = sigma_i^2, V the right Ritz vectors.  With a
 * large spectrum (sigma^2 up to 1e8 at the 12000 x 6000 workload) the
 * recurrence needs PF_FLAG_SCALED with spec_ub >= sigma_max^2. */

/* A matrix operand.  data: device pointer; rows/cols implied by the call;
 * ld: leading dimension in elements (>= rows; a multiple of 16 bytes /
 * element size).  For PF_F8E4M3, tile_scale points to ceil(rows/tile) x
 * ceil(cols/tile) FP32 scales, column-major with leading dimension
 * ceil(rows/tile); element value = code * scale of its tile. */
typedef struct pf_mat {
  const void* data;
  pf_dtype dtype;
  int64_t ld;
  const float* tile_scale;
  int32_t tile;
} pf_mat;

/* Problem description.  struct_size must be sizeof(pf_desc) (versioning). */
typedef struct pf_desc {
  uint32_t struct_size;
  pf_op op;
  int64_t n;        /* order of A (columns of M for PF_OP_GRAM) */
  int64_t m;        /* rows of M (PF_OP_GRAM only) */
  int32_t p;        /* block size, 1 <= p <= min(n, 128) */
  int32_t degree;   /* Chebyshev degree d >= 1 */
  int32_t q;        /* filter power q >= 1 (eq. pfpg2) */
  double a, b;      /* damping interval, a < b: eigenvalues in [a, b] are
                       damped, those above b amplified (section 4.1) */
  double spec_ub;   /* PF_FLAG_SCALED: an upper bound of the spectrum of A
                       (> b); ignored otherwise */
  pf_dtype work;    /* PF_F64 or PF_F32: storage of U, Y, Q, V */
  uint32_t flags;
  int32_t reserved;   /* must be 0 */
} pf_desc;

/* Written by the device at the end of an extraction (device memory). */
typedef struct pf_info {
  int32_t status;       /* pf_status of the numerical phase */
  int32_t n_pos;        /* #{theta_i > 0} */
  int32_t dense_rr;     /* 1: the Rayleigh-Ritz eigensolve needed the dense
                           solver, on the whole matrix (the refinement could
                           not converge) or on its clusters of coupled Ritz
                           values (dense_rows) */
  int32_t dense_pre;    /* 1: the pre-rotation needed the dense solver */
  int32_t deficient;    /* columns replaced because the block lost rank */
  int32_t refine_rr;    /* refinement iterations of the Rayleigh-Ritz
                           eigensolve (meaningless when dense_rr = 1) */
  int32_t refine_pre;   /* refinement iterations of the pre-rotation */
  int32_t dense_rows;   /* when dense_rr = 1 after a refinement that left
                           clusters of coupled Ritz values (refine_rr > 0):
                           the rows of the block the dense solver took (the
                           clusters only); otherwise 0 */
} pf_info;

/* One extraction (section 2.1 then eq. RR).
 *  X_filter: the operator the filter applies (X n-by-n, or M m-by-n for
 *            PF_OP_GRAM); F64 (work F64), F32/BF16/F8E4M3 (work F32).
 *  X_rr:     the operator Rayleigh-Ritz projects; same shape; F64 or F32
 *            (may equal X_filter).  BF16/FP8 filters need an F32 X_rr.
 *            PF_OP_SYM: X is symmetric, and Rayleigh-Ritz reads the
 *            entries X_rr[i][j] with i <= j only (on and above the
 *            diagonal; Q^T X Q as the symmetric part of 2 Q^T (L + D/2) Q,
 *            L the strict lower triangle, whose values these hold) unless
 *            residual norms are asked for (pf_extras.resid), which use the
 *            whole X_rr.
 *  U_inout:  n-by-p block in the work dtype, leading dimension ldu >= n.
 *            In: start block (any full-rank block; Ritz vectors of the
 *            previous call for a warm start).  Out: the Ritz vectors V,
 *            ordered by descending theta.  Left untouched if the device
 *            reports a numerical error.
 *  theta_out: p doubles (device), Ritz values in descending order
 *            (sigma^2 for PF_OP_GRAM).
 *  info_out: device pf_info, may be NULL.
 *  stream:   hipStream_t or NULL.
 * Returns PF_OK once enqueued (PF_ERR_ARG / PF_ERR_NOMEM / PF_ERR_DEVICE
 * synchronously).  Workspace is allocated on first use for a shape and
 * reused; the call is stream-ordered with respect to it. */
pf_status pf_extract(const pf_desc* desc, const pf_mat* X_filter, const pf_mat* X_rr,
                     void* U_inout, int64_t ldu, double* theta_out, pf_info* info_out,
                     void* stream);

/* Optional outputs of an extraction, computed from the Rayleigh-Ritz step's
 * own buffers after the Ritz vectors are written (struct_size must be
 * sizeof(pf_extras); unused members NULL / 0).
 *  resid:       device, p doubles, or NULL.  Residual norms
 *               ||A v_i - theta_i v_i||_2 of the Ritz pairs (the convergence
 *               measure of eq. RR), in the order of theta.  Formed in FP64
 *               as the column norms of E Z with E = A Q - Q H (Q the
 *               orthonormal block, H = Q^T A Q, Z its eigenvectors), so they
 *               are those of the FP64 Ritz vectors Q Z; one Gram product of
 *               E and one block apply.  PF_OP_GRAM adds one product M^T (M Q)
 *               over X_rr.  Not available with a caller-supplied operator.
 *  shrink_left: PF_OP_GRAM only: device m-by-p block (work dtype, leading
 *               dimension ld_shrink >= m), or NULL.  The singular-value
 *               shrinkage of section 5.2.1 (the proximal map of
 *               shrink_tau * nuclear norm) applied to M restricted to the
 *               Ritz subspace: M P_V = B V^T with B = M V, whose columns are
 *               orthogonal with norms sigma_i = sqrt(theta_i), so
 *                 shrink_tau(M P_V) = L V^T,
 *                 L = B diag(max(sigma_i - shrink_tau, 0) / sigma_i)
 *               (columns with sigma_i = 0 are zero).  The library writes L;
 *               the right factor is the V the call returns.
 *  shrink_tau:  the threshold, finite and >= 0.
 * Outputs are written even when the step reports a numerical error in
 * pf_info (they are then meaningless). */
typedef struct pf_extras {
  uint32_t struct_size;
  int32_t reserved;          /* must be 0 */
  double* resid;
  double shrink_tau;
  void* shrink_left;
  int64_t ld_shrink;
} pf_extras;

/* pf_extract with optional outputs (extras may be NULL: then exactly
 * pf_extract). */
pf_status pf_extract_ex(const pf_desc* desc, const pf_mat* X_filter, const pf_mat* X_rr, void* U_inout,
                        int64_t ldu, double* theta_out, pf_info* info_out, const pf_extras* extras,
                        void* stream);

/* pf_extract without device allocation, for callers that cannot call
 * hipMalloc: code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation.  Same arguments, semantics and results as
 * pf_extract for PF_OP_SYM (bitwise: the same kernels run); the workspace is
 * a fixed device array inside the library, 64 MiB on every device the
 * library runs on (pf_extract_noalloc_max_bytes()), held until the process
 * ends.  Shapes whose workspace (pf_workspace_size) exceeds it are rejected
 * with PF_ERR_ARG; PF_OP_GRAM with PF_ERR_UNSUPPORTED.  Each call clears the
 * part of the array it uses with a kernel (no memset, so it can be
 * captured).  All calls on one device share that array: calls that overlap
 * on one device (on different streams, or from several threads without
 * stream order between them) race and give undefined results. */
pf_status pf_extract_noalloc(const pf_desc* desc, const pf_mat* X_filter, const pf_mat* X_rr,
                             void* U_inout, int64_t ldu, double* theta_out, pf_info* info_out,
                             void* stream);
size_t pf_extract_noalloc_max_bytes(void);

/* Many independent extractions in one call: the blocks of a block-diagonal
 * operator (the per-block filtering of block-diagonal SDPs in section 5),
 * or any set of small problems.  Block i is exactly
 *   pf_extract(&descs[i], &X_filter[i], &X_rr[i], U_inout[i], ldu[i],
 *              theta_out[i], info_out ? info_out[i] : NULL, ...)
 * (the same kernels, bitwise the same results), but the blocks share their
 * launches: every phase of the extraction (a filter product, a Gram matrix,
 * a Cholesky factor, a p x p eigensolve, a block apply) is one grouped
 * launch per kernel instance over all blocks, enqueued on `stream`, each
 * block with its own workspace (cached per stream and shape, one per block
 * of a shape in the call).  Blocks on PF_OP_GRAM run one after another
 * before the grouped ones.
 * Every block is validated before any work is enqueued (PF_ERR_ARG names
 * the block in pf_last_error); numerical outcomes land in each info_out[i].
 * Arrays are host arrays of count entries; info_out may be NULL. */
pf_status pf_extract_batch(int32_t count, const pf_desc* descs, const pf_mat* X_filter, const pf_mat* X_rr,
                           void* const* U_inout, const int64_t* ldu, double* const* theta_out,
                           pf_info* const* info_out, void* stream);

/* A caller-supplied symmetric operator in place of a dense X (matrix-free
 * or sparse A; the paper's extraction only ever needs the products A Y).
 * apply(ctx, Y, ldy, AY, lday, cols, stream) enqueues AY = A Y on stream for
 * an n-by-cols device block Y in the work dtype (column-major; cols is p
 * rounded up to a multiple of 16, the columns past p are zero) into AY of
 * the same shape and dtype, and returns PF_OK once enqueued (any other
 * value aborts the extraction with that status).  The library calls it d q
 * + 1 times per extraction (every filter product and the Rayleigh-Ritz
 * product) from the calling thread; the recurrence, CholeskyQR,
 * Rayleigh-Ritz Gram and p x p eigensolve stay in the library's kernels
 * (the Gram accumulated in FP64; the product's own precision is the
 * caller's).  Forms: PF_OP_SYM with work FP32 or FP64; PF_FLAG_NATIVE_F32
 * is implied (no BF16 split). */
typedef pf_status (*pf_apply_fn)(void* ctx, const void* Y, int64_t ldy, void* AY, int64_t lday, int32_t cols,
                                 void* stream);
typedef struct pf_operator {
  pf_apply_fn apply;
  void* ctx;
} pf_operator;

/* pf_extract with the operator in place of X_filter and X_rr. */
pf_status pf_extract_op(const pf_desc* desc, const pf_operator* op, void* U_inout, int64_t ldu,
                        double* theta_out, pf_info* info_out, void* stream);

/* Sessions: a warm-started chain of extractions (eq. pfpg2 / eq. PFAM2:
 * U^{k+1} = orth(rho(X^{k+1}) U^k)), whose subspace stays on the device.
 *  U0: device n-by-p block in the work dtype (ld ldu0), or NULL for an
 *      N(0,1) start drawn on the device from seed. */
typedef struct pf_session pf_session;

typedef struct pf_result {
  int32_t status;          /* host copy of pf_info.status (after wait) */
  int32_t n_pos;           /* host copy of pf_info.n_pos (after wait) */
  const double* theta;     /* device, p values, valid until next step/close */
  const void* V;           /* device n-by-p Ritz vectors (work dtype) */
  int64_t ldv;
  const pf_info* info;     /* device */
  const double* resid;     /* device residual norms of the last step
                              (pf_session_step_ex with extras->resid), else NULL */
  double resid_max;        /* their maximum (after wait), else NaN */
} pf_result;

pf_status pf_session_open(const pf_desc* desc, const void* U0, int64_t ldu0, uint64_t seed,
                          pf_session** out);
/* Enqueue one step on X (and X_rr) on the stream; out (host) receives
 * device pointers immediately and host status fields after pf_session_wait. */
pf_status pf_session_step(pf_session* s, const pf_mat* X_filter, const pf_mat* X_rr,
                          pf_result* out, void* stream);
/* pf_session_step with optional outputs (pf_extras; NULL: pf_session_step).
 * extras->resid and extras->shrink_left are caller-owned device buffers
 * written by this step. */
pf_status pf_session_step_ex(pf_session* s, const pf_mat* X_filter, const pf_mat* X_rr, const pf_extras* extras,
                             pf_result* out, void* stream);
/* Block until the session's last step is done; fills out->status/n_pos. */
pf_status pf_session_wait(pf_session* s, pf_result* out);
/* Free the session.  PF_ERR_BUSY if a step is still in flight. */
pf_status pf_session_close(pf_session* s);

/* Checkpoint and resume of a session.  The state of a warm chain is its
 * subspace: the block U (the Ritz vectors of the last step), theta, the
 * descriptor (interval, degree and power as last set) and the step count
 * (a session's first step is a cold start, later ones are warm).
 * pf_session_export waits for the session's last step, then copies U
 * (n-by-p, work dtype, into the caller's device buffer U_out, ld ldu >= n)
 * and theta (p doubles, device, may be NULL) on stream, and fills *state.
 * pf_session_import opens a session from such a state: its next step is
 * the step the exported session would have taken, bitwise (the same
 * kernels on the same U).  U and theta are device pointers (theta may be
 * NULL: then the session's theta reads zero until its first step); the
 * import reads them on the null stream and returns once they are copied,
 * so work that writes them must be complete (or ordered before the null
 * stream) when it is called. */
typedef struct pf_session_state {
  uint32_t struct_size;    /* sizeof(pf_session_state) */
  int32_t reserved;        /* 0 */
  pf_desc desc;
  int64_t steps;           /* steps taken */
} pf_session_state;
pf_status pf_session_export(pf_session* s, void* U_out, int64_t ldu, double* theta_out, pf_session_state* state,
                            void* stream);
pf_status pf_session_import(const pf_session_state* state, const void* U, int64_t ldu, const double* theta,
                            pf_session** out);

/* ------------------------------------------------------------------------
 * Serving loop: many warm-started sessions of different n, p, degree and
 * operator, driven by a stream of step requests (the per-iteration calls of
 * many PFPG/PFAM solvers sharing one GPU).
 *
 *  - Admission by HBM footprint: a session is resident (workspace, V, theta)
 *    only while its footprint fits the budget; sessions opened while the
 *    budget is full wait in FIFO order and are admitted as closed sessions
 *    free memory.  footprint = the session's device bytes + operator_bytes
 *    (what the caller declares for its X, so that the budget covers it).
 *  - Continuous batching: a worker thread takes the next requested step of
 *    every ready resident session (its previous step done) on PF_OP_SYM into
 *    one batch of grouped launches: each phase of the extraction is one
 *    launch per kernel instance for the whole batch, whatever the sessions'
 *    n, p, degree and interval; steps requested while max_batches batches
 *    run wait and form the next batch (on the next of the worker's
 *    streams) when one finishes, so batches stay large under load and
 *    overlap on the device.
 *  - HIP graphs: sessions on PF_OP_GRAM run their own steps; a session's
 *    first step runs eagerly (cold start); its warm step is captured once
 *    as a graph and replayed for later steps whose operator buffers are the
 *    ones captured (re-captured when they change).
 *  - Closed sessions leave their device memory to later sessions of the
 *    same shape; it is freed (a device synchronisation) only when the budget
 *    needs the room for another shape.
 *  - Every finished step produces a pf_server_event with host timestamps
 *    (steady clock, ns) of submission, launch and observed completion.
 *  - Results of a session are bitwise the same whether it runs alone or in
 *    a mix (its kernels are deterministic and touch only its own buffers).
 * All pf_server_* calls are thread-safe.  Operator buffers passed to
 * pf_server_submit must stay valid and unmodified until that step's event.
 * While a server runs, other threads synchronise their own streams or
 * events, not the whole device: hipDeviceSynchronize fails while the worker
 * is capturing a graph. */
typedef struct pf_server pf_server;

#define PF_SERVER_NO_GRAPHS 0x1u    /* launch warm steps eagerly, no capture */
#define PF_SERVER_NO_GROUPING 0x2u  /* every session runs its own steps (no batches) */

typedef struct pf_server_config {
  uint32_t struct_size;   /* sizeof(pf_server_config) */
  uint32_t flags;
  size_t hbm_budget;      /* bytes sessions may hold together (> 0) */
  int32_t max_active;     /* resident sessions at most (0 = 64) */
  int32_t streams;        /* HIP streams of the worker (0 = 8, at most 64) */
  int32_t max_batches;    /* batches in flight at most (0 = 4): ready steps
                             wait for the next batch while this many run */
  int32_t reserved;       /* 0 */
} pf_server_config;

typedef struct pf_server_event {
  int32_t session;
  int32_t status;         /* pf_status of the step (numerical or PF_ERR_DEVICE) */
  int32_t n_pos;
  int32_t graph;          /* 1 if the step ran as a graph replay */
  int64_t step;           /* 0-based index of the step within its session */
  uint64_t tag;           /* the caller's tag from pf_server_submit */
  int64_t submit_ns, launch_ns, done_ns;
} pf_server_event;

typedef struct pf_server_stats {
  int32_t active, waiting;
  size_t used_bytes;
  int64_t launched, completed, graph_launches, captures;
  int64_t batches;        /* batches of grouped launches */
  int64_t batched_steps;  /* steps that ran in them */
} pf_server_stats;

pf_status pf_server_create(const pf_server_config* cfg, pf_server** out);
/* Open a session (waits for admission inside the server; returns at once).
 * U0: device n x p block in the work dtype that stays valid until the
 * session's first step has completed, or NULL for an N(0,1) start from seed.
 * PF_ERR_NOMEM if its footprint alone exceeds the budget. */
pf_status pf_server_open(pf_server* s, const pf_desc* desc, const void* U0, int64_t ldu0, uint64_t seed,
                         size_t operator_bytes, int32_t* session);
/* Queue one step of a session on (X_filter, X_rr); steps of one session run
 * in submission order. */
pf_status pf_server_submit(pf_server* s, int32_t session, const pf_mat* X_filter, const pf_mat* X_rr,
                           uint64_t tag);
/* Up to max finished-step events; waits up to timeout_ns for the first. */
pf_status pf_server_poll(pf_server* s, pf_server_event* events, int32_t max, int32_t* count, int64_t timeout_ns);
/* Device pointers of a resident session's theta / V (valid until its next
 * step is launched or it is closed). PF_ERR_BUSY while a step is queued or
 * running, PF_ERR_ARG if the session is not resident. */
pf_status pf_server_result(pf_server* s, int32_t session, pf_result* out);
/* Close a session once its queued steps are done; frees its memory. */
pf_status pf_server_close(pf_server* s, int32_t session);
pf_status pf_server_stats_get(pf_server* s, pf_server_stats* out);
/* Finish every queued step, free every session, stop the worker. */
pf_status pf_server_destroy(pf_server* s);

/* Quantise an FP32 matrix (rows x cols, ld) into BF16 (dst ld = ld_dst) or
 * FP8-E4M3 codes with FP32 per-tile scales amax/448 (tile x tile,
 * column-major scale grid).  Round to nearest even; FP8 saturates at 448. */
pf_status pf_quantize(void* dst, int64_t ld_dst, float* tile_scale, int32_t tile,
                      pf_dtype dtype, const float* src, int64_t rows, int64_t cols,
                      int64_t ld_src, void* stream);

/* The p x p eigenproblem of Rayleigh-Ritz (section 2.2, eq. RR) on its own:
 * H = Z diag(theta) Z^T for the symmetric part (H + H^T)/2 of an FP64
 * matrix, 1 <= p <= 128, by the solver an extraction falls back to (a
 * direct dense solver in one workgroup: Householder tridiagonalisation,
 * bisection, inverse iteration with reorthogonalisation in clusters).
 *  H:     device, column-major p x p, ldh >= p; read only.
 *  theta: device, p values, written in descending order.
 *  Z:     device, column-major, ldz >= p; columns 0..p-1 (rows 0..p-1)
 *         written with the orthonormal eigenvectors in theta's order.
 * H and Z must not overlap.  Asynchronous on stream.  For p > 64 the
 * solver runs as a chain of kernels whose state (about 1.3 MB) is taken
 * with a stream-ordered allocation and freed on the stream after it; a
 * failed allocation returns PF_ERR_NOMEM.  A non-finite entry in H gives
 * NaN theta and Z = I; H = 0 gives theta = 0 and Z = I.
 * Accuracy: |theta_i - lambda_i| and ||H z_i - theta_i z_i|| of a few
 * eps ||H||, Z orthonormal to ~1e-13. */
pf_status pf_eigh(const double* H, int64_t ldh, int32_t p, double* theta, double* Z, int64_t ldz,
                  void* stream);

/* Dense PSD projection P_+ = V_+ diag(theta_+) V_+^T (eq. PFAM1) from the
 * Ritz pairs of an extraction: out n-by-n (work dtype), ld_out >= n. */
pf_status pf_psd_dense(const void* V, int64_t ldv, const double* theta, int64_t n, int32_t p,
                       pf_dtype work, void* out, int64_t ld_out, void* stream);

/* Spectrum bounds by block Lanczos: the estimate of the smallest eigenvalue
 * that places the left end a of the damping interval (section 4.1, which
 * names the Lanczos method for it).  The start block V0 (n-by-16 FP64,
 * device, ld ldv0 >= n; the caller draws it) spans the first block of the
 * Krylov space K = span{V0, X V0, ..., X^(steps-1) V0}; each block step is
 * one pass over X (products accumulated in FP64), the new block is
 * orthogonalised against all earlier ones and orthonormalised by block
 * Gram-Schmidt and CholeskyQR, twice (a dependent column becomes a fixed
 * pseudo-random direction, orthogonalised in turn); the Rayleigh-Ritz
 * values of X on K (16 * steps of them, via pf_eigh's solver) give
 *   theta_min >= lambda_min and theta_max <= lambda_max (Cauchy interlacing),
 * and the residual norms ||X y - theta y|| of their Ritz vectors y give
 * intervals [theta - res, theta + res] that each hold an eigenvalue.
 *  X:     n-by-n symmetric, FP32 or FP64 (column-major, ld >= n).
 *  steps: 1..8 block steps, 16 * steps <= n.
 *  out:   device pf_bounds, written stream-ordered (status 0, or
 *         PF_ERR_NONFINITE when X or V0 holds Inf/NaN).
 * Scratch (about 8 n (32 + 16 steps) bytes) is allocated and freed
 * stream-ordered on the stream. */
typedef struct pf_bounds {
  double theta_min, theta_max;  /* extreme Ritz values of X on K */
  double res_min, res_max;      /* their residual norms */
  int32_t status;               /* pf_status of the run (0 = PF_OK) */
  int32_t replaced;             /* dependent columns replaced (an invariant subspace reached) */
} pf_bounds;
pf_status pf_lanczos_bounds(const pf_mat* X, int64_t n, const double* V0, int64_t ldv0, int32_t steps,
                            pf_bounds* out, void* stream);

/* Damping interval of section 4.1, host arithmetic.  a = lam_min - margin
 * (lam_min an estimate of the smallest eigenvalue, e.g. pf_bounds'
 * theta_min; margin >= 0, e.g. its res_min, keeps a below the spectrum).
 *  top_r <= 0 (all positive eigenvalues wanted): b = eta * a, which needs
 *      a < 0;
 *  top_r > 0 (the r largest wanted): b = (1 - eta) * theta_r + eta * a,
 *      theta_r the r-th largest Ritz value of the previous iterate.
 * eta in (0, 1) (the paper uses 0.1 to 0.2).  PF_ERR_ARG unless a < b and
 * every input is finite. */
pf_status pf_interval_policy(double lam_min, double margin, double eta, int32_t top_r, double theta_r,
                             double* a, double* b);

/* Block size of section 4.2, host arithmetic.  top_r > 0: p = 5 + q * r
 * (rounded up; q > 1 the guard factor); top_r <= 0 (all positive wanted):
 * p = n_pos + guards, n_pos the positive Ritz count of the previous iterate
 * (pf_info.n_pos).  The result is clamped to [1, 128]; PF_ERR_ARG for
 * q <= 1, negative counts or non-finite q. */
pf_status pf_block_size_policy(int32_t top_r, double q, int32_t n_pos, int32_t guards, int32_t* p);

/* pf_session_step with a caller-supplied operator (see pf_operator). */
pf_status pf_session_step_op(pf_session* s, const pf_operator* op, pf_result* out, void* stream);

/* Move a session's damping interval [a, b] (a < b, finite) for its next
 * steps, as the interval policy of section 4.1 follows the iterates. */
pf_status pf_session_set_interval(pf_session* s, double a, double b);

/* Filter degree for a tolerance (section 3, Lemma ctr1), host arithmetic.
 * A wanted eigenvalue theta_r > b maps to 1 + l past the damping interval,
 * l = 2 (theta_r - b) / (b - a); the unwanted part maps into [-1, 1].  After
 * one filtered step (power q) the subspace error is bounded by a factor of
 * the start angle times 1 / T_d(1 + l)^q (the step of the proof before
 * Lemma cheb-est's lower bound on T_d is used), so sin <= eps needs
 *   T_d(1 + l)^q >= 1 / eps,  d = ceil(acosh(eps^(-1/q)) / acosh(1 + l)).
 * The result is clamped to [d_min, d_max].  The O(log k) degree schedule of
 * Theorem conv1 is this rule with eps = eps_0 / k at outer iteration k.
 * PF_ERR_ARG unless a < b < theta_r, 0 < eps < 1, q >= 1 and
 * 1 <= d_min <= d_max. */
pf_status pf_degree_policy(double theta_r, double a, double b, int32_t q, double eps, int32_t d_min,
                           int32_t d_max, int32_t* degree);

/* Change a session's filter degree d and power q for its next steps (the
 * degree schedule of Theorem conv1, q_k of eq. pfpg2); validated like
 * pf_desc. */
pf_status pf_session_set_filter(pf_session* s, int32_t degree, int32_t q);

/* Nearest correlation estimation by PFPG (section 5.1; eq. pfpg1-pfpg2
 * with R = 0 on the dual of eq. NCE-dual): minimise
 *   F(x) = 1/2 sum_i max(lambda_i(G + Diag(x)), 0)^2 - 1^T x
 * by x <- x - tau (diag(P_+(P_U(B(x)))) - 1), B(x) = G + Diag(x), where
 * P_U(B) = V Theta V^T is the Rayleigh-Ritz projection of one extraction
 * (filter degree d on [a, b], FP64) warm-started from the previous one.
 * Every extrapolation_len + 1 steps the last points are combined by the
 * regularised extrapolation of section 4.3 (coefficients from the Gram of
 * their successive differences, lambda relative to its Frobenius norm).
 * The interval follows section 4.1 for all positive eigenvalues:
 * a = theta_min - res_min of pf_lanczos_bounds on B(x) (start block V0),
 * b = eta a, refreshed every lanczos_every steps (0: once).  The block size
 * follows section 4.2: the previous positive count plus guards, rounded up
 * to a multiple of 16, within [16, p_max]; while more than p_max
 * eigenvalues are positive the gradient uses the p_max largest Ritz pairs.
 * Columns added when the block grows are the next columns of U0.
 * Stops when ||g|| <= tol ||g_0|| (the paper's criterion) or after
 * max_iter steps.
 *  G:       device n-by-n FP64 symmetric (ld ldg), not modified.
 *  x:       device n FP64: in the start point (the paper takes
 *           1 - diag(G)), out the last iterate (the point whose gradient
 *           met the test, when converged).
 *  U0:      device n-by-p_max FP64 start block (ld ldu0).
 *  V0:      device n-by-16 FP64 Lanczos start block (ld ldv0).
 *  out:     host result.  history: host, max_iter x 6 doubles (row k:
 *           F, ||g||, n_pos, p, a, b at step k), or NULL.
 * Synchronous: returns when the loop ends (the host reads ||g|| and the
 * positive count after every step).  Device scratch (about
 * 8 n (n + 2 p_max + extrapolation_len + 8) bytes plus one extraction
 * workspace per block size) is allocated stream-ordered and freed before
 * return.  PF_ERR_ARG for invalid options, and when the Lanczos bound finds
 * no negative eigenvalue of B(x) (the all-positive interval rule needs
 * a < 0; then P_+(B) = B, no extraction is needed, and at x = 1 - diag(G)
 * G is already a correlation matrix); a failed extraction or
 * Lanczos run stops the loop with its status in out->status (and as the
 * return value), x holding the last good iterate. */
typedef struct pf_nce_opts {
  uint32_t struct_size;     /* sizeof(pf_nce_opts) */
  int32_t degree;           /* Chebyshev degree d >= 1 */
  int32_t guards;           /* guard columns >= 0 */
  int32_t p_max;            /* 16 <= p_max <= min(n, 128) */
  int32_t max_iter;         /* >= 1 */
  int32_t extrapolation_len;  /* l of section 4.3, 0 (off) .. 7 */
  int32_t lanczos_steps;    /* 1..8 block steps, 16 steps <= n */
  int32_t lanczos_every;    /* >= 0 */
  double tau;               /* step size > 0 (F has a 1-Lipschitz gradient: tau < 2) */
  double eta;               /* b = eta a, 0 < eta < 1 */
  double tol;               /* > 0 */
  double extrapolation_lambda;  /* >= 0 */
  uint32_t flags;           /* extraction flags of every step: 0 or
                               PF_FLAG_NO_PREROTATE (the pre-rotation is a
                               precision aid of the FP32 forms; in FP64 it
                               costs a second p x p eigensolve per step) */
  int32_t reserved;         /* must be 0 */
} pf_nce_opts;
typedef struct pf_nce_result {
  int32_t status;           /* pf_status of the run */
  int32_t iters;            /* steps taken (the index of the last evaluated iterate) */
  int32_t converged;        /* 1: ||g|| <= tol ||g_0|| */
  int32_t n_pos;            /* positive Ritz values at the last iterate */
  int32_t p;                /* block size at the last iterate */
  int32_t extrapolations;   /* extrapolation steps taken */
  double F;                 /* F at the last iterate (from its Ritz values) */
  double gnorm, gnorm0;     /* ||g|| there and at x0 */
  double a, b;              /* the last damping interval */
} pf_nce_result;
pf_status pf_nce_pfpg(const pf_nce_opts* opts, int64_t n, const double* G, int64_t ldg, double* x,
                      const double* U0, int64_t ldu0, const double* V0, int64_t ldv0, pf_nce_result* out,
                      double* history, void* stream);

/* Nearest correlation estimation on the primal by PFAM (eq. PFAM1-PFAM2):
 * Douglas-Rachford splitting of min 1/2 ||X - G||_F^2 + indicator(diag(X)
 * = 1) + indicator(X PSD), the PSD projection taken in the extracted
 * subspace:
 *   P = P_+(P_U(Z)) = V_+ Theta_+ V_+^T   (one FP64 extraction on Z,
 *                                          warm-started from the last one)
 *   Z <- prox_tG(2 P - Z) - P + Z, prox_tG(Y)_ij = (t G_ij + Y_ij)/(1 + t)
 *        off the diagonal and 1 on it.
 * Interval, block size and U0 columns follow the rules of pf_nce_pfpg,
 * applied to Z.  Stops when ||dZ||_F <= tol ||dZ_0||_F or after max_iter
 * steps.
 *  G:  device n-by-n FP64 symmetric (ld ldg), not modified.
 *  Z:  device n-by-n FP64 symmetric (ld ldz, 16-byte aligned, ldz * 8 a
 *      multiple of 16): in the start (G itself is the usual one), out Z
 *      after the last step.
 *  X:  device n-by-n FP64 (ld ldx), out: P of the last evaluated step,
 *      the primal iterate (PSD by construction; its diagonal converges to 1).
 *  U0, V0: start blocks as in pf_nce_pfpg.
 *  out: host result.  history: host, max_iter x 7 doubles (row k:
 *      ||dZ||, 1/2 ||G - P||_F^2, n_pos, p, a, b, max |diag(P) - 1|), or NULL.
 * Synchronous, with device scratch allocated stream-ordered and freed before
 * return (about 8 (n p_max + 3 n^2 / 256) bytes plus one extraction
 * workspace per block size).  Errors as pf_nce_pfpg; after a numerical
 * failure Z holds the last good iterate and X is unspecified. */
typedef struct pf_pfam_opts {
  uint32_t struct_size;     /* sizeof(pf_pfam_opts) */
  int32_t degree;           /* Chebyshev degree d >= 1 */
  int32_t guards;           /* guard columns >= 0 */
  int32_t p_max;            /* 16 <= p_max <= min(n, 128) */
  int32_t max_iter;         /* >= 1 */
  int32_t lanczos_steps;    /* 1..8 block steps, 16 steps <= n */
  int32_t lanczos_every;    /* >= 0 */
  uint32_t flags;           /* 0 or PF_FLAG_NO_PREROTATE */
  double t;                 /* DRS step > 0 */
  double eta;               /* b = eta a, 0 < eta < 1 */
  double tol;               /* > 0 */
} pf_pfam_opts;
typedef struct pf_pfam_result {
  int32_t status;           /* pf_status of the run */
  int32_t iters;            /* index of the last evaluated step */
  int32_t converged;        /* 1: ||dZ|| <= tol ||dZ_0|| */
  int32_t n_pos;            /* positive Ritz values at the last step */
  int32_t p;                /* block size at the last step */
  int32_t reserved;
  double residual, residual0;  /* ||dZ||_F at the last and the first step */
  double objective;         /* 1/2 ||G - X||_F^2 */
  double diag_err;          /* max |diag(X) - 1| */
  double a, b;              /* the last damping interval */
} pf_pfam_result;
pf_status pf_nce_pfam(const pf_pfam_opts* opts, int64_t n, const double* G, int64_t ldg, double* Z, int64_t ldz,
                      double* X, int64_t ldx, const double* U0, int64_t ldu0, const double* V0, int64_t ldv0,
                      pf_pfam_result* out, double* history, void* stream);

/* Kernel timing hooks (diagnostics).  While enabled, the library records a
 * HIP event pair on the launch stream around every kernel launch of the
 * given class; pf_profile_read synchronises on the recorded events and
 * returns the number of launches and their summed duration in ms.
 * Classes: PF_PROF_FILTER (the filter product kernel of the Chebyshev
 * recurrence, without its split-K sum), PF_PROF_FILTER_REDUCE (that sum),
 * PF_PROF_RR (the Rayleigh-Ritz product X Q), PF_PROF_EXTRACT (one whole
 * extraction, first to last launch), PF_PROF_FILTER_PRODUCT (one whole
 * filter product: the product kernel and its split-K sum under a single
 * event pair, with no event recorded between them).
 * pf_profile_set(1) times FILTER, FILTER_REDUCE, RR and EXTRACT;
 * pf_profile_set(PF_PROF_MODE_PRODUCT) times FILTER_PRODUCT, RR and EXTRACT;
 * pf_profile_set(0) stops.  Every call clears the counts. */
#define PF_PROF_FILTER 0
#define PF_PROF_FILTER_REDUCE 1
#define PF_PROF_RR 2
#define PF_PROF_EXTRACT 3
#define PF_PROF_FILTER_PRODUCT 4
#define PF_PROF_MODE_PRODUCT 2
pf_status pf_profile_set(int enable);
pf_status pf_profile_read(int which, int64_t* launches, double* total_ms);

/* Device workspace bytes pf_extract uses for desc (allocated on first use). */
pf_status pf_workspace_size(const pf_desc* desc, size_t* bytes);
/* The workspace cache of pf_extract / pf_extract_batch: one workspace per
 * device, stream and shape (n, m, p, work dtype, operator; degree, power,
 * interval and flags do not make a new one).  pf_workspace_cached reports
 * the device bytes and the number of cached workspaces (all devices and
 * streams, operator copies of the Gram form included).  pf_workspace_release
 * waits for the stream (on the current device), then frees the workspaces
 * cached for it; later calls on that stream allocate again.  Sessions and
 * servers own their workspaces and are not affected. */
pf_status pf_workspace_cached(size_t* bytes, int32_t* count);
pf_status pf_workspace_release(void* stream);

const char* pf_status_string(pf_status s);
const char* pf_last_error(void);
int pf_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PF_H */
