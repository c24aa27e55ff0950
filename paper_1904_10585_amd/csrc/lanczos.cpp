// Block Lanczos bounds of the spectrum of a symmetric operator X.
//
// Section 4.1 puts the left end a of the damping interval at the smallest
// eigenvalue of the input matrix and names the Lanczos method to estimate
// it.  Here the Krylov space K = span{V0, X V0, ..., X^(s-1) V0} of a
// 16-column start block is built one block per pass over X (products
// accumulated in FP64 by the contraction kernel), each new block
// orthogonalised against all earlier ones by block classical Gram-Schmidt
// with re-orthogonalisation: Gram-Schmidt, CholeskyQR, Gram-Schmidt,
// CholeskyQR (a dependent column, which CholeskyQR turns into a fixed
// pseudo-random direction, is put back into the orthogonal complement by
// the second pair).  The Rayleigh-Ritz matrix H = V^T X V is assembled
// from the first Gram-Schmidt coefficients of every step (block j of H's
// columns is V^T (X V_j)) and decomposed by the dense p x p solver.  The
// residual of a Ritz vector y = V z is (I - V V^T) X V z = W_r z_r (W_r the
// last step's block after orthogonalisation, z_r the last 16 entries of z),
// so its norm comes from the 16 x 16 Gram matrix of W_r.
#include "pf_internal.h"

#include <algorithm>

namespace pfx {

namespace {

constexpr int kS = 16;   // block width: one MFMA column tile

struct Arena {
  char* base = nullptr;
  size_t used = 0;
  template <typename T>
  T* take(size_t count) {
    T* p = reinterpret_cast<T*>(base + used);
    used += round_up((int64_t)(count * sizeof(T)), 256);
    return p;
  }
};

// The block steps on carved scratch (see enqueue_lanczos).
void lanczos_steps(const pf_mat& X, int64_t n, const double* V0, int64_t ldv0, int steps, pf_bounds* out,
                   hipStream_t st, double* V, double* W, double* W1, double* H, double* S, double* G, double* R,
                   double* Gl, double* Z, double* th, int* def, pf_info* info, void* pb, size_t part, double* E) {
  const Elem tx = X.dtype == PF_F64 ? Elem::F64 : Elem::F32;
  const int m = kS * steps;
  const int64_t ld = round_up(n, 16);
  PFX_HIP(hipMemsetAsync(info, 0, sizeof(pf_info), st));
  // C (M x N, ld ldc) = A^T B, contracted over n rows in FP64
  auto product = [&](const void* A, int64_t lda, Elem ta, int64_t M, const double* B, int64_t ldb, double* C,
                     int64_t ldc) {
    ContractArgs c;
    c.A = A; c.lda = lda; c.ta = ta;
    c.B = B; c.ldb = ldb; c.tb = Elem::F64;
    c.K = n; c.M = M; c.N = kS;
    c.out = C; c.ldo = ldc; c.to = Elem::F64;
    c.D1 = nullptr; c.ld1 = ldc; c.D2 = nullptr; c.ld2 = ldc;
    c.alpha = 1.0; c.beta = 0.0; c.gamma = 0.0;
    c.part = pb; c.part_bytes = part; c.splitk = 0; c.f64_mfma = true;
    contract(c, st);
  };
  // C1 (n x p) = A1 S, S p x p (ld lds)
  auto rotate = [&](const double* A1, int p, const double* Sm, int lds, double* C1, const int* deficient) {
    ApplyArgs ap;
    ap.n = n; ap.p = p;
    ap.A1 = A1; ap.lda1 = ld; ap.ta1 = Elem::F64;
    ap.A2 = nullptr; ap.lda2 = ld; ap.ta2 = Elem::F64;
    ap.S = Sm; ap.lds_ = lds;
    ap.C1 = C1; ap.ldc1 = ld; ap.tc1 = Elem::F64;
    ap.C2 = nullptr; ap.ldc2 = ld; ap.tc2 = Elem::F64;
    ap.alpha = 0.0; ap.beta = 0.0;
    ap.deficient = deficient;
    ap.gate = nullptr;
    launch_apply(ap, st);
  };
  // one Gram-Schmidt pass of Y against V_{0..j}: C = V^T Y ((j+1) kS x kS,
  // ld ldc), then Y -= V C in one rectangular apply
  auto gs_pass = [&](double* Y, int j, double* C, int ldc) {
    const int rows = (j + 1) * kS;
    product(V, ld, Elem::F64, rows, Y, ld, C, ldc);
    ApplyArgs ap;
    ap.n = n; ap.p = rows; ap.q = kS;
    ap.A1 = V; ap.lda1 = ld; ap.ta1 = Elem::F64;
    ap.A2 = nullptr; ap.lda2 = ld; ap.ta2 = Elem::F64;
    ap.S = C; ap.lds_ = ldc;
    ap.C1 = Y; ap.ldc1 = ld; ap.tc1 = Elem::F64;
    ap.C2 = nullptr; ap.ldc2 = ld; ap.tc2 = Elem::F64;
    ap.alpha = 0.0; ap.beta = 0.0;
    ap.deficient = nullptr;
    ap.gate = nullptr;
    ap.D = Y; ap.ldd = ld;
    launch_apply(ap, st);
  };
  // CholeskyQR pass: dst = src R^{-1}, dependent columns replaced
  auto cholqr = [&](const double* src, double* dst) {
    product(src, ld, Elem::F64, kS, src, ld, G, kS);
    launch_chol_rinv(G, kS, kS, R, kS, def, info, 1, st);
    rotate(src, kS, R, kS, dst, def);
  };

  // orthonormal start block
  launch_copy_block(V0, ldv0, Elem::F64, W, ld, Elem::F64, n, kS, ld, kS, st);
  cholqr(W, W1);
  cholqr(W1, V);
  for (int j = 0; j < steps; ++j) {
    const double* Vj = V + (int64_t)j * kS * ld;
    product(X.data, X.ld, tx, n, Vj, ld, W, ld);      // W = X V_j (X symmetric: X^T V_j)
    gs_pass(W, j, H + (int64_t)j * kS * m, m);        // H[0..(j+1)kS, block j] = V^T X V_j
    if (j + 1 < steps) {
      cholqr(W, W1);
      gs_pass(W1, j, S, m);
      cholqr(W1, V + (int64_t)(j + 1) * kS * ld);
    } else {
      gs_pass(W, j, S, m);
      product(W, ld, Elem::F64, kS, W, ld, Gl, kS);   // Gram of the residual block
    }
  }
  launch_sym_from_block_upper(H, m, m, kS, st);
  launch_eigh(H, m, m, th, Z, m, m, nullptr, 1, st, E);
  launch_lanczos_out(th, Z, m, m, kS, Gl, info, out, st);
}

}  // namespace

void enqueue_lanczos(const pf_mat& X, int64_t n, const double* V0, int64_t ldv0, int steps, pf_bounds* out,
                     hipStream_t st) {
  const Elem tx = X.dtype == PF_F64 ? Elem::F64 : Elem::F32;
  const int m = kS * steps;
  const int64_t ld = round_up(n, 16);

  const size_t part = std::max({contract_part_bytes(n, n, kS, tx, Elem::F64, true, 0),
                                contract_part_bytes(n, m, kS, Elem::F64, Elem::F64, true, 0),
                                contract_part_bytes(n, kS, kS, Elem::F64, Elem::F64, true, 0)});
  // sizes first (a null arena counts), then one stream-ordered allocation
  auto carve = [&](Arena& a, double*& V, double*& W, double*& W1, double*& H, double*& S, double*& G,
                   double*& R, double*& Gl, double*& Z, double*& th, int*& def, pf_info*& info, void*& pb,
                   double*& E) {
    V = a.take<double>((size_t)ld * m);
    W = a.take<double>((size_t)ld * kS);
    W1 = a.take<double>((size_t)ld * kS);
    H = a.take<double>((size_t)m * m);
    S = a.take<double>((size_t)m * m);
    G = a.take<double>(kS * kS);
    R = a.take<double>(kS * kS);
    Gl = a.take<double>(kS * kS);
    Z = a.take<double>((size_t)m * m);
    th = a.take<double>(m);
    def = a.take<int>(kS);
    info = a.take<pf_info>(1);
    pb = a.take<char>(std::max<size_t>(part, 256));
    E = a.take<double>(eig_scratch_bytes(m) / sizeof(double) + 1);
  };
  double *V, *W, *W1, *H, *S, *G, *R, *Gl, *Z, *th, *E;
  int* def;
  pf_info* info;
  void* pb;
  Arena a;
  carve(a, V, W, W1, H, S, G, R, Gl, Z, th, def, info, pb, E);
  void* mem = nullptr;
  if (hipMallocAsync(&mem, a.used, st) != hipSuccess) {
    (void)hipGetLastError();
    fail(PF_ERR_NOMEM, "lanczos: scratch allocation failed");
  }
  a.base = static_cast<char*>(mem);
  a.used = 0;
  carve(a, V, W, W1, H, S, G, R, Gl, Z, th, def, info, pb, E);
  try {
    lanczos_steps(X, n, V0, ldv0, steps, out, st, V, W, W1, H, S, G, R, Gl, Z, th, def, info, pb, part, E);
  } catch (...) {
    (void)hipFreeAsync(mem, st);                       // the scratch goes back with the error
    throw;
  }
  PFX_HIP(hipFreeAsync(mem, st));
}

}  // namespace pfx
