// Nearest correlation estimation by PFPG (section 5.1; eq. pfpg1-pfpg2
// with R = 0) on the dual F(x) = 1/2 sum max(lambda(G + Diag(x)), 0)^2 -
// 1^T x.  Each step: one FP64 extraction on B(x) = G + Diag(x), warm-started
// from the previous Ritz vectors; the gradient diag(V Theta_+ V^T) - 1 and
// its norm on the device; the host reads the norm and the positive count,
// then the device takes the step and rewrites the diagonal of B in place
// (the off-diagonal part of B is G, copied once).  Extrapolation of
// section 4.3 every l + 1 steps (the (l+1)^2 regularised system solved on
// the host), interval of section 4.1 from the block Lanczos bound, block
// size of section 4.2 from the positive count.
#include "pf_internal.h"

#include <cmath>
#include <map>
#include <vector>

namespace pfx {

namespace {

// c = (M / ||M||_F + lambda I)^{-1} 1 normalised to sum 1 (Gaussian
// elimination with partial pivoting on an m x m system, m <= 8); false
// when the system is singular.
bool rna_coefficients(const double* M, int m, double lambda, double* c) {
  double fro = 0.0;
  for (int i = 0; i < m * m; ++i) fro += M[i] * M[i];
  fro = std::sqrt(fro);
  if (!(fro > 0.0) || !std::isfinite(fro)) return false;
  double A[kNceMaxRna + 1][kNceMaxRna + 2];
  for (int i = 0; i < m; ++i) {
    for (int j = 0; j < m; ++j) A[i][j] = M[i + j * m] / fro + (i == j ? lambda : 0.0);
    A[i][m] = 1.0;
  }
  for (int k = 0; k < m; ++k) {
    int piv = k;
    for (int i = k + 1; i < m; ++i)
      if (std::fabs(A[i][k]) > std::fabs(A[piv][k])) piv = i;
    if (A[piv][k] == 0.0) return false;
    if (piv != k)
      for (int j = 0; j <= m; ++j) std::swap(A[k][j], A[piv][j]);
    for (int i = k + 1; i < m; ++i) {
      const double f = A[i][k] / A[k][k];
      for (int j = k; j <= m; ++j) A[i][j] -= f * A[k][j];
    }
  }
  double sum = 0.0;
  for (int i = m - 1; i >= 0; --i) {
    double v = A[i][m];
    for (int j = i + 1; j < m; ++j) v -= A[i][j] * c[j];
    c[i] = v / A[i][i];
    sum += c[i];
  }
  if (!(std::fabs(sum) > 0.0) || !std::isfinite(sum)) return false;
  for (int i = 0; i < m; ++i) c[i] /= sum;
  return true;
}

struct Scratch {
  void* mem = nullptr;
  hipStream_t st = nullptr;
  std::map<int, Plan*> plans;
  ~Scratch() {
    (void)hipStreamSynchronize(st);
    for (auto& kv : plans) plan_destroy(kv.second);
    if (mem) (void)hipFreeAsync(mem, st);
    (void)hipStreamSynchronize(st);
  }
};

}  // namespace

void run_nce_pfpg(const pf_nce_opts& o, int64_t n, const double* G, int64_t ldg, double* x, const double* U0,
                  int64_t ldu0, const double* V0, int64_t ldv0, pf_nce_result* out, double* history,
                  hipStream_t st) {
  const int64_t ld = round_up(n, 16);
  const int l = o.extrapolation_len;
  const int hcols = l > 0 ? l + 2 : 0;
  const int nblk = nce_partial_blocks(n);
  // carve: B, U, gd, g, hist, partials, stats, M, theta, info, bounds
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t at = off; off += (size_t)round_up((int64_t)bytes, 256); return at; };
  const size_t oB = take(sizeof(double) * ld * n);
  const size_t oU = take(sizeof(double) * ld * o.p_max);
  const size_t ogd = take(sizeof(double) * n);
  const size_t og = take(sizeof(double) * n);
  const size_t oh = take(sizeof(double) * ld * (hcols ? hcols : 1));
  const size_t opart = take(sizeof(double) * 2 * nblk);
  const size_t ostats = take(sizeof(double) * 4);
  const size_t oM = take(sizeof(double) * (kNceMaxRna + 1) * (kNceMaxRna + 1));
  const size_t oth = take(sizeof(double) * 128);
  const size_t oinfo = take(sizeof(pf_info));
  const size_t obnd = take(sizeof(pf_bounds));
  Scratch S;
  S.st = st;
  if (hipMallocAsync(&S.mem, off, st) != hipSuccess) {
    (void)hipGetLastError();
    S.mem = nullptr;
    fail(PF_ERR_NOMEM, "nce: scratch allocation failed");
  }
  char* base = static_cast<char*>(S.mem);
  double* B = reinterpret_cast<double*>(base + oB);
  double* U = reinterpret_cast<double*>(base + oU);
  double* gd = reinterpret_cast<double*>(base + ogd);
  double* g = reinterpret_cast<double*>(base + og);
  double* hist = hcols ? reinterpret_cast<double*>(base + oh) : nullptr;
  double* part = reinterpret_cast<double*>(base + opart);
  double* stats = reinterpret_cast<double*>(base + ostats);
  double* M = reinterpret_cast<double*>(base + oM);
  double* theta = reinterpret_cast<double*>(base + oth);
  pf_info* info = reinterpret_cast<pf_info*>(base + oinfo);
  pf_bounds* bnd = reinterpret_cast<pf_bounds*>(base + obnd);

  PFX_HIP(hipMemcpy2DAsync(B, ld * sizeof(double), G, ldg * sizeof(double), n * sizeof(double), n,
                           hipMemcpyDeviceToDevice, st));
  PFX_HIP(hipMemcpy2DAsync(U, ld * sizeof(double), U0, ldu0 * sizeof(double), n * sizeof(double), o.p_max,
                           hipMemcpyDeviceToDevice, st));
  launch_nce_init(x, gd, B, ld, n, hist, st);
  const pf_mat Bm{B, PF_F64, ld, nullptr, 0};

  double a = 0.0, b = 0.0;
  auto interval = [&]() {
    enqueue_lanczos(Bm, n, V0, ldv0, o.lanczos_steps, bnd, st);
    pf_bounds hb{};
    PFX_HIP(hipMemcpyAsync(&hb, bnd, sizeof(hb), hipMemcpyDeviceToHost, st));
    PFX_HIP(hipStreamSynchronize(st));
    if (hb.status != 0) fail((pf_status)hb.status, "nce: Lanczos bound failed on B(x)");
    a = hb.theta_min - hb.res_min;
    if (!(a < 0.0)) fail(PF_ERR_ARG, "nce: the all-positive interval rule needs a negative smallest eigenvalue");
    b = o.eta * a;
  };
  auto plan_for = [&](int p) {
    auto it = S.plans.find(p);
    if (it != S.plans.end()) return it->second;
    pf_desc d{};
    d.struct_size = sizeof(pf_desc);
    d.op = PF_OP_SYM; d.n = n; d.p = p; d.degree = o.degree; d.q = 1;
    d.a = a; d.b = b; d.work = PF_F64;
    Plan* P = plan_create(d, st, true);
    S.plans[p] = P;
    return P;
  };

  interval();
  *out = pf_nce_result{};
  int p = o.p_max;
  bool cold = true;
  int slot = 1, extrap = 0;
  double g0 = 0.0;
  for (int k = 0;; ++k) {
    pf_desc d{};
    d.struct_size = sizeof(pf_desc);
    d.op = PF_OP_SYM; d.n = n; d.p = p; d.degree = o.degree; d.q = 1;
    d.a = a; d.b = b; d.work = PF_F64;
    d.flags = (cold ? PF_FLAG_COLD : 0u) | o.flags;
    Plan* P = plan_for(p);
    plan_set_desc(P, d);
    enqueue_extraction(P, Bm, Bm, U, ld, U, ld, theta, info, st);
    launch_nce_grad(U, ld, p, theta, x, g, n, info, part, stats, st);
    double hs[4];
    pf_info hi{};
    PFX_HIP(hipMemcpyAsync(hs, stats, sizeof(hs), hipMemcpyDeviceToHost, st));
    PFX_HIP(hipMemcpyAsync(&hi, info, sizeof(hi), hipMemcpyDeviceToHost, st));
    PFX_HIP(hipStreamSynchronize(st));
    if (hi.status != 0) {
      out->status = hi.status;
      out->iters = k;
      out->p = p;
      out->a = a;
      out->b = b;
      out->gnorm0 = g0;
      out->extrapolations = extrap;
      return;
    }
    const double gn = std::sqrt(hs[0]);
    const double F = hs[2] - hs[1];
    const int npos = hi.n_pos;
    if (k == 0) g0 = gn;
    if (history) {
      double* row = history + (size_t)6 * k;
      row[0] = F; row[1] = gn; row[2] = npos; row[3] = p; row[4] = a; row[5] = b;
    }
    out->iters = k;
    out->n_pos = npos;
    out->p = p;
    out->F = F;
    out->gnorm = gn;
    out->gnorm0 = g0;
    out->a = a;
    out->b = b;
    out->extrapolations = extrap;
    if (gn <= o.tol * g0) {
      out->converged = 1;
      return;
    }
    if (k + 1 >= o.max_iter) return;
    // the step, then the extrapolation when the window is full
    launch_nce_step(x, g, o.tau, gd, B, ld, n, hist, ld, slot, st);
    if (l > 0 && ++slot == l + 2) {
      launch_nce_diff_gram(hist, ld, n, l + 1, M, st);
      double hM[(kNceMaxRna + 1) * (kNceMaxRna + 1)];
      PFX_HIP(hipMemcpyAsync(hM, M, sizeof(double) * (l + 1) * (l + 1), hipMemcpyDeviceToHost, st));
      PFX_HIP(hipStreamSynchronize(st));
      double c[kNceMaxRna + 1];
      if (rna_coefficients(hM, l + 1, o.extrapolation_lambda, c)) {
        launch_nce_combine(c, l + 1, hist, ld, x, gd, B, ld, n, st);
        ++extrap;
      } else {
        // a zero or singular difference Gram: keep the last point
        PFX_HIP(hipMemcpyAsync(hist, hist + (size_t)(l + 1) * ld, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
      }
      slot = 1;
    }
    // block size for the next step (section 4.2), guard columns rounded up
    int p_new = (int)round_up((int64_t)npos + o.guards, 16);
    p_new = std::max(16, std::min(o.p_max, p_new));
    cold = false;
    if (p_new > p) {
      PFX_HIP(hipMemcpy2DAsync(U + (size_t)p * ld, ld * sizeof(double), U0 + (size_t)p * ldu0, ldu0 * sizeof(double),
                               n * sizeof(double), p_new - p, hipMemcpyDeviceToDevice, st));
      cold = true;
    }
    p = p_new;
    if (o.lanczos_every > 0 && (k + 1) % o.lanczos_every == 0) interval();
  }
}

// PFAM (eq. PFAM1-PFAM2) on the NCE primal: per step one FP64 extraction on
// Z (warm-started), P = V_+ Theta_+ V_+^T into X, then the DRS step on Z
// entrywise; the host reads ||dZ|| and the positive count.  Interval and
// block size as in the PFPG loop, applied to Z.
void run_nce_pfam(const pf_pfam_opts& o, int64_t n, const double* G, int64_t ldg, double* Z, int64_t ldz, double* X,
                  int64_t ldx, const double* U0, int64_t ldu0, const double* V0, int64_t ldv0, pf_pfam_result* out,
                  double* history, hipStream_t st) {
  const int64_t ld = round_up(n, 16);
  const int64_t nblk = drs_partial_blocks(n);
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t at = off; off += (size_t)round_up((int64_t)bytes, 256); return at; };
  const size_t oU = take(sizeof(double) * ld * o.p_max);
  const size_t opart = take(sizeof(double) * 3 * nblk);
  const size_t ostats = take(sizeof(double) * 4);
  const size_t oth = take(sizeof(double) * 128);
  const size_t oinfo = take(sizeof(pf_info));
  const size_t obnd = take(sizeof(pf_bounds));
  Scratch S;
  S.st = st;
  if (hipMallocAsync(&S.mem, off, st) != hipSuccess) {
    (void)hipGetLastError();
    S.mem = nullptr;
    fail(PF_ERR_NOMEM, "pfam: scratch allocation failed");
  }
  char* base = static_cast<char*>(S.mem);
  double* U = reinterpret_cast<double*>(base + oU);
  double* part = reinterpret_cast<double*>(base + opart);
  double* stats = reinterpret_cast<double*>(base + ostats);
  double* theta = reinterpret_cast<double*>(base + oth);
  pf_info* info = reinterpret_cast<pf_info*>(base + oinfo);
  pf_bounds* bnd = reinterpret_cast<pf_bounds*>(base + obnd);
  PFX_HIP(hipMemcpy2DAsync(U, ld * sizeof(double), U0, ldu0 * sizeof(double), n * sizeof(double), o.p_max,
                           hipMemcpyDeviceToDevice, st));
  const pf_mat Zm{Z, PF_F64, ldz, nullptr, 0};

  double a = 0.0, b = 0.0;
  auto interval = [&]() {
    enqueue_lanczos(Zm, n, V0, ldv0, o.lanczos_steps, bnd, st);
    pf_bounds hb{};
    PFX_HIP(hipMemcpyAsync(&hb, bnd, sizeof(hb), hipMemcpyDeviceToHost, st));
    PFX_HIP(hipStreamSynchronize(st));
    if (hb.status != 0) fail((pf_status)hb.status, "pfam: Lanczos bound failed on Z");
    a = hb.theta_min - hb.res_min;
    if (!(a < 0.0)) fail(PF_ERR_ARG, "pfam: the all-positive interval rule needs a negative smallest eigenvalue");
    b = o.eta * a;
  };
  auto desc_for = [&](int p, bool cold) {
    pf_desc d{};
    d.struct_size = sizeof(pf_desc);
    d.op = PF_OP_SYM; d.n = n; d.p = p; d.degree = o.degree; d.q = 1;
    d.a = a; d.b = b; d.work = PF_F64;
    d.flags = (cold ? PF_FLAG_COLD : 0u) | o.flags;
    return d;
  };

  interval();
  *out = pf_pfam_result{};
  int p = o.p_max;
  bool cold = true;
  double r0 = 0.0;
  for (int k = 0;; ++k) {
    const pf_desc d = desc_for(p, cold);
    auto it = S.plans.find(p);
    Plan* P = it != S.plans.end() ? it->second : (S.plans[p] = plan_create(d, st, true));
    plan_set_desc(P, d);
    enqueue_extraction(P, Zm, Zm, U, ld, U, ld, theta, info, st);
    launch_psd_dense(U, ld, Elem::F64, theta, n, p, X, ldx, st);
    launch_drs_step(Z, ldz, X, ldx, G, ldg, n, o.t, info, theta, p, part, stats, st);
    double hs[4];
    pf_info hi{};
    PFX_HIP(hipMemcpyAsync(hs, stats, sizeof(hs), hipMemcpyDeviceToHost, st));
    PFX_HIP(hipMemcpyAsync(&hi, info, sizeof(hi), hipMemcpyDeviceToHost, st));
    PFX_HIP(hipStreamSynchronize(st));
    out->iters = k;
    out->p = p;
    out->a = a;
    out->b = b;
    if (hi.status != 0) {
      out->status = hi.status;
      out->residual0 = r0;
      return;
    }
    const double r = std::sqrt(hs[0]);
    const int npos = hi.n_pos;
    if (k == 0) r0 = r;
    if (history) {
      double* row = history + (size_t)7 * k;
      row[0] = r; row[1] = 0.5 * hs[1]; row[2] = npos; row[3] = p; row[4] = a; row[5] = b; row[6] = hs[2];
    }
    out->n_pos = npos;
    out->residual = r;
    out->residual0 = r0;
    out->objective = 0.5 * hs[1];
    out->diag_err = hs[2];
    if (r <= o.tol * r0) {
      out->converged = 1;
      return;
    }
    if (k + 1 >= o.max_iter) return;
    int p_new = (int)round_up((int64_t)npos + o.guards, 16);
    p_new = std::max(16, std::min(o.p_max, p_new));
    cold = false;
    if (p_new > p) {
      PFX_HIP(hipMemcpy2DAsync(U + (size_t)p * ld, ld * sizeof(double), U0 + (size_t)p * ldu0, ldu0 * sizeof(double),
                               n * sizeof(double), p_new - p, hipMemcpyDeviceToDevice, st));
      cold = true;
    }
    p = p_new;
    if (o.lanczos_every > 0 && (k + 1) % o.lanczos_every == 0) interval();
  }
}

}  // namespace pfx
