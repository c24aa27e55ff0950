// The C ABI of include/pf.h: argument validation, error reporting, the
// per-stream workspace cache of pf_extract, and sessions.
#include "pf_internal.h"
#include "group.h"

#include <dlfcn.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <limits>
#include <map>
#include <mutex>
#include <tuple>
#include <utility>
#include <vector>

namespace pfx {

[[noreturn]] void fail(pf_status s, const std::string& msg) { throw Error{s, msg}; }

void check_hip(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) fail(PF_ERR_NOMEM, std::string(what) + ": out of memory");
    fail(PF_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  }
}

size_t session_bytes(const pf_desc& d) {
  const size_t esz = d.work == PF_F64 ? 8 : 4;
  return plan_bytes(d) + (size_t)round_up(d.n, 64) * d.p * esz + sizeof(double) * d.p + sizeof(pf_info) + 3 * 256;
}

SessionCore* session_create(const pf_desc& d, const void* U0, int64_t ldu0, uint64_t seed, hipStream_t st,
                            bool sync) {
  SessionCore* s = new SessionCore();
  try {
    PFX_HIP(hipGetDevice(&s->device));
    s->desc = d;
    s->plan = plan_create(d, st, true);                // cleared in order with st's later work
    const Elem W = d.work == PF_F64 ? Elem::F64 : Elem::F32;
    const size_t esz = W == Elem::F64 ? 8 : 4;
    s->ldu = round_up(d.n, 64);
    const size_t ubytes = (size_t)s->ldu * d.p * esz;
    PFX_HIP(hipMalloc(&s->U, ubytes));
    PFX_HIP(hipMalloc(&s->theta, sizeof(double) * d.p));
    PFX_HIP(hipMalloc(&s->info, sizeof(pf_info)));
    PFX_HIP(hipMemsetAsync(s->U, 0, ubytes, st));
    PFX_HIP(hipMemsetAsync(s->theta, 0, sizeof(double) * d.p, st));
    PFX_HIP(hipMemsetAsync(s->info, 0, sizeof(pf_info), st));
    if (U0) launch_copy_block(U0, ldu0, W, s->U, s->ldu, W, d.n, d.p, d.n, d.p, st);
    else launch_normal_block(s->U, s->ldu, W, d.n, d.p, seed, st);
    if (sync) PFX_HIP(hipStreamSynchronize(st));
  } catch (...) {
    session_destroy(s);
    throw;
  }
  return s;
}

void session_destroy(SessionCore* s) {
  if (!s) return;
  if (s->U) (void)hipFree(s->U);
  if (s->theta) (void)hipFree(s->theta);
  if (s->info) (void)hipFree(s->info);
  plan_destroy(s->plan);
  delete s;
}

void session_enqueue_step(SessionCore* s, const pf_mat& Xf, const pf_mat& Xr, hipStream_t st,
                          const pf_operator* op, const pf_extras* ex) {
  pf_desc d = s->desc;
  if (s->steps == 0) d.flags |= PF_FLAG_COLD;        // first step starts from U0
  plan_set_desc(s->plan, d);
  enqueue_extraction(s->plan, Xf, Xr, s->U, s->ldu, s->U, s->ldu, s->theta, s->info, st, op, ex);
  s->steps++;
}

namespace {

thread_local std::string g_last_error;

template <typename F>
pf_status guarded(F&& f) {
  try {
    f();
    return PF_OK;
  } catch (const Error& e) {
    g_last_error = e.msg;
    return e.status;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return PF_ERR_NOMEM;
  } catch (...) {
    g_last_error = "unexpected internal error";
    return PF_ERR_DEVICE;
  }
}

}  // namespace

pf_status run_guarded(const std::function<void()>& f) { return guarded(f); }

namespace {

// pf_extract workspaces: one per (device, stream, shape); calls on one
// stream are ordered, so a workspace is never used by two extractions at once.
// The key holds exactly what the workspace layout depends on (n, m, p, work
// dtype, operator kind): degree, power, interval and flags only change the
// descriptor, which every call installs with plan_set_desc.
// pf_extract_batch keeps one workspace per block of a shape (slot).
using PlanKey = std::tuple<int, uintptr_t, int64_t, int64_t, int, int, int, int>;
std::mutex g_plans_mu;
std::map<PlanKey, Plan*> g_plans;

PlanKey plan_key(const pf_desc& d, hipStream_t st, int slot) {
  int dev = 0;
  PFX_HIP(hipGetDevice(&dev));
  return PlanKey{dev, (uintptr_t)st, d.n, d.op == PF_OP_GRAM ? d.m : 0, d.p, (int)d.work, (int)d.op, slot};
}

Plan* cached_plan(const pf_desc& d, hipStream_t st, int slot = 0) {
  const PlanKey key = plan_key(d, st, slot);
  std::lock_guard<std::mutex> lk(g_plans_mu);
  auto it = g_plans.find(key);
  if (it != g_plans.end()) return it->second;
  // cleared on the stream it serves, ordered before its first extraction: a
  // clear on the null stream would not be ordered with a non-blocking stream
  Plan* P = plan_create(d, st, true);
  g_plans[key] = P;
  return P;
}

}  // namespace

// ---------------------------------------------------------------------------
// Kernel timing hooks.  Event pairs are pooled per class and reused after
// pf_profile_set(1); recording is stream-ordered and adds no synchronisation.
namespace {
struct ProfClass {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
  size_t used = 0;
  bool open = false;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
int g_prof_mode = 0;
ProfClass g_prof[kProfClasses];

// classes timed in the current mode: per kernel (1), or the filter product
// as one pair (PF_PROF_MODE_PRODUCT)
bool prof_class_on(int cls) {
  if (cls == PF_PROF_RR || cls == PF_PROF_EXTRACT) return true;
  return g_prof_mode == PF_PROF_MODE_PRODUCT ? cls == PF_PROF_FILTER_PRODUCT : cls != PF_PROF_FILTER_PRODUCT;
}
}  // namespace

// (launches being recorded for a grouped enqueue are not timed one by one)
bool prof_enabled() { return g_prof_on && current_recorder() == nullptr; }

// roctx ranges (host-side, per thread) around the phases of an extraction,
// for rocprofv3 --marker-trace.  On when PF_ROCTX=1 is in the environment at
// the first range; the functions are resolved from ROCm's roctx library
// (missing library: no ranges).
namespace {
struct Roctx {
  int (*push)(const char*) = nullptr;
  int (*pop)() = nullptr;
};
const Roctx& roctx() {
  static const Roctx r = [] {
    Roctx x;
    const char* e = std::getenv("PF_ROCTX");
    if (!e || std::strcmp(e, "1") != 0) return x;
    void* h = dlopen("librocprofiler-sdk-roctx.so.1", RTLD_NOW | RTLD_LOCAL);
    if (!h) h = dlopen("libroctx64.so.4", RTLD_NOW | RTLD_LOCAL);
    if (!h) return x;
    x.push = reinterpret_cast<int (*)(const char*)>(dlsym(h, "roctxRangePushA"));
    x.pop = reinterpret_cast<int (*)()>(dlsym(h, "roctxRangePop"));
    if (!x.push || !x.pop) x = Roctx{};
    return x;
  }();
  return r;
}
}  // namespace

void trace_push(const char* name) {
  if (auto f = roctx().push) f(name);
}
void trace_pop() {
  if (auto f = roctx().pop) f();
}

Recorder*& current_recorder() {
  static thread_local Recorder* r = nullptr;
  return r;
}

void prof_begin(int cls, hipStream_t st) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (!prof_class_on(cls)) return;
  ProfClass& c = g_prof[cls];
  if (c.used == c.pool.size()) {
    hipEvent_t a, b;
    PFX_HIP(hipEventCreate(&a));
    PFX_HIP(hipEventCreate(&b));
    c.pool.emplace_back(a, b);
  }
  PFX_HIP(hipEventRecord(c.pool[c.used].first, st));
  c.open = true;
}

void prof_end(int cls, hipStream_t st) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (!prof_class_on(cls)) return;
  ProfClass& c = g_prof[cls];
  if (!c.open) return;
  PFX_HIP(hipEventRecord(c.pool[c.used].second, st));
  c.used++;
  c.open = false;
}

}  // namespace pfx

struct pf_session {
  pfx::SessionCore* core = nullptr;
  hipEvent_t done = nullptr;
  bool stepped = false;
  const double* resid = nullptr;   // the caller's residual buffer of the last step
};
using namespace pfx;

namespace {

// The optional outputs of an extraction, checked before anything is enqueued.
void check_extras(const pf_desc& d, const pf_extras* ex, bool op) {
  if (!ex) return;
  if (ex->struct_size != sizeof(pf_extras)) fail(PF_ERR_ARG, "pf_extras.struct_size must be sizeof(pf_extras)");
  if (ex->reserved != 0) fail(PF_ERR_ARG, "pf_extras.reserved must be 0");
  if (ex->resid && op) fail(PF_ERR_UNSUPPORTED, "residual norms need a dense operator");
  if (ex->shrink_left) {
    if (d.op != PF_OP_GRAM) fail(PF_ERR_ARG, "shrink_left needs PF_OP_GRAM");
    if (!std::isfinite(ex->shrink_tau) || ex->shrink_tau < 0.0) fail(PF_ERR_ARG, "shrink_tau must be finite and >= 0");
    if (ex->ld_shrink < d.m) fail(PF_ERR_ARG, "ld_shrink is smaller than m");
  }
}

void fill_result(const pf_session* s, pf_result* out) {
  out->status = 0;
  out->n_pos = 0;
  out->theta = s->core->theta;
  out->V = s->core->U;
  out->ldv = s->core->ldu;
  out->info = s->core->info;
  out->resid = s->resid;
  out->resid_max = std::numeric_limits<double>::quiet_NaN();
}

}  // namespace

extern "C" {

const char* pf_status_string(pf_status s) {
  switch (s) {
    case PF_OK: return "PF_OK";
    case PF_ERR_ARG: return "PF_ERR_ARG: invalid argument";
    case PF_ERR_NOMEM: return "PF_ERR_NOMEM: allocation failed";
    case PF_ERR_DEVICE: return "PF_ERR_DEVICE: HIP runtime error";
    case PF_ERR_BREAKDOWN: return "PF_ERR_BREAKDOWN: Cholesky of the Gram matrix broke down";
    case PF_ERR_NOCONV: return "PF_ERR_NOCONV: an iteration did not converge";
    case PF_ERR_NONFINITE: return "PF_ERR_NONFINITE: non-finite values in the filtered block";
    case PF_ERR_BUSY: return "PF_ERR_BUSY: work in flight";
    case PF_ERR_UNSUPPORTED: return "PF_ERR_UNSUPPORTED: not implemented by the library";
  }
  return "unknown pf_status";
}

const char* pf_last_error(void) { return g_last_error.c_str(); }

int pf_abi_version(void) { return PF_ABI_VERSION; }

pf_status pf_profile_set(int enable) {
  return guarded([&] {
    if (enable != 0 && enable != 1 && enable != PF_PROF_MODE_PRODUCT) fail(PF_ERR_ARG, "unknown profiling mode");
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = enable != 0;
    g_prof_mode = enable;
    for (auto& c : g_prof) { c.used = 0; c.open = false; }
  });
}

pf_status pf_profile_read(int which, int64_t* launches, double* total_ms) {
  return guarded([&] {
    if (which < 0 || which >= kProfClasses) fail(PF_ERR_ARG, "unknown profiling class");
    if (!launches || !total_ms) fail(PF_ERR_ARG, "NULL output");
    std::lock_guard<std::mutex> lk(g_prof_mu);
    ProfClass& c = g_prof[which];
    double tot = 0.0;
    for (size_t i = 0; i < c.used; ++i) {
      PFX_HIP(hipEventSynchronize(c.pool[i].second));
      float ms = 0.f;
      PFX_HIP(hipEventElapsedTime(&ms, c.pool[i].first, c.pool[i].second));
      tot += ms;
    }
    *launches = (int64_t)c.used;
    *total_ms = tot;
  });
}

pf_status pf_workspace_cached(size_t* bytes, int32_t* count) {
  return guarded([&] {
    if (!bytes || !count) fail(PF_ERR_ARG, "NULL output");
    std::lock_guard<std::mutex> lk(g_plans_mu);
    size_t b = 0;
    for (const auto& kv : g_plans) b += plan_device_bytes(kv.second);
    *bytes = b;
    *count = (int32_t)g_plans.size();
  });
}

pf_status pf_workspace_release(void* stream) {
  return guarded([&] {
    hipStream_t st = static_cast<hipStream_t>(stream);
    int dev = 0;
    PFX_HIP(hipGetDevice(&dev));
    std::vector<Plan*> gone;
    {
      std::lock_guard<std::mutex> lk(g_plans_mu);
      for (auto it = g_plans.begin(); it != g_plans.end();) {
        if (std::get<0>(it->first) == dev && std::get<1>(it->first) == reinterpret_cast<uintptr_t>(st)) {
          gone.push_back(it->second);
          it = g_plans.erase(it);
        } else {
          ++it;
        }
      }
    }
    if (gone.empty()) return;
    PFX_HIP(hipStreamSynchronize(st));        // the stream's extractions are done with them
    for (Plan* P : gone) plan_destroy(P);
  });
}

pf_status pf_workspace_size(const pf_desc* desc, size_t* bytes) {
  return guarded([&] {
    if (!desc || !bytes) fail(PF_ERR_ARG, "NULL argument");
    plan_validate(*desc, nullptr, nullptr);
    *bytes = plan_bytes(*desc);
  });
}

pf_status pf_extract(const pf_desc* desc, const pf_mat* X_filter, const pf_mat* X_rr, void* U_inout, int64_t ldu,
                     double* theta_out, pf_info* info_out, void* stream) {
  return pf_extract_ex(desc, X_filter, X_rr, U_inout, ldu, theta_out, info_out, nullptr, stream);
}

pf_status pf_extract_ex(const pf_desc* desc, const pf_mat* X_filter, const pf_mat* X_rr, void* U_inout,
                        int64_t ldu, double* theta_out, pf_info* info_out, const pf_extras* extras,
                        void* stream) {
  return guarded([&] {
    if (!desc) fail(PF_ERR_ARG, "desc is NULL");
    plan_validate(*desc, X_filter, X_rr);
    if (!U_inout) fail(PF_ERR_ARG, "U_inout is NULL");
    if (ldu < desc->n) fail(PF_ERR_ARG, "ldu is smaller than n");
    if (!theta_out) fail(PF_ERR_ARG, "theta_out is NULL");
    check_extras(*desc, extras, false);
    hipStream_t st = static_cast<hipStream_t>(stream);
    Plan* P = cached_plan(*desc, st);
    plan_set_desc(P, *desc);
    enqueue_extraction(P, *X_filter, *X_rr, U_inout, ldu, U_inout, ldu, theta_out, info_out, st, nullptr, extras);
  });
}


pf_status pf_extract_batch(int32_t count, const pf_desc* descs, const pf_mat* X_filter, const pf_mat* X_rr,
                           void* const* U_inout, const int64_t* ldu, double* const* theta_out,
                           pf_info* const* info_out, void* stream) {
  return guarded([&] {
    if (count < 0) fail(PF_ERR_ARG, "count must be >= 0");
    if (count == 0) return;
    if (!descs || !X_filter || !X_rr || !U_inout || !ldu || !theta_out) fail(PF_ERR_ARG, "NULL array");
    // every block is checked before any work is enqueued
    for (int i = 0; i < count; ++i) {
      try {
        plan_validate(descs[i], &X_filter[i], &X_rr[i]);
        if (!U_inout[i]) fail(PF_ERR_ARG, "U_inout is NULL");
        if (ldu[i] < descs[i].n) fail(PF_ERR_ARG, "ldu is smaller than n");
        if (!theta_out[i]) fail(PF_ERR_ARG, "theta_out is NULL");
      } catch (const Error& e) {
        fail(e.status, "block " + std::to_string(i) + ": " + e.msg);
      }
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    // a workspace per block: the k-th block of a shape takes the k-th
    // workspace of that shape on this stream
    std::map<PlanKey, int> seen;
    std::vector<ExtractionJob> jobs;
    jobs.reserve(count);
    for (int i = 0; i < count; ++i) {
      const pf_desc& d = descs[i];
      const int slot = seen[plan_key(d, st, 0)]++;
      Plan* P = cached_plan(d, st, slot);
      if (d.op != PF_OP_SYM) {
        // the Gram operator (transposed copies made on first use) runs on its own
        plan_set_desc(P, d);
        enqueue_extraction(P, X_filter[i], X_rr[i], U_inout[i], ldu[i], U_inout[i], ldu[i], theta_out[i],
                           info_out ? info_out[i] : nullptr, st);
        continue;
      }
      ExtractionJob j;
      j.plan = P;
      j.desc = d;
      j.Xf = X_filter[i];
      j.Xr = X_rr[i];
      j.U_in = U_inout[i];
      j.ldu_in = ldu[i];
      j.U_out = U_inout[i];
      j.ldu_out = ldu[i];
      j.theta_out = theta_out[i];
      j.info_out = info_out ? info_out[i] : nullptr;
      jobs.push_back(j);
    }
    // the blocks' phases as grouped launches on the caller's stream
    enqueue_extractions_grouped((int)jobs.size(), jobs.data(), st);
  });
}

namespace {
// the operator forms: a symmetric operator given by its products
void check_operator(const pf_desc& d, const pf_operator* op) {
  if (!op || !op->apply) fail(PF_ERR_ARG, "operator or its apply callback is NULL");
  if (d.op != PF_OP_SYM) fail(PF_ERR_ARG, "an operator extraction takes pf_desc.op = PF_OP_SYM");
}
}  // namespace

pf_status pf_extract_op(const pf_desc* desc, const pf_operator* op, void* U_inout, int64_t ldu, double* theta_out,
                        pf_info* info_out, void* stream) {
  return guarded([&] {
    if (!desc) fail(PF_ERR_ARG, "desc is NULL");
    plan_validate(*desc, nullptr, nullptr);
    check_operator(*desc, op);
    if (!U_inout) fail(PF_ERR_ARG, "U_inout is NULL");
    if (ldu < desc->n) fail(PF_ERR_ARG, "ldu is smaller than n");
    if (!theta_out) fail(PF_ERR_ARG, "theta_out is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    Plan* P = cached_plan(*desc, st);
    plan_set_desc(P, *desc);
    const pf_mat none{};
    enqueue_extraction(P, none, none, U_inout, ldu, U_inout, ldu, theta_out, info_out, st, op);
  });
}

pf_status pf_session_open(const pf_desc* desc, const void* U0, int64_t ldu0, uint64_t seed, pf_session** out) {
  return guarded([&] {
    if (!desc || !out) fail(PF_ERR_ARG, "NULL argument");
    plan_validate(*desc, nullptr, nullptr);
    if (U0 && ldu0 < desc->n) fail(PF_ERR_ARG, "ldu0 is smaller than n");
    pf_session* s = new pf_session();
    try {
      s->core = session_create(*desc, U0, ldu0, seed, nullptr, true);
      PFX_HIP(hipEventCreateWithFlags(&s->done, hipEventDisableTiming));
    } catch (...) {
      session_destroy(s->core);
      delete s;
      throw;
    }
    *out = s;
  });
}

pf_status pf_session_step(pf_session* s, const pf_mat* X_filter, const pf_mat* X_rr, pf_result* out,
                          void* stream) {
  return pf_session_step_ex(s, X_filter, X_rr, nullptr, out, stream);
}

pf_status pf_session_step_ex(pf_session* s, const pf_mat* X_filter, const pf_mat* X_rr, const pf_extras* extras,
                             pf_result* out, void* stream) {
  return guarded([&] {
    if (!s) fail(PF_ERR_ARG, "session is NULL");
    plan_validate(s->core->desc, X_filter, X_rr);
    check_extras(s->core->desc, extras, false);
    hipStream_t st = static_cast<hipStream_t>(stream);
    session_enqueue_step(s->core, *X_filter, *X_rr, st, nullptr, extras);
    PFX_HIP(hipEventRecord(s->done, st));
    s->stepped = true;
    s->resid = extras ? extras->resid : nullptr;
    if (out) fill_result(s, out);
  });
}

pf_status pf_session_step_op(pf_session* s, const pf_operator* op, pf_result* out, void* stream) {
  return guarded([&] {
    if (!s) fail(PF_ERR_ARG, "session is NULL");
    check_operator(s->core->desc, op);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const pf_mat none{};
    session_enqueue_step(s->core, none, none, st, op);
    PFX_HIP(hipEventRecord(s->done, st));
    s->stepped = true;
    s->resid = nullptr;
    if (out) fill_result(s, out);
  });
}

pf_status pf_session_wait(pf_session* s, pf_result* out) {
  pf_info host{};
  pf_status st = guarded([&] {
    if (!s) fail(PF_ERR_ARG, "session is NULL");
    if (s->stepped) PFX_HIP(hipEventSynchronize(s->done));
    PFX_HIP(hipMemcpy(&host, s->core->info, sizeof(pf_info), hipMemcpyDeviceToHost));
    if (out) {
      fill_result(s, out);
      out->status = host.status;
      out->n_pos = host.n_pos;
      if (s->resid) {
        std::vector<double> r(s->core->desc.p);
        PFX_HIP(hipMemcpy(r.data(), s->resid, sizeof(double) * r.size(), hipMemcpyDeviceToHost));
        double mx = 0.0;
        for (double v : r) mx = std::isnan(v) || v > mx ? v : mx;
        out->resid_max = mx;
      }
    }
  });
  if (st != PF_OK) return st;
  if (host.status != 0) {
    g_last_error = pf_status_string((pf_status)host.status);
    return (pf_status)host.status;
  }
  return PF_OK;
}

pf_status pf_session_export(pf_session* s, void* U_out, int64_t ldu, double* theta_out, pf_session_state* state,
                            void* stream) {
  return guarded([&] {
    if (!s || !U_out || !state) fail(PF_ERR_ARG, "NULL argument");
    const pf_desc& d = s->core->desc;
    if (ldu < d.n) fail(PF_ERR_ARG, "ldu is smaller than n");
    hipStream_t st = static_cast<hipStream_t>(stream);
    // the last step's U, in order after it
    if (s->stepped) PFX_HIP(hipStreamWaitEvent(st, s->done, 0));
    const Elem W = d.work == PF_F64 ? Elem::F64 : Elem::F32;
    launch_copy_block(s->core->U, s->core->ldu, W, U_out, ldu, W, d.n, d.p, d.n, d.p, st);
    if (theta_out)
      PFX_HIP(hipMemcpyAsync(theta_out, s->core->theta, sizeof(double) * d.p, hipMemcpyDeviceToDevice, st));
    pf_session_state out{};
    out.struct_size = sizeof(pf_session_state);
    out.desc = d;
    out.steps = s->core->steps;
    *state = out;
  });
}

pf_status pf_session_import(const pf_session_state* state, const void* U, int64_t ldu, const double* theta,
                            pf_session** out) {
  return guarded([&] {
    if (!state || !U || !out) fail(PF_ERR_ARG, "NULL argument");
    if (state->struct_size != sizeof(pf_session_state))
      fail(PF_ERR_ARG, "pf_session_state.struct_size must be sizeof(pf_session_state)");
    if (state->reserved != 0) fail(PF_ERR_ARG, "pf_session_state.reserved must be 0");
    if (state->steps < 0) fail(PF_ERR_ARG, "pf_session_state.steps must be >= 0");
    const pf_desc& d = state->desc;
    plan_validate(d, nullptr, nullptr);
    if (ldu < d.n) fail(PF_ERR_ARG, "ldu is smaller than n");
    pf_session* s = new pf_session();
    try {
      s->core = session_create(d, U, ldu, 0, nullptr, false);
      if (theta)
        PFX_HIP(hipMemcpyAsync(s->core->theta, theta, sizeof(double) * d.p, hipMemcpyDeviceToDevice, nullptr));
      PFX_HIP(hipStreamSynchronize(nullptr));
      s->core->steps = state->steps;
      PFX_HIP(hipEventCreateWithFlags(&s->done, hipEventDisableTiming));
    } catch (...) {
      session_destroy(s->core);
      delete s;
      throw;
    }
    *out = s;
  });
}

pf_status pf_session_close(pf_session* s) {
  return guarded([&] {
    if (!s) fail(PF_ERR_ARG, "session is NULL");
    if (s->stepped) {
      hipError_t q = hipEventQuery(s->done);
      if (q == hipErrorNotReady) fail(PF_ERR_BUSY, "session has a step in flight");
    }
    session_destroy(s->core);
    (void)hipEventDestroy(s->done);
    delete s;
  });
}

pf_status pf_quantize(void* dst, int64_t ld_dst, float* tile_scale, int32_t tile, pf_dtype dtype, const float* src,
                      int64_t rows, int64_t cols, int64_t ld_src, void* stream) {
  return guarded([&] {
    if (!dst || !src) fail(PF_ERR_ARG, "NULL matrix pointer");
    if (rows < 1 || cols < 1) fail(PF_ERR_ARG, "empty matrix");
    if (ld_src < rows || ld_dst < rows) fail(PF_ERR_ARG, "leading dimension smaller than rows");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (dtype == PF_BF16) {
      launch_quantize_bf16(src, rows, cols, ld_src, static_cast<uint16_t*>(dst), ld_dst, st);
    } else if (dtype == PF_F8E4M3) {
      if (!tile_scale) fail(PF_ERR_ARG, "FP8 needs tile_scale");
      if (tile < 1) fail(PF_ERR_ARG, "tile must be >= 1");
      launch_quantize_fp8(src, rows, cols, ld_src, static_cast<uint8_t*>(dst), ld_dst, tile_scale, tile, st);
    } else {
      fail(PF_ERR_ARG, "pf_quantize: dtype must be PF_BF16 or PF_F8E4M3");
    }
  });
}

pf_status pf_psd_dense(const void* V, int64_t ldv, const double* theta, int64_t n, int32_t p, pf_dtype work,
                       void* out, int64_t ld_out, void* stream) {
  return guarded([&] {
    if (!V || !theta || !out) fail(PF_ERR_ARG, "NULL argument");
    if (n < 1 || p < 1 || p > n) fail(PF_ERR_ARG, "bad n / p");
    if (ldv < n || ld_out < n) fail(PF_ERR_ARG, "leading dimension smaller than n");
    if (work != PF_F32 && work != PF_F64) fail(PF_ERR_ARG, "work must be F32 or F64");
    launch_psd_dense(V, ldv, work == PF_F64 ? Elem::F64 : Elem::F32, theta, n, p, out, ld_out,
                     static_cast<hipStream_t>(stream));
  });
}

pf_status pf_eigh(const double* H, int64_t ldh, int32_t p, double* theta, double* Z, int64_t ldz, void* stream) {
  return guarded([&] {
    if (!H || !theta || !Z) fail(PF_ERR_ARG, "NULL argument");
    if (p < 1 || p > 128) fail(PF_ERR_ARG, "p must be in [1, 128]");
    if (ldh < p || ldz < p) fail(PF_ERR_ARG, "leading dimension smaller than p");
    if (ldh > INT32_MAX || ldz > INT32_MAX) fail(PF_ERR_ARG, "leading dimension too large");
    const char* h0 = reinterpret_cast<const char*>(H);
    const char* h1 = h0 + ((size_t)(p - 1) * ldh + p) * sizeof(double);
    const char* z0 = reinterpret_cast<const char*>(Z);
    const char* z1 = z0 + ((size_t)(p - 1) * ldz + p) * sizeof(double);
    if (h0 < z1 && z0 < h1) fail(PF_ERR_ARG, "H and Z overlap");
    const hipStream_t st = static_cast<hipStream_t>(stream);
    if (p <= 64) {
      launch_eigh(H, (int)ldh, p, theta, Z, (int)ldz, p, nullptr, 1, st);
      return;
    }
    // the kernel chain of the dense solver keeps its state in device scratch
    void* mem = nullptr;
    if (hipMallocAsync(&mem, eig_scratch_bytes(p), st) != hipSuccess) {
      (void)hipGetLastError();
      fail(PF_ERR_NOMEM, "eigensolver scratch allocation failed");
    }
    try {
      launch_eigh(H, (int)ldh, p, theta, Z, (int)ldz, p, nullptr, 1, st, static_cast<double*>(mem));
    } catch (...) {
      (void)hipFreeAsync(mem, st);
      throw;
    }
    PFX_HIP(hipFreeAsync(mem, st));
  });
}

pf_status pf_lanczos_bounds(const pf_mat* X, int64_t n, const double* V0, int64_t ldv0, int32_t steps,
                            pf_bounds* out, void* stream) {
  return guarded([&] {
    if (!X || !X->data || !V0 || !out) fail(PF_ERR_ARG, "NULL argument");
    if (X->dtype != PF_F32 && X->dtype != PF_F64) fail(PF_ERR_ARG, "X must be FP32 or FP64");
    if (steps < 1 || steps > 8) fail(PF_ERR_ARG, "steps must be in [1, 8]");
    if (n < 16 * (int64_t)steps) fail(PF_ERR_ARG, "n must be at least 16 * steps");
    if (X->ld < n || ldv0 < n) fail(PF_ERR_ARG, "leading dimension smaller than n");
    const size_t esz = X->dtype == PF_F64 ? 8 : 4;
    if (reinterpret_cast<uintptr_t>(X->data) % 16 != 0) fail(PF_ERR_ARG, "X.data must be 16-byte aligned");
    if (((size_t)X->ld * esz) % 16 != 0) fail(PF_ERR_ARG, "X.ld * element size must be a multiple of 16 bytes");
    enqueue_lanczos(*X, n, V0, ldv0, steps, out, static_cast<hipStream_t>(stream));
  });
}

pf_status pf_interval_policy(double lam_min, double margin, double eta, int32_t top_r, double theta_r, double* a,
                             double* b) {
  return guarded([&] {
    if (!a || !b) fail(PF_ERR_ARG, "NULL argument");
    if (!std::isfinite(lam_min) || !std::isfinite(margin) || margin < 0.0) fail(PF_ERR_ARG, "lam_min and margin >= 0 must be finite");
    if (!(eta > 0.0 && eta < 1.0)) fail(PF_ERR_ARG, "eta must be in (0, 1)");
    const double lo = lam_min - margin;
    double hi;
    if (top_r <= 0) {
      hi = eta * lo;                                  // all positive eigenvalues
    } else {
      if (!std::isfinite(theta_r)) fail(PF_ERR_ARG, "theta_r must be finite");
      hi = (1.0 - eta) * theta_r + eta * lo;          // the r largest
    }
    if (!(lo < hi)) fail(PF_ERR_ARG, "the policy gives a >= b (all-positive case needs a < 0; top-r needs theta_r > a)");
    *a = lo;
    *b = hi;
  });
}

pf_status pf_block_size_policy(int32_t top_r, double q, int32_t n_pos, int32_t guards, int32_t* p) {
  return guarded([&] {
    if (!p) fail(PF_ERR_ARG, "NULL argument");
    double v;
    if (top_r > 0) {
      if (!std::isfinite(q) || !(q > 1.0)) fail(PF_ERR_ARG, "q must be a finite number above 1");
      v = std::ceil(5.0 + q * top_r);
    } else {
      if (n_pos < 0 || guards < 0) fail(PF_ERR_ARG, "n_pos and guards must be non-negative");
      v = (double)n_pos + guards;
    }
    *p = (int32_t)std::min(128.0, std::max(1.0, v));
  });
}

pf_status pf_session_set_interval(pf_session* s, double a, double b) {
  return guarded([&] {
    if (!s) fail(PF_ERR_ARG, "session is NULL");
    pf_desc d = s->core->desc;
    d.a = a;
    d.b = b;
    plan_validate(d, nullptr, nullptr);             // finite a < b; spec_ub > b when scaled
    s->core->desc = d;
  });
}

pf_status pf_degree_policy(double theta_r, double a, double b, int32_t q, double eps, int32_t d_min,
                           int32_t d_max, int32_t* degree) {
  return guarded([&] {
    if (!degree) fail(PF_ERR_ARG, "NULL argument");
    if (!std::isfinite(theta_r) || !std::isfinite(a) || !std::isfinite(b) || !(a < b) || !(b < theta_r))
      fail(PF_ERR_ARG, "need finite a < b < theta_r");
    if (!(eps > 0.0 && eps < 1.0)) fail(PF_ERR_ARG, "eps must be in (0, 1)");
    if (q < 1) fail(PF_ERR_ARG, "q must be >= 1");
    if (d_min < 1 || d_max < d_min) fail(PF_ERR_ARG, "need 1 <= d_min <= d_max");
    const double l = 2.0 * (theta_r - b) / (b - a);
    // T_d(1 + l) = cosh(d acosh(1 + l)) >= eps^(-1/q)
    const double d = std::ceil(std::acosh(std::pow(eps, -1.0 / q)) / std::acosh(1.0 + l));
    *degree = (int32_t)std::min<double>(d_max, std::max<double>(d_min, d));
  });
}

pf_status pf_session_set_filter(pf_session* s, int32_t degree, int32_t q) {
  return guarded([&] {
    if (!s) fail(PF_ERR_ARG, "session is NULL");
    pf_desc d = s->core->desc;
    d.degree = degree;
    d.q = q;
    plan_validate(d, nullptr, nullptr);             // degree >= 1, q >= 1
    s->core->desc = d;
  });
}

pf_status pf_nce_pfpg(const pf_nce_opts* opts, int64_t n, const double* G, int64_t ldg, double* x, const double* U0,
                      int64_t ldu0, const double* V0, int64_t ldv0, pf_nce_result* out, double* history,
                      void* stream) {
  if (out) *out = pf_nce_result{};
  const pf_status s = guarded([&] {
    if (!opts || !G || !x || !U0 || !V0 || !out) fail(PF_ERR_ARG, "NULL argument");
    const pf_nce_opts& o = *opts;
    if (o.struct_size != sizeof(pf_nce_opts)) fail(PF_ERR_ARG, "opts.struct_size must be sizeof(pf_nce_opts)");
    if (o.p_max < 16 || o.p_max > 128 || o.p_max > n) fail(PF_ERR_ARG, "p_max must be in [16, min(n, 128)]");
    if (o.degree < 1 || o.guards < 0 || o.max_iter < 1) fail(PF_ERR_ARG, "need degree >= 1, guards >= 0, max_iter >= 1");
    if (o.extrapolation_len < 0 || o.extrapolation_len > kNceMaxRna) fail(PF_ERR_ARG, "extrapolation_len must be in [0, 7]");
    if (o.lanczos_steps < 1 || o.lanczos_steps > 8 || n < 16 * (int64_t)o.lanczos_steps)
      fail(PF_ERR_ARG, "lanczos_steps must be in [1, 8] with 16 * lanczos_steps <= n");
    if (o.lanczos_every < 0) fail(PF_ERR_ARG, "lanczos_every must be >= 0");
    if (!(o.tau > 0.0) || !std::isfinite(o.tau)) fail(PF_ERR_ARG, "tau must be positive and finite");
    if (!(o.eta > 0.0 && o.eta < 1.0)) fail(PF_ERR_ARG, "eta must be in (0, 1)");
    if (!(o.tol > 0.0) || !std::isfinite(o.tol)) fail(PF_ERR_ARG, "tol must be positive and finite");
    if (!(o.extrapolation_lambda >= 0.0) || !std::isfinite(o.extrapolation_lambda))
      fail(PF_ERR_ARG, "extrapolation_lambda must be >= 0 and finite");
    if ((o.flags & ~PF_FLAG_NO_PREROTATE) != 0 || o.reserved != 0)
      fail(PF_ERR_ARG, "opts.flags may hold only PF_FLAG_NO_PREROTATE; opts.reserved must be 0");
    if (ldg < n || ldu0 < n || ldv0 < n) fail(PF_ERR_ARG, "leading dimension smaller than n");
    run_nce_pfpg(o, n, G, ldg, x, U0, ldu0, V0, ldv0, out, history, static_cast<hipStream_t>(stream));
    if (out->status != 0) fail((pf_status)out->status, "nce: an extraction reported a numerical failure");
  });
  if (s != PF_OK && out && out->status == 0) out->status = s;
  return s;
}

pf_status pf_nce_pfam(const pf_pfam_opts* opts, int64_t n, const double* G, int64_t ldg, double* Z, int64_t ldz,
                      double* X, int64_t ldx, const double* U0, int64_t ldu0, const double* V0, int64_t ldv0,
                      pf_pfam_result* out, double* history, void* stream) {
  if (out) *out = pf_pfam_result{};
  const pf_status s = guarded([&] {
    if (!opts || !G || !Z || !X || !U0 || !V0 || !out) fail(PF_ERR_ARG, "NULL argument");
    const pf_pfam_opts& o = *opts;
    if (o.struct_size != sizeof(pf_pfam_opts)) fail(PF_ERR_ARG, "opts.struct_size must be sizeof(pf_pfam_opts)");
    if (o.p_max < 16 || o.p_max > 128 || o.p_max > n) fail(PF_ERR_ARG, "p_max must be in [16, min(n, 128)]");
    if (o.degree < 1 || o.guards < 0 || o.max_iter < 1) fail(PF_ERR_ARG, "need degree >= 1, guards >= 0, max_iter >= 1");
    if (o.lanczos_steps < 1 || o.lanczos_steps > 8 || n < 16 * (int64_t)o.lanczos_steps)
      fail(PF_ERR_ARG, "lanczos_steps must be in [1, 8] with 16 * lanczos_steps <= n");
    if (o.lanczos_every < 0) fail(PF_ERR_ARG, "lanczos_every must be >= 0");
    if ((o.flags & ~PF_FLAG_NO_PREROTATE) != 0) fail(PF_ERR_ARG, "opts.flags may hold only PF_FLAG_NO_PREROTATE");
    if (!(o.t > 0.0) || !std::isfinite(o.t)) fail(PF_ERR_ARG, "t must be positive and finite");
    if (!(o.eta > 0.0 && o.eta < 1.0)) fail(PF_ERR_ARG, "eta must be in (0, 1)");
    if (!(o.tol > 0.0) || !std::isfinite(o.tol)) fail(PF_ERR_ARG, "tol must be positive and finite");
    if (n > 65535) fail(PF_ERR_ARG, "n must be at most 65535");
    if (ldg < n || ldz < n || ldx < n || ldu0 < n || ldv0 < n) fail(PF_ERR_ARG, "leading dimension smaller than n");
    if (Z == X || Z == G || X == G) fail(PF_ERR_ARG, "G, Z and X must be distinct buffers");
    if (reinterpret_cast<uintptr_t>(Z) % 16 != 0 || ((size_t)ldz * 8) % 16 != 0)
      fail(PF_ERR_ARG, "Z must be 16-byte aligned with ldz * 8 a multiple of 16");
    {
      // the extraction's own checks on Z at the largest block
      pf_desc d{};
      d.struct_size = sizeof(pf_desc);
      d.op = PF_OP_SYM; d.n = n; d.p = o.p_max; d.degree = o.degree; d.q = 1;
      d.a = -1.0; d.b = 0.0; d.work = PF_F64; d.flags = o.flags;
      const pf_mat zm{Z, PF_F64, ldz, nullptr, 0};
      plan_validate(d, &zm, &zm);
    }
    run_nce_pfam(o, n, G, ldg, Z, ldz, X, ldx, U0, ldu0, V0, ldv0, out, history, static_cast<hipStream_t>(stream));
    if (out->status != 0) fail((pf_status)out->status, "pfam: an extraction reported a numerical failure");
  });
  if (s != PF_OK && out && out->status == 0) out->status = s;
  return s;
}

}  // extern "C"
