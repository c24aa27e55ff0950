// The serving loop of include/pf.h: admission by HBM footprint, continuous
// batching of many sessions' steps, and HIP graph replay of the sessions
// that run on their own.
//
// One worker thread owns every HIP call on session state.  Caller threads
// only queue work (open / submit / close) under the server mutex and read
// finished-step events.  Per session at most one step is in flight: a step
// starts from the V its predecessor wrote, so a session is ready again when
// its previous step's event has completed.  Every pass of the worker takes
// all ready sessions on the symmetric operator and enqueues their steps as
// one batch of grouped launches (each phase of the extraction -- a filter
// product, a Gram matrix, a Cholesky factor, a p x p eigensolve, a block
// apply -- one launch per kernel instance for the whole batch); steps that
// arrive while batches run form the next batch, on the next stream.  Other
// sessions (the Gram operator) run their own steps, warm steps as graph
// replays.  A finished step's status reaches the host through a mapped
// pinned pf_info written by the last launch of the step.
//
// Device memory of closed sessions is kept for sessions of the same shape
// (a slot: workspace, block, theta, pf_info, event, pinned record) and only
// freed when the budget needs the room, so opening and closing sessions
// does not synchronise the device.
#include "pf_internal.h"
#include "group.h"
#include "admission.h"

#include <chrono>
#include <condition_variable>
#include <deque>
#include <functional>
#include <limits>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

namespace pfx {
namespace {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

bool same_mat(const pf_mat& a, const pf_mat& b) {
  return a.data == b.data && a.dtype == b.dtype && a.ld == b.ld && a.tile_scale == b.tile_scale && a.tile == b.tile;
}

struct Request {
  pf_mat xf, xr;
  uint64_t tag;
  int64_t submit_ns;
};

struct InFlight {
  Request req;
  int64_t step;
  int64_t launch_ns;
  bool graph;
};

// Device resources of a session, recycled across sessions of one layout.
struct Slot {
  SessionCore* core = nullptr;
  hipEvent_t done = nullptr;
  pf_info* host_info = nullptr;     // mapped pinned: host address
  pf_info* host_info_dev = nullptr; // the same memory as the device sees it
  size_t bytes = 0;                 // device bytes held
};

// what a slot's layout depends on
using SlotKey = std::tuple<int64_t, int64_t, int, int, int>;
SlotKey slot_key(const pf_desc& d) { return SlotKey{d.n, d.op == PF_OP_GRAM ? d.m : 0, d.p, (int)d.work, (int)d.op}; }

struct SrvSession {
  int32_t id = 0;
  pf_desc desc{};
  size_t footprint = 0;
  bool resident = false;
  bool closing = false;
  const void* U0 = nullptr;
  int64_t ldu0 = 0;
  uint64_t seed = 0;
  Slot slot;
  hipStream_t stream = nullptr;
  std::deque<Request> pending;
  bool busy = false;
  InFlight cur{};
  hipGraphExec_t exec = nullptr;
  pf_mat g_xf{}, g_xr{};
};

}  // namespace
}  // namespace pfx

using namespace pfx;

struct pf_server {
  pf_server_config cfg{};
  int device = 0;
  std::mutex mu;
  std::condition_variable cv;       // work for the worker
  std::condition_variable done_cv;  // events for pollers
  std::map<int32_t, SrvSession*> sessions;
  std::deque<int32_t> waitq;
  std::deque<pf_server_event> events;
  Admission<SlotKey, Slot>* adm = nullptr;   // budget, residents, pool of closed sessions' slots
  int32_t next_id = 1;
  std::vector<hipStream_t> streams;
  int next_stream = 0;
  std::vector<hipEvent_t> batch_running;   // one event per batch in flight
  std::vector<hipEvent_t> batch_free;
  bool stop = false;
  pf_server_stats stats{};
  std::thread worker;
};

namespace {

void free_slot(Slot& t) {
  if (t.done) (void)hipEventDestroy(t.done);
  if (t.host_info) (void)hipHostFree(t.host_info);
  session_destroy(t.core);
  t = Slot{};
}

// Close: the session is drained (no step queued or running), so its slot
// goes back to the pool as it is; no HIP call.
void free_session(pf_server* S, SrvSession* s) {
  if (s->exec) (void)hipGraphExecDestroy(s->exec);
  if (s->resident) {
    S->adm->release(s->footprint, slot_key(s->desc), s->slot, s->slot.bytes);
    s->slot = Slot{};
  }
  delete s;
}

// Free pooled slots until `need` more bytes fit the budget (the mutex is
// released while the device memory is freed).
void make_room(pf_server* S, std::unique_lock<std::mutex>& lk, size_t need) {
  std::vector<Slot> out = S->adm->evict_for(need);
  if (out.empty()) return;
  lk.unlock();
  for (Slot& t : out) free_slot(t);
  lk.lock();
}

// Admit s on its stream: a pooled slot of its shape when there is one
// (the start block re-initialised in place), a new one otherwise.  The
// slot's event marks the end of the initialisation.
void admit(pf_server* S, SrvSession* s) {
  s->stream = S->streams[S->next_stream];
  S->next_stream = (S->next_stream + 1) % (int)S->streams.size();
  if (S->adm->take(slot_key(s->desc), s->slot)) {
    SessionCore* c = s->slot.core;
    c->desc = s->desc;
    c->steps = 0;
    plan_set_desc(c->plan, s->desc);
    const Elem W = s->desc.work == PF_F64 ? Elem::F64 : Elem::F32;
    // the previous user's last step has completed (its session was drained)
    if (s->U0) launch_copy_block(s->U0, s->ldu0, W, c->U, c->ldu, W, s->desc.n, s->desc.p, s->desc.n, s->desc.p,
                                 s->stream);
    else launch_normal_block(c->U, c->ldu, W, s->desc.n, s->desc.p, s->seed, s->stream);
  } else {
    Slot t;
    try {
      PFX_HIP(hipEventCreateWithFlags(&t.done, hipEventDisableTiming));
      PFX_HIP(hipHostMalloc(reinterpret_cast<void**>(&t.host_info), sizeof(pf_info), hipHostMallocMapped));
      PFX_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&t.host_info_dev), t.host_info, 0));
      t.core = session_create(s->desc, s->U0, s->ldu0, s->seed, s->stream, false);
      t.bytes = session_bytes(s->desc);
    } catch (...) {
      free_slot(t);
      throw;
    }
    s->slot = t;
  }
  PFX_HIP(hipEventRecord(s->slot.done, s->stream));
  s->resident = true;
  S->adm->admit(s->footprint);
}

void finish(pf_server* S, SrvSession* s, int32_t status, int32_t n_pos);
void launch_step(pf_server* S, SrvSession* s, const Request& r, int64_t step);

// Launch the next queued step of s (caller holds the mutex).  A failure to
// enqueue finishes the step at once with its status.
void launch(pf_server* S, SrvSession* s) {
  Request r = s->pending.front();
  s->pending.pop_front();
  const int64_t step = s->slot.core->steps;
  try {
    launch_step(S, s, r, step);
  } catch (const Error& e) {
    s->cur = InFlight{r, step, now_ns(), false};
    finish(S, s, e.status, 0);
  }
}

void launch_step(pf_server* S, SrvSession* s, const Request& r, int64_t step) {
  const bool warm = step > 0;
  bool graph = warm && !(S->cfg.flags & PF_SERVER_NO_GRAPHS) && !prof_enabled();
  if (graph && !(s->exec && same_mat(s->g_xf, r.xf) && same_mat(s->g_xr, r.xr))) {
    // capture the warm step on these operator buffers
    if (s->exec) {
      (void)hipGraphExecDestroy(s->exec);
      s->exec = nullptr;
    }
    PFX_HIP(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
    hipGraph_t g = nullptr;
    try {
      pf_desc d = s->desc;                          // warm: no cold-start flag
      SessionCore* c = s->slot.core;
      plan_set_desc(c->plan, d);
      enqueue_extraction(c->plan, r.xf, r.xr, c->U, c->ldu, c->U, c->ldu, c->theta, c->info, s->stream);
      launch_info_to_host(c->info, s->slot.host_info_dev, s->stream);
    } catch (...) {
      (void)hipStreamEndCapture(s->stream, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    PFX_HIP(hipStreamEndCapture(s->stream, &g));
    hipError_t e = hipGraphInstantiate(&s->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    PFX_HIP(e);
    s->g_xf = r.xf;
    s->g_xr = r.xr;
    S->stats.captures++;
  }
  if (graph) {
    PFX_HIP(hipGraphLaunch(s->exec, s->stream));
    s->slot.core->steps++;
    S->stats.graph_launches++;
  } else {
    session_enqueue_step(s->slot.core, r.xf, r.xr, s->stream);
    launch_info_to_host(s->slot.core->info, s->slot.host_info_dev, s->stream);
  }
  PFX_HIP(hipEventRecord(s->slot.done, s->stream));
  s->busy = true;
  s->cur = InFlight{r, step, now_ns(), graph};
  S->stats.launched++;
}

void finish(pf_server* S, SrvSession* s, int32_t status, int32_t n_pos) {
  pf_server_event ev{};
  ev.session = s->id;
  ev.status = status;
  ev.n_pos = n_pos;
  ev.graph = s->cur.graph ? 1 : 0;
  ev.step = s->cur.step;
  ev.tag = s->cur.req.tag;
  ev.submit_ns = s->cur.req.submit_ns;
  ev.launch_ns = s->cur.launch_ns;
  ev.done_ns = now_ns();
  S->events.push_back(ev);
  S->stats.completed++;
  s->busy = false;
}

void fail_request(pf_server* S, SrvSession* s, const Request& r, int32_t status) {
  s->cur = InFlight{r, s->slot.core ? s->slot.core->steps : 0, now_ns(), false};
  finish(S, s, status, 0);
}

// One batch: the next step of every session in `members` (ready, on the
// symmetric operator), as grouped launches on the next stream.  Each
// member's stream order with its earlier work (initialisation, previous
// step) comes from its slot event.
void launch_batch(pf_server* S, const std::vector<SrvSession*>& members) {
  TraceRange trace("pf.server.batch");
  hipStream_t B = S->streams[S->next_stream];
  S->next_stream = (S->next_stream + 1) % (int)S->streams.size();
  std::vector<ExtractionJob> jobs(members.size());
  std::vector<Request> reqs(members.size());
  for (size_t i = 0; i < members.size(); ++i) {
    SrvSession* m = members[i];
    reqs[i] = m->pending.front();
    SessionCore* c = m->slot.core;
    ExtractionJob& j = jobs[i];
    j.plan = c->plan;
    j.desc = m->desc;
    if (c->steps == 0) j.desc.flags |= PF_FLAG_COLD;     // the first step starts from U0
    j.Xf = reqs[i].xf;
    j.Xr = reqs[i].xr;
    j.U_in = c->U;
    j.ldu_in = c->ldu;
    j.U_out = c->U;
    j.ldu_out = c->ldu;
    j.theta_out = c->theta;
    j.info_out = c->info;
    j.info_host = m->slot.host_info_dev;
  }
  try {
    for (SrvSession* m : members) PFX_HIP(hipStreamWaitEvent(B, m->slot.done, 0));
    enqueue_extractions_grouped((int)jobs.size(), jobs.data(), B);
  } catch (const Error& e) {
    for (size_t i = 0; i < members.size(); ++i) {
      members[i]->pending.pop_front();
      fail_request(S, members[i], reqs[i], e.status);
    }
    return;
  }
  const int64_t t = now_ns();
  for (size_t i = 0; i < members.size(); ++i) {
    SrvSession* m = members[i];
    m->pending.pop_front();
    const hipError_t e = hipEventRecord(m->slot.done, B);
    m->cur = InFlight{reqs[i], m->slot.core->steps, t, false};
    m->slot.core->steps++;
    if (e != hipSuccess) {
      finish(S, m, PF_ERR_DEVICE, 0);
      continue;
    }
    m->busy = true;
    S->stats.launched++;
  }
  S->stats.batches++;
  S->stats.batched_steps += (int64_t)members.size();
  hipEvent_t be = nullptr;
  if (!S->batch_free.empty()) {
    be = S->batch_free.back();
    S->batch_free.pop_back();
  } else if (hipEventCreateWithFlags(&be, hipEventDisableTiming) != hipSuccess) {
    be = nullptr;
  }
  if (be) {
    if (hipEventRecord(be, B) == hipSuccess) S->batch_running.push_back(be);
    else S->batch_free.push_back(be);
  }
}

// Batches still running (finished ones leave the list).
int batches_in_flight(pf_server* S) {
  for (size_t i = 0; i < S->batch_running.size();) {
    if (hipEventQuery(S->batch_running[i]) != hipErrorNotReady) {
      S->batch_free.push_back(S->batch_running[i]);
      S->batch_running[i] = S->batch_running.back();
      S->batch_running.pop_back();
    } else {
      ++i;
    }
  }
  return (int)S->batch_running.size();
}

constexpr size_t kMaxBatch = 256;

void worker_loop(pf_server* S) {
  (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    bool progress = false;
    // completions
    for (auto& kv : S->sessions) {
      SrvSession* s = kv.second;
      if (!s->busy) continue;
      const hipError_t q = hipEventQuery(s->slot.done);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) {
        finish(S, s, PF_ERR_DEVICE, 0);
      } else {
        const volatile pf_info* hi = s->slot.host_info;
        finish(S, s, hi->status, hi->n_pos);
      }
      progress = true;
    }
    // closes of drained sessions
    for (auto it = S->sessions.begin(); it != S->sessions.end();) {
      SrvSession* s = it->second;
      if (s->closing && !s->busy && s->pending.empty()) {
        if (!s->resident) {
          for (auto w = S->waitq.begin(); w != S->waitq.end(); ++w)
            if (*w == s->id) { S->waitq.erase(w); break; }
        }
        free_session(S, s);
        it = S->sessions.erase(it);
        progress = true;
      } else {
        ++it;
      }
    }
    // admission in FIFO order
    while (!S->waitq.empty()) {
      SrvSession* s = S->sessions[S->waitq.front()];
      if (!S->adm->fits(s->footprint)) break;
      if (!S->adm->pooled(slot_key(s->desc))) make_room(S, lk, s->footprint);
      S->waitq.pop_front();
      try {
        admit(S, s);
      } catch (const Error&) {
        // could not allocate: fail its queued steps; it stays closed-out
        while (!s->pending.empty()) {
          fail_request(S, s, s->pending.front(), PF_ERR_NOMEM);
          s->pending.pop_front();
        }
        s->closing = true;
      }
      progress = true;
    }
    // launches: the ready sessions on the symmetric operator as one batch
    // of grouped launches while fewer than max_batches batches run (they
    // wait for the next batch otherwise), the others one by one
    std::vector<SrvSession*> batch;
    const bool group = !(S->cfg.flags & PF_SERVER_NO_GROUPING);
    const bool room = group && batches_in_flight(S) < S->cfg.max_batches;
    for (auto& kv : S->sessions) {
      SrvSession* s = kv.second;
      if (!s->resident || s->busy || s->pending.empty()) continue;
      if (group && s->desc.op == PF_OP_SYM) {
        if (!room) continue;
        batch.push_back(s);
        if (batch.size() == kMaxBatch) {
          launch_batch(S, batch);
          batch.clear();
        }
      } else {
        launch(S, s);
      }
      progress = true;
    }
    if (!batch.empty()) launch_batch(S, batch);
    if (!S->events.empty()) S->done_cv.notify_all();
    if (S->stop) {
      bool idle = S->waitq.empty();
      for (auto& kv : S->sessions) idle = idle && !kv.second->busy && kv.second->pending.empty();
      if (idle) break;
    }
    if (!progress) {
      bool any_busy = false;
      for (auto& kv : S->sessions) any_busy = any_busy || kv.second->busy;
      // poll quickly while steps run; otherwise sleep until work arrives
      if (any_busy) S->cv.wait_for(lk, std::chrono::microseconds(20));
      else S->cv.wait_for(lk, std::chrono::milliseconds(5));
    }
  }
  for (hipEvent_t e : S->batch_running) (void)hipEventDestroy(e);
  for (hipEvent_t e : S->batch_free) (void)hipEventDestroy(e);
  S->batch_running.clear();
  S->batch_free.clear();
  for (auto& kv : S->sessions) free_session(S, kv.second);
  S->sessions.clear();
  for (Slot& t : S->adm->drain()) free_slot(t);
  S->waitq.clear();
  S->done_cv.notify_all();
}

}  // namespace

// guarded() of capi.cpp is file-local; the server reports errors the same way.
namespace pfx {
pf_status run_guarded(const std::function<void()>& f);
}

extern "C" {

pf_status pf_server_create(const pf_server_config* cfg, pf_server** out) {
  return run_guarded([&] {
    if (!cfg || !out) fail(PF_ERR_ARG, "NULL argument");
    if (cfg->struct_size != sizeof(pf_server_config)) fail(PF_ERR_ARG, "pf_server_config.struct_size mismatch");
    if (cfg->hbm_budget == 0) fail(PF_ERR_ARG, "pf_server_config.hbm_budget must be > 0");
    if (cfg->max_active < 0 || cfg->streams < 0 || cfg->streams > 64 || cfg->max_batches < 0)
      fail(PF_ERR_ARG, "bad server limits");
    if (cfg->reserved != 0) fail(PF_ERR_ARG, "pf_server_config.reserved must be 0");
    if (cfg->flags & ~(PF_SERVER_NO_GRAPHS | PF_SERVER_NO_GROUPING))
      fail(PF_ERR_ARG, "unknown bits in pf_server_config.flags");
    pf_server* S = new pf_server();
    S->cfg = *cfg;
    if (S->cfg.max_active == 0) S->cfg.max_active = 64;
    if (S->cfg.streams == 0) S->cfg.streams = 8;
    if (S->cfg.max_batches == 0) S->cfg.max_batches = 4;
    S->adm = new Admission<SlotKey, Slot>(S->cfg.hbm_budget, S->cfg.max_active);
    try {
      PFX_HIP(hipGetDevice(&S->device));
      for (int i = 0; i < S->cfg.streams; ++i) {
        hipStream_t st;
        PFX_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));   // default priority
        S->streams.push_back(st);
      }
      S->worker = std::thread(worker_loop, S);
    } catch (...) {
      for (hipStream_t st : S->streams) (void)hipStreamDestroy(st);
      delete S->adm;
      delete S;
      throw;
    }
    *out = S;
  });
}

pf_status pf_server_open(pf_server* S, const pf_desc* desc, const void* U0, int64_t ldu0, uint64_t seed,
                         size_t operator_bytes, int32_t* session) {
  return run_guarded([&] {
    if (!S || !desc || !session) fail(PF_ERR_ARG, "NULL argument");
    plan_validate(*desc, nullptr, nullptr);
    if (U0 && ldu0 < desc->n) fail(PF_ERR_ARG, "ldu0 is smaller than n");
    const size_t fp = session_bytes(*desc) + operator_bytes;
    if (fp > S->cfg.hbm_budget) fail(PF_ERR_NOMEM, "session footprint exceeds the server's HBM budget");
    SrvSession* s = new SrvSession();
    s->desc = *desc;
    s->footprint = fp;
    s->U0 = U0;
    s->ldu0 = ldu0;
    s->seed = seed;
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) {
      delete s;
      fail(PF_ERR_ARG, "server is shutting down");
    }
    s->id = S->next_id++;
    S->sessions[s->id] = s;
    S->waitq.push_back(s->id);
    *session = s->id;
    S->cv.notify_one();
  });
}

pf_status pf_server_submit(pf_server* S, int32_t session, const pf_mat* X_filter, const pf_mat* X_rr,
                           uint64_t tag) {
  return run_guarded([&] {
    if (!S) fail(PF_ERR_ARG, "server is NULL");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->sessions.find(session);
    if (it == S->sessions.end() || it->second->closing) fail(PF_ERR_ARG, "unknown or closing session");
    plan_validate(it->second->desc, X_filter, X_rr);
    it->second->pending.push_back(Request{*X_filter, *X_rr, tag, now_ns()});
    S->cv.notify_one();
  });
}

pf_status pf_server_poll(pf_server* S, pf_server_event* events, int32_t max, int32_t* count, int64_t timeout_ns) {
  return run_guarded([&] {
    if (!S || !count || (max > 0 && !events)) fail(PF_ERR_ARG, "NULL argument");
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->events.empty() && timeout_ns > 0)
      S->done_cv.wait_for(lk, std::chrono::nanoseconds(timeout_ns), [&] { return !S->events.empty(); });
    int32_t n = 0;
    while (n < max && !S->events.empty()) {
      events[n++] = S->events.front();
      S->events.pop_front();
    }
    *count = n;
  });
}

pf_status pf_server_result(pf_server* S, int32_t session, pf_result* out) {
  return run_guarded([&] {
    if (!S || !out) fail(PF_ERR_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->sessions.find(session);
    if (it == S->sessions.end() || !it->second->resident) fail(PF_ERR_ARG, "session is not resident");
    SrvSession* s = it->second;
    if (s->busy || !s->pending.empty()) fail(PF_ERR_BUSY, "session has steps queued or running");
    out->status = s->slot.host_info->status;
    out->n_pos = s->slot.host_info->n_pos;
    out->theta = s->slot.core->theta;
    out->V = s->slot.core->U;
    out->ldv = s->slot.core->ldu;
    out->info = s->slot.core->info;
    out->resid = nullptr;
    out->resid_max = std::numeric_limits<double>::quiet_NaN();
  });
}

pf_status pf_server_close(pf_server* S, int32_t session) {
  return run_guarded([&] {
    if (!S) fail(PF_ERR_ARG, "server is NULL");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->sessions.find(session);
    if (it == S->sessions.end() || it->second->closing) fail(PF_ERR_ARG, "unknown or closing session");
    it->second->closing = true;
    S->cv.notify_one();
  });
}

pf_status pf_server_stats_get(pf_server* S, pf_server_stats* out) {
  return run_guarded([&] {
    if (!S || !out) fail(PF_ERR_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->stats;
    out->active = S->adm->active();
    out->waiting = (int32_t)S->waitq.size();
    out->used_bytes = S->adm->used();
  });
}

pf_status pf_server_destroy(pf_server* S) {
  return run_guarded([&] {
    if (!S) fail(PF_ERR_ARG, "server is NULL");
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->stop = true;
      for (auto& kv : S->sessions) kv.second->closing = true;
      S->cv.notify_one();
    }
    S->worker.join();
    for (hipStream_t st : S->streams) (void)hipStreamDestroy(st);
    delete S->adm;
    delete S;
  });
}

}  // extern "C"
