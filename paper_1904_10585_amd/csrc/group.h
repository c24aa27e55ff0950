// Grouped launches: one launch of a kernel serving many independent
// problems (the extractions of many sessions, or the blocks of a
// block-diagonal operator), each with its own arguments and grid.
//
// A kernel is a struct K with
//   using Args = ...;                          its argument record
//   static constexpr int kThreads, kMinWaves;  block size, launch bounds
//   static __device__ void body(const Args&, uint3 bid);
// and is only ever launched through grouped_kernel<K, N>: a single problem
// is a group of one.  A problem runs the same kernel body whether it is
// launched alone or beside others (the instances for one member and for
// many differ only in the size of their argument block), and its results
// are bitwise the same either way (checked by the batch and serving tests).
//
// Members' block ranges are laid end to end, each starting at a multiple of
// 8 (the XCD count, so a member's block b lands on XCD b mod 8 as it would
// alone); blocks past a member's own grid return at once.  A group of one
// is launched on the member's own grid.
#pragma once

#include "pf_internal.h"

#include <algorithm>
#include <cstring>
#include <vector>

namespace pfx {

// kernel-argument budget of one grouped launch (the member records, their
// block offsets and grid shapes)
constexpr size_t kGroupArgBytes = 3584;
constexpr int kGroupMaxMembers = 32;
constexpr size_t kRecArgBytes = 512;     // largest Args record

template <typename A>
constexpr int group_n() {
  constexpr size_t per = sizeof(A) + 16;
  constexpr size_t n = (kGroupArgBytes - 16) / per;
  return (int)(n > (size_t)kGroupMaxMembers ? (size_t)kGroupMaxMembers : (n < 1 ? 1 : n));
}

template <typename A, int N>
struct GroupArgs {
  A a[N];
  int first[N + 1];      // first flat block of each member; first[count] = total
  unsigned gx[N], gy[N], nb[N];
  int count;
};

template <typename K, int N>
__global__ __launch_bounds__(K::kThreads, K::kMinWaves) void grouped_kernel(GroupArgs<typename K::Args, N> g) {
  if constexpr (N == 1) {
    // one member: launched on its own grid, its arguments at fixed offsets
    K::body(g.a[0], make_uint3(blockIdx.x, blockIdx.y, blockIdx.z));
  } else {
    const int b = (int)blockIdx.x;
    int i = 0;
    while (i + 1 < g.count && b >= g.first[i + 1]) ++i;
    const unsigned local = (unsigned)(b - g.first[i]);
    if (local >= g.nb[i]) return;
    const unsigned gx = g.gx[i], gy = g.gy[i];
    const uint3 bid = make_uint3(local % gx, (local / gx) % gy, local / (gx * gy));
    K::body(g.a[i], bid);
  }
}

// One recorded launch: its kernel instance, arguments, grid and where it
// sits in the sequence of its problem (phase, then order within the phase).
struct LaunchRec {
  void (*flush)(LaunchRec* const* recs, int count, hipStream_t st) = nullptr;
  dim3 grid;
  size_t lds = 0;
  int64_t phase = 0;
  int sub = 0;
  int member = 0;
  alignas(16) unsigned char args[kRecArgBytes];
};

// While a recorder is installed on the calling thread, launches are recorded
// instead of enqueued (grouped_enqueue installs one).
struct Recorder {
  std::vector<LaunchRec> recs;
  int64_t phase = 0;
  int sub = 0;
  int member = 0;
};
Recorder*& current_recorder();

// Mark the start of a phase of the problem being recorded (a no-op when
// launches go straight to the stream).
inline void set_phase(int64_t phase) {
  if (Recorder* R = current_recorder()) {
    R->phase = phase;
    R->sub = 0;
  }
}

// Launches of at most N members each (N = 1: a single problem, with a
// kernel-argument block of one record; larger blocks cost launch time).
template <typename K, int N>
void flush_n(LaunchRec* const* recs, int count, hipStream_t st) {
  using A = typename K::Args;
  static_assert(sizeof(GroupArgs<A, N>) <= kGroupArgBytes, "group record too large");
  static size_t cur_lds = 0;
  for (int c0 = 0; c0 < count; c0 += N) {
    const int cnt = std::min(N, count - c0);
    GroupArgs<A, N> g;
    std::memset(&g, 0, sizeof(g));
    int total = 0;
    size_t lds = 0;
    for (int i = 0; i < cnt; ++i) {
      const LaunchRec& r = *recs[c0 + i];
      std::memcpy(&g.a[i], r.args, sizeof(A));
      g.first[i] = total;
      g.gx[i] = r.grid.x;
      g.gy[i] = r.grid.y;
      g.nb[i] = r.grid.x * r.grid.y * r.grid.z;
      total += (int)round_up((int64_t)g.nb[i], 8);
      lds = std::max(lds, r.lds);
    }
    g.first[cnt] = total;
    g.count = cnt;
    if (total == 0) continue;
    ensure_lds((const void*)grouped_kernel<K, N>, lds, cur_lds);
    const dim3 grid = N == 1 ? recs[c0]->grid : dim3((unsigned)total);
    grouped_kernel<K, N><<<grid, dim3(K::kThreads), lds, st>>>(g);
    PFX_HIP(hipGetLastError());
  }
}

template <typename K>
void flush_group(LaunchRec* const* recs, int count, hipStream_t st) {
  if (count == 1) flush_n<K, 1>(recs, 1, st);
  else flush_n<K, group_n<typename K::Args>()>(recs, count, st);
}

// Launch kernel K on one problem, or record the launch when a recorder is
// installed on this thread.
template <typename K>
void emit(const typename K::Args& a, dim3 grid, size_t lds, hipStream_t st) {
  static_assert(sizeof(typename K::Args) <= kRecArgBytes, "argument record too large");
  static_assert(std::is_trivially_copyable<typename K::Args>::value, "argument records are copied as bytes");
  if (Recorder* R = current_recorder()) {
    R->recs.emplace_back();
    LaunchRec& r = R->recs.back();
    r.flush = &flush_group<K>;
    r.grid = grid;
    r.lds = lds;
    r.phase = R->phase;
    r.sub = R->sub++;
    r.member = R->member;
    std::memcpy(r.args, &a, sizeof(a));
    return;
  }
  LaunchRec r;
  r.grid = grid;
  r.lds = lds;
  std::memcpy(r.args, &a, sizeof(a));
  LaunchRec* p = &r;
  flush_group<K>(&p, 1, st);
}

// Enqueue many independent problems on st as grouped launches.  enqueue(i)
// enqueues problem i (every launch through emit, every phase marked with
// set_phase, phases in increasing order); launches of equal (phase, order
// within the phase) and kernel instance run as one grouped launch, in
// problem order.  Launches of different problems never depend on each
// other; each problem's own launches keep their order.
template <typename F>
void grouped_enqueue(int count, F&& enqueue, hipStream_t st) {
  Recorder R;
  Recorder*& slot = current_recorder();
  Recorder* saved = slot;
  slot = &R;
  try {
    for (int i = 0; i < count; ++i) {
      R.member = i;
      R.phase = 0;
      R.sub = 0;
      enqueue(i);
    }
  } catch (...) {
    slot = saved;
    throw;
  }
  slot = saved;
  std::vector<LaunchRec*> order(R.recs.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = &R.recs[i];
  std::stable_sort(order.begin(), order.end(), [](const LaunchRec* x, const LaunchRec* y) {
    return x->phase != y->phase ? x->phase < y->phase : x->sub < y->sub;
  });
  std::vector<LaunchRec*> bucket;
  size_t i = 0;
  while (i < order.size()) {
    size_t j = i;
    while (j < order.size() && order[j]->phase == order[i]->phase && order[j]->sub == order[i]->sub) ++j;
    // one grouped launch per kernel instance among launches [i, j)
    std::vector<bool> done(j - i, false);
    for (size_t a = i; a < j; ++a) {
      if (done[a - i]) continue;
      bucket.clear();
      for (size_t b = a; b < j; ++b)
        if (!done[b - i] && order[b]->flush == order[a]->flush) {
          bucket.push_back(order[b]);
          done[b - i] = true;
        }
      order[a]->flush(bucket.data(), (int)bucket.size(), st);
    }
    i = j;
  }
}

}  // namespace pfx
