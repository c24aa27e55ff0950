// Host check of the serving loop's admission bookkeeping (admission.h)
// against a fake allocator, built with address and undefined-behaviour
// sanitizers.  Scripted cases, then a seeded random open/close stream with
// the invariants checked after every event:
//   - resident footprints never exceed the budget, nor the active limit;
//   - a new slot is allocated only after the pool gave up enough slots for
//     resident + pooled + new bytes to fit the budget;
//   - a pooled slot is reused only by a session of its own shape;
//   - every allocation is freed exactly once by the end (no leak, no
//     double free).
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <set>
#include <vector>

#include "../../paper_1904_10585_amd/csrc/admission.h"

namespace {

int failures = 0;
#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
      ++failures;                                                       \
    }                                                                   \
  } while (0)

struct FakeAlloc {
  std::map<int, size_t> live;   // slot id -> bytes
  int next = 1;
  size_t bytes = 0;
  int alloc(size_t b) {
    live[next] = b;
    bytes += b;
    return next++;
  }
  void free(int id) {
    auto it = live.find(id);
    CHECK(it != live.end());      // no double free, no free of unknown memory
    if (it == live.end()) return;
    bytes -= it->second;
    live.erase(it);
  }
};

struct Slot {
  int id = 0;
  int key = -1;
};

using Adm = pfx::Admission<int, Slot>;

// Admit one session of shape key (slot of slot_bytes, footprint bytes): the
// server's order of operations.  Returns false if it does not fit now.
bool admit(Adm& a, FakeAlloc& fa, int key, size_t slot_bytes, size_t footprint, Slot& out) {
  if (!a.fits(footprint)) return false;
  if (a.take(key, out)) {
    CHECK(out.key == key);
  } else {
    for (Slot& s : a.evict_for(footprint)) fa.free(s.id);
    CHECK(a.used() + a.pooled_bytes() + footprint <= a.budget());
    out.id = fa.alloc(slot_bytes);
    out.key = key;
  }
  a.admit(footprint);
  CHECK(a.used() <= a.budget());
  return true;
}

void scripted() {
  FakeAlloc fa;
  Adm a(100, 2);
  Slot A, B, C, D;
  CHECK(admit(a, fa, 1, 30, 40, A));
  CHECK(admit(a, fa, 2, 30, 40, B));
  CHECK(!admit(a, fa, 1, 30, 40, C));            // active limit (and 120 > 100 bytes)
  a.release(40, 1, A, 30);                       // A's slot goes to the pool
  CHECK(a.active() == 1 && a.used() == 40 && a.pooled_bytes() == 30);
  CHECK(admit(a, fa, 1, 30, 40, C));             // same shape: A's slot again, nothing allocated
  CHECK(C.id == A.id && fa.live.size() == 2);
  CHECK(!admit(a, fa, 3, 30, 40, D));
  a.release(40, 2, B, 30);
  CHECK(admit(a, fa, 3, 30, 40, D));             // other shape: B's pooled slot is freed first
  CHECK(fa.live.count(B.id) == 0 && fa.live.size() == 2 && a.pooled_bytes() == 0);
  a.release(40, 1, C, 30);
  a.release(40, 3, D, 30);
  for (Slot& s : a.drain()) fa.free(s.id);
  CHECK(fa.live.empty() && a.used() == 0 && a.active() == 0 && a.pooled_bytes() == 0);
}

void random_stream(unsigned seed) {
  std::mt19937 g(seed);
  FakeAlloc fa;
  const size_t budget = 1000;
  Adm a(budget, 6);
  std::vector<std::pair<Slot, size_t>> resident;   // slot, footprint
  const size_t slot_bytes[5] = {50, 80, 120, 200, 260};
  for (int ev = 0; ev < 20000; ++ev) {
    if (!resident.empty() && (g() % 3 == 0 || resident.size() == 6)) {
      const size_t i = g() % resident.size();
      const Slot s = resident[i].first;
      a.release(resident[i].second, s.key, s, slot_bytes[s.key]);
      resident.erase(resident.begin() + i);
    } else {
      const int key = (int)(g() % 5);
      const size_t fp = slot_bytes[key] + g() % 100;   // declared operator bytes on top
      Slot s;
      if (admit(a, fa, key, slot_bytes[key], fp, s)) resident.push_back({s, fp});
    }
    size_t used = 0;
    for (auto& r : resident) used += r.second;
    CHECK(used == a.used() && used <= budget && (int)resident.size() == a.active());
    // device memory held = resident slots + pooled slots, all live allocations
    size_t held = 0;
    std::set<int> ids;
    for (auto& r : resident) {
      held += slot_bytes[r.first.key];
      ids.insert(r.first.id);
    }
    CHECK(fa.bytes == held + a.pooled_bytes());
    CHECK(ids.size() == resident.size());              // no slot handed to two sessions
  }
  for (auto& r : resident) a.release(r.second, r.first.key, r.first, slot_bytes[r.first.key]);
  for (Slot& s : a.drain()) fa.free(s.id);
  CHECK(fa.live.empty() && fa.bytes == 0);
}

}  // namespace

int main() {
  scripted();
  for (unsigned seed = 1; seed <= 5; ++seed) random_stream(seed);
  if (failures) {
    std::fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  std::printf("admission checks passed\n");
  return 0;
}
