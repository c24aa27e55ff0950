// Admission bookkeeping of the serving loop, free of HIP so that it can be
// checked on the host alone (tests/host/admission_check.cpp builds it with
// address and undefined-behaviour sanitizers against a fake allocator).
//
// A session holds `footprint` bytes of the budget while it is resident (its
// device memory plus the operator bytes its caller declares).  The device
// memory of a closed session (a slot) stays in a pool keyed by its shape and
// is handed to the next session of that shape; pooled bytes count against
// the budget too, and pooled slots of any shape are given up (oldest key
// first) when a new allocation needs the room.
#pragma once

#include <cstddef>
#include <map>
#include <utility>
#include <vector>

namespace pfx {

template <typename Key, typename Slot>
class Admission {
 public:
  Admission(size_t budget, int max_active) : budget_(budget), max_active_(max_active) {}

  // Room for one more resident session of this footprint.
  bool fits(size_t footprint) const { return used_ + footprint <= budget_ && active_ < max_active_; }

  bool pooled(const Key& k) const { return pool_.find(k) != pool_.end(); }

  // Slots to free (in order) so that a new slot of `need` bytes fits beside
  // the resident sessions and the pool.
  std::vector<Slot> evict_for(size_t need) {
    std::vector<Slot> out;
    while (!pool_.empty() && used_ + pooled_ + need > budget_) {
      auto it = pool_.begin();
      pooled_ -= it->second.second;
      out.push_back(it->second.first);
      pool_.erase(it);
    }
    return out;
  }

  // A pooled slot of this shape (and true), or false when there is none.
  bool take(const Key& k, Slot& slot) {
    auto it = pool_.find(k);
    if (it == pool_.end()) return false;
    slot = it->second.first;
    pooled_ -= it->second.second;
    pool_.erase(it);
    return true;
  }

  // A session of this footprint becomes resident / leaves (its slot of
  // slot_bytes device bytes goes to the pool).
  void admit(size_t footprint) {
    used_ += footprint;
    ++active_;
  }
  void release(size_t footprint, const Key& k, const Slot& slot, size_t slot_bytes) {
    used_ -= footprint;
    --active_;
    pooled_ += slot_bytes;
    pool_.emplace(k, std::make_pair(slot, slot_bytes));
  }
  // A resident session that leaves without a slot to keep.
  void drop(size_t footprint) {
    used_ -= footprint;
    --active_;
  }

  // Every pooled slot (for freeing at shutdown); the pool is left empty.
  std::vector<Slot> drain() {
    std::vector<Slot> out;
    for (auto& kv : pool_) out.push_back(kv.second.first);
    pool_.clear();
    pooled_ = 0;
    return out;
  }

  size_t used() const { return used_; }
  size_t pooled_bytes() const { return pooled_; }
  int active() const { return active_; }
  size_t budget() const { return budget_; }

 private:
  size_t budget_;
  int max_active_;
  size_t used_ = 0;
  size_t pooled_ = 0;
  int active_ = 0;
  std::multimap<Key, std::pair<Slot, size_t>> pool_;
};

}  // namespace pfx
