// Host-only building blocks of the engine, free of HIP calls so that they can
// be exercised without a GPU: the device-memory arena (first-fit with
// coalescing), the footprint of a solve and the FIFO admission queue of the
// served path.
#pragma once
#include <stdint.h>

#include <deque>
#include <map>
#include <vector>

#include "solve_desc.hpp"

namespace mppi {

constexpr uint64_t kAlign = 256;

inline uint64_t align_up(uint64_t x, uint64_t a = kAlign) { return (x + a - 1) / a * a; }

// First-fit allocator over offsets [0, capacity) with neighbour coalescing.
class Arena {
 public:
  explicit Arena(uint64_t capacity = 0) { reset(capacity); }
  void reset(uint64_t capacity) {
    cap_ = capacity;
    in_use_ = 0;
    peak_ = 0;
    free_.clear();
    if (capacity) free_[0] = capacity;
  }
  bool alloc(uint64_t bytes, uint64_t* offset) {
    bytes = align_up(bytes ? bytes : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const uint64_t off = it->first, rest = it->second - bytes;
        free_.erase(it);
        if (rest) free_[off + bytes] = rest;
        in_use_ += bytes;
        if (in_use_ > peak_) peak_ = in_use_;
        *offset = off;
        return true;
      }
    }
    return false;
  }
  void release(uint64_t offset, uint64_t bytes) {
    bytes = align_up(bytes ? bytes : 1);
    in_use_ -= bytes;
    auto it = free_.emplace(offset, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  uint64_t capacity() const { return cap_; }
  uint64_t in_use() const { return in_use_; }
  uint64_t peak() const { return peak_; }
  uint64_t largest_free() const {
    uint64_t m = 0;
    for (auto& kv : free_) m = kv.second > m ? kv.second : m;
    return m;
  }
  size_t fragments() const { return free_.size(); }

 private:
  uint64_t cap_ = 0, in_use_ = 0, peak_ = 0;
  std::map<uint64_t, uint64_t> free_;
};

// Instance id -> slot map with its storage sized once (open addressing,
// linear probing, a power-of-two table of at least twice the capacity), so
// lookups and inserts never allocate.
class IdTable {
 public:
  void reset(int capacity) {
    size_t n = 16;
    while (n < 2 * (size_t)(capacity > 0 ? capacity : 1)) n <<= 1;
    keys_.assign(n, 0);
    vals_.assign(n, -1);
    mask_ = n - 1;
    cap_ = capacity;
    count_ = 0;
  }
  int find(uint64_t id) const {
    for (size_t i = mix(id) & mask_;; i = (i + 1) & mask_) {
      if (vals_[i] < 0) return -1;
      if (keys_[i] == id) return vals_[i];
    }
  }
  bool contains(uint64_t id) const { return find(id) >= 0; }
  // false when the table already holds `capacity` ids (id new)
  bool insert(uint64_t id, int value) {
    size_t i = mix(id) & mask_;
    for (; vals_[i] >= 0; i = (i + 1) & mask_)
      if (keys_[i] == id) {
        vals_[i] = value;
        return true;
      }
    if (count_ >= cap_) return false;
    keys_[i] = id;
    vals_[i] = value;
    ++count_;
    return true;
  }
  int size() const { return count_; }

 private:
  // 64-bit finaliser of MurmurHash3 (public domain): spreads sequential ids
  static uint64_t mix(uint64_t x) {
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ull;
    x ^= x >> 33;
    return x;
  }
  std::vector<uint64_t> keys_;
  std::vector<int> vals_;
  size_t mask_ = 0;
  int cap_ = 0, count_ = 0;
};

// Byte layout of one solve's device block (descriptor, request data, buffers).
struct SolveLayout {
  uint64_t desc, U, Rt, base, z, los;                // request part (uploaded)
  uint64_t cfold, samples, pos, sdf, Jpart, J, wt, wn, result, partials;
  uint64_t upload_bytes, total;
};

// fused_sdf: a fused solve that exports its field values ([T][K] floats).
inline SolveLayout solve_layout(int K, int T, int G, int H, bool fused, int n_tiles, bool fused_sdf = false) {
  SolveLayout L{};
  uint64_t o = 0;
  auto take = [&](uint64_t bytes) { const uint64_t r = o; o = align_up(o + bytes); return r; };
  L.desc = take(sizeof(SolveDesc));
  L.U = take(8ull * 4 * T);
  L.Rt = take(4ull * 9 * G);
  L.base = take(4ull * 3 * G * (T + 1));
  L.z = take(4ull * G * 64);
  L.los = take(4ull * 2 * T);
  L.upload_bytes = o;
  L.cfold = take(4ull * G * H);
  L.result = take(8ull * (4 * T + 10));
  L.J = take(4ull * K);
  L.wn = take(8ull * K);
  if (!fused) {
    L.samples = take(4ull * 4 * T * K);
    L.pos = take(4ull * 3 * (T + 1) * K);
    L.sdf = take(4ull * T * K);
    L.Jpart = take(4ull * K);
    L.wt = take(8ull * K);
  } else {
    L.partials = take(8ull * (4 + 4 * T) * n_tiles);
    if (fused_sdf) L.sdf = take(4ull * T * K);
  }
  L.total = o;
  return L;
}

// FIFO queue with budget admission: the head is admitted when its footprint
// fits the free budget and an in-flight slot is free; requests never overtake
// the head (no starvation of large requests), except that a head blocked only
// by its instance being busy lets later requests of other instances pass.
// One admit() pass forms one batch; it stops once the batch holds max_work
// units of work (the first item is always taken), so that no launch grows
// without bound under a burst and a request waits for at most one bounded
// batch per stream.  Memory taken outside the queue (blocking solves, staged
// batches) is counted against the same budget through reserve().
struct AdmissionItem {
  uint64_t ticket;
  uint64_t instance_id;
  uint64_t footprint;
  uint64_t work = 0;
};

class Admission {
 public:
  Admission(uint64_t budget, int max_inflight, int queue_depth)
      : budget_(budget), max_inflight_(max_inflight), depth_(queue_depth) {}
  // 0 = queued, -3 = queue full, -2 = can never fit
  int push(const AdmissionItem& it) {
    if (it.footprint > budget_) return -2;
    if ((int)q_.size() >= depth_) return -3;
    q_.push_back(it);
    return 0;
  }
  // Pops the items admissible now, in FIFO order, given the busy instances,
  // up to max_work units of work in total (0: no limit; the first item is
  // taken whatever its work).
  template <class BusyFn>
  std::vector<AdmissionItem> admit(BusyFn instance_busy, uint64_t max_work = 0) {
    std::vector<AdmissionItem> out;
    uint64_t work = 0;
    auto taken = [&](uint64_t id) {
      for (auto& o : out) if (o.instance_id == id) return true;
      return false;
    };
    for (auto it = q_.begin(); it != q_.end();) {
      if (inflight_ >= max_inflight_) break;
      if (instance_busy(it->instance_id) || taken(it->instance_id)) { ++it; continue; }
      if (in_use_ + it->footprint > budget_) break;
      if (max_work && !out.empty() && work + it->work > max_work) break;
      in_use_ += it->footprint;
      work += it->work;
      ++inflight_;
      out.push_back(*it);
      it = q_.erase(it);
    }
    return out;
  }
  // Budget for memory held outside the queue: 0 = taken, -2 = can never fit,
  // -3 = does not fit now.
  int reserve(uint64_t bytes) {
    if (bytes > budget_) return -2;
    if (in_use_ + bytes > budget_) return -3;
    in_use_ += bytes;
    return 0;
  }
  void unreserve(uint64_t bytes) { in_use_ -= bytes; }
  void complete(uint64_t footprint) {
    in_use_ -= footprint;
    --inflight_;
  }
  // Undo admit() for items that could not be placed yet: back to the queue
  // front, in their original order.
  void requeue_front(const std::vector<AdmissionItem>& items) {
    for (auto it = items.rbegin(); it != items.rend(); ++it) {
      in_use_ -= it->footprint;
      --inflight_;
      q_.push_front(*it);
    }
  }
  size_t queued() const { return q_.size(); }
  int inflight() const { return inflight_; }
  uint64_t in_use() const { return in_use_; }
  uint64_t budget() const { return budget_; }

 private:
  uint64_t budget_;
  int max_inflight_, depth_;
  int inflight_ = 0;
  uint64_t in_use_ = 0;
  std::deque<AdmissionItem> q_;
};

}  // namespace mppi
