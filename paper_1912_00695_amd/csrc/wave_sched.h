// wave_sched.h -- host-only scheduling logic of the serving engine: the device
// pool's first-fit allocator, the admission policy and the latency percentiles.
// Plain C++ (no HIP), so the same code the engine runs is also exercised by a
// host-only self-test.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <iterator>
#include <map>
#include <vector>

namespace wave {
namespace sched {

constexpr size_t kGranule = 256;
inline size_t round_up(size_t v) { return (v + kGranule - 1) / kGranule * kGranule; }

// First-fit allocator over [0, size) with 256-byte granularity; freed blocks
// coalesce with their neighbours.
class PoolAlloc {
 public:
  explicit PoolAlloc(size_t size) {
    if (size >= kGranule) free_[0] = size / kGranule * kGranule;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = round_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes, base = it->first + bytes;
        free_.erase(it);
        if (rest) free_[base] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = round_up(bytes);
    auto it = free_.emplace(off, bytes).first;
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
  size_t free_bytes() const {
    size_t s = 0;
    for (auto& kv : free_) s += kv.second;
    return s;
  }
  size_t largest_free() const {
    size_t m = 0;
    for (auto& kv : free_) m = std::max(m, kv.second);
    return m;
  }
  size_t blocks() const { return free_.size(); }

 private:
  std::map<size_t, size_t> free_;  // offset -> length
};

// Admission: walk the queue in arrival order and admit every request for which
// a slot is free and the pool has room, so a request that does not fit does not
// block later ones that do (first-come first-served with skip-ahead). Returns
// the admitted queue positions and their pool offsets; allocations are made in
// `pool`.
struct Admission {
  size_t pos;
  size_t off;
};
inline std::vector<Admission> admit(const std::vector<size_t>& queued_bytes, PoolAlloc& pool,
                                    int free_slots) {
  std::vector<Admission> out;
  for (size_t i = 0; i < queued_bytes.size() && free_slots > 0; ++i) {
    size_t off = 0;
    if (pool.alloc(queued_bytes[i], &off)) {
      out.push_back({i, off});
      --free_slots;
    }
  }
  return out;
}

// Nearest-rank percentile q in (0, 1] of a sample (the smallest value with at
// least q of the sample at or below it); 0 for an empty sample.
inline double percentile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  size_t k = (size_t)std::ceil(q * (double)v.size());
  k = std::min(v.size(), std::max<size_t>(k, 1));
  return v[k - 1];
}

}  // namespace sched
}  // namespace wave
