// vegas_sched.hpp — host-side building blocks of the serving loop, with no
// HIP calls so that they are testable on any CPU:
//   Arena       first-fit allocator of byte ranges inside one device
//               allocation (the server's memory budget)
//   Admission   FIFO admission of requests by free slot and free arena bytes
//   chunk_events  the event-chunk size of an integral (a function of its
//               event count only, so an integral is cut the same way alone
//               and in a mix)
//   pick_lane   the stream (lane) a newly admitted integral joins
//   chain_ticks how many ticks a lane runs before returning to the host
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <deque>
#include <iterator>
#include <map>
#include <tuple>
#include <vector>

namespace vegas {

class Arena {
 public:
  explicit Arena(size_t bytes = 0, size_t align = 256) : size_(bytes), align_(align) {
    if (bytes) free_[0] = bytes;
  }
  size_t size() const { return size_; }
  size_t used() const { return used_; }
  // Offset of a free range of `bytes` (rounded up to the alignment), or
  // SIZE_MAX if none is large enough.
  size_t alloc(size_t bytes) {
    const size_t need = round(bytes);
    if (need == 0 || need > size_) return SIZE_MAX;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= need) {
        const size_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > need) free_[off + need] = len - need;
        live_[off] = need;
        used_ += need;
        return off;
      }
    }
    return SIZE_MAX;
  }
  // Release a range returned by alloc; false if `off` is not a live range.
  bool release(size_t off) {
    auto it = live_.find(off);
    if (it == live_.end()) return false;
    size_t len = it->second;
    live_.erase(it);
    used_ -= len;
    size_t start = off;
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && nx->first == off + len) {
      len += nx->second;
      nx = free_.erase(nx);
    }
    if (nx != free_.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == start) {
        start = pv->first;
        len += pv->second;
        free_.erase(pv);
      }
    }
    free_[start] = len;
    return true;
  }
  size_t largest_free() const {
    size_t m = 0;
    for (const auto& kv : free_) m = std::max(m, kv.second);
    return m;
  }
  size_t live_ranges() const { return live_.size(); }

 private:
  size_t round(size_t b) const { return (b + align_ - 1) / align_ * align_; }
  size_t size_, align_;
  size_t used_ = 0;
  std::map<size_t, size_t> free_;  // offset -> length, coalesced
  std::map<size_t, size_t> live_;  // offset -> length
};

// Strict FIFO admission: the head of the queue is admitted when a slot is
// free and the arena has room for it; later requests wait behind it (no
// overtaking, so no request starves).
template <class Req>
class Admission {
 public:
  Admission(int max_slots, Arena* arena) : arena_(arena) {
    for (int i = max_slots - 1; i >= 0; --i) free_slots_.push_back(i);
  }
  void push(Req r) { queue_.push_back(r); }
  size_t pending() const { return queue_.size(); }
  size_t free_slots() const { return free_slots_.size(); }
  // Admit as many queued requests as fit; bytes_of(req) gives the device
  // bytes of a request. Returns (request, slot, arena offset) triples.
  template <class BytesOf>
  std::vector<std::tuple<Req, int, size_t>> admit(BytesOf bytes_of) {
    std::vector<std::tuple<Req, int, size_t>> out;
    while (!queue_.empty() && !free_slots_.empty()) {
      const size_t off = arena_->alloc(bytes_of(queue_.front()));
      if (off == SIZE_MAX) break;
      const int slot = free_slots_.back();
      free_slots_.pop_back();
      out.emplace_back(queue_.front(), slot, off);
      queue_.pop_front();
    }
    return out;
  }
  void finish(int slot, size_t off) {
    arena_->release(off);
    free_slots_.push_back(slot);
  }

 private:
  Arena* arena_;
  std::deque<Req> queue_;
  std::vector<int> free_slots_;
};

// Events per chunk for an integral of n events per iteration: about n/512,
// a multiple of 256 (one event per thread of a 256-thread workgroup), between
// 256 and 262144 (or `fixed` when non-zero). A chunk is one workgroup, which
// holds one wave per SIMD, so its events run latency-bound: small chunks
// spread an integral over more CUs and shorten its iteration. Measured on
// the serving trace at 200 requests/s, median latency of integrals below
// 1e5 events: 0.199 ms with chunks of at least 2048 events, 0.131 ms with
// 256; from 1e5 to 1e6 events: 0.222 and 0.171 ms (512).
inline int64_t chunk_events(int64_t n, int64_t fixed) {
  if (fixed > 0) return fixed;
  int64_t c = (n + 511) / 512;
  c = (c + 255) / 256 * 256;
  return std::min<int64_t>(std::max<int64_t>(c, 256), 262144);
}

// The lane a newly admitted integral joins, of n lanes with busy[i] (a chain
// in flight) and members[i] (integrals assigned): the first idle lane
// without integrals, where it starts at once; else the lane holding the
// fewest integrals (the first of equals), whose next chain it joins.
inline int pick_lane(int n, const bool* busy, const size_t* members) {
  int best = 0;
  for (int i = 1; i < n; ++i) {
    const bool free_i = !busy[i] && members[i] == 0;
    const bool free_b = !busy[best] && members[best] == 0;
    if ((free_i && !free_b) || (free_i == free_b && members[i] < members[best])) best = i;
  }
  return best;
}

// Ticks of a lane's next chain: up to the first completion among its
// integrals (remaining[i] iterations left, events[i] per iteration), at most
// max_ticks, and at most max_events events in all unless one tick alone
// carries more; at least 1.
inline int chain_ticks(int n, const int* remaining, const int64_t* events, int max_ticks,
                       int64_t max_events) {
  int K = max_ticks;
  int64_t tick_events = 0;
  for (int i = 0; i < n; ++i) {
    K = std::min(K, remaining[i]);
    tick_events += events[i];
  }
  while (K > 1 && (int64_t)K * tick_events > max_events) --K;
  return std::max(K, 1);
}

}  // namespace vegas
