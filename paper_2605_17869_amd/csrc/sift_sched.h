// Host-side scheduling pieces of the serving front end: the first-fit arena
// allocator and the arrival-order batch former with admission by footprint.
// Plain C++ (no HIP): the server uses them under its mutex, and a CPU test
// drives them against a simulated device.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <iterator>
#include <map>

#include "sift_internal.h"

namespace sift {

constexpr int64_t kArenaAlign = 256;

inline int64_t align_up256(int64_t v) { return (v + kArenaAlign - 1) / kArenaAlign * kArenaAlign; }

// First-fit allocator over [0, size); ranges are multiples of 256 bytes and
// free neighbours coalesce, so an idle arena is one free range again.
class Arena {
 public:
  void reset(int64_t size) {
    free_.clear();
    size_ = size / kArenaAlign * kArenaAlign;
    if (size_ > 0) free_[0] = size_;
  }
  int64_t size() const { return size_; }
  int64_t largest() const {
    int64_t m = 0;
    for (const auto& f : free_) m = std::max(m, f.second);
    return m;
  }
  int64_t free_bytes() const {
    int64_t t = 0;
    for (const auto& f : free_) t += f.second;
    return t;
  }
  // Offset of a range of `bytes` (rounded up to 256), or -1 if none fits.
  int64_t take(int64_t bytes) {
    bytes = align_up256(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const int64_t off = it->first, rest = it->second - bytes;
        free_.erase(it);
        if (rest > 0) free_[off + bytes] = rest;
        return off;
      }
    }
    return -1;
  }
  // Returns a range obtained from take(bytes).
  void give(int64_t off, int64_t bytes) {
    bytes = align_up256(bytes);
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  int64_t size_ = 0;
  std::map<int64_t, int64_t> free_;
};

inline int64_t header_bytes(int n) {
  Header hd;
  make_header(n, &hd);
  return hd.bytes;
}

// Workspace bytes that cover a batch of n images whose regions sum to
// `regions`, however the batched call splits it: at most min(n, kMaxParts)
// sub-batches, each with a header no larger than the whole batch's.
inline int64_t batch_bytes(int n, int64_t regions) {
  return align_up256((int64_t)std::min(n, kMaxParts) * header_bytes(n) + regions);
}

// The next batch from the head of `pending` (a sequence of requests with a
// `region` member, in arrival order): the longest prefix of at most max_batch
// requests whose batch bytes fit in `room`.  Returns its length (0: the head
// waits for space) and its bytes in *bytes.
template <class Seq>
int next_batch(const Seq& pending, int max_batch, int64_t room, int64_t* bytes) {
  int n = 0;
  int64_t regions = 0;
  while (n < (int)pending.size() && n < max_batch) {
    const int64_t need = batch_bytes(n + 1, regions + pending[n].region);
    if (need > room) break;
    regions += pending[n].region;
    ++n;
  }
  *bytes = n ? batch_bytes(n, regions) : 0;
  return n;
}

}  // namespace sift
