// Device-memory arena of the request server: first-fit allocation of byte
// ranges of [0, size) from address-ordered free ranges, coalesced on
// release.  Pure host code (offsets only), not thread-safe.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <iterator>
#include <map>

namespace ffp {

class Arena {
 public:
  void init(uint64_t size) {
    size_ = size;
    free_.clear();
    if (size) free_[0] = size;
  }
  bool alloc(uint64_t n, uint64_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      *off = it->first;
      const uint64_t rest = it->second - n, start = it->first + n;
      free_.erase(it);
      if (rest) free_[start] = rest;
      used_ += n;
      peak_ = std::max(peak_, used_);
      return true;
    }
    return false;
  }
  void release(uint64_t off, uint64_t n) {
    used_ -= n;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + n == next->first) {
      n += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += n;
        return;
      }
    }
    free_[off] = n;
  }
  uint64_t size() const { return size_; }
  uint64_t used() const { return used_; }
  uint64_t peak() const { return peak_; }
  const std::map<uint64_t, uint64_t>& free_ranges() const { return free_; }

 private:
  uint64_t size_ = 0, used_ = 0, peak_ = 0;
  std::map<uint64_t, uint64_t> free_;  // offset -> length
};

}  // namespace ffp
