// First-fit range allocator over a fixed byte range (the server's device
// arena and its pinned host pool).  Pure C++: no HIP, so its behaviour can be
// checked on a machine without a GPU.
#pragma once

#include <stdint.h>

#include <iterator>
#include <map>

namespace jefi {

class Arena {
 public:
  Arena() = default;
  explicit Arena(uint64_t size) { reset(size); }

  void reset(uint64_t size) {
    free_.clear();
    size_ = size;
    used_ = 0;
    high_ = 0;
    if (size > 0) free_[0] = size;
  }

  // Allocation granule; every block is a multiple of it and aligned to it.
  static constexpr uint64_t kGranule = 256;

  static uint64_t round_up(uint64_t bytes) { return (bytes + kGranule - 1) / kGranule * kGranule; }

  // First fit.  Returns false (and changes nothing) when no free block holds
  // round_up(bytes).  A zero-byte request gets one granule.
  bool alloc(uint64_t bytes, uint64_t* off) {
    const uint64_t need = round_up(bytes == 0 ? 1 : bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= need) {
        const uint64_t at = it->first;
        const uint64_t rest = it->second - need;
        free_.erase(it);
        if (rest > 0) free_[at + need] = rest;
        used_ += need;
        if (used_ > high_) high_ = used_;
        *off = at;
        return true;
      }
    }
    return false;
  }

  // Return a block obtained from alloc() with the same byte count.
  void release(uint64_t off, uint64_t bytes) {
    uint64_t need = round_up(bytes == 0 ? 1 : bytes);
    used_ -= need;
    auto next = free_.lower_bound(off);
    // merge with the following block
    if (next != free_.end() && off + need == next->first) {
      need += next->second;
      next = free_.erase(next);
    }
    // merge with the preceding block
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += need;
        return;
      }
    }
    free_[off] = need;
  }

  // True when a block of `bytes` could be allocated right now.
  bool fits(uint64_t bytes) const { return largest_free() >= round_up(bytes == 0 ? 1 : bytes); }

  uint64_t largest_free() const {
    uint64_t m = 0;
    for (auto& kv : free_)
      if (kv.second > m) m = kv.second;
    return m;
  }

  uint64_t size() const { return size_; }
  uint64_t used() const { return used_; }
  uint64_t high_water() const { return high_; }
  size_t free_blocks() const { return free_.size(); }

 private:
  std::map<uint64_t, uint64_t> free_;  // offset -> length, non-adjacent blocks
  uint64_t size_ = 0, used_ = 0, high_ = 0;
};

}  // namespace jefi
