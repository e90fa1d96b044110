// First-fit bookkeeping of one contiguous block: the gaps as (offset -> length), kept sorted
// and merged with their neighbours on release.  No device code and no locking: the arena
// allocator wraps it in a mutex; a host-only test drives it under the address, undefined-
// behaviour and thread sanitizers.
#pragma once

#include <cstddef>
#include <iterator>
#include <map>

namespace rsv {

class FirstFit {
 public:
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
    size_ = size;
    used_ = 0;
  }
  // Takes `bytes` from the first gap that holds them; false if none does.
  bool take(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t o = it->first, len = it->second;
      free_.erase(it);
      if (len > bytes) free_[o + bytes] = len - bytes;
      used_ += bytes;
      *off = o;
      return true;
    }
    return false;
  }
  // Returns [off, off + bytes) (taken earlier) and merges it with adjacent gaps.
  void give(size_t off, size_t bytes) {
    used_ -= bytes;
    size_t len = bytes;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + len == next->first) {  // merge with the following gap
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {  // merge with the preceding gap
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += len;
        return;
      }
    }
    free_[off] = len;
  }
  size_t used() const { return used_; }
  size_t size() const { return size_; }
  const std::map<size_t, size_t>& gaps() const { return free_; }

 private:
  std::map<size_t, size_t> free_;
  size_t size_ = 0, used_ = 0;
};

}  // namespace rsv
