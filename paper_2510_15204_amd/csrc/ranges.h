// First-fit map of the free ranges of one device-memory chunk, coalesced on release (the context's
// device pool hands out slot arenas as such ranges).  Host-only bookkeeping: no device calls.
#pragma once
#include <cstddef>
#include <iterator>
#include <map>

namespace psint {

class RangeMap {
 public:
  explicit RangeMap(size_t size = 0) : size_(size) {
    if (size) free_[0] = size;
  }
  size_t size() const { return size_; }
  // Take `bytes` from the lowest free range that holds them; false if none does.
  bool take(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t o = it->first, len = it->second;
      free_.erase(it);
      if (len > bytes) free_[o + bytes] = len - bytes;
      *off = o;
      return true;
    }
    return false;
  }
  // Give back [off, off + len) (taken before), merged with the free ranges next to it.
  void give(size_t off, size_t len) {
    auto next = free_.lower_bound(off);
    if (next != free_.end() && next->first == off + len) {
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        off = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    free_[off] = len;
  }
  // Nothing taken.
  bool unused() const { return free_.size() == 1 && free_.begin()->first == 0 && free_.begin()->second == size_; }
  const std::map<size_t, size_t>& free_ranges() const { return free_; }

 private:
  size_t size_;
  std::map<size_t, size_t> free_;  // offset -> length
};

}  // namespace psint
