// First-fit range allocator over one pre-allocated region (host-only C++, no HIP).
//
// The request server carves every request's device memory (input, scratch, results) and
// pinned host memory (staged input, unread results) out of two regions allocated once, so
// serving never calls the HIP allocator. Free ranges are kept by offset and merged with
// their neighbours on release; allocation takes the lowest-offset range that fits.
#pragma once
#include <cstddef>
#include <iterator>
#include <map>

namespace tmfg {

class RangeAllocator {
 public:
  RangeAllocator() = default;
  RangeAllocator(size_t capacity, size_t align) { reset(capacity, align); }

  void reset(size_t capacity, size_t align) {
    align_ = align ? align : 1;
    capacity_ = capacity / align_ * align_;
    free_.clear();
    if (capacity_) free_[0] = capacity_;
    used_ = 0;
  }

  size_t round(size_t bytes) const { return (bytes + align_ - 1) / align_ * align_; }
  size_t capacity() const { return capacity_; }
  size_t used() const { return used_; }
  size_t ranges() const { return free_.size(); }

  // Offset of a new range of `bytes` (rounded up to the alignment), or false if none fits.
  bool alloc(size_t bytes, size_t* offset) {
    const size_t need = round(bytes ? bytes : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < need) continue;
      *offset = it->first;
      const size_t rest = it->second - need, at = it->first + need;
      free_.erase(it);
      if (rest) free_[at] = rest;
      used_ += need;
      return true;
    }
    return false;
  }

  // Returns a range from alloc (same offset and byte count).
  void release(size_t offset, size_t bytes) {
    size_t size = round(bytes ? bytes : 1);
    used_ -= size;
    auto next = free_.lower_bound(offset);
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == offset) {
        offset = prev->first;
        size += prev->second;
        free_.erase(prev);
      }
    }
    if (next != free_.end() && offset + size == next->first) {
      size += next->second;
      free_.erase(next);
    }
    free_[offset] = size;
  }

  // Largest range alloc could return now.
  size_t largest() const {
    size_t m = 0;
    for (const auto& kv : free_) m = kv.second > m ? kv.second : m;
    return m;
  }

 private:
  size_t align_ = 1, capacity_ = 0, used_ = 0;
  std::map<size_t, size_t> free_;   // offset -> bytes
};

}  // namespace tmfg
