// arena.hpp -- first-fit placement of the serving loop's outputs.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <iterator>
#include <map>

namespace ec {

// First-fit allocator over [0, size) whose free ranges are coalesced; sizes
// are rounded up to `align`.
class FirstFit {
 public:
  FirstFit(size_t size, size_t align) : align_(align) {
    if (size) free_[0] = size;
  }
  // Offset of n bytes rounded up to the alignment (the rounded size in
  // *got), or SIZE_MAX when no free range holds them.
  size_t alloc(size_t n, size_t *got) {
    n = (n + align_ - 1) / align_ * align_;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      const size_t off = it->first, len = it->second;
      free_.erase(it);
      if (len > n) free_[off + n] = len - n;
      *got = n;
      return off;
    }
    return SIZE_MAX;
  }
  // Returns [off, off + n), as given by alloc, to the free ranges.
  void release(size_t off, size_t n) {
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
  const std::map<size_t, size_t> &free_ranges() const { return free_; }

 private:
  size_t align_;
  std::map<size_t, size_t> free_;  // offset -> length
};

}  // namespace ec
