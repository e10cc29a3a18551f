// arena.hpp -- first-fit placement of the serving loop's outputs.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <map>
#include <utility>
#include <vector>

namespace ec {

// First-fit allocator over [0, size) whose free ranges are coalesced; sizes
// are rounded up to `align`.  Free ranges are kept by their end offset, so
// that taking space from the front of a range, and growing a range at
// either side, change it in place (or re-key its node) without allocating:
// a serving loop allocates and releases an output per request.
class FirstFit {
 public:
  FirstFit(size_t size, size_t align) : align_(align) {
    if (size) free_[size] = 0;
  }
  // Offset of n bytes rounded up to the alignment (the rounded size in
  // *got), or SIZE_MAX when no free range holds them.
  size_t alloc(size_t n, size_t *got) {
    n = (n + align_ - 1) / align_ * align_;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      const size_t start = it->second, end = it->first;
      if (end - start < n) continue;
      if (end - start == n) free_.erase(it);
      else it->second = start + n;
      *got = n;
      return start;
    }
    return SIZE_MAX;
  }
  // Returns [off, off + n), as given by alloc, to the free ranges.
  void release(size_t off, size_t n) {
    const size_t end = off + n;
    auto prev = free_.find(off);         // the free range ending where this one starts
    auto next = free_.upper_bound(end);  // the first free range ending after this one
    const bool join_next = next != free_.end() && next->second == end;
    if (prev != free_.end() && join_next) {
      next->second = prev->second;
      free_.erase(prev);
    } else if (prev != free_.end()) {
      auto node = free_.extract(prev);  // the range now ends at `end`: re-key its node
      node.key() = end;
      free_.insert(std::move(node));
    } else if (join_next) {
      next->second = off;
    } else {
      free_[end] = off;
    }
  }
  // The free ranges as (offset, length), in address order.
  std::vector<std::pair<size_t, size_t>> free_ranges() const {
    std::vector<std::pair<size_t, size_t>> out;
    for (const auto &r : free_) out.push_back({r.second, r.first - r.second});
    return out;
  }

 private:
  size_t align_;
  std::map<size_t, size_t> free_;  // end offset -> start offset
};

}  // namespace ec
