// First-fit sub-allocator over the byte range [0, size), used by the serving loop for its
// device arena (the HBM budget) and its pinned host staging arena.  Sizes are rounded up to
// 256 bytes, so every offset handed out is 256-byte aligned; released ranges are merged with
// free neighbours, so a run of frees restores one free range.  Plain C++ (no HIP), not
// thread-safe: the serving loop calls it under its own lock.
#pragma once

#include <cstddef>
#include <iterator>
#include <map>

namespace snf {

class Arena {
 public:
  static constexpr size_t kAlign = 256;

  void init(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
  }
  // First free range (lowest offset) that holds the rounded size; false if none does.
  bool alloc(size_t bytes, size_t* off) {
    bytes = round(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes, start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        return true;
      }
    }
    return false;
  }
  // Return [off, off + bytes) (bytes as passed to alloc).
  void release(size_t off, size_t bytes) {
    bytes = round(bytes);
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
  // Free ranges (offset, length) in offset order.
  const std::map<size_t, size_t>& free_ranges() const { return free_; }

 private:
  static size_t round(size_t b) { return (b + kAlign - 1) & ~(kAlign - 1); }
  std::map<size_t, size_t> free_;
};

}  // namespace snf
