// Sub-allocation of a server's output arena (the caller's HBM budget): best
// fit over the free blocks, which are kept by offset (to coalesce a released
// block with its neighbours) and by size (to find the smallest block that
// fits), so an allocation or a release is logarithmic in the free blocks.
// Plain host code: the arena is only offsets here, never dereferenced.
#pragma once

#include <algorithm>
#include <cstdint>
#include <map>
#include <set>
#include <utility>

namespace ranmar {

class ArenaAlloc {
 public:
  explicit ArenaAlloc(uint64_t bytes = 0) { reset(bytes); }

  void reset(uint64_t bytes) {
    free_off_.clear();
    free_size_.clear();
    in_use_ = peak_ = 0;
    if (bytes) add(0, bytes);
  }

  // The offset of `bytes` free bytes (the smallest free block that holds
  // them, its start), or false if no free block does.  bytes > 0.
  bool alloc(uint64_t bytes, uint64_t* off) {
    const auto b = free_size_.lower_bound({bytes, 0});
    if (b == free_size_.end()) return false;
    const uint64_t size = b->first, at = b->second;
    free_size_.erase(b);
    free_off_.erase(at);
    if (size > bytes) add(at + bytes, size - bytes);
    *off = at;
    in_use_ += bytes;
    peak_ = std::max(peak_, in_use_);
    return true;
  }

  // Returns [off, off + bytes), which alloc handed out, merging it with free
  // neighbours.  bytes == 0 does nothing.
  void release(uint64_t off, uint64_t bytes) {
    if (!bytes) return;
    in_use_ -= bytes;
    auto nx = free_off_.lower_bound(off);
    if (nx != free_off_.end() && off + bytes == nx->first) {
      bytes += nx->second;
      drop(nx++);
    }
    if (nx != free_off_.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == off) {
        off = pv->first;
        bytes += pv->second;
        drop(pv);
      }
    }
    add(off, bytes);
  }

  uint64_t in_use() const { return in_use_; }
  uint64_t peak() const { return peak_; }
  size_t free_blocks() const { return free_off_.size(); }
  const std::map<uint64_t, uint64_t>& free_by_offset() const { return free_off_; }

 private:
  void add(uint64_t off, uint64_t bytes) {
    free_off_.emplace(off, bytes);
    free_size_.emplace(bytes, off);
  }
  void drop(std::map<uint64_t, uint64_t>::iterator it) {
    free_size_.erase({it->second, it->first});
    free_off_.erase(it);
  }

  std::map<uint64_t, uint64_t> free_off_;           // offset -> size
  std::set<std::pair<uint64_t, uint64_t>> free_size_;  // (size, offset)
  uint64_t in_use_ = 0, peak_ = 0;
};

}  // namespace ranmar
