// Host-side buddy allocator for the server's device arena (plain C++; no
// device code).
#pragma once

#include <algorithm>
#include <cstdint>
#include <set>
#include <utility>
#include <vector>

namespace gx {

// Buddy allocator over [0, size): the range is cut into power-of-two top
// blocks, largest first (each at an offset that is a multiple of its size),
// and every allocation is a power-of-two block of at least 4 KiB, split
// from the smallest free block that holds it; a freed block merges with its
// free buddy up to its top block.
class Buddy {
 public:
  static constexpr int kMinShift = 12;  // 4 KiB
  void init(uint64_t size) {
    free_.assign(64, {});
    tops_.clear();
    uint64_t off = 0;
    for (int o = 63 - kMinShift; o >= 0; --o) {
      const uint64_t b = uint64_t(1) << (o + kMinShift);
      if (size - off >= b) {
        tops_.push_back({off, o});
        free_[o].insert(off);
        off += b;
      }
    }
  }
  uint64_t largest() const {
    return tops_.empty() ? 0 : uint64_t(1) << (tops_.front().second + kMinShift);
  }
  // offset of a block of at least n bytes, or ~0 when none is free
  uint64_t alloc(uint64_t n) {
    const int o = order(n);
    int k = o;
    while (k < 64 && free_[k].empty()) ++k;
    if (k >= 64) return ~0ull;
    const uint64_t off = *free_[k].begin();
    free_[k].erase(free_[k].begin());
    while (k > o) {
      --k;
      free_[k].insert(off + (uint64_t(1) << (k + kMinShift)));
    }
    return off;
  }
  void release(uint64_t off, uint64_t n) {
    int o = order(n);
    const int top = top_order(off);
    while (o < top) {
      const uint64_t buddy = off ^ (uint64_t(1) << (o + kMinShift));
      auto it = free_[o].find(buddy);
      if (it == free_[o].end()) break;
      free_[o].erase(it);
      off = std::min(off, buddy);
      ++o;
    }
    free_[o].insert(off);
  }
  static uint64_t block_bytes(uint64_t n) { return uint64_t(1) << (order(n) + kMinShift); }

 private:
  static int order(uint64_t n) {
    int o = 0;
    while ((uint64_t(1) << (o + kMinShift)) < n) ++o;
    return o;
  }
  int top_order(uint64_t off) const {
    for (const auto& t : tops_)
      if (off >= t.first && off < t.first + (uint64_t(1) << (t.second + kMinShift)))
        return t.second;
    return 0;
  }
  std::vector<std::set<uint64_t>> free_;
  std::vector<std::pair<uint64_t, int>> tops_;  // offset, order
};

}  // namespace gx
