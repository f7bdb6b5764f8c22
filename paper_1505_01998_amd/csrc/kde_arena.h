// kde_arena.h -- first-fit allocator of byte ranges inside one reserved
// device allocation (the server's HBM budget).  Host-only bookkeeping: the
// arena hands out offsets; the caller adds them to its base address.
// Ranges are multiples of kAlign bytes; freed ranges merge with free
// neighbours, so a drained arena is one free range again.
#pragma once

#include <stdint.h>

#include <iterator>
#include <map>

namespace kde {

class Arena {
 public:
  static constexpr uint64_t kAlign = 256;

  explicit Arena(uint64_t bytes = 0) { reset(bytes); }

  void reset(uint64_t bytes) {
    free_.clear();
    used_.clear();
    size_ = bytes / kAlign * kAlign;
    if (size_) free_[0] = size_;
    in_use_ = 0;
  }

  // Offset of a range of at least `bytes`, or -1 when no free range is large
  // enough (the lowest-offset range that fits is taken).
  int64_t alloc(uint64_t bytes) {
    const uint64_t want = round(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < want) continue;
      const uint64_t off = it->first, len = it->second;
      free_.erase(it);
      if (len > want) free_[off + want] = len - want;
      used_[off] = want;
      in_use_ += want;
      return (int64_t)off;
    }
    return -1;
  }

  // Returns a range given by alloc; false for an offset alloc did not give.
  bool release(int64_t off) {
    auto u = used_.find((uint64_t)off);
    if (off < 0 || u == used_.end()) return false;
    uint64_t start = u->first, len = u->second;
    in_use_ -= len;
    used_.erase(u);
    auto next = free_.lower_bound(start);
    if (next != free_.end() && next->first == start + len) {
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == start) {
        prev->second += len;
        return true;
      }
    }
    free_[start] = len;
    return true;
  }

  static uint64_t round(uint64_t bytes) { return (bytes + kAlign - 1) / kAlign * kAlign + (bytes == 0 ? kAlign : 0); }
  uint64_t size() const { return size_; }
  uint64_t in_use() const { return in_use_; }
  uint64_t largest_free() const {
    uint64_t m = 0;
    for (const auto& f : free_) m = f.second > m ? f.second : m;
    return m;
  }
  size_t free_ranges() const { return free_.size(); }
  size_t used_ranges() const { return used_.size(); }

 private:
  std::map<uint64_t, uint64_t> free_, used_;  // offset -> length
  uint64_t size_ = 0, in_use_ = 0;
};

}  // namespace kde
