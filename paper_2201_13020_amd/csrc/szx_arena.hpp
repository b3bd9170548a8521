// szx_arena.hpp -- offset allocator over one device arena (host-side
// bookkeeping only; no HIP calls, so it builds and is tested without a GPU).
//
// First fit by address over a free list kept coalesced; every allocation is
// rounded up to kAlign bytes and starts on a kAlign boundary. shrink() gives
// back the tail of an allocation in place (a compressed stream is reserved at
// its worst-case size and shrunk to its real size once that is known). Not
// thread-safe: the owner serialises calls.
#pragma once

#include <stdint.h>

#include <iterator>
#include <map>

namespace szx {

class Arena {
 public:
  static constexpr uint64_t kAlign = 256;
  static constexpr uint64_t kFail = ~0ull;

  explicit Arena(uint64_t bytes = 0) { reset(bytes); }

  void reset(uint64_t bytes) {
    free_.clear();
    used_.clear();
    cap_ = bytes / kAlign * kAlign;
    in_use_ = peak_ = 0;
    if (cap_) free_[0] = cap_;
  }

  static uint64_t round(uint64_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

  // Offset of a new allocation of n bytes (n = 0 takes kAlign), or kFail.
  uint64_t alloc(uint64_t n) {
    const uint64_t need = round(n ? n : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < need) continue;
      const uint64_t off = it->first, rest = it->second - need;
      free_.erase(it);
      if (rest) free_[off + need] = rest;
      used_[off] = need;
      in_use_ += need;
      if (in_use_ > peak_) peak_ = in_use_;
      return off;
    }
    return kFail;
  }

  // Would alloc(n) succeed now?
  bool fits(uint64_t n) const {
    const uint64_t need = round(n ? n : 1);
    for (const auto& f : free_)
      if (f.second >= need) return true;
    return false;
  }

  // Keep the first n bytes of the allocation at off; false if off is unknown
  // or n exceeds its size.
  bool shrink(uint64_t off, uint64_t n) {
    auto it = used_.find(off);
    if (it == used_.end()) return false;
    const uint64_t keep = round(n ? n : 1);
    if (keep > it->second) return false;
    const uint64_t tail = it->second - keep;
    if (tail == 0) return true;
    it->second = keep;
    in_use_ -= tail;
    give_back(off + keep, tail);
    return true;
  }

  bool release(uint64_t off) {
    auto it = used_.find(off);
    if (it == used_.end()) return false;
    const uint64_t n = it->second;
    used_.erase(it);
    in_use_ -= n;
    give_back(off, n);
    return true;
  }

  uint64_t capacity() const { return cap_; }
  uint64_t in_use() const { return in_use_; }
  uint64_t peak() const { return peak_; }
  uint64_t size_of(uint64_t off) const {
    auto it = used_.find(off);
    return it == used_.end() ? 0 : it->second;
  }
  size_t free_ranges() const { return free_.size(); }
  size_t allocations() const { return used_.size(); }
  uint64_t largest_free() const {
    uint64_t m = 0;
    for (const auto& f : free_) m = f.second > m ? f.second : m;
    return m;
  }

 private:
  void give_back(uint64_t off, uint64_t n) {
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

  std::map<uint64_t, uint64_t> free_;  // offset -> bytes, coalesced
  std::map<uint64_t, uint64_t> used_;  // offset -> bytes
  uint64_t cap_ = 0, in_use_ = 0, peak_ = 0;
};

}  // namespace szx
