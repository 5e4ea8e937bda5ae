// serve.hpp -- pieces of the request server that are plain host code: the
// pool allocator behind its HBM budget and the backend interface.
#pragma once

#include <cstddef>
#include <cstdint>
#include <map>

namespace fftpde {

// First-fit allocator over one contiguous region [0, size): offsets aligned
// to 256 bytes, neighbouring free blocks merged on free.
class Pool {
 public:
  static constexpr size_t kAlign = 256;
  static constexpr size_t kNone = SIZE_MAX;

  void reset(size_t size) {
    free_.clear();
    used_.clear();
    size_ = size / kAlign * kAlign;
    if (size_) free_[0] = size_;
  }
  size_t size() const { return size_; }

  // offset of a block of at least n bytes, or kNone
  size_t alloc(size_t n) {
    n = (n + kAlign - 1) / kAlign * kAlign;
    if (n == 0) n = kAlign;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      const size_t off = it->first, len = it->second;
      free_.erase(it);
      if (len > n) free_[off + n] = len - n;
      used_[off] = n;
      return off;
    }
    return kNone;
  }

  // false if off is not a live block
  bool release(size_t off) {
    auto u = used_.find(off);
    if (u == used_.end()) return false;
    size_t start = off, len = u->second;
    used_.erase(u);
    auto next = free_.lower_bound(start);
    if (next != free_.end() && next->first == start + len) {
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == start) {
        start = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    free_[start] = len;
    return true;
  }

  size_t largest_free() const {
    size_t m = 0;
    for (auto& f : free_) m = f.second > m ? f.second : m;
    return m;
  }
  size_t blocks_in_use() const { return used_.size(); }

 private:
  std::map<size_t, size_t> free_;  // offset -> length
  std::map<size_t, size_t> used_;
  size_t size_ = 0;
};

}  // namespace fftpde
