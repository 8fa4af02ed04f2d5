// Host-side first-fit allocator over a caller-owned device pool, used by the serving scheduler to
// place each admitted request's resident state.  Pure C++ (no HIP), so that it can be exercised
// on its own, also under the address and undefined-behaviour sanitizers.
#pragma once

#include <cstddef>
#include <iterator>
#include <map>

namespace fm {
namespace cx {

// Offsets into [0, size): alloc(n) returns the lowest offset of a free range of at least n bytes
// (first fit); release(off, n) returns a range and merges it with free neighbours, so that
// releasing everything leaves one range [0, size).  The caller passes back exactly what alloc
// handed out; ranges are not checked for overlap.
class PoolAlloc {
 public:
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
  }
  bool alloc(size_t n, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n;
        const size_t at = it->first + n;
        free_.erase(it);
        if (rest) free_[at] = rest;
        return true;
      }
    return false;
  }
  void release(size_t off, size_t n) {
    auto it = free_.emplace(off, n).first;
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

 private:
  std::map<size_t, size_t> free_;
};

}  // namespace cx
}  // namespace fm
