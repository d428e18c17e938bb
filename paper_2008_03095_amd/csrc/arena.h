// Sub-allocator over one reservation (host code only): best fit among the
// free ranges, which are merged with their neighbours when freed.  Used for
// a context's whole HBM budget, so that a serving process keeps a fixed
// footprint and never returns to the device allocator while it runs.
#pragma once

#include <cstddef>
#include <iterator>
#include <map>

namespace infuse {

struct Arena {
  char* base = nullptr;
  size_t size = 0;
  std::map<size_t, size_t> by_off;        // free ranges: offset -> size
  std::multimap<size_t, size_t> by_size;  // free ranges: size -> offset

  void reset(void* b, size_t bytes) {
    base = static_cast<char*>(b);
    size = bytes;
    by_off.clear();
    by_size.clear();
    if (bytes) {
      by_off[0] = bytes;
      by_size.emplace(bytes, 0);
    }
  }

  // The smallest free range that fits, or nullptr.
  void* take(size_t bytes) {
    auto it = by_size.lower_bound(bytes);
    if (it == by_size.end()) return nullptr;
    const size_t sz = it->first, off = it->second;
    by_size.erase(it);
    by_off.erase(off);
    if (sz > bytes) {
      by_off[off + bytes] = sz - bytes;
      by_size.emplace(sz - bytes, off + bytes);
    }
    return base + off;
  }

  // Returns [p, p + bytes) and merges it with free neighbours.
  void give(void* p, size_t bytes) {
    size_t off = static_cast<size_t>(static_cast<char*>(p) - base), sz = bytes;
    auto erase_range = [&](std::map<size_t, size_t>::iterator r) {
      auto range = by_size.equal_range(r->second);
      for (auto q = range.first; q != range.second; ++q)
        if (q->second == r->first) {
          by_size.erase(q);
          break;
        }
      return by_off.erase(r);
    };
    auto next = by_off.lower_bound(off);
    if (next != by_off.end() && next->first == off + sz) {
      sz += next->second;
      next = erase_range(next);
    }
    if (next != by_off.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        off = prev->first;
        sz += prev->second;
        erase_range(prev);
      }
    }
    by_off[off] = sz;
    by_size.emplace(sz, off);
  }

  size_t free_bytes() const {
    size_t t = 0;
    for (const auto& r : by_off) t += r.second;
    return t;
  }
};

}  // namespace infuse
