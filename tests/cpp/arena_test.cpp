// Randomised test of the budget arena (host code): allocations never
// overlap and stay inside the reservation, freed ranges merge so that the
// whole reservation is one range again when everything is freed, and best
// fit reuses the smallest range that fits.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <vector>

#include "arena.h"

#define CHECK(c)                                                  \
  do {                                                            \
    if (!(c)) {                                                   \
      std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
      return 1;                                                   \
    }                                                             \
  } while (0)

int main() {
  const size_t total = 1 << 20;
  std::vector<char> mem(total);
  infuse::Arena a;
  a.reset(mem.data(), total);
  CHECK(a.free_bytes() == total && a.by_off.size() == 1);

  // best fit: free ranges of 4096 and 1024 bytes, a 1000-byte request takes the 1024 one
  void* x = a.take(4096);
  void* y = a.take(256);
  void* z = a.take(1024);
  void* w = a.take(256);
  CHECK(x && y && z && w);
  a.give(x, 4096);
  a.give(z, 1024);
  void* t = a.take(1000);
  CHECK(t == z);
  a.give(t, 1000);
  a.give(y, 256);
  a.give(w, 256);
  // z's range came back as 1000 + the 24-byte tail merged in again: one range
  CHECK(a.by_off.size() == 1 && a.free_bytes() == total);

  std::mt19937_64 rng(7);
  std::map<size_t, size_t> live;  // offset -> bytes
  size_t used = 0;
  for (int it = 0; it < 200000; ++it) {
    const bool alloc = live.empty() || (rng() % 100) < 55;
    if (alloc) {
      const size_t bytes = 256 * (1 + rng() % 64);
      void* p = a.take(bytes);
      if (!p) {
        CHECK(a.free_bytes() == total - used);  // fragmentation only, no leak
        continue;
      }
      const size_t off = static_cast<size_t>(static_cast<char*>(p) - mem.data());
      CHECK(off + bytes <= total);
      auto nx = live.lower_bound(off);
      if (nx != live.end()) CHECK(off + bytes <= nx->first);
      if (nx != live.begin()) {
        auto pv = std::prev(nx);
        CHECK(pv->first + pv->second <= off);
      }
      live[off] = bytes;
      used += bytes;
    } else {
      auto victim = live.begin();
      std::advance(victim, rng() % live.size());
      a.give(mem.data() + victim->first, victim->second);
      used -= victim->second;
      live.erase(victim);
    }
    // the free ranges never touch each other (they would have been merged)
    if (it % 997 == 0) {
      size_t prev_end = SIZE_MAX;
      for (const auto& r : a.by_off) {
        CHECK(r.first != prev_end);
        prev_end = r.first + r.second;
      }
      CHECK(a.by_off.size() == a.by_size.size());
      CHECK(a.free_bytes() == total - used);
    }
  }
  for (const auto& r : live) a.give(mem.data() + r.first, r.second);
  CHECK(a.by_off.size() == 1 && a.free_bytes() == total);
  std::printf("arena ok\n");
  return 0;
}
