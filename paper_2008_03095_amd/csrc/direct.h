// Launchers of the memo-free sigma kernels (direct.hip).
#pragma once

#include "common.h"

namespace infuse {

// Several searches can run side by side as copies of the graph: virtual
// vertex c * gn + v is vertex v of copy c (gn = the graph's n); n counts the
// virtual vertices.  A copy's arrays are those of one search.
struct BfsView {
  uint32_t n, ntiles;
  uint32_t gn;          // vertices of the graph (n / copies)
  uint64_t* V;          // [n][ntiles][4] visited columns (ballot layout)
  const uint64_t* F;    // frontier of this level
  uint64_t* N;          // frontier of the next level
  const uint32_t* cur;  // frontier vertices of this level
  uint32_t* next;       // frontier vertices of the next level
  uint32_t* ncount;     // |next|
  uint32_t* stamp;      // [n] last level a vertex joined a frontier list
  uint32_t* levels;     // largest level with a non-empty frontier
};

void launch_bfs_seed(const MemoView& m, const BfsView& b, const uint32_t* S, uint32_t len, hipStream_t st);
// The frontier size is read on the device (*ncur), so levels can be
// enqueued without waiting for the host; an empty frontier makes both no-ops.
void launch_bfs_level(const GraphView& g, const MemoView& m, const BfsView& b, const uint32_t* ncur,
                      uint32_t level, hipStream_t st);
void launch_bfs_clear(uint64_t* F, const uint32_t* cur, const uint32_t* ncur, uint32_t ntiles, hipStream_t st);
void launch_bfs_count(const uint64_t* V, uint64_t words, unsigned long long* out, hipStream_t st);
// Set bits of each copy's words: out[c] += popcount(V[c * words .. (c + 1) * words)).
void launch_bfs_count_copies(const uint64_t* V, uint64_t words, uint32_t copies, unsigned long long* out,
                             hipStream_t st);
// V[c * words + i] = src[i] for every copy c < copies.
void launch_bfs_replicate(const uint64_t* src, uint64_t* V, uint64_t words, uint32_t copies, hipStream_t st);

}  // namespace infuse
