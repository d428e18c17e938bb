// Launchers of the memo-free sigma kernels (direct.hip).
#pragma once

#include "common.h"

namespace infuse {

// Several searches can run side by side as copies of the graph: virtual
// vertex c * gn + v is vertex v of copy c (gn = the graph's n); n counts the
// virtual vertices.  A copy's arrays are those of one search.
// Per copy, new bits are summed into kCountSlots counters (blocks spread
// over them; fewer slots made the adds of one level's wavefronts contend);
// the copy's count is the sum of its slots.
constexpr uint32_t kCountSlots = 128;

// Items of long rows are split: an item of a vertex with more than
// kSplitArcs arcs is listed kPieces times, entry = item | piece << kPieceShift,
// and each piece walks an eighth of the row, so no item of a level waits on
// a whole hub row.  Only when item ids fit below 2^kPieceShift.
constexpr uint32_t kSplitArcs = 256;
constexpr uint32_t kPieces = 8;
constexpr uint32_t kPieceShift = 29;

struct BfsView {
  uint32_t n, ntiles;
  uint32_t pieces;                // kPieces when long rows are split, else 1
  const uint64_t* hubmask;        // [ceil(n * ntiles / 64)] items of long rows (when split)
  uint32_t gn;                    // vertices of the graph (n / copies)
  uint64_t* V;                    // [n][ntiles][4] visited columns (ballot layout)
  uint64_t* F;                    // frontier of this level (cleared as it is read)
  uint64_t* N;                    // frontier of the next level
  const uint32_t* cur;            // frontier entries of this level: vertex * ntiles + tile (+ piece)
  uint32_t* next;                 // frontier entries of the next level
  uint32_t* lcount;               // [3] list sizes, level l reads lcount[l % 3]; lcount[1] zero before the seeds
  uint64_t* nbits;                // [ceil(n * ntiles / 64)] items of the next frontier (zero between levels)
  uint32_t* levels;               // largest level with a non-empty frontier
  unsigned long long* counts;     // [copies][kCountSlots] new bits
  unsigned long long* stats;      // [kCountSlots][3] work counts (items, arcs, live pairs), or nullptr
};

// Seeds S[i] (virtual ids) join the visited sets and the first frontier
// (entries of the items (S[i], t) appended to b.next, b.lcount[1] counting
// them); their uncovered columns are counted.  Item ids (n * ntiles) must
// fit in 32 bits.
void launch_bfs_seed(const GraphView& g, const MemoView& m, const BfsView& b, const uint32_t* S, uint32_t len,
                     hipStream_t st);
// The items of long rows, as a bitmap over b.n * b.ntiles items.
void launch_bfs_hubmask(const GraphView& g, const BfsView& b, uint64_t* mask, hipStream_t st);
// One level, then the listing of the next frontier: the frontier size is
// read on the device, so levels can be enqueued without waiting for the
// host; an empty frontier makes both kernels no-ops.
void launch_bfs_level(const GraphView& g, const MemoView& m, const BfsView& b, uint32_t level, hipStream_t st);
void launch_bfs_compact(const BfsView& b, uint32_t level, hipStream_t st);
// V[c * words + i] = src[i] for every copy c < copies.
void launch_bfs_replicate(const uint64_t* src, uint64_t* V, uint64_t words, uint32_t copies, hipStream_t st);

}  // namespace infuse
