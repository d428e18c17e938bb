// Column tiles of the memo and the candidate test (shared by the labelling
// kernels and the memo-free sigma kernels).
//
// A tile is 256 columns: lane l of a wavefront holds columns 4l .. 4l+3.
// Columns are sorted by X, so a tile spans a narrow X interval and an edge
// with hash h can be live in it only if h >> k lies in [X_lo >> k, X_hi >> k]
// with k = bitlen(T - 1): one compare and one ballot per tile rule out all
// other edges before the per-column test (h ^ X) <= T - 1.
#pragma once

#include "common.h"

namespace infuse {

struct TileCtx {
  uint32_t q0;      // first column of this lane
  uint32_t x[4];    // X of the lane's 4 columns
  uint32_t klo, khi;
  bool valid[4];
};

__device__ inline uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// X of the lane's four columns of tile t (one 16-byte load per lane).
__device__ inline uint4 load_tile_x(const MemoView& m, uint32_t t, uint32_t lane) {
  return *reinterpret_cast<const uint4*>(m.xs + t * kTile + lane * kPerLane);
}

// Tile context from the loaded X values: the tile's X range comes from lane
// 0 (first column) and the lane holding the last used column.
__device__ inline void tile_from_x(const MemoView& m, uint32_t t, uint32_t lane, uint4 x4, uint32_t kshift,
                                   TileCtx& tc, bool per_edge) {
  tc.q0 = t * kTile + lane * kPerLane;
  tc.x[0] = x4.x;
  tc.x[1] = x4.y;
  tc.x[2] = x4.z;
  tc.x[3] = x4.w;
#pragma unroll
  for (int i = 0; i < 4; ++i) tc.valid[i] = tc.q0 + i < m.R;
  const uint32_t qlast = min(t * kTile + kTile - 1, m.R - 1) - t * kTile;  // R > t * kTile
  const uint32_t c = qlast & 3;
  const uint32_t pick = c == 0 ? x4.x : c == 1 ? x4.y : c == 2 ? x4.z : x4.w;
  const uint32_t xlo = __builtin_amdgcn_readlane(x4.x, 0);
  const uint32_t xhi = __builtin_amdgcn_readlane(pick, qlast >> 2);
  if (!per_edge) {
    tc.klo = (uint32_t)((uint64_t)xlo >> kshift);
    tc.khi = (uint32_t)((uint64_t)xhi >> kshift);
  } else {
    tc.klo = xlo;  // shifted per edge
    tc.khi = xhi;
  }
}

// Can an edge with hash h and bit length k be live in the tile?
__device__ inline bool cand_uniform(uint32_t h, uint32_t kshift, const TileCtx& tc) {
  const uint32_t hk = (uint32_t)((uint64_t)h >> kshift);
  return hk - tc.klo <= tc.khi - tc.klo;
}
__device__ inline bool cand_per_edge(uint32_t h, uint32_t k, const TileCtx& tc) {
  const uint32_t hk = (uint32_t)((uint64_t)h >> k);
  const uint32_t lo = (uint32_t)((uint64_t)tc.klo >> k), hi = (uint32_t)((uint64_t)tc.khi >> k);
  return hk - lo <= hi - lo;
}

// Visits the candidate edges of v in the tile, calling f(u, h, tm1, small)
// for each in slot order.  Returns whether any candidate exists.
template <bool PER_EDGE, bool SMALL_ONLY, typename F>
__device__ inline bool for_candidates(const GraphView& g, const MemoView& m, uint32_t v,
                                      uint32_t beg, uint32_t end, uint32_t split, uint32_t lane,
                                      bool inreg, uint32_t rcol, uint32_t rh, uint32_t rtm1,
                                      const TileCtx& tc, F&& f) {
  bool any = false;
  const uint32_t last = SMALL_ONLY ? split : end;
  if (m.never_live) return false;
  if (inreg) {
    const uint32_t j = beg + lane;
    bool c = j < last;
    if (PER_EDGE) c = c && cand_per_edge(rh, bitlen32(rtm1), tc);
    else c = c && cand_uniform(rh, m.kshift, tc);
    uint64_t mask = __ballot(c);
    any = mask != 0;
    while (mask) {
      const int b = __builtin_ctzll(mask);
      mask &= mask - 1;
      const uint32_t u = __builtin_amdgcn_readlane(rcol, b);
      const uint32_t h = __builtin_amdgcn_readlane(rh, b);
      const uint32_t tt = PER_EDGE ? __builtin_amdgcn_readlane(rtm1, b) : m.tm1;
      f(u, h, tt, beg + (uint32_t)b < split);
    }
  } else {
    for (uint32_t base = beg; base < last; base += kWave) {
      const uint32_t j = base + lane;
      uint32_t col = kInvalid, h = 0, tm1 = 0;
      bool c = false;
      if (j < last) {
        const uint2 e = m.edges[j];
        col = e.x;
        h = e.y;
        if (PER_EDGE) {
          tm1 = g.tm1[j];
          c = cand_per_edge(h, bitlen32(tm1), tc);
        } else {
          c = cand_uniform(h, m.kshift, tc);
        }
      }
      uint64_t mask = __ballot(c);
      any = any || mask != 0;
      while (mask) {
        const int b = __builtin_ctzll(mask);
        mask &= mask - 1;
        const uint32_t u = __builtin_amdgcn_readlane(col, b);
        const uint32_t hh = __builtin_amdgcn_readlane(h, b);
        const uint32_t tt = PER_EDGE ? __builtin_amdgcn_readlane(tm1, b) : m.tm1;
        f(u, hh, tt, base + (uint32_t)b < split);
      }
    }
  }
  return any;
}


}  // namespace infuse
