// Work lists of a memo construction (entries v * ntiles + t in kSubLists
// sub-lists by vertex range) walked by wavefronts: shared by the labelling
// kernels and the set-up of a selection.
#pragma once

#include "common.h"
#include "tile.h"  // uni()

namespace infuse {

// Wavefront iteration over the concatenation of the kSubLists sub-lists of a
// work list: every wavefront of the grid strides over all entries (so the
// heavy tiles of hub vertices spread over the whole grid).  The sub-list
// sizes are prefix-summed in LDS by each workgroup (blockDim.x == 256 ==
// kSubLists) and an entry's sub-list found by binary search.
struct ListIter {
  const uint32_t* list;
  const uint32_t* pre;  // LDS, kSubLists + 1 prefix sums
  uint32_t cap, total, first, stride;
  __device__ uint32_t at(uint32_t idx) const {
    uint32_t lo = 0, hi = kSubLists;  // pre[lo] <= idx < pre[hi]
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (pre[mid] <= idx) lo = mid; else hi = mid;
    }
    return list[(uint64_t)lo * cap + (idx - pre[lo])];
  }
};
__device__ inline ListIter list_iter(const MemoView& m, const uint32_t* base, int which, uint32_t* pre,
                                     uint32_t bid, uint32_t nblk) {
  static_assert(kSubLists == 256, "one prefix element per thread of a 256-thread workgroup");
  const uint32_t tid = threadIdx.x;
  uint32_t x = m.counts[2 * tid + which];
  pre[tid + 1] = x;
  if (tid == 0) pre[0] = 0;
  __syncthreads();
  for (uint32_t off = 1; off < kSubLists; off <<= 1) {
    const uint32_t y = tid + 1 > off ? pre[tid + 1 - off] : 0u;
    __syncthreads();
    x += y;
    pre[tid + 1] = x;
    __syncthreads();
  }
  ListIter it;
  it.list = base;
  it.pre = pre;
  it.cap = m.list_cap;
  it.total = uni(pre[kSubLists]);
  it.first = uni(bid * (blockDim.x >> 6) + (threadIdx.x >> 6));
  it.stride = nblk * (blockDim.x >> 6);
  return it;
}

// A wavefront's entries of a work list, 64 at a time: the entries of the
// wavefront are first + k * stride (k = 0, 1, ...); lane l resolves entry
// k0 + l of them.  `count` receives how many of the 64 exist (a prefix of
// the lanes).  One load brings 64 entries, so the per-entry work that
// follows does not wait for the list.
__device__ inline uint32_t list_chunk(const ListIter& it, uint32_t k0, uint32_t lane, uint32_t& count) {
  const uint64_t idx = (uint64_t)it.first + (uint64_t)(k0 + lane) * it.stride;
  const bool ok = idx < it.total;
  count = (uint32_t)__popcll(__ballot(ok));
  return ok ? it.at((uint32_t)idx) : 0u;
}

}  // namespace infuse
