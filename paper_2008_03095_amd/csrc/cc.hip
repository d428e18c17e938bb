// Fused multi-simulation connected components and the component-size memo
// (Section III-B, Algorithms 5-6; Section III-C).
//
// The paper labels R sampled subgraphs by min-label propagation, 8
// simulations per AVX2 op, re-testing each edge's hash-liveness as it is
// read.  Here a wavefront owns one vertex row of the vertex-major memo and
// its 64 lanes x 4 columns are 256 simulations of that vertex (coalesced
// 16-byte accesses).  Instead of iterating propagation sweeps to a fixed
// point, components are built as a union-find forest whose roots are the
// component minima:
//
//   k_hook     one streaming pass over the memo: M[v][q] = smallest live
//              neighbour u < v of v in column q (a parent pointer), or -1
//              when v has none (a root).  This is the first propagation step
//              of Algorithm 5 restricted to smaller neighbours; it reads no
//              label, so the pass is a pure write of n*Rs words.
//   k_link     the remaining live edges (u < v, u not the hook of v) are
//              merged by lock-free union: the larger root is linked under the
//              smaller with compare-and-swap, so every root stays the minimum
//              of its tree in any interleaving.  The hook parent stored in the
//              memo stands for v, so no second scan for it is needed.  A
//              wavefront queues its live (edge, column) pairs and joins them
//              64 at a time, one per lane.
//   k_flatten  every non-root entry is replaced by its root;
//   k_count    each member decrements its root's -1 once: afterwards roots
//              hold -|component| (the size memo) and members hold the label.
//   k_gain0    mg_v = sum over columns of |C_q(v)| (Algorithm 5, int64).
//
// Work skipping.  Columns are sorted by X, so a 256-column tile spans a
// narrow X interval; edge e can be live in the tile only if h_e >> k lies in
// [X_lo >> k, X_hi >> k] where k = bitlen(T - 1).  The wavefront tests all
// (up to 64) adjacent edges with one compare and one ballot per tile and runs
// the per-column test only for the candidates.  k_hook records, per
// (vertex, tile), whether any candidate exists (tmask, and the work list
// tlist: the tile may hold a non-singleton column) and whether some column
// has two or more live smaller neighbours (work list llist: the tile needs
// k_link); the later kernels visit only those tiles.
#include <algorithm>

#include "common.h"
#include "lists.h"
#include "tile.h"

namespace infuse {

// Adds the wavefront's sum of x to work count i (one atomic per wavefront;
// only while the construction is counted).
__device__ inline void work_add(const MemoView& m, uint32_t i, uint32_t x) {
  if (!m.work) return;
  uint64_t s = x;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0 && s) atomicAdd(&m.work[i], (unsigned long long)s);
}

// Hook of one tile: for each of the lane's columns, the smallest live
// neighbour u < v (or -1), stored as one 16-byte write when the tile has a
// candidate edge at all; otherwise v is a singleton in every column of the
// tile and nothing is written (readers consult tmask first).  Returns
// whether the tile has any candidate edge (tmask bit) and whether some
// column has two or more live smaller neighbours (lmask bit).
template <bool PER_EDGE>
__device__ inline void hook_tile(const GraphView& g, const MemoView& m, uint32_t v, uint32_t beg, uint32_t end,
                                 uint32_t split, uint32_t lane, bool inreg, uint32_t rcol, uint32_t rh,
                                 uint32_t rtm1, const TileCtx& tc, int32_t* row, bool& any, bool& need) {
  int32_t mn[4] = {INT32_MAX, INT32_MAX, INT32_MAX, INT32_MAX};
  uint32_t cnt[4] = {0, 0, 0, 0};
  // candidates among all neighbours mark the tile; smaller ones hook
  any = for_candidates<PER_EDGE, false>(
      g, m, v, beg, end, split, lane, inreg, rcol, rh, rtm1, tc,
      [&](uint32_t u, uint32_t h, uint32_t tt, bool small) {
        if (!small) return;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const bool live = tc.valid[i] && (h ^ tc.x[i]) <= tt;
          cnt[i] += live ? 1u : 0u;
          mn[i] = live ? min(mn[i], (int32_t)u) : mn[i];
        }
      });
  int4 out;
  out.x = cnt[0] ? mn[0] : -1;
  out.y = cnt[1] ? mn[1] : -1;
  out.z = cnt[2] ? mn[2] : -1;
  out.w = cnt[3] ? mn[3] : -1;
  // streaming store: the row is not read again before the next kernel
  typedef int int4v __attribute__((ext_vector_type(4)));
  const int4v ov = {out.x, out.y, out.z, out.w};
  if (any) __builtin_nontemporal_store(ov, reinterpret_cast<int4v*>(row + tc.q0));
  need = __ballot(cnt[0] > 1 || cnt[1] > 1 || cnt[2] > 1 || cnt[3] > 1) != 0;
  if (m.work) {
    work_add(m, kWorkLivePairs, cnt[0] + cnt[1] + cnt[2] + cnt[3]);
    work_add(m, inreg ? kWorkRowTiles : kWorkHubTiles, (any && (threadIdx.x & 63) == 0) ? 1u : 0u);
  }
}

// k_hook_rows: one wavefront per vertex with at most kWave neighbours (the
// neighbour list sits in registers).  Per 32 tiles, lane i reads the X
// bounds of tile i and tests them against every edge of the vertex (one lane
// read and a compare per edge): the tiles with a candidate edge form the
// tmask word.  Only those tiles are
// then hooked and written, the X values of the next one loaded before the
// current one is processed.  The wave owns the vertex's mask words and
// stores them directly.
template <bool PER_EDGE>
__device__ inline void hook_rows_body(const GraphView& g, const MemoView& m, uint32_t bid) {
  const uint32_t v = uni(bid * 4 + (threadIdx.x >> 6));
  if (v >= g.n) return;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t beg = uni(g.row_ptr[v]), end = uni(g.row_ptr[v + 1]);
  // no edge: the vertex is a singleton in every column, its mask words stay
  // as cleared and its memo row is never read
  if (end == beg || end - beg > (uint32_t)kWave) return;  // more than kWave: k_hook_hubs
  const uint32_t split = uni(g.split[v]);
  const bool has = beg + lane < end;
  uint32_t rcol = kInvalid, rh = 0, rtm1 = 0;
  if (has) {
    const uint2 e = m.edges[beg + lane];
    rcol = e.x;
    rh = e.y;
    if (PER_EDGE) rtm1 = g.tm1[beg + lane];
  }
  const uint32_t kb = m.kshift;  // uniform mode
  int32_t* row = m.M + (uint64_t)v * m.Rs;
  uint32_t* tw = m.tmask + (uint64_t)v * m.mwords;
  uint32_t* lw = m.lmask + (uint64_t)v * m.mwords;
  for (uint32_t w = 0; w < m.mwords; ++w) {
    const uint32_t t0 = w * 32, nt = min(32u, m.ntiles - t0);
    // X of the first and of the last used column of tile t0 + lane
    uint32_t xlo = 0, xhi = 0;
    if (lane < nt) {
      const uint32_t t = t0 + lane;
      xlo = m.xs[t * kTile];
      xhi = m.xs[min(t * kTile + kTile - 1, m.R - 1)];
    }
    // lane i tests tile t0 + i against every edge (one lane read per edge)
    bool hit = false;
    if (!m.never_live) {
      const uint32_t deg = end - beg;
      if (PER_EDGE) {
        for (uint32_t j = 0; j < deg; ++j) {
          const uint32_t kj = bitlen32((uint32_t)__builtin_amdgcn_readlane((int)rtm1, (int)j));
          const uint32_t hj = (uint32_t)((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)rh, (int)j) >> kj);
          const uint32_t lo = (uint32_t)((uint64_t)xlo >> kj), hi = (uint32_t)((uint64_t)xhi >> kj);
          hit = hit || hj - lo <= hi - lo;
        }
      } else {
        const uint32_t lo = (uint32_t)((uint64_t)xlo >> kb), hi = (uint32_t)((uint64_t)xhi >> kb);
        for (uint32_t j = 0; j < deg; ++j) {
          const uint32_t hj = (uint32_t)((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)rh, (int)j) >> kb);
          hit = hit || hj - lo <= hi - lo;
        }
      }
    }
    const uint32_t cm = (uint32_t)__ballot(hit && lane < nt);
    uint32_t lbits = 0;
    uint32_t rem = cm;
    uint4 xn = load_tile_x(m, t0 + (rem ? (uint32_t)__builtin_ctz(rem) : 0u), lane);
    while (rem) {
      const uint32_t t = t0 + (uint32_t)__builtin_ctz(rem);
      rem &= rem - 1;
      const uint4 xc = xn;
      xn = load_tile_x(m, t0 + (rem ? (uint32_t)__builtin_ctz(rem) : 0u), lane);
      TileCtx tc;
      tile_from_x(m, t, lane, xc, m.kshift, tc, PER_EDGE);
      bool any, need;
      hook_tile<PER_EDGE>(g, m, v, beg, end, split, lane, true, rcol, rh, rtm1, tc, row, any, need);
      lbits |= (need ? 1u : 0u) << (t & 31);
    }
    if (lane == 0) {
      tw[w] = cm;
      lw[w] = lbits;
    }
  }
}

// k_hook_hubs: vertices with more than kWave neighbours, one wavefront per
// (vertex, chunk of tiles); the neighbour list is streamed in 64-slot
// pieces.  Several wavefronts share a vertex's mask words (atomic or).
template <bool PER_EDGE>
__device__ inline void hook_hubs_body(const GraphView& g, const MemoView& m, uint32_t chunk, uint32_t wpv,
                                      uint32_t bid) {
  const uint64_t wid = (uint64_t)bid * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const uint32_t hi = uni((uint32_t)(wid / wpv));
  if (hi >= g.nhubs) return;
  const uint32_t c = uni((uint32_t)(wid % wpv));
  const uint32_t t0 = c * chunk, t1 = min(t0 + chunk, m.ntiles);
  const uint32_t lane = threadIdx.x & 63, v = uni(g.hubs[hi]);
  const uint32_t beg = uni(g.row_ptr[v]), end = uni(g.row_ptr[v + 1]), split = uni(g.split[v]);
  int32_t* row = m.M + (uint64_t)v * m.Rs;
  uint32_t tbits = 0, lbits = 0;
  for (uint32_t t = t0; t < t1; ++t) {
    TileCtx tc;
    tile_from_x(m, t, lane, load_tile_x(m, t, lane), m.kshift, tc, PER_EDGE);
    bool any, need;
    hook_tile<PER_EDGE>(g, m, v, beg, end, split, lane, false, kInvalid, 0, 0, tc, row, any, need);
    tbits |= (any ? 1u : 0u) << (t - t0);
    lbits |= (need ? 1u : 0u) << (t - t0);
  }
  if (lane == 0) {  // chunk <= 32 tiles, aligned: one mask word
    const uint64_t word = (uint64_t)v * m.mwords + (t0 >> 5);
    if (tbits) atomicOr(&m.tmask[word], tbits << (t0 & 31));
    if (lbits) atomicOr(&m.lmask[word], lbits << (t0 & 31));
  }
}

// k_lists: sub-list j lists, in vertex order, the tiles of the vertices
// [j * vps, (j + 1) * vps) whose tmask (tlist) or lmask (llist) bit is set.
// One workgroup per sub-list; positions come from workgroup prefix sums, so
// no global counter is contended.  It also sets mg_v = R, the gain of an all
// singleton row, to which k_gain0 adds the listed tiles.
__device__ inline void lists_body(const MemoView& m, uint32_t bid) {
  __shared__ uint32_t wsum[2][4];
  const uint32_t j = bid, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint32_t vps = (m.n + kSubLists - 1) / kSubLists;
  const uint32_t v0 = min(m.n, j * vps), v1 = min(m.n, v0 + vps);
  uint32_t* tout = m.tlist + (uint64_t)j * m.list_cap;
  uint32_t* lout = m.llist + (uint64_t)j * m.list_cap;
  uint32_t tbase = 0, lbase = 0;
  for (uint32_t vb = v0; vb < v1; vb += 256) {
    const uint32_t v = vb + threadIdx.x;
    uint32_t tc = 0, lc = 0;
    if (v < v1) m.g0[v] = (int64_t)m.R;
    if (v < v1)
      for (uint32_t w = 0; w < m.mwords; ++w) {
        tc += __popc(m.tmask[(uint64_t)v * m.mwords + w]);
        lc += __popc(m.lmask[(uint64_t)v * m.mwords + w]);
      }
    // exclusive prefix sums of tc and lc over the workgroup
    uint32_t ts = tc, ls = lc;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t a = __shfl_up(ts, off), b = __shfl_up(ls, off);
      if (lane >= (uint32_t)off) {
        ts += a;
        ls += b;
      }
    }
    if (lane == 63) {
      wsum[0][wv] = ts;
      wsum[1][wv] = ls;
    }
    __syncthreads();
    uint32_t tpre = 0, lpre = 0, ttot = 0, ltot = 0;
#pragma unroll
    for (uint32_t i = 0; i < 4; ++i) {
      tpre += i < wv ? wsum[0][i] : 0;
      lpre += i < wv ? wsum[1][i] : 0;
      ttot += wsum[0][i];
      ltot += wsum[1][i];
    }
    __syncthreads();
    uint32_t ta = tbase + tpre + ts - tc, la = lbase + lpre + ls - lc;
    if (v < v1)
      for (uint32_t w = 0; w < m.mwords; ++w) {
        const uint32_t first = v * m.ntiles + w * 32;
        for (uint32_t b = m.tmask[(uint64_t)v * m.mwords + w]; b; b &= b - 1) tout[ta++] = first + __ffs(b) - 1;
        for (uint32_t b = m.lmask[(uint64_t)v * m.mwords + w]; b; b &= b - 1) lout[la++] = first + __ffs(b) - 1;
      }
    tbase += ttot;
    lbase += ltot;
  }
  if (threadIdx.x == 0) {
    m.counts[2 * j] = tbase;
    m.counts[2 * j + 1] = lbase;
  }
}

// Root of x in column q, with path halving.  Every parent has a smaller id
// than its child (hook parents are smaller neighbours, unions put the larger
// root under the smaller), and while linking an entry only moves from
// "root" (-1) to a parent, or from a parent to one of its ancestors.  So a
// stale value read from a non-coherent cache is still an ancestor (or the
// root state of a vertex linked meanwhile, caught by the compare-and-swap in
// unite_root), every step goes to a smaller id and the walk ends.  Each
// visited entry is re-pointed to its grandparent with an atomic store (the
// memo is written only by atomics while linking); a value written from a
// stale read is still an ancestor.
// The walk also ends at `stop` (a root the caller holds, or kInvalid):
// reaching it shows that x is in the caller's tree, which is all a union
// needs to know.
__device__ inline uint32_t find_root_halving(int32_t* M, uint32_t Rs, uint32_t x, uint32_t q,
                                             uint32_t stop = kInvalid) {
  while (true) {
    if (x == stop) return x;
    const int32_t p = M[(uint64_t)x * Rs + q];
    if (p < 0 || (uint32_t)p == stop) return p < 0 ? x : stop;
    const int32_t gp = M[(uint64_t)p * Rs + q];
    if (gp < 0) return (uint32_t)p;
    __hip_atomic_store(&M[(uint64_t)x * Rs + q], gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    x = (uint32_t)gp;
  }
}

// Joins root a with the tree of b in column q and returns the smallest root
// reached.  Roots hold -1 during linking; the larger root is linked under
// the smaller with compare-and-swap, so every root stays the minimum of its
// tree in any interleaving.  A failed compare-and-swap returns the entry's
// current parent, from which the walk continues: each retry moves one side
// to a strictly smaller id, so the loop ends.  The memo is written only by
// atomics in this kernel (the XCD L2 caches are not coherent within a
// kernel, so plain stores must not share lines with atomics).
__device__ inline uint32_t unite_root(int32_t* M, uint32_t Rs, uint32_t a, uint32_t b, uint32_t q) {
  b = find_root_halving(M, Rs, b, q, a);
  while (a != b) {
    if (a < b) {
      const uint32_t t = a;
      a = b;
      b = t;
    }
    int32_t expected = -1;
    if (__hip_atomic_compare_exchange_strong(&M[(uint64_t)a * Rs + q], &expected, (int32_t)b,
                                             __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT))
      return b;
    a = find_root_halving(M, Rs, (uint32_t)expected, q, b);
    b = find_root_halving(M, Rs, b, q, a);
  }
  return a;
}

// Row words of entry e (vertex e / ntiles, tile e % ntiles) for this lane.
__device__ inline int4 list_row(const MemoView& m, uint32_t e, uint32_t lane) {
  const uint32_t v = e / m.ntiles, t = e % m.ntiles;
  return *reinterpret_cast<const int4*>(m.M + (uint64_t)v * m.Rs + t * kTile + lane * kPerLane);
}

// Live (candidate, column) pairs of a wavefront queued in LDS (a ring of
// kQueue entries) and joined 64 at a time, one union per lane: a
// candidate's live columns are a contiguous run (columns are sorted by X),
// so unions taken per lane would leave most lanes idle while a few walk four
// columns each.  root[c] is a vertex of the tree being joined in column c
// (its root when last seen), shared by the lanes that join in that column.
constexpr uint32_t kQueue = 512;
struct PairQueue {
  uint32_t u[kQueue];    // candidate
  uint8_t c[kQueue];     // column within the tile
  uint32_t root[kTile];
};
__device__ inline void lds_wave_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// Columns (bits 0-3) of this lane where candidate u is live and still has to
// be joined: v has a hook parent there (mn >= 0) and it is not u.
__device__ inline uint32_t join_mask(const TileCtx& tc, const int32_t (&mn)[4], uint32_t u, uint32_t h, uint32_t tt) {
  uint32_t m4 = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    m4 |= (tc.valid[i] && (h ^ tc.x[i]) <= tt && mn[i] >= 0 && (int32_t)u != mn[i]) ? 1u << i : 0u;
  return m4;
}

// Appends the lanes' pairs of candidate u at tail (lane order); returns how
// many the wavefront added.  Wave-uniform call.
__device__ inline uint32_t pq_push(PairQueue& Q, uint32_t tail, uint32_t u, uint32_t m4, uint32_t lane) {
  const uint32_t cnt = (uint32_t)__builtin_popcount(m4);
  uint32_t incl = cnt;
#pragma unroll
  for (uint32_t off = 1; off < 64; off <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int)incl, off);
    if (lane >= off) incl += y;
  }
  uint32_t k = tail + incl - cnt;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if ((m4 >> i) & 1u) {
      Q.u[k & (kQueue - 1)] = u;
      Q.c[k & (kQueue - 1)] = (uint8_t)(lane * kPerLane + i);
      ++k;
    }
  lds_wave_sync();
  return (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
}

// Joins the cnt (<= 64) pairs from head, one per lane, in tile t.
// Wave-uniform call.
__device__ inline void pq_run(const MemoView& m, PairQueue& Q, uint32_t head, uint32_t cnt, uint32_t t,
                              uint32_t lane) {
  if (lane < cnt) {
    const uint32_t slot = (head + lane) & (kQueue - 1);
    const uint32_t u = Q.u[slot], ci = Q.c[slot], q = t * kTile + ci;
    const uint32_t a = find_root_halving(m.M, m.Rs, Q.root[ci], q);
    Q.root[ci] = unite_root(m.M, m.Rs, a, u, q);
  }
  lds_wave_sync();
}

template <bool PER_EDGE>
__device__ inline void link_body(const GraphView& g, const MemoView& m, uint32_t bid, uint32_t nblk) {
  const uint32_t lane = threadIdx.x & 63;
  __shared__ uint32_t pre[kSubLists + 1];
  __shared__ PairQueue pq[4];
  PairQueue& Q = pq[threadIdx.x >> 6];
  const ListIter it = list_iter(m, m.llist, 1, pre, bid, nblk);
  for (uint32_t idx = it.first; idx < it.total; idx += it.stride) {
    const uint32_t e = uni(it.at(idx));
    const uint32_t v = e / m.ntiles, t = e % m.ntiles;
    const uint32_t beg = uni(g.row_ptr[v]), end = uni(g.row_ptr[v + 1]), split = uni(g.split[v]);
    if (end - beg > (uint32_t)kWave) continue;  // hub: k_link_hubs
    uint32_t rcol = kInvalid, rh = 0, rtm1 = 0;
    if (beg + lane < end) {
      const uint2 ed = m.edges[beg + lane];
      rcol = ed.x;
      rh = ed.y;
      if (PER_EDGE) rtm1 = g.tm1[beg + lane];
    }
    TileCtx tc;
    tile_from_x(m, t, lane, load_tile_x(m, t, lane), m.kshift, tc, PER_EDGE);
    // v's hook parent per column: its smallest live smaller neighbour, which
    // linking never changes (only roots are re-pointed).  A negative entry
    // means v has no live smaller neighbour in that column.
    const int4 hp = *reinterpret_cast<const int4*>(m.M + (uint64_t)v * m.Rs + tc.q0);
    const int32_t mn[4] = {hp.x, hp.y, hp.z, hp.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) Q.root[lane * kPerLane + i] = (uint32_t)mn[i];  // read only where mn >= 0
    lds_wave_sync();
    uint32_t head = 0, tail = 0;
    for_candidates<PER_EDGE, true>(g, m, v, beg, end, split, lane, true, rcol, rh, rtm1, tc,
                                   [&](uint32_t u, uint32_t h, uint32_t tt, bool) {
                                     tail += pq_push(Q, tail, u, join_mask(tc, mn, u, h, tt), lane);
                                     for (; tail - head >= 64; head += 64) pq_run(m, Q, head, 64, t, lane);
                                   });
    for (; tail != head; head += min(64u, tail - head)) pq_run(m, Q, head, min(64u, tail - head), t, lane);
    work_add(m, kWorkUnions, lane == 0 ? tail : 0u);
  }
}

// k_link_hubs: the unions of hub vertices, one wavefront per (hub, tile,
// piece of kHubPiece smaller neighbours, walked 64 at a time); tiles without
// an lmask bit are skipped.  The piece table gives the hub and the piece's
// first slot.
template <bool PER_EDGE>
__device__ inline void link_hubs_body(const GraphView& g, const MemoView& m, uint32_t bid) {
  __shared__ PairQueue pq[4];
  const uint64_t wid = (uint64_t)bid * 4 + (threadIdx.x >> 6);
  const uint32_t pg = uni((uint32_t)(wid / m.ntiles)), t = uni((uint32_t)(wid % m.ntiles));
  if (pg >= g.hub_pieces) return;
  const uint2 pc = g.hub_piece[pg];
  const uint32_t v = uni(pc.x);
  if (!((m.lmask[(uint64_t)v * m.mwords + (t >> 5)] >> (t & 31)) & 1u)) return;
  const uint32_t lane = threadIdx.x & 63;
  PairQueue& Q = pq[threadIdx.x >> 6];
  const uint32_t pbeg = uni(pc.y);
  const uint32_t pend = min(pbeg + kHubPiece, uni(g.split[v]));  // smaller neighbours only
  TileCtx tc;
  tile_from_x(m, t, lane, load_tile_x(m, t, lane), m.kshift, tc, PER_EDGE);
  const int4 hp = *reinterpret_cast<const int4*>(m.M + (uint64_t)v * m.Rs + tc.q0);
  const int32_t mn[4] = {hp.x, hp.y, hp.z, hp.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) Q.root[lane * kPerLane + i] = (uint32_t)mn[i];  // read only where mn >= 0
  lds_wave_sync();
  uint32_t head = 0, tail = 0;
  for (uint32_t beg = pbeg; beg < pend; beg += kWave) {
    const uint32_t end = min(beg + (uint32_t)kWave, pend);
    uint32_t rcol = kInvalid, rh = 0, rtm1 = 0;
    if (beg + lane < end) {
      const uint2 ed = m.edges[beg + lane];
      rcol = ed.x;
      rh = ed.y;
      if (PER_EDGE) rtm1 = g.tm1[beg + lane];
    }
    for_candidates<PER_EDGE, true>(g, m, v, beg, end, end, lane, true, rcol, rh, rtm1, tc,
                                   [&](uint32_t u, uint32_t h, uint32_t tt, bool) {
                                     tail += pq_push(Q, tail, u, join_mask(tc, mn, u, h, tt), lane);
                                     for (; tail - head >= 64; head += 64) pq_run(m, Q, head, 64, t, lane);
                                   });
  }
  for (; tail != head; head += min(64u, tail - head)) pq_run(m, Q, head, min(64u, tail - head), t, lane);
  if (m.work) {
    work_add(m, kWorkUnions, lane == 0 ? tail : 0u);
    work_add(m, kWorkHubLinkWaves, lane == 0 ? 1u : 0u);
  }
}

// k_flatten: every non-root entry of a listed tile is replaced by its root
// (plain loads and stores only; a stale value read during the walk is an
// older ancestor, so every walk still ends at the root).  A wavefront takes
// two list entries at a time, the rows of the next two requested first; the
// eight columns of a lane (four per entry) walk together, one load each per
// step.
__device__ inline void flatten_body(const MemoView& m, uint32_t bid, uint32_t nblk) {
  const uint32_t lane = threadIdx.x & 63;
  __shared__ uint32_t pre[kSubLists + 1];
  const ListIter it = list_iter(m, m.tlist, 0, pre, bid, nblk);
  for (uint32_t k0 = 0; (uint64_t)it.first + (uint64_t)k0 * it.stride < it.total; k0 += 64) {
    uint32_t cnt;
    const uint32_t ent = list_chunk(it, k0, lane, cnt);
    uint32_t ea = uni(__builtin_amdgcn_readfirstlane(ent));
    uint32_t eb = (uint32_t)__builtin_amdgcn_readlane(ent, (int)min(1u, cnt - 1));
    int4 na = list_row(m, ea, lane), nb = list_row(m, eb, lane);
    for (uint32_t j = 0; j < cnt; j += 2) {
      const uint32_t ec[2] = {ea, eb};
      int4 out[2] = {na, nb};
      const bool hasb = j + 1 < cnt;
      ea = (uint32_t)__builtin_amdgcn_readlane(ent, (int)min(j + 2, cnt - 1));
      eb = (uint32_t)__builtin_amdgcn_readlane(ent, (int)min(j + 3, cnt - 1));
      na = list_row(m, ea, lane);
      nb = list_row(m, eb, lane);
      uint32_t c[8], q0[2];
      bool act[8];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        q0[x] = (ec[x] % m.ntiles) * kTile + lane * kPerLane;
        const int32_t* o = &out[x].x;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          act[4 * x + i] = (x == 0 || hasb) && q0[x] + i < m.R && o[i] >= 0;
          c[4 * x + i] = act[4 * x + i] ? (uint32_t)o[i] : 0u;
        }
      }
      bool any = true;
      while (any) {
        int32_t p[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) p[k] = act[k] ? m.M[(uint64_t)c[k] * m.Rs + q0[k >> 2] + (k & 3)] : -1;
        any = false;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          if (act[k] && p[k] >= 0) c[k] = (uint32_t)p[k];
          else act[k] = false;
          any = any || act[k];
        }
      }
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        if (x == 1 && !hasb) break;
        const uint32_t v = ec[x] / m.ntiles;
        int32_t* o = &out[x].x;
        uint32_t changed = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (q0[x] + i < m.R && o[i] >= 0 && c[4 * x + i] != (uint32_t)o[i]) {
            o[i] = (int32_t)c[4 * x + i];
            ++changed;
          }
        if (changed) *reinterpret_cast<int4*>(m.M + (uint64_t)v * m.Rs + q0[x]) = out[x];
        work_add(m, kWorkRewrites, changed);
      }
    }
  }
}

// k_count: each member entry (now pointing at its root) decrements its
// root's -1 once, so roots end at -|component|.  Only atomics write the memo
// here.  Workgroup = one 256-column tile x a block of vertices; counts for
// roots below kHotRoots are summed in LDS first, because large components
// (in power-law graphs the giant one) are rooted at small ids and their
// members would otherwise all hit the same words.
constexpr uint32_t kHotRoots = 8;
constexpr uint32_t kCountMaxBlockVerts = 4096;

// Vertices per workgroup of k_count: many workgroups (about 32768, so that
// the row loads of many wavefronts are in flight), multiples of 256, at most
// kCountMaxBlockVerts.
static uint32_t count_block_verts(const MemoView& m) {
  const uint64_t want = ((uint64_t)m.n * m.ntiles + 32767) / 32768;
  const uint64_t vb = (want + 255) / 256 * 256;
  return (uint32_t)std::min<uint64_t>(kCountMaxBlockVerts, std::max<uint64_t>(256, vb));
}

__device__ inline void count_body(const MemoView& m, uint32_t block_verts, uint32_t bid) {
  __shared__ uint32_t hot[kHotRoots][kTile];
  const uint32_t t = bid % m.ntiles;
  const uint32_t v0 = (bid / m.ntiles) * block_verts;
  const uint32_t v1 = min(v0 + block_verts, m.n);
  const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (uint32_t i = threadIdx.x; i < kHotRoots * kTile; i += blockDim.x) (&hot[0][0])[i] = 0;
  __syncthreads();
  const uint32_t word = t >> 5, bit = t & 31;
  const uint32_t q0 = t * kTile + lane * kPerLane;
  // 64 vertices' mask words per load; the wave then visits the flagged ones,
  // four rows requested together
  constexpr int kRows = 4;
  uint32_t nat = 0;  // root decrements made in device memory (work count)
  for (uint32_t vb = v0 + wv * 64; vb < v1; vb += 4 * 64) {
    const uint32_t vl = vb + lane;
    const bool flagged = vl < v1 && ((m.tmask[(uint64_t)vl * m.mwords + word] >> bit) & 1u);
    uint64_t fm = __ballot(flagged);
    while (fm) {
      uint32_t vv[kRows];
      bool on[kRows];
#pragma unroll
      for (int r = 0; r < kRows; ++r) {
        on[r] = fm != 0;
        vv[r] = on[r] ? vb + (uint32_t)__builtin_ctzll(fm) : vb + (uint32_t)__builtin_ctzll(__ballot(flagged));
        fm &= fm - 1;
      }
      int4 rows[kRows];
#pragma unroll
      for (int r = 0; r < kRows; ++r) rows[r] = *reinterpret_cast<const int4*>(m.M + (uint64_t)vv[r] * m.Rs + q0);
#pragma unroll
      for (int r = 0; r < kRows; ++r) {
        if (!on[r]) continue;
        const int32_t vals[4] = {rows[r].x, rows[r].y, rows[r].z, rows[r].w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const uint32_t q = q0 + i;
          const int32_t c = vals[i];
          if (q >= m.R || c < 0) continue;
          if ((uint32_t)c < kHotRoots) atomicAdd(&hot[c][lane * kPerLane + i], 1u);
          else atomicAdd(&m.M[(uint64_t)c * m.Rs + q], -1);
          nat += (uint32_t)c >= kHotRoots ? 1u : 0u;
        }
      }
    }
  }
  work_add(m, kWorkCountAtomics, nat);
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < kHotRoots * kTile; i += blockDim.x) {
    const uint32_t cnt = (&hot[0][0])[i];
    if (!cnt) continue;
    const uint32_t c = i / kTile, q = t * kTile + i % kTile;
    atomicAdd(&m.M[(uint64_t)c * m.Rs + q], -(int32_t)cnt);
    if (m.work) atomicAdd(&m.work[kWorkCountAtomics], 1ull);
  }
}

__device__ inline uint64_t wave_sum_u64(uint64_t x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off);
  return x;
}

// mg_v = sum_q |C_q(v)| = R + sum over the listed tiles of v of
// sum_q (|C_q(v)| - 1): unlisted tiles hold only singleton columns.

__device__ inline void gain0_body(const MemoView& m, uint32_t bid, uint32_t nblk) {
  const uint32_t lane = threadIdx.x & 63;
  __shared__ uint32_t pre[kSubLists + 1];
  const ListIter it = list_iter(m, m.tlist, 0, pre, bid, nblk);
  for (uint32_t k0 = 0; (uint64_t)it.first + (uint64_t)k0 * it.stride < it.total; k0 += 64) {
    uint32_t cnt;
    const uint32_t ent = list_chunk(it, k0, lane, cnt);
    // the next entry's row is requested before the current one's root
    // sizes are gathered; every gather has a valid address (a root or a
    // singleton reads its own entry), so none waits behind a branch
    uint32_t e = uni(__builtin_amdgcn_readfirstlane(ent));
    int4 nrow = list_row(m, e, lane);
    for (uint32_t j = 0; j < cnt; ++j) {
      const uint32_t ec = e;
      const int4 cur = nrow;
      e = (uint32_t)__builtin_amdgcn_readlane(ent, (int)min(j + 1, cnt - 1));
      nrow = list_row(m, e, lane);
      const uint32_t v = ec / m.ntiles, t = ec % m.ntiles;
      const uint32_t q0 = t * kTile + lane * kPerLane;
      const int32_t vals[4] = {cur.x, cur.y, cur.z, cur.w};
      int32_t raw[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) raw[i] = m.M[(uint64_t)(vals[i] >= 0 ? (uint32_t)vals[i] : v) * m.Rs + q0 + i];
      uint64_t sum = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int32_t sz = vals[i] < 0 ? -vals[i] : -raw[i];
        sum += (q0 + i < m.R) ? (uint64_t)(sz - 1) : 0;
      }
      if (m.work)
        work_add(m, kWorkGathers, (uint32_t)(vals[0] >= 0) + (vals[1] >= 0) + (vals[2] >= 0) + (vals[3] >= 0));
      sum = wave_sum_u64(sum);
      if (lane == 0 && sum) atomicAdd((unsigned long long*)&m.g0[v], (unsigned long long)sum);
    }
  }
}

// ---- kernels: one graph per launch, or many graphs per launch (batching) ----

template <bool PER_EDGE>
__global__ void __launch_bounds__(256) k_hook_rows(GraphView g, MemoView m) {
  hook_rows_body<PER_EDGE>(g, m, blockIdx.x);
}
template <bool PER_EDGE>
__global__ void __launch_bounds__(256) k_hook_hubs(GraphView g, MemoView m, uint32_t chunk, uint32_t wpv) {
  hook_hubs_body<PER_EDGE>(g, m, chunk, wpv, blockIdx.x);
}
__global__ void __launch_bounds__(256) k_lists(MemoView m) { lists_body(m, blockIdx.x); }
template <bool PER_EDGE>
__global__ void __launch_bounds__(256) k_link(GraphView g, MemoView m) {
  link_body<PER_EDGE>(g, m, blockIdx.x, gridDim.x);
}
template <bool PER_EDGE>
__global__ void __launch_bounds__(256) k_link_hubs(GraphView g, MemoView m) {
  link_hubs_body<PER_EDGE>(g, m, blockIdx.x);
}
__global__ void __launch_bounds__(256) k_flatten(MemoView m) { flatten_body(m, blockIdx.x, gridDim.x); }
__global__ void __launch_bounds__(256) k_count(MemoView m, uint32_t block_verts) {
  count_body(m, block_verts, blockIdx.x);
}
__global__ void __launch_bounds__(256) k_gain0(MemoView m) { gain0_body(m, blockIdx.x, gridDim.x); }

// Batched: workgroup blockIdx.x of the phase belongs to the graph found in
// the phase's prefix sums; per-slot and uniform probabilities are chosen per
// graph (uniform over a workgroup).
__global__ void __launch_bounds__(256) k_hook_rows_batch(BuildBatch b) {
  uint32_t local, nblk;
  const BuildJob& J = b.jobs[batch_job(b, kBpHookRows, blockIdx.x, local, nblk)];
  const GraphView g = J.g;
  const MemoView m = J.m;
  if (g.tm1) hook_rows_body<true>(g, m, local);
  else hook_rows_body<false>(g, m, local);
}
__global__ void __launch_bounds__(256) k_hook_hubs_batch(BuildBatch b) {
  uint32_t local, nblk;
  const BuildJob& J = b.jobs[batch_job(b, kBpHookHubs, blockIdx.x, local, nblk)];
  const GraphView g = J.g;
  const MemoView m = J.m;
  if (g.tm1) hook_hubs_body<true>(g, m, J.hub_chunk, J.hub_wpv, local);
  else hook_hubs_body<false>(g, m, J.hub_chunk, J.hub_wpv, local);
}
__global__ void __launch_bounds__(256) k_lists_batch(BuildBatch b) {
  uint32_t local, nblk;
  const MemoView m = b.jobs[batch_job(b, kBpLists, blockIdx.x, local, nblk)].m;
  lists_body(m, local);
}
__global__ void __launch_bounds__(256) k_link_batch(BuildBatch b) {
  uint32_t local, nblk;
  const BuildJob& J = b.jobs[batch_job(b, kBpLink, blockIdx.x, local, nblk)];
  const GraphView g = J.g;
  const MemoView m = J.m;
  if (g.tm1) link_body<true>(g, m, local, nblk);
  else link_body<false>(g, m, local, nblk);
}
__global__ void __launch_bounds__(256) k_link_hubs_batch(BuildBatch b) {
  uint32_t local, nblk;
  const BuildJob& J = b.jobs[batch_job(b, kBpLinkHubs, blockIdx.x, local, nblk)];
  const GraphView g = J.g;
  const MemoView m = J.m;
  if (g.tm1) link_hubs_body<true>(g, m, local);
  else link_hubs_body<false>(g, m, local);
}
__global__ void __launch_bounds__(256) k_flatten_batch(BuildBatch b) {
  uint32_t local, nblk;
  const MemoView m = b.jobs[batch_job(b, kBpFlatten, blockIdx.x, local, nblk)].m;
  flatten_body(m, local, nblk);
}
__global__ void __launch_bounds__(256) k_count_batch(BuildBatch b) {
  uint32_t local, nblk;
  const BuildJob& J = b.jobs[batch_job(b, kBpCount, blockIdx.x, local, nblk)];
  const MemoView m = J.m;
  count_body(m, J.count_bv, local);
}
__global__ void __launch_bounds__(256) k_gain0_batch(BuildBatch b) {
  uint32_t local, nblk;
  const MemoView m = b.jobs[batch_job(b, kBpGain0, blockIdx.x, local, nblk)].m;
  gain0_body(m, local, nblk);
}

__global__ void k_fill_u32(uint32_t* p, uint64_t count, uint32_t value) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

// ---- launchers -----------------------------------------------------------

static uint32_t waves_per_vertex(const MemoView& m, uint32_t chunk) {
  return (m.ntiles + chunk - 1) / chunk;
}

static dim3 grid_for(uint32_t n, uint32_t wpv) {
  const uint64_t waves = (uint64_t)n * wpv;
  return dim3((uint32_t)((waves + 3) / 4));
}

void launch_fill_u32(uint32_t* p, uint64_t count, uint32_t value, hipStream_t st) {
  if (!count) return;
  uint64_t blocks = (count + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_fill_u32, dim3((uint32_t)blocks), dim3(256), 0, st, p, count, value);
}

void launch_hook_rows(const GraphView& g, const MemoView& m, hipStream_t st) {
  const dim3 rows((g.n + 3) / 4);
  if (g.tm1)
    hipLaunchKernelGGL(k_hook_rows<true>, rows, dim3(256), 0, st, g, m);
  else
    hipLaunchKernelGGL(k_hook_rows<false>, rows, dim3(256), 0, st, g, m);
}

void launch_hook_hubs(const GraphView& g, const MemoView& m, uint32_t chunk, hipStream_t st) {
  if (!g.nhubs) return;
  const uint32_t wpv = waves_per_vertex(m, chunk);
  if (g.tm1)
    hipLaunchKernelGGL(k_hook_hubs<true>, grid_for(g.nhubs, wpv), dim3(256), 0, st, g, m, chunk, wpv);
  else
    hipLaunchKernelGGL(k_hook_hubs<false>, grid_for(g.nhubs, wpv), dim3(256), 0, st, g, m, chunk, wpv);
}

void launch_lists(const MemoView& m, hipStream_t st) {
  hipLaunchKernelGGL(k_lists, dim3(kSubLists), dim3(256), 0, st, m);
}


void launch_link(const GraphView& g, const MemoView& m, uint32_t blocks, hipStream_t st) {
  if (g.tm1)
    hipLaunchKernelGGL(k_link<true>, dim3(blocks), dim3(256), 0, st, g, m);
  else
    hipLaunchKernelGGL(k_link<false>, dim3(blocks), dim3(256), 0, st, g, m);
}

void launch_link_hubs(const GraphView& g, const MemoView& m, hipStream_t st) {
  if (!g.hub_pieces) return;
  const uint64_t waves = (uint64_t)g.hub_pieces * m.ntiles;
  const dim3 grid((uint32_t)((waves + 3) / 4));
  if (g.tm1)
    hipLaunchKernelGGL(k_link_hubs<true>, grid, dim3(256), 0, st, g, m);
  else
    hipLaunchKernelGGL(k_link_hubs<false>, grid, dim3(256), 0, st, g, m);
}

void launch_flatten(const MemoView& m, uint32_t blocks, hipStream_t st) {
  hipLaunchKernelGGL(k_flatten, dim3(blocks), dim3(256), 0, st, m);
}

void launch_count(const MemoView& m, hipStream_t st) {
  const uint32_t bv = count_block_verts(m);
  const uint32_t vblocks = (m.n + bv - 1) / bv;
  hipLaunchKernelGGL(k_count, dim3(vblocks * m.ntiles), dim3(256), 0, st, m, bv);
}

void launch_gain0(const MemoView& m, uint32_t blocks, hipStream_t st) {
  hipLaunchKernelGGL(k_gain0, dim3(blocks), dim3(256), 0, st, m);
}

// Workgroups of one graph in each labelling phase of a batched launch: the
// single-graph grids, except the list kernels, whose grid scales with the
// graph's (vertex, tile) pairs (64 per workgroup, at most list_blocks).
void build_job_shape(const GraphView& g, const MemoView& m, uint32_t chunk_tiles, uint32_t list_blocks,
                     BuildJob* job, uint32_t* blocks) {
  job->hub_chunk = chunk_tiles;
  job->hub_wpv = waves_per_vertex(m, chunk_tiles);
  job->count_bv = count_block_verts(m);
  const uint64_t pairs = (uint64_t)m.n * m.ntiles;
  const uint32_t lb = (uint32_t)std::min<uint64_t>(list_blocks, std::max<uint64_t>(1, (pairs + 63) / 64));
  blocks[kBpHookRows] = (m.n + 3) / 4;
  blocks[kBpHookHubs] = g.nhubs ? grid_for(g.nhubs, job->hub_wpv).x : 0;
  blocks[kBpLists] = kSubLists;
  blocks[kBpLink] = lb;
  blocks[kBpLinkHubs] = g.hub_pieces ? (uint32_t)(((uint64_t)g.hub_pieces * m.ntiles + 3) / 4) : 0;
  blocks[kBpFlatten] = lb;
  blocks[kBpCount] = ((m.n + job->count_bv - 1) / job->count_bv) * m.ntiles;
  blocks[kBpGain0] = lb;
}

void launch_build_batch(const BuildBatch& b, uint32_t phase, uint32_t blocks, hipStream_t st) {
  if (!blocks) return;
  const dim3 grid(blocks), block(256);
  switch (phase) {
    case kBpHookRows: hipLaunchKernelGGL(k_hook_rows_batch, grid, block, 0, st, b); break;
    case kBpHookHubs: hipLaunchKernelGGL(k_hook_hubs_batch, grid, block, 0, st, b); break;
    case kBpLists: hipLaunchKernelGGL(k_lists_batch, grid, block, 0, st, b); break;
    case kBpLink: hipLaunchKernelGGL(k_link_batch, grid, block, 0, st, b); break;
    case kBpLinkHubs: hipLaunchKernelGGL(k_link_hubs_batch, grid, block, 0, st, b); break;
    case kBpFlatten: hipLaunchKernelGGL(k_flatten_batch, grid, block, 0, st, b); break;
    case kBpCount: hipLaunchKernelGGL(k_count_batch, grid, block, 0, st, b); break;
    case kBpGain0: hipLaunchKernelGGL(k_gain0_batch, grid, block, 0, st, b); break;
    default: break;
  }
}

}  // namespace infuse
