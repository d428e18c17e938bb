// sigma(S) without a memo (Algorithm 4, RandCas, on all R samples at once):
// a level-synchronous breadth-first search from S over the live edges of
// every sample, for parameter sets whose memo would not fit.
//
// Per (vertex, 256-column tile) the visited set V and the frontier F hold
// one bit per column, as four 64-bit words: bit l of word i is column
// 4l + i of the tile (the layout of a ballot over the wavefront's lanes).
// A level visits, for every item (vertex, tile) of the frontier list, the
// candidate edges of the tile (tile prefilter), and ors the columns where
// the edge is live and the vertex is in the frontier into V and the next
// frontier N of the neighbour; a neighbour that gains columns in the tile is
// marked in a bitmap of items, which a second kernel turns into the next
// frontier list (in item order), so only (vertex, tile) pairs whose
// frontier is not empty are visited.  V and N are written only by atomics
// while a level runs; F is only read, then cleared by the wavefront that
// owns the item (for an item split into pieces, by the listing kernel after
// the level), so both frontier sets are all zero again once a search ends.
// The count is the number of bits the search sets in V, summed from the
// atomics' old values: sum over samples of |R_r(S)|, seeds included (beyond
// the set V starts from).
#include <algorithm>

#include "common.h"
#include "direct.h"
#include "tile.h"

namespace infuse {

// Columns of tile t that are samples (q < R), in the ballot layout.
__device__ inline uint64_t valid_word(uint32_t R, uint32_t t, uint32_t i) {
  uint64_t w = 0;
  for (uint32_t l = 0; l < 64; ++l) w |= (uint64_t)(t * kTile + 4 * l + i < R) << l;
  return w;
}

// New bits of a copy's count: summed over the wavefront, one atomic add by
// lane 0 into one of the copy's slots.
__device__ inline void add_count(const BfsView& b, uint32_t copy, uint32_t pc) {
  uint32_t c = pc;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off);
  if ((threadIdx.x & 63) == 0 && c)
    atomicAdd(&b.counts[(uint64_t)copy * kCountSlots + blockIdx.x % kCountSlots], (unsigned long long)c);
}

// Seeds (virtual ids): every sample column of every tile is visited; the
// columns where the seed was not visited before join the frontier and the
// count (V may start from a covered set, whose vertices add nothing).  The
// items (seed, tile) are appended to the first list, kPieces entries for a
// split row: positions from a scan over the wavefront, one add per
// wavefront.
__global__ void k_bfs_seed(GraphView g, MemoView m, BfsView b, const uint32_t* S, uint32_t len) {
  const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t lane = threadIdx.x & 63;
  const bool act = k < (uint64_t)len * m.ntiles * 4;
  uint32_t v = 0, t = 0, cnt = 0;
  if (act) {
    const uint32_t s = (uint32_t)(k / (m.ntiles * 4)), r = (uint32_t)(k % (m.ntiles * 4)), i = r % 4;
    v = S[s];
    t = r / 4;
    const uint64_t w = valid_word(m.R, t, i);
    const uint64_t at = ((uint64_t)v * m.ntiles + t) * 4 + i;
    const uint64_t nb = w & ~(uint64_t)atomicOr((unsigned long long*)&b.V[at], (unsigned long long)w);
    if (nb) {
      atomicOr((unsigned long long*)&b.N[at], (unsigned long long)nb);
      atomicAdd(&b.counts[(uint64_t)(v / b.gn) * kCountSlots + k % kCountSlots], (unsigned long long)__popcll(nb));
    }
    if (i == 0) {
      const uint32_t gv = v % b.gn;
      cnt = b.pieces > 1 && g.row_ptr[gv + 1] - g.row_ptr[gv] > kSplitArcs ? b.pieces : 1u;
    }
  }
  uint32_t incl = cnt;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(incl, off);
    if (lane >= (uint32_t)off) incl += y;
  }
  const uint32_t total = __shfl(incl, 63);
  if (!total) return;
  uint32_t base = 0;
  if (lane == 63) base = atomicAdd(&b.lcount[1], total);
  base = __shfl(base, 63);
  const uint32_t item = v * m.ntiles + t;
  for (uint32_t p = 0; p < cnt; ++p) b.next[base + incl - cnt + p] = item | (cnt > 1 ? p << kPieceShift : 0u);
}

// One level.  A wavefront takes list entries, each an item (frontier
// vertex, tile) or a piece of one; for each candidate edge of the item's
// tile (of the piece's arcs) it forms the 256-bit set of columns where the
// edge is live and the vertex is in the frontier, and parks it in four
// lanes (lane 4j + i holds word i of the j-th pending target).  Sixteen
// targets are then updated at once: each lane ors its word into V (the
// atomic's old value decides which bits are new, so every bit is counted
// once) and the new ones into N, and one lane per target that gained
// columns marks it in the next frontier's bitmap.  An unsplit item's
// frontier words are cleared once read: each (vertex, tile) is one item of
// the level.
template <bool PER_EDGE>
__global__ void __launch_bounds__(256) k_bfs_level(GraphView g, MemoView m, BfsView b, uint32_t level) {
  if (blockIdx.x == 0 && threadIdx.x == 0) b.lcount[(level + 2) % 3] = 0;  // the next level's next list
  const uint32_t ncur = b.lcount[level % 3];
  if (ncur == 0) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) atomicMax(b.levels, level);
  const uint32_t lane = threadIdx.x & 63, wsel = lane & 3, pslot = lane >> 2;
  // item ids (vertex * ntiles + tile) fit in 32 bits (checked by the host);
  // the entry index is wave-uniform.  The item's frontier words, row bounds
  // and tile X are requested together, and the next entry one entry ahead.
  // Listed items have frontier bits (seeds aside), so none is skipped: a
  // test would defer the loads past it.
  const uint64_t nw = gridDim.x * 4;
  const uint64_t items = ncur;
  uint32_t pc = 0;        // new bits set by this lane for copy pcopy
  uint32_t pcopy = 0;
  uint64_t s_items = 0, s_arcs = 0, s_live = 0;  // work counts of this wavefront (kept when b.stats)
  const uint64_t it0 = blockIdx.x * 4 + uni(threadIdx.x >> 6);
  uint32_t en = b.cur[min(it0, items - 1)];
  for (uint64_t it = it0; it < items; it += nw) {
    const uint32_t e0 = uni(en);
    en = b.cur[min(it + nw, items - 1)];
    const uint32_t item = b.pieces > 1 ? e0 & ((1u << kPieceShift) - 1) : e0;
    const uint32_t piece = b.pieces > 1 ? e0 >> kPieceShift : 0u;
    const uint32_t vv = item / m.ntiles, t = item % m.ntiles;
    const uint32_t v = vv % b.gn, cb = vv - v;  // graph vertex, first virtual id of its copy
    if (cb / b.gn != pcopy) {  // counts are added when the copy changes, and at the end
      if (__ballot(pc != 0)) add_count(b, pcopy, pc);
      pc = 0;
      pcopy = cb / b.gn;
    }
    uint64_t* fw = b.F + ((uint64_t)vv * m.ntiles + t) * 4;
    const uint64_t f0 = fw[0], f1 = fw[1], f2 = fw[2], f3 = fw[3];
    const uint32_t rb = g.row_ptr[v], re = g.row_ptr[v + 1];
    const uint4 x4 = load_tile_x(m, t, lane);
    uint32_t beg = uni(rb), end = uni(re);
    const bool split = b.pieces > 1 && end - beg > kSplitArcs;
    // a split item's frontier words are cleared after the level, once every
    // piece has read them
    if (!split) {
      if (lane < 4) fw[lane] = 0;
      ++s_items;
    } else {
      s_items += piece == 0;
      const uint32_t len = ((end - beg + b.pieces - 1) / b.pieces + kWave - 1) & ~(uint32_t)(kWave - 1);
      beg = min(end, beg + piece * len);
      end = min(end, beg + len);
    }
    uint32_t fb[4];
    fb[0] = (uint32_t)(f0 >> lane) & 1u;
    fb[1] = (uint32_t)(f1 >> lane) & 1u;
    fb[2] = (uint32_t)(f2 >> lane) & 1u;
    fb[3] = (uint32_t)(f3 >> lane) & 1u;
    TileCtx tc;
    tile_from_x(m, t, lane, x4, m.kshift, tc, PER_EDGE);
    const bool inreg = !split && end - beg <= (uint32_t)kWave;
    s_arcs += end - beg;
    uint32_t rcol = kInvalid, rh = 0, rtm1 = 0;
    if (inreg && beg + lane < end) {
      const uint2 e = m.edges[beg + lane];
      rcol = e.x;
      rh = e.y;
      if (PER_EDGE) rtm1 = g.tm1[beg + lane];
    }
    uint32_t pu = 0;   // this lane's pending target (graph id)
    uint64_t pm = 0;   // word wsel of its live frontier columns
    uint32_t np = 0;   // pending targets (uniform)
    auto flush = [&]() {
      uint64_t nb = 0;
      if (pm) {
        const uint64_t at = ((uint64_t)(cb + pu) * m.ntiles + t) * 4 + wsel;
        nb = pm & ~(uint64_t)atomicOr((unsigned long long*)&b.V[at], (unsigned long long)pm);
        if (nb) atomicOr((unsigned long long*)&b.N[at], (unsigned long long)nb);
      }
      pc += (uint32_t)__popcll(nb);
      const uint64_t hit = __ballot(nb != 0);
      if (wsel == 0 && pslot < np && ((hit >> lane) & 0xFull)) {
        const uint32_t ui = (cb + pu) * m.ntiles + t;  // item (target, tile) of the next level
        atomicOr((unsigned long long*)&b.nbits[ui >> 6], 1ull << (ui & 63));
      }
      np = 0;
      pm = 0;
    };
    for_candidates<PER_EDGE, false>(
        g, m, v, beg, end, end, lane, inreg, rcol, rh, rtm1, tc, [&](uint32_t u, uint32_t h, uint32_t tt, bool) {
          uint32_t lb[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) lb[i] = (fb[i] && tc.valid[i] && (h ^ tc.x[i]) <= tt) ? 1u : 0u;
          const uint64_t w0 = __ballot(lb[0]), w1 = __ballot(lb[1]), w2 = __ballot(lb[2]), w3 = __ballot(lb[3]);
          if (!(w0 | w1 | w2 | w3)) return;
          ++s_live;
          if (pslot == np) {
            pu = u;
            pm = wsel == 0 ? w0 : wsel == 1 ? w1 : wsel == 2 ? w2 : w3;
          }
          if (++np == kWave / 4) flush();
        });
    if (np) flush();
  }
  if (__ballot(pc != 0)) add_count(b, pcopy, pc);
  if (b.stats) {  // block sums in LDS, then one add per counter and block
    __shared__ unsigned long long ws[3];
    if (threadIdx.x < 3) ws[threadIdx.x] = 0;
    __syncthreads();
    if (lane == 0 && (s_items | s_arcs)) {  // a wavefront may have run pieces of split items only
      atomicAdd(&ws[0], (unsigned long long)s_items);
      atomicAdd(&ws[1], (unsigned long long)s_arcs);
      atomicAdd(&ws[2], (unsigned long long)s_live);
    }
    __syncthreads();
    if (threadIdx.x < 3 && ws[threadIdx.x])
      atomicAdd(&b.stats[(blockIdx.x % kCountSlots) * 3 + threadIdx.x], ws[threadIdx.x]);
  }
}

// The next frontier list from the bitmap left by level `level` (item
// order; the bitmap is cleared; kPieces entries for an item of a split
// row): two bitmap words per thread, positions from a scan over the
// workgroup and one atomic add per workgroup (one add per wavefront made the
// adds of a launch contend on the list size).  It also clears the frontier
// words of the level's split items, which their pieces left in place.
constexpr uint32_t kCompactWords = 2;

__global__ void __launch_bounds__(256) k_bfs_compact(BfsView b, uint32_t level) {
  const uint32_t ncur = b.lcount[level % 3];
  if (ncur == 0) return;  // an empty level marks nothing
  __shared__ uint32_t wsum[4];
  __shared__ uint32_t base_sh;
  const uint64_t gtid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b.pieces > 1) {
    // piece 1 is listed once per split item; the list is read four entries
    // per load, two loads in flight per thread
    const uint64_t nthr = (uint64_t)gridDim.x * blockDim.x;
    auto clear = [&](uint32_t e) {
      if (e >> kPieceShift == 1) {
        uint64_t* fw = b.F + (uint64_t)(e & ((1u << kPieceShift) - 1)) * 4;
        fw[0] = 0;
        fw[1] = 0;
        fw[2] = 0;
        fw[3] = 0;
      }
    };
    const uint64_t quads = ncur / 4;
    const uint4* cq = reinterpret_cast<const uint4*>(b.cur);
    for (uint64_t k = gtid; k < quads; k += 2 * nthr) {
      const uint4 a = cq[k];
      const uint4 c2 = k + nthr < quads ? cq[k + nthr] : make_uint4(0, 0, 0, 0);
      clear(a.x);
      clear(a.y);
      clear(a.z);
      clear(a.w);
      clear(c2.x);
      clear(c2.y);
      clear(c2.z);
      clear(c2.w);
    }
    if (gtid < ncur % 4) clear(b.cur[quads * 4 + gtid]);
  }
  const uint64_t words = ((uint64_t)b.n * b.ntiles + 63) / 64;
  const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint64_t w0 = gtid * kCompactWords;
  uint64_t w[kCompactWords], hm[kCompactWords];
  uint32_t c = 0;
#pragma unroll
  for (uint32_t k = 0; k < kCompactWords; ++k) {
    w[k] = w0 + k < words ? b.nbits[w0 + k] : 0ull;
    if (w[k]) b.nbits[w0 + k] = 0;
    hm[k] = b.pieces > 1 && w0 + k < words ? w[k] & b.hubmask[w0 + k] : 0ull;
    c += (uint32_t)__popcll(w[k] & ~hm[k]) + b.pieces * (uint32_t)__popcll(hm[k]);
  }
  uint32_t incl = c;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(incl, off);
    if (lane >= (uint32_t)off) incl += y;
  }
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t total = 0;
    for (uint32_t i = 0; i < blockDim.x / 64; ++i) {
      const uint32_t x = wsum[i];
      wsum[i] = total;  // exclusive prefix of the wavefronts
      total += x;
    }
    base_sh = total ? atomicAdd(&b.lcount[(level + 1) % 3], total) : 0u;
  }
  __syncthreads();
  uint32_t pos = base_sh + wsum[wv] + incl - c;
#pragma unroll
  for (uint32_t k = 0; k < kCompactWords; ++k) {
    uint64_t x = w[k];
    while (x) {
      const uint32_t bit = (uint32_t)__builtin_ctzll(x);
      const uint32_t item = (uint32_t)((w0 + k) * 64 + bit);
      x &= x - 1;
      if ((hm[k] >> bit) & 1ull)
        for (uint32_t p = 0; p < b.pieces; ++p) b.next[pos++] = item | p << kPieceShift;
      else
        b.next[pos++] = item;
    }
  }
}

// Bit (vertex * ntiles + t) is set when the vertex (its graph vertex, for
// a copy) has more than kSplitArcs arcs.
__global__ void k_bfs_hubmask(GraphView g, BfsView b, uint64_t* mask) {
  const uint64_t items = (uint64_t)b.n * b.ntiles, words = (items + 63) / 64;
  for (uint64_t wi = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; wi < words;
       wi += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t bits = 0;
    for (uint32_t k = 0; k < 64 && wi * 64 + k < items; ++k) {
      const uint32_t v = (uint32_t)((wi * 64 + k) / b.ntiles % b.gn);
      if (g.row_ptr[v + 1] - g.row_ptr[v] > kSplitArcs) bits |= 1ull << k;
    }
    mask[wi] = bits;
  }
}

__global__ void k_bfs_replicate(const uint64_t* src, uint64_t* V, uint64_t words) {
  const uint32_t c = blockIdx.y;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < words; k += (uint64_t)gridDim.x * blockDim.x)
    V[(uint64_t)c * words + k] = src[k];
}

// ---- launchers ---------------------------------------------------------------

void launch_bfs_seed(const GraphView& g, const MemoView& m, const BfsView& b, const uint32_t* S, uint32_t len,
                     hipStream_t st) {
  const uint64_t k = (uint64_t)len * m.ntiles * 4;
  if (k) hipLaunchKernelGGL(k_bfs_seed, dim3((uint32_t)((k + 255) / 256)), dim3(256), 0, st, g, m, b, S, len);
}

void launch_bfs_hubmask(const GraphView& g, const BfsView& b, uint64_t* mask, hipStream_t st) {
  const uint64_t words = ((uint64_t)b.n * b.ntiles + 63) / 64;
  if (words)
    hipLaunchKernelGGL(k_bfs_hubmask, dim3((uint32_t)std::min<uint64_t>(4096, (words + 255) / 256)), dim3(256), 0,
                       st, g, b, mask);
}

// A fixed grid (the frontier size is known only on the device): four
// rounds of resident wavefronts, striding over the (vertex, tile) items.
// Larger grids pay per-wavefront set-up and count adds for nothing.
void launch_bfs_level(const GraphView& g, const MemoView& m, const BfsView& b, uint32_t level, hipStream_t st) {
  constexpr uint32_t kBlocks = 8192;
  if (g.tm1)
    hipLaunchKernelGGL(k_bfs_level<true>, dim3(kBlocks), dim3(256), 0, st, g, m, b, level);
  else
    hipLaunchKernelGGL(k_bfs_level<false>, dim3(kBlocks), dim3(256), 0, st, g, m, b, level);
}

void launch_bfs_compact(const BfsView& b, uint32_t level, hipStream_t st) {
  const uint64_t words = ((uint64_t)b.n * b.ntiles + 63) / 64;
  const uint64_t per_block = 256ull * kCompactWords;
  hipLaunchKernelGGL(k_bfs_compact, dim3((uint32_t)((words + per_block - 1) / per_block)), dim3(256), 0, st, b, level);
}

void launch_bfs_replicate(const uint64_t* src, uint64_t* V, uint64_t words, uint32_t copies, hipStream_t st) {
  if (!copies || !words) return;
  const uint32_t bx = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(256, (words + 255) / 256));
  hipLaunchKernelGGL(k_bfs_replicate, dim3(bx, copies), dim3(256), 0, st, src, V, words);
}

}  // namespace infuse
