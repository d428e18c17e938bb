// sigma(S) without a memo (Algorithm 4, RandCas, on all R samples at once):
// a level-synchronous breadth-first search from S over the live edges of
// every sample, for parameter sets whose memo would not fit.
//
// Per (vertex, 256-column tile) the visited set V and the frontier F hold
// one bit per column, as four 64-bit words: bit l of word i is column
// 4l + i of the tile (the layout of a ballot over the wavefront's lanes).
// A level visits, for every vertex of the frontier list and every tile where
// its frontier is not empty, the candidate edges of the tile (tile
// prefilter), and ors the columns where the edge is live and the vertex is
// in the frontier into V and the next frontier N of the neighbour; a
// neighbour that gains columns joins the next frontier list once (level
// stamp).  V and N are written only by atomics while a level runs (stale
// reads of V only cause redundant atomics); F is read-only.  The count is
// the number of set bits of V: sum over samples of |R_r(S)|, seeds included.
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

// Seeds (virtual ids): every sample column of every tile is visited; the
// columns where the seed was not visited before join the frontier (V may
// start from a covered set, whose vertices add nothing).
__global__ void k_bfs_seed(MemoView m, BfsView b, const uint32_t* S, uint32_t len) {
  const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (uint64_t)len * m.ntiles * 4) return;
  const uint32_t s = (uint32_t)(k / (m.ntiles * 4)), r = (uint32_t)(k % (m.ntiles * 4));
  const uint32_t v = S[s], t = r / 4, i = r % 4;
  const uint64_t w = valid_word(m.R, t, i);
  const uint64_t old = b.V[((uint64_t)v * m.ntiles + t) * 4 + i];
  b.V[((uint64_t)v * m.ntiles + t) * 4 + i] = old | w;
  b.N[((uint64_t)v * m.ntiles + t) * 4 + i] = w & ~old;
  if (r == 0) {
    b.stamp[v] = 1;
    b.next[s] = v;
  }
}

template <bool PER_EDGE>
__global__ void __launch_bounds__(256) k_bfs_level(GraphView g, MemoView m, BfsView b, const uint32_t* ncur_p,
                                                   uint32_t level) {
  const uint32_t ncur = *ncur_p;
  if (ncur == 0) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) atomicMax(b.levels, level);
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t nw = (uint64_t)gridDim.x * 4;
  const uint64_t items = (uint64_t)ncur * m.ntiles;
  for (uint64_t it = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6); it < items; it += nw) {
    const uint32_t vv = uni(b.cur[it / m.ntiles]), t = (uint32_t)(it % m.ntiles);
    const uint32_t v = vv % b.gn, cb = vv - v;  // graph vertex, first virtual id of its copy
    const uint64_t* fw = b.F + ((uint64_t)vv * m.ntiles + t) * 4;
    const uint64_t f0 = fw[0], f1 = fw[1], f2 = fw[2], f3 = fw[3];
    if (!(f0 | f1 | f2 | f3)) continue;
    uint32_t fb[4];
    fb[0] = (uint32_t)(f0 >> lane) & 1u;
    fb[1] = (uint32_t)(f1 >> lane) & 1u;
    fb[2] = (uint32_t)(f2 >> lane) & 1u;
    fb[3] = (uint32_t)(f3 >> lane) & 1u;
    TileCtx tc;
    tile_from_x(m, t, lane, load_tile_x(m, t, lane), m.kshift, tc, PER_EDGE);
    const uint32_t beg = uni(g.row_ptr[v]), end = uni(g.row_ptr[v + 1]);
    const bool inreg = end - beg <= (uint32_t)kWave;
    uint32_t rcol = kInvalid, rh = 0, rtm1 = 0;
    if (inreg && beg + lane < end) {
      const uint2 e = m.edges[beg + lane];
      rcol = e.x;
      rh = e.y;
      if (PER_EDGE) rtm1 = g.tm1[beg + lane];
    }
    for_candidates<PER_EDGE, false>(
        g, m, v, beg, end, end, lane, inreg, rcol, rh, rtm1, tc, [&](uint32_t u, uint32_t h, uint32_t tt, bool) {
          uint32_t lb[4];
          bool any = false;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            lb[i] = (fb[i] && tc.valid[i] && (h ^ tc.x[i]) <= tt) ? 1u : 0u;
            any = any || lb[i];
          }
          if (!__ballot(any)) return;
          const uint32_t uv = cb + u;  // virtual id of the neighbour
          uint64_t* vw = b.V + ((uint64_t)uv * m.ntiles + t) * 4;
          const uint64_t v0 = vw[0], v1 = vw[1], v2 = vw[2], v3 = vw[3];
          const uint64_t n0 = __ballot(lb[0] && !((v0 >> lane) & 1u));
          const uint64_t n1 = __ballot(lb[1] && !((v1 >> lane) & 1u));
          const uint64_t n2 = __ballot(lb[2] && !((v2 >> lane) & 1u));
          const uint64_t n3 = __ballot(lb[3] && !((v3 >> lane) & 1u));
          if (!(n0 | n1 | n2 | n3)) return;
          if (lane == 0) {
            uint64_t* nw4 = b.N + ((uint64_t)uv * m.ntiles + t) * 4;
            const uint64_t nn[4] = {n0, n1, n2, n3};
            for (int i = 0; i < 4; ++i)
              if (nn[i]) {
                atomicOr((unsigned long long*)&vw[i], (unsigned long long)nn[i]);
                atomicOr((unsigned long long*)&nw4[i], (unsigned long long)nn[i]);
              }
            if (atomicMax(&b.stamp[uv], level + 1) < level + 1) b.next[atomicAdd(b.ncount, 1u)] = uv;
          }
        });
  }
}

// Clears the frontier words of this level's vertices.
__global__ void k_bfs_clear(uint64_t* F, const uint32_t* cur, const uint32_t* ncur_p, uint32_t ntiles) {
  const uint64_t total = (uint64_t)(*ncur_p) * ntiles * 4;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t v = cur[k / (ntiles * 4)];
    F[(uint64_t)v * ntiles * 4 + k % (ntiles * 4)] = 0;
  }
}

__global__ void k_bfs_count(const uint64_t* V, uint64_t words, unsigned long long* out) {
  uint64_t c = 0;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < words; k += (uint64_t)gridDim.x * blockDim.x)
    c += (uint64_t)__popcll(V[k]);
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(out, (unsigned long long)c);
}

// Per-copy counts: block (x, c) sums a stretch of copy c's words.
__global__ void k_bfs_count_copies(const uint64_t* V, uint64_t words, unsigned long long* out) {
  const uint32_t c = blockIdx.y;
  const uint64_t* p = V + (uint64_t)c * words;
  uint64_t cnt = 0;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < words; k += (uint64_t)gridDim.x * blockDim.x)
    cnt += (uint64_t)__popcll(p[k]);
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off);
  if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(&out[c], (unsigned long long)cnt);
}

__global__ void k_bfs_replicate(const uint64_t* src, uint64_t* V, uint64_t words) {
  const uint32_t c = blockIdx.y;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < words; k += (uint64_t)gridDim.x * blockDim.x)
    V[(uint64_t)c * words + k] = src[k];
}

// ---- launchers ---------------------------------------------------------------

void launch_bfs_seed(const MemoView& m, const BfsView& b, const uint32_t* S, uint32_t len, hipStream_t st) {
  const uint64_t k = (uint64_t)len * m.ntiles * 4;
  if (k) hipLaunchKernelGGL(k_bfs_seed, dim3((uint32_t)((k + 255) / 256)), dim3(256), 0, st, m, b, S, len);
}

// Fixed grids (the frontier size is known only on the device): enough
// wavefronts to fill the device, striding over the (vertex, tile) items.
void launch_bfs_level(const GraphView& g, const MemoView& m, const BfsView& b, const uint32_t* ncur,
                      uint32_t level, hipStream_t st) {
  constexpr uint32_t kBlocks = 16384;
  if (g.tm1)
    hipLaunchKernelGGL(k_bfs_level<true>, dim3(kBlocks), dim3(256), 0, st, g, m, b, ncur, level);
  else
    hipLaunchKernelGGL(k_bfs_level<false>, dim3(kBlocks), dim3(256), 0, st, g, m, b, ncur, level);
}

void launch_bfs_clear(uint64_t* F, const uint32_t* cur, const uint32_t* ncur, uint32_t ntiles, hipStream_t st) {
  hipLaunchKernelGGL(k_bfs_clear, dim3(1024), dim3(256), 0, st, F, cur, ncur, ntiles);
}

void launch_bfs_count(const uint64_t* V, uint64_t words, unsigned long long* out, hipStream_t st) {
  const uint32_t blocks = (uint32_t)std::min<uint64_t>(8192, (words + 255) / 256);
  hipLaunchKernelGGL(k_bfs_count, dim3(std::max(1u, blocks)), dim3(256), 0, st, V, words, out);
}

void launch_bfs_count_copies(const uint64_t* V, uint64_t words, uint32_t copies, unsigned long long* out,
                             hipStream_t st) {
  if (!copies) return;
  const uint32_t bx = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(256, (words + 255) / 256));
  hipLaunchKernelGGL(k_bfs_count_copies, dim3(bx, copies), dim3(256), 0, st, V, words, out);
}

void launch_bfs_replicate(const uint64_t* src, uint64_t* V, uint64_t words, uint32_t copies, hipStream_t st) {
  if (!copies || !words) return;
  const uint32_t bx = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(256, (words + 255) / 256));
  hipLaunchKernelGGL(k_bfs_replicate, dim3(bx, copies), dim3(256), 0, st, src, V, words);
}

}  // namespace infuse
