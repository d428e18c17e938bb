// Hash edge sampler set-up (Section III-A, Eq. 1-2).
//
// k_edge_hash   h_e = fmix32(s ^ key32(u, v)) for every CSR slot (the key of
//               the ordered pair for an arc of a directed graph), stored
//               beside the neighbour id ({v, h_e}, 8 bytes per slot), since
//               the paper precomputes the m hashes once instead of hashing
//               during traversal.
// k_x_sort_*    X_r = fmix32(s + r) for r < R and the column order: columns
//               hold the simulations sorted by X (ascending).  X values are
//               distinct (fmix32 is a bijection and s + r takes R distinct
//               values), so the order is unique.
#include "common.h"

namespace infuse {

// One thread per CSR slot (its row from g.src), strided over the `nblk`
// workgroups: consecutive threads read and write consecutive slots.
__device__ inline void edge_hash_body(const GraphView& g, uint32_t seed, uint2* edges, uint32_t bid, uint32_t nblk) {
  const uint32_t stride = nblk * blockDim.x;
  for (uint32_t j = bid * blockDim.x + threadIdx.x; j < g.nnz; j += stride) {
    const uint32_t u = g.src[j], v = g.col[j];
    edges[j] = make_uint2(v, fmix32(seed ^ (g.directed ? arc_key32(u, v, g.n) : edge_key32(u, v, g.n))));
  }
}

__global__ void __launch_bounds__(256) k_edge_hash(GraphView g, uint32_t seed, uint2* edges) {
  edge_hash_body(g, seed, edges, blockIdx.x, gridDim.x);
}

constexpr int kSortChunk = 4096;  // elements sorted per block in LDS

// Sorts chunk blockIdx.x of the (X_r, r) pairs; pads with all-ones keys.  A
// single chunk sorts only the next power of two above R.
__global__ void __launch_bounds__(1024) k_x_sort_chunk(uint32_t seed, uint32_t R, uint64_t* out) {
  __shared__ uint64_t a[kSortChunk];
  const uint32_t base = blockIdx.x * kSortChunk;
  uint32_t len = kSortChunk;
  if (gridDim.x == 1)
    while (len > 2 && len / 2 >= R) len /= 2;
  for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) {
    const uint32_t r = base + i;
    a[i] = r < R ? ((uint64_t)fmix32(seed + r) << 32) | r : ~0ull;
  }
  __syncthreads();
  for (uint32_t k = 2; k <= len; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) {
        const uint32_t ixj = i ^ j;
        if (ixj > i) {
          const bool asc = (i & k) == 0;
          const uint64_t x = a[i], y = a[ixj];
          if ((x > y) == asc) {
            a[i] = y;
            a[ixj] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  for (uint32_t i = threadIdx.x; i < kSortChunk; i += blockDim.x) out[base + i] = i < len ? a[i] : ~0ull;
}

// R <= kSortChunk: one workgroup (of any size) sorts and writes the column
// order and the padding columns directly.
__device__ inline void x_sort_single_body(uint32_t seed, uint32_t R, uint32_t Rs, uint32_t* xs, uint32_t* inv,
                                          uint32_t* pos) {
  __shared__ uint64_t a[kSortChunk];
  uint32_t len = kSortChunk;
  while (len > 2 && len / 2 >= R) len /= 2;
  for (uint32_t i = threadIdx.x; i < len; i += blockDim.x)
    a[i] = i < R ? ((uint64_t)fmix32(seed + i) << 32) | i : ~0ull;
  __syncthreads();
  for (uint32_t k = 2; k <= len; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) {
        const uint32_t ixj = i ^ j;
        if (ixj > i) {
          const bool asc = (i & k) == 0;
          const uint64_t x = a[i], y = a[ixj];
          if ((x > y) == asc) {
            a[i] = y;
            a[ixj] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  for (uint32_t q = threadIdx.x; q < Rs; q += blockDim.x) {
    if (q < R) {
      const uint64_t key = a[q];
      const uint32_t r = (uint32_t)key;
      xs[q] = (uint32_t)(key >> 32);
      inv[q] = r;
      pos[r] = q;
    } else {
      xs[q] = kInvalid;
      inv[q] = kInvalid;
    }
  }
}

__global__ void __launch_bounds__(1024) k_x_sort_single(uint32_t seed, uint32_t R, uint32_t Rs, uint32_t* xs,
                                                        uint32_t* inv, uint32_t* pos) {
  x_sort_single_body(seed, R, Rs, xs, inv, pos);
}

// R <= kCountSortMax: one workgroup of 1024 threads sorts by counting.  The
// X values are distinct and spread evenly, so their top kCountBits bits
// split them into buckets of about one value: count per bucket (LDS
// atomics), scan the counts into offsets, place each simulation at its
// bucket's next slot, then order the few values of each bucket by X.  The
// X of a simulation is recomputed where needed instead of stored.
constexpr uint32_t kCountBits = 13;
constexpr uint32_t kCountSortMax = 1u << kCountBits;
__global__ void __launch_bounds__(1024) k_x_sort_count(uint32_t seed, uint32_t R, uint32_t Rs, uint32_t* xs,
                                                       uint32_t* inv, uint32_t* pos) {
  constexpr uint32_t NB = kCountSortMax, kPerT = NB / 1024;
  __shared__ uint32_t cnt[NB];   // counts, then running slots, then bucket ends
  __shared__ uint32_t slot[NB];  // simulations in sorted order
  __shared__ uint32_t part[1024 / 64];
  const uint32_t tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (uint32_t i = tid; i < NB; i += 1024) cnt[i] = 0;
  __syncthreads();
  for (uint32_t r = tid; r < R; r += 1024) atomicAdd(&cnt[fmix32(seed + r) >> (32 - kCountBits)], 1u);
  __syncthreads();
  // exclusive scan: each thread its kPerT consecutive buckets, then the
  // workgroup over the threads' sums
  uint32_t loc[kPerT], sum = 0;
#pragma unroll
  for (uint32_t k = 0; k < kPerT; ++k) {
    loc[k] = sum;
    sum += cnt[tid * kPerT + k];
  }
  uint32_t incl = sum;
#pragma unroll
  for (uint32_t off = 1; off < 64; off <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int)incl, off);
    if (lane >= off) incl += y;
  }
  if (lane == 63) part[wv] = incl;
  __syncthreads();
  uint32_t base = 0;
  for (uint32_t w = 0; w < wv; ++w) base += part[w];
  base += incl - sum;
#pragma unroll
  for (uint32_t k = 0; k < kPerT; ++k) cnt[tid * kPerT + k] = base + loc[k];
  __syncthreads();
  for (uint32_t r = tid; r < R; r += 1024) slot[atomicAdd(&cnt[fmix32(seed + r) >> (32 - kCountBits)], 1u)] = r;
  __syncthreads();
  // cnt[b] is now the end of bucket b; insertion sort of each bucket by X
  for (uint32_t b = tid; b < NB; b += 1024) {
    const uint32_t beg = b ? cnt[b - 1] : 0u, end = cnt[b];
    for (uint32_t i = beg + 1; i < end; ++i) {
      const uint32_t r = slot[i], x = fmix32(seed + r);
      uint32_t j = i;
      while (j > beg && fmix32(seed + slot[j - 1]) > x) {
        slot[j] = slot[j - 1];
        --j;
      }
      slot[j] = r;
    }
  }
  __syncthreads();
  for (uint32_t q = tid; q < Rs; q += 1024) {
    if (q < R) {
      const uint32_t r = slot[q];
      xs[q] = fmix32(seed + r);
      inv[q] = r;
      if (r < R) pos[r] = q;  // always: every simulation holds one slot
    } else {
      xs[q] = kInvalid;
      inv[q] = kInvalid;
    }
  }
}

// Batched set-up of many memos: per graph, one workgroup sorts X (when
// R <= kSortChunk; larger R is sorted by the single-graph kernels first),
// the next ones hash the edges and the rest clear the mask arrays.
__global__ void __launch_bounds__(256) k_prep_batch(BuildBatch b) {
  uint32_t local, nblk;
  const uint32_t j = batch_job(b, kBpPrep, blockIdx.x, local, nblk);
  const BuildJob& J = b.jobs[j];
  const uint32_t sort_blocks = J.sort_blocks, hash_blocks = J.hash_blocks;
  if (local < sort_blocks) {
    x_sort_single_body(J.seed, J.m.R, J.m.Rs, J.xs, J.inv, J.pos);
    return;
  }
  local -= sort_blocks;
  if (local < hash_blocks) {
    const GraphView g = J.g;
    edge_hash_body(g, J.seed, J.edges, local, hash_blocks);
    return;
  }
  local -= hash_blocks;
  const uint32_t fb = nblk - sort_blocks - hash_blocks;
  uint32_t* p = J.m.tmask;
  const uint64_t words = J.fill_words;
  for (uint64_t i = (uint64_t)local * blockDim.x + threadIdx.x; i < words; i += (uint64_t)fb * blockDim.x) p[i] = 0u;
}

// Global rank of each element = its rank in its own sorted chunk plus the
// number of smaller X in every other chunk (binary search).
__global__ void __launch_bounds__(256) k_x_sort_merge(const uint64_t* sorted, uint32_t R,
                                                      uint32_t nchunks, uint32_t* xs, uint32_t* inv,
                                                      uint32_t* pos) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t padded = nchunks * kSortChunk;
  if (i >= padded) return;
  const uint64_t key = sorted[i];
  if (key == ~0ull) return;
  const uint32_t x = (uint32_t)(key >> 32), r = (uint32_t)key;
  const uint32_t c = i / kSortChunk;
  uint32_t rank = i - c * kSortChunk;
  for (uint32_t d = 0; d < nchunks; ++d) {
    if (d == c) continue;
    const uint64_t* s = sorted + (uint64_t)d * kSortChunk;
    uint32_t lo = 0, hi = kSortChunk;  // pads (all ones) sort last and are never smaller
    while (lo < hi) {
      const uint32_t mid = (lo + hi) >> 1;
      if ((s[mid] >> 32) < x && s[mid] != ~0ull) lo = mid + 1; else hi = mid;
    }
    rank += lo;
  }
  xs[rank] = x;
  inv[rank] = r;
  pos[r] = rank;
}

__global__ void k_x_pad(uint32_t R, uint32_t Rs, uint32_t* xs, uint32_t* inv) {
  const uint32_t q = R + blockIdx.x * blockDim.x + threadIdx.x;
  if (q < Rs) {
    xs[q] = kInvalid;
    inv[q] = kInvalid;
  }
}

void launch_edge_hash(const GraphView& g, uint32_t seed, uint2* edges, hipStream_t st) {
  uint32_t blocks = (g.nnz + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(k_edge_hash, dim3(blocks), dim3(256), 0, st, g, seed, edges);
}

void launch_prep_batch(const BuildBatch& b, uint32_t blocks, hipStream_t st) {
  if (blocks) hipLaunchKernelGGL(k_prep_batch, dim3(blocks), dim3(256), 0, st, b);
}

uint32_t x_sort_single_max() { return kSortChunk; }

uint32_t x_sort_scratch_elems(uint32_t R) {
  return (R + kSortChunk - 1) / kSortChunk * kSortChunk;
}

void launch_x_sort(uint32_t seed, uint32_t R, uint32_t Rs, uint64_t* scratch, uint32_t* xs,
                   uint32_t* inv, uint32_t* pos, hipStream_t st) {
  if (R <= kCountSortMax) {
    hipLaunchKernelGGL(k_x_sort_count, dim3(1), dim3(1024), 0, st, seed, R, Rs, xs, inv, pos);
    return;
  }
  const uint32_t nchunks = (R + kSortChunk - 1) / kSortChunk;
  if (nchunks == 1) {
    hipLaunchKernelGGL(k_x_sort_single, dim3(1), dim3(1024), 0, st, seed, R, Rs, xs, inv, pos);
    return;
  }
  hipLaunchKernelGGL(k_x_sort_chunk, dim3(nchunks), dim3(1024), 0, st, seed, R, scratch);
  const uint32_t padded = nchunks * kSortChunk;
  hipLaunchKernelGGL(k_x_sort_merge, dim3((padded + 255) / 256), dim3(256), 0, st, scratch, R,
                     nchunks, xs, inv, pos);
  if (Rs > R) hipLaunchKernelGGL(k_x_pad, dim3((Rs - R + 255) / 256), dim3(256), 0, st, R, Rs, xs, inv);
}

}  // namespace infuse
