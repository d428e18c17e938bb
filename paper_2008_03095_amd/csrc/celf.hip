// CELF on the memo (Algorithm 7), on the device.
//
// Queue state: key[v] = gain << B | (2^B - 1 - v) (B = bitlen(n), so larger
// key = larger gain, then smaller id; 0 marks a selected vertex) and iter[v]
// (|S| when key[v] was computed).  Covered components: one bit per
// (label, column), set for every column's component of every seed.
//
// One CELF step commits exactly one seed, in three launches:
//   k_celf_topw  top-(W+1) keys of unselected vertices (per-wave, per-block,
//                then a last-block merge);
//   k_celf_eval  gains of the W candidates for the current S (blocks over
//                (candidate, 1024-column chunk)); the last block sets
//                key/iter of the candidates and commits the best if its key
//                beats the (W+1)-th key; otherwise it asks for
//   k_celf_bulk  re-evaluation of every stale vertex whose key exceeds the
//                best fresh key k*; the last block commits the best key.
// Why this is lazy greedy: gains only fall as S grows (coverage is
// submodular), so a stale key bounds its vertex's gain.  A committed key is
// fresh and larger than every stale key, hence it is the lowest-id maximiser
// of the exact gains, the same vertex plain greedy and the sequential CELF
// queue pick.
#include <cstring>

#include "common.h"
#include "launch.h"
#include "lists.h"

namespace infuse {


// Cross-block hand-off inside a kernel.  Data another block reads later in
// the same kernel is written with atomics or write-through (agent-scope)
// stores; before taking a ticket the writer waits until its memory
// operations completed (on GFX9 vmcnt counts stores and atomics too), and
// the last block reads with agent-scope loads.  An agent-scope fence would
// instead write back and invalidate the whole XCD L2 in every block.
__device__ inline void wait_memory_ops() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Wave-wide maximum of a 64-bit value with DPP row shifts and row
// broadcasts (no LDS round trips): lane 63 ends with the maximum, which is
// then read as a scalar.
template <int CTRL, int ROW_MASK>
__device__ inline uint64_t dpp_u64(uint64_t x) {
  const uint32_t lo = __builtin_amdgcn_update_dpp(0u, (uint32_t)x, CTRL, ROW_MASK, 0xF, false);
  const uint32_t hi = __builtin_amdgcn_update_dpp(0u, (uint32_t)(x >> 32), CTRL, ROW_MASK, 0xF, false);
  return ((uint64_t)hi << 32) | lo;
}
__device__ inline uint64_t umax64(uint64_t a, uint64_t b) { return a > b ? a : b; }
__device__ inline uint64_t wave_max_u64(uint64_t x) {
  x = umax64(x, dpp_u64<0x111, 0xF>(x));  // row_shr:1
  x = umax64(x, dpp_u64<0x112, 0xF>(x));  // row_shr:2
  x = umax64(x, dpp_u64<0x114, 0xF>(x));  // row_shr:4
  x = umax64(x, dpp_u64<0x118, 0xF>(x));  // row_shr:8
  x = umax64(x, dpp_u64<0x142, 0xA>(x));  // row_bcast:15
  x = umax64(x, dpp_u64<0x143, 0xC>(x));  // row_bcast:31
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)x, 63);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(x >> 32), 63);
  return ((uint64_t)hi << 32) | lo;
}
__device__ inline uint64_t wave_sum_u64(uint64_t x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off);
  return x;
}

__device__ inline uint32_t key_id(const CelfView& c, uint64_t k) {
  return (uint32_t)((1ull << c.B) - 1 - (k & ((1ull << c.B) - 1)));
}
__device__ inline uint64_t key_gain(const CelfView& c, uint64_t k) { return k >> c.B; }
__device__ inline uint64_t make_key(const CelfView& c, uint64_t gain, uint32_t v) {
  return (gain << c.B) | ((1ull << c.B) - 1 - v);
}

// Per-lane partial gain of vertex u over tile t: sum over the lane's columns
// of |C_q(u)| when the component is not covered.
__device__ inline uint64_t eval_tile(const CelfView& c, uint32_t u, uint32_t t, uint32_t lane) {
  const MemoView& m = c.m;
  const uint32_t q0 = t * kTile + lane * kPerLane;
  const uint32_t bit = (uni(m.tmask[(uint64_t)u * m.mwords + (t >> 5)]) >> (t & 31)) & 1u;
  if (!bit) return (uint64_t)min(max((int32_t)m.R - (int32_t)q0, 0), 4);
  const int4 cur = *reinterpret_cast<const int4*>(m.M + (uint64_t)u * m.Rs + q0);
  const int32_t vals[4] = {cur.x, cur.y, cur.z, cur.w};
  uint64_t sum = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t q = q0 + i;
    if (q >= m.R) continue;
    const int32_t val = vals[i];
    if (val == -1) {  // u alone: u is unselected, so its component is uncovered
      sum += 1;
      continue;
    }
    const uint32_t root = val < 0 ? u : (uint32_t)val;
    const int32_t size = val < 0 ? -val : -m.M[(uint64_t)val * m.Rs + q];
    const uint32_t w = c.cov[(uint64_t)root * c.cwords + (q >> 5)];
    sum += ((w >> (q & 31)) & 1u) ? 0 : (uint64_t)size;
  }
  return sum;
}

// Commit the vertex of key k as seed number st->s (whole block).
__device__ void commit_block(const CelfView& c, uint64_t k) {
  const MemoView& m = c.m;
  const uint32_t id = key_id(c, k);
  // 32 consecutive columns share a coverage word; when they also share the
  // root (always for singleton columns, mostly for a large component) one
  // atomic sets all their bits
  const uint32_t lane = threadIdx.x & 63;
  constexpr int kBatch = 8;  // loads issued together before their atomics
  for (uint32_t qb = 0; qb < m.R; qb += kBatch * blockDim.x) {
    int32_t vals[kBatch];
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      const uint32_t q = qb + b * blockDim.x + threadIdx.x;
      vals[b] = q < m.R ? memo_entry(m, id, q) : 0;
    }
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      const uint32_t q = qb + b * blockDim.x + threadIdx.x;
      const bool valid = q < m.R;
      const int32_t val = vals[b];
      const uint32_t root = val < 0 ? id : (uint32_t)val;
      const uint32_t r0 = __shfl(root, lane & ~31u);
      const uint32_t sh = lane & 32u;
      const uint32_t same = (uint32_t)(__ballot(valid && root == r0) >> sh);
      const uint32_t vm = (uint32_t)(__ballot(valid) >> sh);
      if (same == vm) {
        if ((lane & 31) == 0 && vm) atomicOr(&c.cov[(uint64_t)r0 * c.cwords + (q >> 5)], vm);
      } else if (valid) {
        atomicOr(&c.cov[(uint64_t)root * c.cwords + (q >> 5)], 1u << (q & 31));
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t s = __hip_atomic_load(&c.st->s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    c.seeds[s] = id;
    c.marginal[s] = (int64_t)key_gain(c, k);
    c.key[id] = 0;
    c.st->s = s + 1;
  }
}

constexpr int kTopPerLane = 16;  // keys per lane in k_celf_topw

// Largest key below `last` among a lane's CNT keys (compile-time count, so
// the array stays in registers), then over the wave.
template <int CNT>
__device__ inline uint64_t next_below(const uint64_t (&kk)[CNT], uint64_t last) {
  uint64_t best = 0;
#pragma unroll
  for (int i = 0; i < CNT; ++i) {
    const uint64_t k = kk[i];
    best = (k < last && k > best) ? k : best;
  }
  return wave_max_u64(best);
}

constexpr int kWaveMergePerLane = 5;     // 4 lists of <= 65 keys over 64 lanes
constexpr int kFinalMergePerThread = 32; // <= 8192 keys over 256 threads

__global__ void __launch_bounds__(256) k_celf_topw(CelfView c) {
  if (c.st->s >= c.K) return;
  __shared__ uint64_t wl[4][65];
  __shared__ uint64_t red[4];
  __shared__ uint32_t last_block;
  const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint32_t W1 = c.W + 1;
  const uint64_t base = ((uint64_t)blockIdx.x * 4 + wv) * (64 * kTopPerLane);
  uint64_t kk[kTopPerLane];
#pragma unroll
  for (int i = 0; i < kTopPerLane; ++i) {
    const uint64_t v = base + (uint64_t)i * 64 + lane;
    kk[i] = v < c.m.n ? c.key[v] : 0;
  }
  uint64_t last = ~0ull;
  for (uint32_t it = 0; it < W1; ++it) {
    last = next_below(kk, last);
    if (lane == 0) wl[wv][it] = last;
  }
  __syncthreads();
  if (wv == 0) {  // merge the 4 wave lists
    uint64_t mk[kWaveMergePerLane];
#pragma unroll
    for (int j = 0; j < kWaveMergePerLane; ++j) {
      const uint32_t i = lane + 64 * j;
      mk[j] = i < 4 * W1 ? wl[i / W1][i % W1] : 0;
    }
    uint64_t l2 = ~0ull;
    for (uint32_t it = 0; it < W1; ++it) {
      l2 = next_below(mk, l2);
      if (lane == 0)
        __hip_atomic_store(&c.lists[(uint64_t)blockIdx.x * W1 + it], l2, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    wait_memory_ops();
    last_block = atomicAdd(&c.st->ticket1, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!last_block) return;
  // final merge over gridDim.x * W1 (<= 8192) keys: every thread loads its
  // share once (all loads in flight together), then W1 rounds of "largest
  // key below the previous one" with a block reduction
  const uint32_t total = gridDim.x * W1;
  uint64_t mine[kFinalMergePerThread];
#pragma unroll
  for (int j = 0; j < kFinalMergePerThread; ++j) {
    const uint32_t i = threadIdx.x + 256 * j;
    mine[j] = i < total ? __hip_atomic_load(&c.lists[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
  }
  uint64_t prev = ~0ull;
  for (uint32_t it = 0; it < W1; ++it) {
    const uint64_t best = next_below(mine, prev);
    if (lane == 0) red[wv] = best;
    __syncthreads();
    uint64_t b = red[0];
    for (int i = 1; i < 4; ++i) b = red[i] > b ? red[i] : b;
    __syncthreads();
    prev = b;
    if (threadIdx.x == 0) {
      if (it < c.W) {
        c.cand[it] = b ? key_id(c, b) : kInvalid;
        c.candgain[it] = 0;
      } else {
        c.st->next_key = b;
      }
    }
    if (b == 0 && threadIdx.x == 0) {
      // fewer than W+1 unselected vertices: pad
      for (uint32_t j = it; j < c.W; ++j) {
        c.cand[j] = kInvalid;
        c.candgain[j] = 0;
      }
      c.st->next_key = 0;
    }
    if (b == 0) break;
  }
  if (threadIdx.x == 0) {
    uint32_t nc = 0;
    for (uint32_t j = 0; j < c.W; ++j) nc += c.cand[j] != kInvalid ? 1u : 0u;
    c.st->ncand = nc;
    c.st->ticket1 = 0;
  }
}

constexpr uint32_t kEvalCols = 1024;  // columns per evaluation block (4 waves x 1 tile)

__global__ void __launch_bounds__(256) k_celf_eval(CelfView c, uint32_t nchunks) {
  if (c.st->s >= c.K) return;
  __shared__ uint64_t red[4];
  __shared__ uint32_t last_block;
  const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint32_t w = blockIdx.x / nchunks, ch = blockIdx.x % nchunks;
  const uint32_t s = c.st->s;
  if (w < c.W) {
    const uint32_t u = c.cand[w];
    if (u != kInvalid && c.iter[u] != s) {
      const uint32_t t = ch * (kEvalCols / kTile) + wv;
      uint64_t part = t < c.m.ntiles ? eval_tile(c, u, t, lane) : 0;
      part = wave_sum_u64(part);
      if (lane == 0) red[wv] = part;
      __syncthreads();
      if (threadIdx.x == 0) {
        const uint64_t tot = red[0] + red[1] + red[2] + red[3];
        if (tot) atomicAdd((unsigned long long*)&c.candgain[w], (unsigned long long)tot);
      }
    }
  }
  if (threadIdx.x == 0) {
    wait_memory_ops();
    last_block = atomicAdd(&c.st->ticket2, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!last_block) return;
  __shared__ uint64_t best_sh;
  __shared__ uint32_t bulk_sh;
  __shared__ uint64_t ck[64];
  __shared__ uint32_t cev[64];
  // candidate j is finished by thread j: all its loads are in flight together
  if (threadIdx.x < c.W) {
    const uint32_t j = threadIdx.x;
    const uint32_t u = c.cand[j];
    uint64_t k = 0;
    uint32_t e = 0;
    if (u != kInvalid) {
      if (c.iter[u] != s) {
        const uint64_t g = __hip_atomic_load(&c.candgain[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        k = make_key(c, g, u);
        c.key[u] = k;
        c.iter[u] = s;
        e = 1;
      } else {
        k = c.key[u];
      }
    }
    ck[j] = k;
    cev[j] = e;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t best = 0, ev = 0;
    for (uint32_t j = 0; j < c.W; ++j) {
      best = ck[j] > best ? ck[j] : best;
      ev += cev[j];
    }
    c.st->evals += ev;
    c.st->ticket2 = 0;
    // decisions travel through LDS: the block's L1 may hold the state line
    bulk_sh = best > c.st->next_key ? 0u : 1u;
    c.st->need_bulk = bulk_sh;
    if (bulk_sh) {
      c.st->kstar = best;
      c.st->bulk_best = best;
      c.st->bulk_rounds += 1;
    }
    best_sh = best;
  }
  __syncthreads();
  if (!bulk_sh) commit_block(c, best_sh);
}

// One wavefront per vertex (grid-stride over vertices), no block barriers.
__global__ void __launch_bounds__(256) k_celf_bulk(CelfView c) {
  if (c.st->s >= c.K || !c.st->need_bulk) return;
  __shared__ uint32_t last_block;
  __shared__ uint64_t wbest[4], wev[4];
  const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint32_t s = c.st->s;
  const uint64_t kstar = c.st->kstar;
  uint64_t ev = 0, best = 0;
  const uint32_t nw = gridDim.x * 4;
  for (uint32_t v = blockIdx.x * 4 + wv; v < c.m.n; v += nw) {
    const uint64_t k = c.key[v];
    if (k <= kstar) continue;
    if (c.iter[v] == s) {
      best = k > best ? k : best;
      continue;
    }
    uint64_t sum = 0;
    for (uint32_t t = 0; t < c.m.ntiles; ++t) sum += eval_tile(c, v, t, lane);
    sum = wave_sum_u64(sum);
    const uint64_t nk = make_key(c, sum, v);
    if (lane == 0) {
      c.key[v] = nk;
      c.iter[v] = s;
    }
    best = nk > best ? nk : best;
    ++ev;
  }
  if (lane == 0) {
    wbest[wv] = best;
    wev[wv] = ev;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    best = umax64(umax64(wbest[0], wbest[1]), umax64(wbest[2], wbest[3]));
    ev = wev[0] + wev[1] + wev[2] + wev[3];
    if (best) atomicMax((unsigned long long*)&c.st->bulk_best, (unsigned long long)best);
    if (ev) atomicAdd((unsigned long long*)&c.st->evals, (unsigned long long)ev);
    wait_memory_ops();
    last_block = atomicAdd(&c.st->ticket3, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!last_block) return;
  __shared__ uint64_t k_sh;
  if (threadIdx.x == 0) {
    k_sh = __hip_atomic_load(&c.st->bulk_best, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    c.st->ticket3 = 0;
    c.st->need_bulk = 0;
  }
  __syncthreads();
  commit_block(c, k_sh);
}

// Key (initial gain, stamp 0) of vertex i; i = 0 also clears the state.
__device__ inline void celf_init_at(const CelfView& c, uint64_t i) {
  if (i < c.m.n) {
    c.key[i] = make_key(c, (uint64_t)c.m.g0[i], (uint32_t)i);
    c.iter[i] = 0;
  }
  if (i == 0) {
    CelfState z = {};
    *c.st = z;
  }
}

// Clears the coverage words a selection can read: those of the listed
// (vertex, tile) pairs, the tile's 256 columns in 8 words.  A coverage word
// is read only for a column whose component is not a singleton, and that
// component's root has a candidate edge in the tile, so its pair is listed;
// the words of unlisted pairs are never read and may hold anything.
__device__ inline void cov_clear_body(const MemoView& m, uint32_t* cov, uint32_t cwords, uint32_t bid,
                                      uint32_t nblk) {
  const uint32_t lane = threadIdx.x & 63;
  __shared__ uint32_t pre[kSubLists + 1];
  const ListIter it = list_iter(m, m.tlist, 0, pre, bid, nblk);
  for (uint32_t k0 = 0; (uint64_t)it.first + (uint64_t)k0 * it.stride < it.total; k0 += 64) {
    uint32_t cnt;
    const uint32_t ent = list_chunk(it, k0, lane, cnt);
    if (lane < cnt) {
      const uint32_t v = ent / m.ntiles, t = ent % m.ntiles;
      uint4* w = reinterpret_cast<uint4*>(cov + (uint64_t)v * cwords + t * (kTile / 32));
      w[0] = make_uint4(0u, 0u, 0u, 0u);
      w[1] = make_uint4(0u, 0u, 0u, 0u);
    }
  }
}

// Set-up of one selection in one launch: cov_blocks workgroups clear the
// coverage words of the listed tiles, init_blocks set the keys, and the last
// one clears the persistent kernel's state and writes its job description
// (passed by value, so no separate upload), or nothing when pjob is null.
__global__ void __launch_bounds__(256) k_celf_setup(CelfView c, uint32_t cov_blocks, uint32_t init_blocks,
                                                    uint32_t* pscratch, uint32_t scratch_words, JobWords job,
                                                    uint32_t* pjob) {
  if (blockIdx.x < cov_blocks) {
    cov_clear_body(c.m, c.cov, c.cwords, blockIdx.x, cov_blocks);
    return;
  }
  const uint32_t b = blockIdx.x - cov_blocks;
  if (b < init_blocks) {
    celf_init_at(c, (uint64_t)b * blockDim.x + threadIdx.x);
    return;
  }
  for (uint32_t i = threadIdx.x; i < scratch_words; i += blockDim.x) pscratch[i] = 0u;
  if (pjob)
    for (uint32_t i = threadIdx.x; i < kJobWords; i += blockDim.x) pjob[i] = job.w[i];
}

// Set-up of many selections in one launch: per selection (found by binary
// search in the prefix sums `first` of its workgroups), cov_blocks
// workgroups clear its coverage bits, init_blocks set its keys, and one
// clears the persistent kernel's state.
__global__ void __launch_bounds__(256) k_celf_prepare_batch(const CelfBatchJob* jobs, const uint32_t* first,
                                                            uint32_t njobs) {
  uint32_t lo = 0, hi = njobs;  // the last lo with first[lo] <= blockIdx.x
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (first[mid] <= blockIdx.x) lo = mid;
    else hi = mid;
  }
  const CelfBatchJob& J = jobs[lo];
  uint32_t local = blockIdx.x - first[lo];
  if (local < J.cov_blocks) {
    const uint64_t words = (uint64_t)J.v.m.n * J.v.cwords;
    for (uint64_t i = (uint64_t)local * blockDim.x + threadIdx.x; i < words; i += (uint64_t)J.cov_blocks * blockDim.x)
      J.v.cov[i] = 0u;
    return;
  }
  local -= J.cov_blocks;
  if (local < J.init_blocks) {
    celf_init_at(J.v, (uint64_t)local * blockDim.x + threadIdx.x);
    return;
  }
  for (uint32_t i = threadIdx.x; i < J.scratch_words; i += blockDim.x) J.pscratch[i] = 0u;
}

// Packs the results of selection blockIdx.x into its record (one download
// for all selections of a batched call).
__global__ void __launch_bounds__(256) k_celf_collect_batch(const CelfBatchJob* jobs, unsigned char* out) {
  const CelfBatchJob& J = jobs[blockIdx.x];
  unsigned char* rec = out + J.rec_off;
  const uint32_t K = J.v.K;
  uint32_t* seeds = reinterpret_cast<uint32_t*>(rec + 8 + sizeof(CelfState));
  int64_t* marg = reinterpret_cast<int64_t*>(rec + 8 + sizeof(CelfState) + (((uint64_t)K * 4 + 7) & ~7ull));
  if (threadIdx.x == 0) {
    *reinterpret_cast<uint64_t*>(rec) = *J.perr;
    *reinterpret_cast<CelfState*>(rec + 8) = *J.v.st;
  }
  for (uint32_t i = threadIdx.x; i < K; i += blockDim.x) {
    seeds[i] = J.v.seeds[i];
    marg[i] = J.v.marginal[i];
  }
}

// ---- launchers -------------------------------------------------------------

uint32_t celf_topw_blocks(uint32_t n) { return (n + 4 * 64 * kTopPerLane - 1) / (4 * 64 * kTopPerLane); }

void launch_celf_prepare_batch(const CelfBatchJob* jobs, const uint32_t* first, uint32_t njobs, uint32_t blocks,
                               hipStream_t st) {
  if (blocks) hipLaunchKernelGGL(k_celf_prepare_batch, dim3(blocks), dim3(256), 0, st, jobs, first, njobs);
}

void launch_celf_collect_batch(const CelfBatchJob* jobs, uint32_t njobs, unsigned char* out, hipStream_t st) {
  if (njobs) hipLaunchKernelGGL(k_celf_collect_batch, dim3(njobs), dim3(256), 0, st, jobs, out);
}

void launch_celf_setup(const CelfView& c, uint32_t* pscratch, uint32_t scratch_words, const void* job,
                       void* pjob, hipStream_t st) {
  constexpr uint32_t cov_blocks = 1024;  // list walkers: light work per entry
  const uint32_t init_blocks = (c.m.n + 255) / 256;
  JobWords jw = {};
  if (job) std::memcpy(jw.w, job, sizeof(jw.w));
  hipLaunchKernelGGL(k_celf_setup, dim3(cov_blocks + init_blocks + 1), dim3(256), 0, st, c, cov_blocks,
                     init_blocks, pscratch, scratch_words, jw, job ? static_cast<uint32_t*>(pjob) : nullptr);
}

void launch_celf_topw(const CelfView& c, hipStream_t st) {
  hipLaunchKernelGGL(k_celf_topw, dim3(celf_topw_blocks(c.m.n)), dim3(256), 0, st, c);
}

void launch_celf_eval(const CelfView& c, hipStream_t st) {
  const uint32_t nchunks = (c.m.Rs + kEvalCols - 1) / kEvalCols;
  hipLaunchKernelGGL(k_celf_eval, dim3(c.W * nchunks), dim3(256), 0, st, c, nchunks);
}

void launch_celf_bulk(const CelfView& c, uint32_t bulk_blocks, hipStream_t st) {
  hipLaunchKernelGGL(k_celf_bulk, dim3(bulk_blocks), dim3(256), 0, st, c);
}

void launch_celf_step(const CelfView& c, uint32_t bulk_blocks, hipStream_t st) {
  launch_celf_topw(c, st);
  launch_celf_eval(c, st);
  launch_celf_bulk(c, bulk_blocks, st);
}


}  // namespace infuse
