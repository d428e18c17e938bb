// CELF on the memo (Algorithm 7) as one persistent kernel.
//
// A grid of co-resident workgroups runs all K greedy steps.  Keys pack the
// gain above the id bits (larger id = smaller key), so key order is gain
// descending, then id ascending.  A key computed for the current |S| is
// "fresh" and exact; older keys are upper bounds (the coverage objective is
// submodular).  Every workgroup holds the same candidate pool in LDS, in two
// parts:
//   S  stale entries, sorted by key, consumed from the front (head);
//   F  entries re-evaluated in this step, unsorted, with their maximum;
// and out_bound, at least every key outside the pool.  Per step:
//   * max F above the S front and above out_bound -> commit it (the exact
//     maximiser, as in lazy greedy);
//   * else, S front above out_bound -> evaluate the next W entries of S with
//     the whole grid (W starts at one grid's worth of candidates and doubles
//     within the step), move them to F;
//   * else (the largest key is outside the pool) -> rebuild the pool; if
//     that already happened in this step, first evaluate every stale vertex
//     whose key exceeds max F at once (bulk), with the whole grid.
// On commit, the rest of F is sorted and merged back into S.  All workgroups
// decide from identical data, so only gains, coverage bits and keys cross
// workgroups.  Evaluations also test the components of the seeds committed
// since the last grid barrier (up to kUnsynced) directly, so a commit needs
// no barrier before the next round.
//
// Look-ahead.  A round that starts with F empty (at most kAheadMax
// candidates) also splits each candidate u's gain by signature: for each of
// u's columns, the subset of the round's first kAheadSet candidates (the
// largest stale keys, the set A) whose component there is u's.  Once seeds
// T of A are committed, u's gain is the sum of its bins whose signature
// misses T, exactly; so while every commit comes from A the pool's keys stay
// fresh and the steps are decided without a round.
//
// Rebuild: a radix select (11-bit digits from the top bit of the largest
// key) finds a threshold above which at most kPool keys lie, the keys above
// it are collected and split into S (sorted) and F.
//
// Memory rules (the XCD L2 caches are not coherent with each other inside a
// kernel): data written during the kernel and read by another workgroup goes
// through device-scope atomics or agent-scope stores and is read with
// agent-scope loads; the memo is read-only here.  Grid barriers are
// hierarchical (16 arrival counters, then one) and give up after a time
// limit: they raise an error flag and every workgroup returns.
#include "common.h"

namespace infuse {

constexpr uint32_t kPool = 2048;               // pool entries per workgroup
constexpr uint32_t kPBlock = 256;              // threads per workgroup
constexpr uint32_t kPer = kPool / kPBlock;     // pool entries per thread
constexpr uint32_t kMaxCand = 1024;            // evaluations per round
constexpr uint32_t kAheadMax = 64;             // largest round that measures look-ahead signatures
constexpr uint32_t kAheadSet = 3;              // candidates of such a round whose components are told apart
constexpr uint32_t kSig = 1u << kAheadSet;     // signatures: subsets of them
constexpr uint32_t kUnsynced = kAheadSet + 1;  // most seeds committed between two grid barriers
constexpr uint32_t kGroups = 16;               // barrier arrival groups
constexpr uint32_t kDigitBits = 11;
constexpr uint32_t kBins = 1u << kDigitBits;
constexpr uint64_t kSpinTicks = 200000000;     // 2 s of the 100 MHz clock
constexpr uint64_t kRunTicks = 3000000000ull;  // 30 s

constexpr uint32_t kGainWords = kMaxCand + kAheadMax * kSig;

// Device scratch of one run (zeroed by the host before the launch).
struct PCelfScratch {
  uint32_t err;  // 1 barrier time-out, 2 inconsistent state, 4 run time-out
  uint32_t pool_cnt;
  uint32_t bulk_cnt;
  uint32_t pad0;
  uint64_t out_bound;
  uint64_t kmax;
  uint64_t pad1[4];
  uint64_t prof[16];                  // workgroup 0's phase clock, then counts
  // profiling: listed (candidate, tile) pairs evaluated and their columns of
  // non-singleton components (each a size gather and a coverage word), added
  // once per wavefront at the end; a line of its own (only atomics write it)
  alignas(128) uint64_t work[2];
  alignas(128) uint32_t arrive[kGroups][32];  // one 128-byte line per group
  uint32_t top[32];
  uint32_t release[kGroups][32];
  // per round: candidate gains [0, kMaxCand), then for a look-ahead round
  // each candidate's gain by signature at kMaxCand + w * kSig + sig; three
  // buffers rotated
  uint64_t gains[3][kGainWords];
  uint32_t hist[kBins];
  uint32_t pool_id[kPool];
  uint64_t pool_key[kPool];
};

// One selection: the graph's CELF state, its scratch and bulk list.
struct PCelfJob {
  CelfView c;
  PCelfScratch* x;
  uint32_t* blist;   // [n] bulk candidates
  uint32_t w0;       // candidates of the first round of a step
  uint32_t prof;     // bit 0: keep the phase clock (each reading is a scalar memory
                     // access); bit 1: count listed tiles and gathers (loads rows again)
};

// The workgroups that run one selection together: their number and this
// workgroup's index among them.  Barriers and every grid-stride loop are
// over the group.
struct Grp {
  uint32_t nb, bi;
};

__device__ inline uint32_t p_uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ inline void p_wait_vm() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
// Workgroup barrier for LDS data only: waits for the wave's LDS (and scalar)
// operations, not its global ones, so global loads, stores and atomics
// issued before it stay in flight (the pool routines touch LDS only; every
// global write a later reader depends on is complete at the next grid
// barrier, which waits for all of them).
__device__ inline void p_lds_sync() {
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}
// Global-memory accessors.  The buffers reach this kernel through a job
// record in memory, so the compiler cannot prove their address space and
// would emit flat instructions, which also hold the LDS wait counter; the
// casts below keep every device-memory access a global one.
#define P_GLOBAL __attribute__((address_space(1)))
typedef int p_i4 __attribute__((ext_vector_type(4)));
template <class T>
__device__ inline P_GLOBAL T* gp(T* p) {
  return (P_GLOBAL T*)p;
}
template <class T>
__device__ inline const P_GLOBAL T* gp(const T* p) {
  return (const P_GLOBAL T*)p;
}
__device__ inline p_i4 ldg4(const int32_t* p) { return *(const P_GLOBAL p_i4*)p; }
__device__ inline int32_t ldg(const int32_t* p) { return *gp(p); }
__device__ inline uint32_t ldg(const uint32_t* p) { return *gp(p); }
__device__ inline uint64_t ld64(const uint64_t* p) {
  return __hip_atomic_load(gp(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint32_t ld32(const uint32_t* p) {
  return __hip_atomic_load(gp(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st64(uint64_t* p, uint64_t v) {
  __hip_atomic_store(gp(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st32(uint32_t* p, uint32_t v) {
  __hip_atomic_store(gp(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint32_t g_add(uint32_t* p, uint32_t v) {
  return __hip_atomic_fetch_add(gp(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void g_add64(uint64_t* p, uint64_t v) {
  __hip_atomic_fetch_add(gp(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void g_or(uint32_t* p, uint32_t v) {
  __hip_atomic_fetch_or(gp(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void g_max64(uint64_t* p, uint64_t v) {
  __hip_atomic_fetch_max(gp(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint64_t p_wsum(uint64_t x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off);
  return x;
}
__device__ inline uint64_t p_wmax(uint64_t x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const uint64_t y = __shfl_xor(x, off);
    x = y > x ? y : x;
  }
  return x;
}

// Phase clock of a workgroup (100 MHz real-time counter); workgroup 0
// reports it.
struct PClock {
  enum { kBarrier = 0, kEval = 1, kCommit = 2, kRestale = 3, kPrep = 4, kPost = 5, kRebuild = 6, kBulk = 7,
         kSort = 8, kMove = 9, kPhases = 10 };
  uint64_t acc[kPhases];
  uint64_t mark;
  uint32_t barriers, rounds, rebuilds, bulks, ahead;
  bool on;
  __device__ void start(bool enable) {
    for (int i = 0; i < kPhases; ++i) acc[i] = 0;
    barriers = rounds = rebuilds = bulks = ahead = 0;
    on = enable;
    mark = on ? __builtin_amdgcn_s_memrealtime() : 0;
  }
  __device__ void lap(int phase) {
    if (!on) return;
    const uint64_t t = __builtin_amdgcn_s_memrealtime();
    acc[phase] += t - mark;
    mark = t;
  }
};

struct PoolLds {
  uint64_t skey[kPool];  // S: stale, sorted descending
  uint32_t sid[kPool];
  uint64_t fkey[kPool];  // F: fresh this step, unsorted
  uint32_t fid[kPool];
  uint32_t wsum[kPBlock / 64];
  uint64_t wmax[kPBlock / 64];
  uint32_t hist[kBins];
  uint32_t cg[64];               // restale of a small F: S entries above each F entry
  uint64_t fbin[kAheadMax][kSig];  // look-ahead: gain of F entry i by signature
  uint32_t aset[kAheadSet];        // look-ahead: the set A of the round F came from
  uint32_t na;                     // |A| (0: F's bins are not valid)
  uint32_t amask;                  // members of A committed since
  uint32_t uns[kUnsynced];         // seeds committed since the last grid barrier, most recent first
  uint32_t nuns;                   // their number (valid until the next barrier)
  uint32_t ns, head, nf, fbest;  // S size, S front, F size, index of max F
  uint64_t out_bound;
  uint64_t prefix;
  uint32_t want, cap, done, shift, width;
};

// Exclusive prefix sum over the workgroup; `total` receives the sum.
__device__ uint32_t block_exscan(PoolLds& L, uint32_t v, uint32_t& total) {
  const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(x, off);
    if (lane >= (uint32_t)off) x += y;
  }
  if (lane == 63) L.wsum[wv] = x;
  __syncthreads();
  uint32_t base = 0, tot = 0;
#pragma unroll
  for (uint32_t i = 0; i < kPBlock / 64; ++i) {
    const uint32_t w = L.wsum[i];
    base += i < wv ? w : 0;
    tot += w;
  }
  __syncthreads();
  total = tot;
  return base + x - v;
}

// Maximum over the workgroup.
__device__ uint64_t block_max(PoolLds& L, uint64_t v) {
  const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  v = p_wmax(v);
  if (lane == 0) L.wmax[wv] = v;
  p_lds_sync();
  uint64_t m = 0;
#pragma unroll
  for (uint32_t i = 0; i < kPBlock / 64; ++i) m = L.wmax[i] > m ? L.wmax[i] : m;
  p_lds_sync();
  return m;
}

// Grid barrier: every wave waits for its own memory operations, then one
// thread per workgroup arrives at its group's counter; the last of a group
// arrives at the top counter, and the last of all releases every group.
__device__ bool grid_sync(PCelfScratch* x, const Grp& G, uint32_t& gen, PClock& clk, int phase) {
  __shared__ uint32_t ok_sh;
  clk.lap(phase);
  ++clk.barriers;
  p_wait_vm();
  __syncthreads();
  ++gen;
  if (threadIdx.x == 0) {
    const uint32_t g = G.bi % kGroups;
    const uint32_t ng = min(kGroups, G.nb);
    const uint32_t members = (G.nb - g + kGroups - 1) / kGroups;
    uint32_t ok = 1;
    if (g_add(&x->arrive[g][0], 1u) + 1 == gen * members)
      if (g_add(&x->top[0], 1u) + 1 == gen * ng)
        for (uint32_t i = 0; i < ng; ++i) st32(&x->release[i][0], gen);
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    while ((int32_t)(ld32(&x->release[g][0]) - gen) < 0) {
      if (ld32(&x->err)) {
        ok = 0;
        break;
      }
      if (__builtin_amdgcn_s_memrealtime() - t0 > kSpinTicks) {
        g_or(&x->err, 1u);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    ok_sh = ok;
  }
  __syncthreads();
  clk.lap(PClock::kBarrier);
  return ok_sh != 0;
}

__device__ inline uint64_t p_make_key(const CelfView& c, uint64_t gain, uint32_t v) {
  return (gain << c.B) | ((1ull << c.B) - 1 - v);
}

// This lane's share of gain(u | S) over tile t: the sizes of u's components
// in the lane's four columns that hold no seed.  uns[0 .. nuns) (LDS) are
// the seeds committed since the last grid barrier: their coverage bits may
// not be visible yet, so their components are tested directly.  With na > 0,
// bins[sig] receives the part of the share in components shared with
// exactly the candidates {aset[j] : bit j of sig} (j < na, LDS); a lane's bin is
// at most four component sizes of at most 2^24 vertices.  The rows and their
// tmask words are loaded together; a row word of a tile without its tmask
// bit is stale and reads as -1 (a singleton), which saves a dependent load
// on this latency-bound path.
__device__ inline uint64_t p_eval_tile(const CelfView& c, uint32_t u, uint32_t t, uint32_t lane,
                                       const uint32_t* uns, uint32_t nuns, const uint32_t* aset, uint32_t na,
                                       uint32_t (&bins)[kSig]) {
  const MemoView& m = c.m;
  const uint32_t q0 = t * kTile + lane * kPerLane;
  const uint32_t bit = t & 31;
  const p_i4 none = p_i4{-1, -1, -1, -1};
  const uint32_t ub = ldg(m.tmask + (uint64_t)u * m.mwords + (t >> 5));
  const p_i4 ru = ldg4(m.M + (uint64_t)u * m.Rs + q0);
  // unused slots read u's own row: every load has a valid address
  uint32_t sid[kUnsynced], sb[kUnsynced];
  p_i4 sr[kUnsynced];
#pragma unroll
  for (uint32_t j = 0; j < kUnsynced; ++j) {
    sid[j] = j < nuns ? uns[j] : u;
    sb[j] = ldg(m.tmask + (uint64_t)sid[j] * m.mwords + (t >> 5));
    sr[j] = ldg4(m.M + (uint64_t)sid[j] * m.Rs + q0);
  }
  uint32_t aid[kAheadSet], ab[kAheadSet];
  p_i4 ar[kAheadSet];
  if (na) {
#pragma unroll
    for (uint32_t j = 0; j < kAheadSet; ++j) {
      aid[j] = j < na ? aset[j] : u;
      ab[j] = ldg(m.tmask + (uint64_t)aid[j] * m.mwords + (t >> 5));
      ar[j] = ldg4(m.M + (uint64_t)aid[j] * m.Rs + q0);
    }
  }
  const p_i4 cur = ((ub >> bit) & 1u) ? ru : none;
  // every load below has a valid address, so none waits behind a branch:
  // a member reads its root's entry, a root or singleton its own
  int32_t raw[4];
  uint32_t word[4], root[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int32_t val = cur[i];
    root[i] = val < 0 ? u : (uint32_t)val;
    raw[i] = ldg(m.M + (uint64_t)root[i] * m.Rs + q0 + i);
    word[i] = ld32(&c.cov[(uint64_t)root[i] * c.cwords + (q0 >> 5)]);
  }
#pragma unroll
  for (uint32_t b = 0; b < kSig; ++b) bins[b] = 0;
  uint64_t sum = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t q = q0 + i;
    const int32_t val = cur[i];
    const bool shared = val != -1;  // a singleton holds no seed
    bool seeded = (word[i] >> (q & 31)) & 1u;
#pragma unroll
    for (uint32_t j = 0; j < kUnsynced; ++j) {
      const int32_t sv = ((sb[j] >> bit) & 1u) ? sr[j][i] : -1;
      seeded = seeded || (j < nuns && (sv < 0 ? sid[j] : (uint32_t)sv) == root[i]);
    }
    const bool counted = q < m.R && !(shared && seeded);
    const uint32_t size = (uint32_t)(-(val < 0 ? val : raw[i]));
    sum += counted ? size : 0u;
    if (na) {
      uint32_t sig = 0;
#pragma unroll
      for (uint32_t j = 0; j < kAheadSet; ++j) {
        const int32_t av = ((ab[j] >> bit) & 1u) ? ar[j][i] : -1;
        sig |= (j < na && shared && (av < 0 ? aid[j] : (uint32_t)av) == root[i]) ? 1u << j : 0u;
      }
#pragma unroll
      for (uint32_t b = 0; b < kSig; ++b) bins[b] += (counted && sig == b) ? size : 0u;
    }
  }
  return sum;
}

// Sums the lanes' signature bins over the wavefront: each butterfly step
// halves the bins a lane holds (a lane keeps the upper half when its lane
// bit is set and adds its partner's), then the groups of lanes that hold the
// same bin are summed.  Returns the wavefront's total of bin
// (lane >> (6 - kAheadSet)) & (kSig - 1), the same in every lane of the
// group.  The halving steps sum at most 16 lanes (2^30 fits 32 bits); the
// rest is summed in 64 bits.
__device__ inline uint64_t p_bins_reduce(uint32_t (&v)[kSig], uint32_t lane) {
#pragma unroll
  for (uint32_t k = 0; k < kAheadSet; ++k) {
    const uint32_t o = 32u >> k, h = kSig >> (k + 1);
    const bool up = (lane & o) != 0;
#pragma unroll
    for (uint32_t i = 0; i < h; ++i) {
      const uint32_t keep = up ? v[i + h] : v[i];
      const uint32_t give = up ? v[i] : v[i + h];
      v[i] = keep + (uint32_t)__shfl_xor((int)give, (int)o);
    }
  }
  uint64_t x = v[0];
#pragma unroll
  for (uint32_t o = 32u >> kAheadSet; o >= 1; o >>= 1) x += __shfl_xor(x, (int)o);
  return x;
}

// The bulk pass visits a candidate's tiles in batches of kBulkB.  With one
// mask word per vertex (Rs <= 8192) only the tiles with their tmask bit are
// visited and the others (singletons only) are counted in closed form;
// otherwise every tile is visited.  tl[b] == kInvalid marks an empty slot.
constexpr int kBulkB = 4;
__device__ inline uint32_t p_tile_or0(uint32_t t) { return t == kInvalid ? 0u : t; }

// Takes the next kBulkB tiles of a candidate: the lowest set bits of `rem`
// (sparse) or the tiles pos, pos + 1, ... (dense).  Scalar work only.
__device__ inline void p_take_tiles(bool sparse, uint32_t ntiles, uint32_t& rem, uint32_t& pos,
                                    uint32_t (&tl)[kBulkB]) {
#pragma unroll
  for (int b = 0; b < kBulkB; ++b) {
    if (sparse) {
      tl[b] = rem ? (uint32_t)__builtin_ctz(rem) : kInvalid;
      rem &= rem - 1;
    } else {
      tl[b] = pos < ntiles ? pos : kInvalid;
      ++pos;
    }
  }
}

// Row words of u for the tiles tl and u's tmask word for them (the tiles of
// a batch share one word).  Every load is issued whatever the tiles are, so
// the number of loads in flight never depends on the data.
__device__ inline void p_load_list(const CelfView& c, uint32_t u, const uint32_t (&tl)[kBulkB], uint32_t lane,
                                   p_i4 (&cur)[kBulkB], uint32_t& word) {
  const MemoView& m = c.m;
  word = ldg(m.tmask + (uint64_t)u * m.mwords + (p_tile_or0(tl[0]) >> 5));
#pragma unroll
  for (int b = 0; b < kBulkB; ++b)
    cur[b] = ldg4(m.M + (uint64_t)u * m.Rs + p_tile_or0(tl[b]) * kTile + lane * kPerLane);
}

// This lane's share of gain(u | S) over the tiles tl whose row words
// p_load_list fetched; a tile without its tmask bit reads as singletons.
// Coverage is read from the bitmap only, so every commit must be visible.
// All loads have valid addresses (a member reads its root's entries,
// anything else its own), so they issue together.
__device__ inline uint64_t p_sum_list(const CelfView& c, uint32_t u, const uint32_t (&tl)[kBulkB], uint32_t lane,
                                      const p_i4 (&row)[kBulkB], uint32_t tword) {
  const MemoView& m = c.m;
  int32_t raw[kBulkB][4];
  uint32_t word[kBulkB][4];
  p_i4 cur[kBulkB];
#pragma unroll
  for (int b = 0; b < kBulkB; ++b)
    cur[b] = (tl[b] != kInvalid && ((tword >> (tl[b] & 31)) & 1u)) ? row[b] : p_i4{-1, -1, -1, -1};
#pragma unroll
  for (int b = 0; b < kBulkB; ++b) {
    const uint32_t q0 = p_tile_or0(tl[b]) * kTile + lane * kPerLane;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int32_t val = cur[b][i];
      const uint32_t root = val < 0 ? u : (uint32_t)val;
      raw[b][i] = ldg(m.M + (uint64_t)root * m.Rs + q0 + i);
      word[b][i] = ld32(&c.cov[(uint64_t)root * c.cwords + (q0 >> 5)]);
    }
  }
  uint64_t sum = 0;
#pragma unroll
  for (int b = 0; b < kBulkB; ++b) {
    if (tl[b] == kInvalid) continue;
    const uint32_t q0 = tl[b] * kTile + lane * kPerLane;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t q = q0 + i;
      const int32_t val = cur[b][i];
      const bool covered = val != -1 && ((word[b][i] >> (q & 31)) & 1u);  // a singleton holds no seed
      const uint64_t size = (uint64_t)(uint32_t)(-(val < 0 ? val : raw[b][i]));
      sum += (q < m.R && !covered) ? size : 0;
    }
  }
  return sum;
}

// Profiling work counts of one (candidate, tile) evaluation: whether the
// tile is listed (its row words hold the candidate's components) and, if so,
// this wavefront's columns of non-singleton components (their size and
// coverage words are gathered).  Only while profiling: it loads the row again.
__device__ inline void p_count_tile(const CelfView& c, uint32_t u, uint32_t t, uint32_t lane, uint64_t& tiles,
                                    uint64_t& cols) {
  const MemoView& m = c.m;
  const uint32_t tw = ldg(m.tmask + (uint64_t)u * m.mwords + (t >> 5));
  if (!((tw >> (t & 31)) & 1u)) return;
  const uint32_t q0 = t * kTile + lane * kPerLane;
  const p_i4 r = ldg4(m.M + (uint64_t)u * m.Rs + q0);
  uint64_t k = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) k += (q0 + i < m.R && r[i] != -1) ? 1u : 0u;
  k = p_wsum(k);
  if (lane == 0) {
    tiles += 1;
    cols += k;
  }
}

// Bitonic sort of key/id[0, cnt) descending, cnt a power of two.
__device__ void lds_sort_desc(uint64_t* key, uint32_t* id, uint32_t cnt) {
  for (uint32_t k = 2; k <= cnt; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t i = threadIdx.x; i < cnt; i += kPBlock) {
        const uint32_t ixj = i ^ j;
        if (ixj > i) {
          const bool desc = (i & k) == 0;
          const uint64_t a = key[i], b = key[ixj];
          if ((a < b) == desc) {
            key[i] = b;
            key[ixj] = a;
            const uint32_t t = id[i];
            id[i] = id[ixj];
            id[ixj] = t;
          }
        }
      }
      p_lds_sync();
    }
  }
}

__device__ inline uint32_t next_pow2(uint32_t v) {
  uint32_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

// Number of entries of the descending array a[0, cnt) larger than k.
__device__ inline uint32_t count_greater(const uint64_t* a, uint32_t cnt, uint64_t k) {
  uint32_t lo = 0, hi = cnt;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (a[mid] > k)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// Recomputes the index of the largest F entry.
__device__ void f_best(PoolLds& L) {
  const uint32_t nf = L.nf;
  uint64_t best = 0;
  for (uint32_t i = threadIdx.x; i < nf; i += kPBlock) best = L.fkey[i] > best ? L.fkey[i] : best;
  best = block_max(L, best);
  for (uint32_t i = threadIdx.x; i < nf; i += kPBlock)
    if (L.fkey[i] == best) L.fbest = i;
  p_lds_sync();
}

// Restale of at most 64 F entries.  Wavefront 0 ranks F across its lanes
// (keys are distinct: the rank of an entry is the number of larger keys,
// read from the other lanes) and finds, by binary search, how many S entries
// lie above each F entry: cg[rank], non-decreasing in the rank.  F entry of
// rank r goes to r + cg[r] and S entry i to i + #{r : cg[r] <= i} (an F
// entry precedes S entry i exactly when cg[r] <= i).
__device__ void pool_restale_small(PoolLds& L, uint32_t nf, uint32_t head, uint32_t ns, PClock& clk) {
  const uint32_t l = threadIdx.x;
  uint64_t fk = 0;
  uint32_t fv = kInvalid, fpos = kPool;
  if (l < 64) {
    fk = l < nf ? L.fkey[l] : 0;  // keys of unselected vertices are >= 1
    fv = l < nf ? L.fid[l] : kInvalid;
    const uint32_t hi = (uint32_t)(fk >> 32), lo = (uint32_t)fk;
    uint32_t rank = 0;
    for (uint32_t j = 0; j < nf; ++j) {
      const uint64_t kj = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)hi, (int)j) << 32) |
                          (uint32_t)__builtin_amdgcn_readlane((int)lo, (int)j);
      rank += kj > fk ? 1u : 0u;
    }
    const uint32_t c = l < nf ? count_greater(L.skey + head, ns, fk) : kPool;
    L.cg[l < nf ? rank : l] = c;  // lanes past nf pad the slots nf .. 63
    fpos = l < nf ? rank + c : kPool;
  }
  clk.lap(PClock::kSort);
  p_lds_sync();
  constexpr uint32_t kR = kPool / kPBlock;
  uint64_t k[kR];
  uint32_t v[kR], sh[kR];
#pragma unroll
  for (uint32_t j = 0; j < kR; ++j) {
    const uint32_t i = threadIdx.x + j * kPBlock;
    k[j] = i < ns ? L.skey[head + i] : 0;
    v[j] = i < ns ? L.sid[head + i] : kInvalid;
    sh[j] = 0;
  }
  // sh[j] = #{r : cg[r] <= i}: eight independent searches, one probe each per step
#pragma unroll
  for (uint32_t step = 32; step > 0; step >>= 1) {
    uint32_t probe[kR];
#pragma unroll
    for (uint32_t j = 0; j < kR; ++j) probe[j] = L.cg[sh[j] + step - 1];
#pragma unroll
    for (uint32_t j = 0; j < kR; ++j) sh[j] += probe[j] <= threadIdx.x + j * kPBlock ? step : 0u;
  }
  p_lds_sync();
#pragma unroll
  for (uint32_t j = 0; j < kR; ++j) {
    const uint32_t i = threadIdx.x + j * kPBlock;
    if (i < ns) {
      L.skey[i + sh[j]] = k[j];
      L.sid[i + sh[j]] = v[j];
    }
  }
  if (fpos < kPool) {
    L.skey[fpos] = fk;
    L.sid[fpos] = fv;
  }
  if (threadIdx.x == 0) {
    L.ns = ns + nf;
    L.head = 0;
    L.nf = 0;
  }
  p_lds_sync();
  clk.lap(PClock::kMove);
}

// After a commit: F (without the seed) becomes stale and is merged into the
// unconsumed part of S; S restarts at position 0.
__device__ void pool_restale(PoolLds& L, PClock& clk) {
  const uint32_t nf = L.nf, head = L.head, ns = L.ns - head;
  if (nf <= 64) {
    pool_restale_small(L, nf, head, ns, clk);
    return;
  }
  // sort F descending (padding keys 0 sort last)
  const uint32_t np2 = next_pow2(nf);
  for (uint32_t i = nf + threadIdx.x; i < np2; i += kPBlock) {
    L.fkey[i] = 0;
    L.fid[i] = kInvalid;
  }
  p_lds_sync();
  lds_sort_desc(L.fkey, L.fid, np2);
  // merge by rank into registers, then write S
  constexpr uint32_t kR = kPool / kPBlock;
  uint64_t k[2 * kR];
  uint32_t v[2 * kR], pos[2 * kR];
#pragma unroll
  for (uint32_t j = 0; j < kR; ++j) {
    const uint32_t i = threadIdx.x + j * kPBlock;
    const bool in = i < ns;
    k[j] = in ? L.skey[head + i] : 0;
    v[j] = in ? L.sid[head + i] : kInvalid;
    pos[j] = in ? i + count_greater(L.fkey, nf, k[j]) : kPool;
    const bool fin = i < nf;
    k[kR + j] = fin ? L.fkey[i] : 0;
    v[kR + j] = fin ? L.fid[i] : kInvalid;
    pos[kR + j] = fin ? i + count_greater(L.skey + head, ns, k[kR + j]) : kPool;
  }
  p_lds_sync();
#pragma unroll
  for (uint32_t j = 0; j < 2 * kR; ++j)
    if (pos[j] < kPool) {
      L.skey[pos[j]] = k[j];
      L.sid[pos[j]] = v[j];
    }
  if (threadIdx.x == 0) {
    L.ns = ns + nf;
    L.head = 0;
    L.nf = 0;
  }
  p_lds_sync();
}

// Rebuilds the pool from the keys of all unselected vertices.
__device__ bool pool_rebuild(const PCelfJob& a, const Grp& G, PoolLds& L, uint32_t s, uint32_t& gen,
                             PClock& clk) {
  const CelfView& c = a.c;
  PCelfScratch* x = a.x;
  const uint32_t n = c.m.n;
  const uint32_t gtid = G.bi * kPBlock + threadIdx.x, gstride = G.nb * kPBlock;
  if (!grid_sync(x, G, gen, clk, PClock::kRebuild)) return false;  // readers of the last staging are done
  if (G.bi == 0) {
    for (uint32_t i = threadIdx.x; i < kBins; i += kPBlock) st32(&x->hist[i], 0u);
    if (threadIdx.x == 0) {
      st32(&x->pool_cnt, 0u);
      st64(&x->out_bound, 0ull);
      st64(&x->kmax, 0ull);
    }
  }
  if (!grid_sync(x, G, gen, clk, PClock::kRebuild)) return false;
  // largest key
  uint64_t mx = 0;
  for (uint32_t v = gtid; v < n; v += gstride) {
    const uint64_t k = ld64(&c.key[v]);
    mx = k > mx ? k : mx;
  }
  mx = block_max(L, mx);  // one max per workgroup, skipped when not above the value seen
  if (threadIdx.x == 0 && mx && mx > ld64(&x->kmax)) g_max64(&x->kmax, mx);
  if (!grid_sync(x, G, gen, clk, PClock::kRebuild)) return false;
  const uint64_t kmax = ld64(&x->kmax);
  if (kmax == 0) {  // nothing unselected: the caller reports it
    if (threadIdx.x == 0) {
      L.ns = L.head = L.nf = 0;
      L.out_bound = 0;
    }
    __syncthreads();
    return true;
  }
  // radix select of a threshold: digits of up to kDigitBits bits from the
  // top bit down; bits [shift, shift + width) form the current digit
  const uint32_t topbit = 63 - __clzll((long long)kmax);
  if (threadIdx.x == 0) {
    L.prefix = 0;
    L.want = kPool / 2;
    L.cap = kPool;
    L.done = 0;
    L.width = min(kDigitBits, topbit + 1);
    L.shift = topbit + 1 - L.width;
  }
  __syncthreads();
  uint64_t thresh = 1;
  for (;;) {
    const uint32_t shift = L.shift, width = L.width;
    const uint64_t prefix = L.prefix;
    for (uint32_t i = threadIdx.x; i < kBins; i += kPBlock) L.hist[i] = 0;
    __syncthreads();
    for (uint32_t v = gtid; v < n; v += gstride) {
      const uint64_t k = ld64(&c.key[v]);
      if (k == 0) continue;
      const uint64_t hi = (shift + width >= 64) ? 0 : (k >> (shift + width));
      if (hi != prefix) continue;
      atomicAdd(&L.hist[(k >> shift) & ((1u << width) - 1)], 1u);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < kBins; i += kPBlock)
      if (L.hist[i]) g_add(&x->hist[i], L.hist[i]);
    if (!grid_sync(x, G, gen, clk, PClock::kRebuild)) return false;
    // bins from the top: thread t holds bins kBins-1-(kBPer*t .. kBPer*t+kBPer-1)
    constexpr uint32_t kBPer = kBins / kPBlock;
    uint32_t h[kBPer], mine = 0;
#pragma unroll
    for (uint32_t j = 0; j < kBPer; ++j) {
      h[j] = ld32(&x->hist[kBins - 1 - (threadIdx.x * kBPer + j)]);
      mine += h[j];
    }
    uint32_t tot;
    uint32_t cum = block_exscan(L, mine, tot);
    const uint32_t want = L.want, cap = L.cap;
    __syncthreads();
#pragma unroll
    for (uint32_t j = 0; j < kBPer; ++j) {
      // bin b holds the want-th largest matching key
      if (cum < want && want <= cum + h[j]) {
        const uint32_t b = kBins - 1 - (threadIdx.x * kBPer + j);  // < 2^width: bins above are empty
        L.prefix = (prefix << width) | b;
        if (cum + h[j] <= cap || shift == 0) {
          L.done = 1;  // threshold = lower edge of bin b
        } else {
          L.want = want - cum;
          L.cap = cap - cum;
          L.width = min(kDigitBits, shift);
          L.shift = shift - L.width;
        }
      }
      cum += h[j];
    }
    if (want > tot && threadIdx.x == 0) {  // fewer matching keys than wanted: take them all
      L.done = 1;
      L.prefix = prefix << width;
    }
    __syncthreads();
    if (L.done) {
      thresh = L.prefix << shift;
      if (thresh == 0) thresh = 1;
      break;
    }
    if (L.shift == shift) {  // no lower digit (cannot happen: shift 0 always finishes)
      if (threadIdx.x == 0) g_or(&x->err, 2u);
      return false;
    }
    // clear the global histogram for the next digit once every reader is done
    if (!grid_sync(x, G, gen, clk, PClock::kRebuild)) return false;
    if (G.bi == 0)
      for (uint32_t i = threadIdx.x; i < kBins; i += kPBlock) st32(&x->hist[i], 0u);
    if (!grid_sync(x, G, gen, clk, PClock::kRebuild)) return false;
  }
  // collect the keys at or above the threshold: positions from a scan over
  // the workgroup, one add per workgroup and pass
  uint64_t outside = 0;
  for (uint32_t vb = G.bi * kPBlock; vb < n; vb += gstride) {  // uniform over the workgroup
    const uint32_t v = vb + threadIdx.x;
    const uint64_t k = v < n ? ld64(&c.key[v]) : 0ull;
    const uint32_t take = k != 0 && k >= thresh;
    if (k != 0 && k < thresh && k > outside) outside = k;
    uint32_t tot;
    const uint32_t pre = block_exscan(L, take, tot);
    if (!tot) continue;
    if (threadIdx.x == 0) L.cg[0] = g_add(&x->pool_cnt, tot);
    __syncthreads();
    const uint32_t at = L.cg[0] + pre;
    if (take && at < kPool) {
      st32(&x->pool_id[at], v);
      st64(&x->pool_key[at], k);
    }
    __syncthreads();  // L.cg[0] is rewritten by the next pass
  }
  outside = block_max(L, outside);
  if (threadIdx.x == 0 && outside && outside > ld64(&x->out_bound)) g_max64(&x->out_bound, outside);
  if (!grid_sync(x, G, gen, clk, PClock::kRebuild)) return false;
  const uint32_t cnt = ld32(&x->pool_cnt);
  if (cnt > kPool) {  // the threshold admits at most kPool keys
    if (threadIdx.x == 0) g_or(&x->err, 2u);
    return false;
  }
  // split into F (fresh: evaluated for this |S|) and S (stale, sorted)
  uint32_t vv[kPer];
  uint64_t kk[kPer];
  uint32_t fr[kPer];
  uint32_t nfm = 0;
#pragma unroll
  for (uint32_t j = 0; j < kPer; ++j) {
    const uint32_t i = threadIdx.x * kPer + j;
    vv[j] = i < cnt ? ld32(&x->pool_id[i]) : kInvalid;
    kk[j] = i < cnt ? ld64(&x->pool_key[i]) : 0;
    fr[j] = (i < cnt && ld32(&c.iter[vv[j]]) == s) ? 1u : 0u;
    nfm += fr[j];
  }
  uint32_t nfresh;
  uint32_t fpos = block_exscan(L, nfm, nfresh);
  uint32_t spos = min(threadIdx.x * kPer, cnt) - fpos;  // stale entries before this thread's
#pragma unroll
  for (uint32_t j = 0; j < kPer; ++j) {
    const uint32_t i = threadIdx.x * kPer + j;
    if (i >= cnt) continue;
    if (fr[j]) {
      L.fkey[fpos] = kk[j];
      L.fid[fpos] = vv[j];
      ++fpos;
    } else {
      L.skey[spos] = kk[j];
      L.sid[spos] = vv[j];
      ++spos;
    }
  }
  if (threadIdx.x == 0) {
    L.ns = cnt - nfresh;
    L.nf = nfresh;
    L.head = 0;
    L.out_bound = ld64(&x->out_bound);
  }
  __syncthreads();
  const uint32_t ns = L.ns;
  const uint32_t np2 = next_pow2(ns);
  for (uint32_t i = ns + threadIdx.x; i < np2; i += kPBlock) {
    L.skey[i] = 0;
    L.sid[i] = kInvalid;
  }
  __syncthreads();
  lds_sort_desc(L.skey, L.sid, np2);
  f_best(L);
  ++clk.rebuilds;
  clk.lap(PClock::kRebuild);
  return true;
}

// Bulk evaluation of every stale vertex whose key exceeds kstar.
__device__ bool bulk_eval(const PCelfJob& a, const Grp& G, PoolLds& L, uint32_t s, uint64_t kstar, uint64_t& ptiles,
                          uint64_t& pcols, uint32_t& gen,
                          PClock& clk, uint64_t& evals) {
  const CelfView& c = a.c;
  PCelfScratch* x = a.x;
  const uint32_t n = c.m.n, ntiles = c.m.ntiles;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t gtid = G.bi * kPBlock + threadIdx.x, gstride = G.nb * kPBlock;
  const uint32_t nw = G.nb * (kPBlock / 64);
  const uint32_t gw = G.bi * (kPBlock / 64) + (threadIdx.x >> 6);
  // the last commit's key store and the counter reset must be visible
  if (G.bi == 0 && threadIdx.x == 0) st32(&x->bulk_cnt, 0u);
  if (!grid_sync(x, G, gen, clk, PClock::kBulk)) return false;
  // 1. list the candidates: positions from a scan over the workgroup and one
  // add per workgroup and pass (an add per wavefront made them contend)
  for (uint32_t vb = G.bi * kPBlock; vb < n; vb += gstride) {  // uniform over the workgroup
    const uint32_t v = vb + threadIdx.x;
    uint32_t take = 0;
    if (v < n) {
      const uint64_t k = ld64(&c.key[v]);
      take = k > kstar && ld32(&c.iter[v]) != s;
    }
    uint32_t tot;
    const uint32_t pre = block_exscan(L, take, tot);
    if (!tot) continue;
    if (threadIdx.x == 0) L.cg[0] = g_add(&x->bulk_cnt, tot);
    __syncthreads();
    if (take) st32(&a.blist[L.cg[0] + pre], v);
    __syncthreads();  // L.cg[0] is rewritten by the next pass
  }
  if (!grid_sync(x, G, gen, clk, PClock::kBulk)) return false;
  const uint32_t cnt = ld32(&x->bulk_cnt);
  // 2. one wavefront per candidate: the gain over all tiles, kB at a time;
  // the keys are read by the rebuild that follows, after its barrier.  A
  // wavefront's candidates are w = gw + j * nw; one load brings the ids of
  // the next 64.  The row words of the next batch (the next candidate's
  // first batch after the last one) are requested before the gathers of
  // the current batch, so a batch costs one memory latency, not two.
  const MemoView& m = c.m;
  const bool sparse = m.mwords == 1;
  for (uint32_t base = gw; base < cnt; base += 64 * nw) {
    const uint32_t nloc = min(64u, (cnt - base + nw - 1) / nw);
    const uint32_t ids = ld32(&a.blist[min(base + lane * nw, cnt - 1)]);
    const uint32_t tws = ldg(m.tmask + (uint64_t)ids * m.mwords);  // word 0 of each lane's candidate
    uint32_t v = (uint32_t)__builtin_amdgcn_readfirstlane(ids);
    uint32_t vb = (uint32_t)__builtin_amdgcn_readfirstlane(tws);
    uint32_t rem = vb, pos = 0;
    uint32_t nt[kBulkB];
    p_i4 nxt[kBulkB];
    uint32_t nword;
    p_take_tiles(sparse, ntiles, rem, pos, nt);
    p_load_list(c, v, nt, lane, nxt, nword);
    for (uint32_t j = 0; j < nloc; ++j) {
      const int jn = (int)min(j + 1, nloc - 1);
      const uint32_t vn = (uint32_t)__builtin_amdgcn_readlane(ids, jn);
      const uint32_t vnb = (uint32_t)__builtin_amdgcn_readlane(tws, jn);
      // batches of v; in the sparse case its unvisited tiles hold R minus the
      // visited tiles' columns of singletons, each of gain 1
      const uint32_t nbat = sparse ? max(1u, ((uint32_t)__builtin_popcount(vb) + kBulkB - 1) / kBulkB)
                                   : (ntiles + kBulkB - 1) / kBulkB;
      uint64_t singles = 0;
      if (sparse) {
        const uint32_t lastpad = ((vb >> (ntiles - 1)) & 1u) ? ntiles * kTile - m.R : 0u;
        singles = (uint64_t)(m.R - ((uint32_t)__builtin_popcount(vb) * kTile - lastpad));
      }
      uint32_t nrem = vnb, npos = 0;
      uint64_t sum = 0;
      for (uint32_t i = 0; i < nbat; ++i) {
        uint32_t ct[kBulkB];
        p_i4 cur[kBulkB];
#pragma unroll
        for (int b = 0; b < kBulkB; ++b) {
          ct[b] = nt[b];
          cur[b] = nxt[b];
        }
        const uint32_t cword = nword;
        const bool more = i + 1 < nbat;
        if (more)
          p_take_tiles(sparse, ntiles, rem, pos, nt);
        else
          p_take_tiles(sparse, ntiles, nrem, npos, nt);
        p_load_list(c, more ? v : vn, nt, lane, nxt, nword);
        sum += p_sum_list(c, v, ct, lane, cur, cword);
        if (a.prof & 2u)
#pragma unroll
          for (int b = 0; b < kBulkB; ++b)
            if (ct[b] != kInvalid) p_count_tile(c, v, ct[b], lane, ptiles, pcols);
      }
      sum = p_wsum(sum) + singles;
      if (lane == 0) {
        st64(&c.key[v], p_make_key(c, sum, v));
        st32(&c.iter[v], s);
      }
      v = vn;
      vb = vnb;
      rem = nrem;
      pos = npos;
    }
  }
  evals += cnt;
  ++clk.bulks;
  clk.lap(PClock::kBulk);
  return true;
}

__device__ void run_celf(const PCelfJob& a, const Grp& G, PoolLds& L) {
  const CelfView& c = a.c;
  PCelfScratch* x = a.x;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t nw = G.nb * (kPBlock / 64);
  const uint32_t gw = G.bi * (kPBlock / 64) + (threadIdx.x >> 6);
  const uint32_t ntiles = c.m.ntiles;
  uint32_t gen = 0, s = 0, rounds = 0, ev_round = 0, step_rebuilds = 0;

  bool synced = true;  // a grid barrier has passed since the last commit
  uint64_t evals = 0;
  uint64_t ptiles = 0, pcols = 0;  // profiling work counts of this wavefront
  PClock clk;
  clk.start((a.prof & 1u) != 0);
  const uint64_t t_start = __builtin_amdgcn_s_memrealtime();
  if (threadIdx.x == 0) L.na = L.nuns = 0;
  if (!pool_rebuild(a, G, L, s, gen, clk)) return;
  bool just_rebuilt = true;
  while (s < c.K) {
    if (__builtin_amdgcn_s_memrealtime() - t_start > kRunTicks) {
      if (threadIdx.x == 0) g_or(&x->err, 4u);
      return;
    }
    const uint32_t ns = L.ns, head = L.head, nf = L.nf;
    const uint64_t stop = head < ns ? L.skey[head] : 0;
    const uint64_t fbest = nf ? L.fkey[L.fbest] : 0;
    const uint64_t ob = L.out_bound;
    if (nf && fbest > stop && fbest > ob) {
      // ---- commit the exact maximiser; each workgroup marks a slice of columns
      const uint32_t id = L.fid[L.fbest];
      const uint32_t per = (c.m.R + G.nb - 1) / G.nb;
      const uint32_t q_lo = min(G.bi * per, c.m.R), q_hi = min(q_lo + per, c.m.R);
      for (uint32_t q = q_lo + threadIdx.x; q < q_hi; q += kPBlock) {
        const uint32_t t = q / kTile;
        const int32_t raw = ldg(c.m.M + (uint64_t)id * c.m.Rs + q);
        const int32_t val = ((ldg(c.m.tmask + (uint64_t)id * c.m.mwords + (t >> 5)) >> (t & 31)) & 1u) ? raw : -1;
        const uint32_t root = val < 0 ? id : (uint32_t)val;
        g_or(&c.cov[(uint64_t)root * c.cwords + (q >> 5)], 1u << (q & 31));
      }
      if (G.bi == 0 && threadIdx.x == 0) {
        *gp(c.seeds + s) = id;  // global stores: a flat one would hold the LDS waits below
        *gp(c.marginal + s) = (int64_t)(fbest >> c.B);
        st64(&c.key[id], 0ull);
      }
      // look-ahead: F came from a round that measured every entry's gain by
      // signature over A, and every seed since is in A; if id is in A too,
      // F holds every entry's key for the step after this one
      const uint32_t na = L.na;
      uint32_t jm = kAheadSet;
#pragma unroll
      for (uint32_t j = 0; j < kAheadSet; ++j)
        if (j < na && L.aset[j] == id) jm = j;
      const bool ahead = jm < kAheadSet;
      // A's members and one more seed can follow each other without a grid
      // barrier: at most kUnsynced
      const uint32_t nu = synced ? 0u : L.nuns;
      if (nu == kUnsynced) {  // cannot happen; every workgroup decides the same
        if (G.bi == 0 && threadIdx.x == 0) g_or(&x->err, 2u);
        return;
      }
      clk.lap(PClock::kCommit);
      p_lds_sync();  // the marking atomics stay in flight through the pool work
      if (threadIdx.x == 0) {  // drop the seed from F
        const uint32_t b = L.fbest;
        L.fkey[b] = L.fkey[nf - 1];
        L.fid[b] = L.fid[nf - 1];
        if (ahead) {  // nf <= kAheadMax here
#pragma unroll
          for (uint32_t g = 0; g < kSig; ++g) L.fbin[b][g] = L.fbin[nf - 1][g];
          L.amask |= 1u << jm;
        } else {
          L.na = 0;
        }
        L.nf = nf - 1;
        for (uint32_t j = kUnsynced - 1; j > 0; --j) L.uns[j] = L.uns[j - 1];
        L.uns[0] = id;
        L.nuns = nu + 1;
      }
      p_lds_sync();
      if (ahead) {
        // the keys for the next step are exact: F stays fresh, S unchanged
        const uint32_t mask = L.amask;
        for (uint32_t i = threadIdx.x; i + 1 < nf; i += kPBlock) {
          uint64_t gain = 0;
#pragma unroll 4
          for (uint32_t g = 0; g < kSig; ++g) gain += (g & mask) ? 0ull : L.fbin[i][g];
          const uint64_t k = p_make_key(c, gain, L.fid[i]);
          L.fkey[i] = k;
          if (G.bi == 0) {
            st64(&c.key[L.fid[i]], k);
            st32(&c.iter[L.fid[i]], s + 1);
          }
        }
        p_lds_sync();
        f_best(L);
        ++clk.ahead;
      } else {
        pool_restale(L, clk);
      }
      synced = false;
      ++s;
      rounds = 0;
      step_rebuilds = 0;
      just_rebuilt = false;
      clk.lap(PClock::kRestale);
      continue;
    }
    if (stop > ob && stop > fbest) {
      // ---- evaluate the next W entries of S (only those above max F can win)
      const uint32_t want = min(kMaxCand, a.w0 << min(rounds, 10u));
      uint32_t nc = min(want, ns - head);
      if (fbest) nc = min(nc, count_greater(L.skey + head, nc, fbest));
      nc = min(nc, kPool - nf);
      // look-ahead when F is empty: the round also splits each candidate's
      // gain by signature over its first kAheadSet candidates (the set A)
      const bool ahead = nf == 0 && nc <= kAheadMax;
      const uint32_t na = ahead ? min(nc, kAheadSet) : 0u;
      const uint32_t nuns = L.nuns;
      uint64_t* g = x->gains[ev_round % 3];
      if (G.bi == 0) {
        uint64_t* nxt = x->gains[(ev_round + 1) % 3];
        for (uint32_t i = threadIdx.x; i < kGainWords; i += kPBlock) st64(&nxt[i], 0ull);
      }
      clk.lap(PClock::kPrep);
      const uint32_t items = nc * ntiles;
      for (uint32_t it = gw; it < items; it += nw) {
        const uint32_t w = it / ntiles, t = it - w * ntiles;
        const uint32_t u = L.sid[head + w];
        uint32_t bins[kSig];
        const uint64_t part = p_wsum(p_eval_tile(c, u, t, lane, L.uns, nuns, L.sid + head, na, bins));
        if (a.prof & 2u) p_count_tile(c, u, t, lane, ptiles, pcols);
        if (lane == 0 && part) g_add64(&g[w], part);
        if (na) {
          const uint64_t tot = p_bins_reduce(bins, lane);
          if ((lane & ((64u >> kAheadSet) - 1)) == 0 && tot)
            g_add64(&g[kMaxCand + w * kSig + ((lane >> (6 - kAheadSet)) & (kSig - 1))], tot);
        }
      }
      if (!grid_sync(x, G, gen, clk, PClock::kEval)) return;
      synced = true;  // every commit so far is visible in the coverage bitmap
      // move the evaluated entries from S to F
      for (uint32_t w = threadIdx.x; w < nc; w += kPBlock) {
        const uint32_t v = L.sid[head + w];
        const uint64_t gain = ld64(&g[w]);
        const uint64_t k = p_make_key(c, gain, v);
        L.fkey[nf + w] = k;
        L.fid[nf + w] = v;
        if (G.bi == 0) {
          st64(&c.key[v], k);
          st32(&c.iter[v], s);
        }
      }
      // a look-ahead round's bins (F was empty: entry w is candidate w)
      if (na)
        for (uint32_t i = threadIdx.x; i < nc * kSig; i += kPBlock) L.fbin[i / kSig][i % kSig] = ld64(&g[kMaxCand + i]);
      __syncthreads();
      if (threadIdx.x == 0) {
        L.head = head + nc;
        L.nf = nf + nc;
        // F's bins are valid only when F is this round's candidates alone
        L.na = na;
        L.amask = 0;
#pragma unroll
        for (uint32_t j = 0; j < kAheadSet; ++j) L.aset[j] = j < na ? L.sid[head + j] : kInvalid;
      }
      __syncthreads();
      f_best(L);
      evals += nc;
      ++rounds;
      ++ev_round;
      ++clk.rounds;
      just_rebuilt = false;
      clk.lap(PClock::kPost);
      continue;
    }
    // ---- the pool cannot decide: the largest key is outside.  Refill the
    // pool; when that already happened in this step, first evaluate every
    // stale vertex above max F at once (a lower bound of this step's gain).
    if (just_rebuilt) {  // a fresh pool always decides
      if (G.bi == 0 && threadIdx.x == 0) g_or(&x->err, 2u);
      return;
    }
    if (nf && step_rebuilds > 0)
      if (!bulk_eval(a, G, L, s, fbest, ptiles, pcols, gen, clk, evals)) return;
    if (threadIdx.x == 0) L.na = 0;  // the rebuilt F did not come from one round
    if (!pool_rebuild(a, G, L, s, gen, clk)) return;
    synced = true;
    ++step_rebuilds;
    if (L.ns == 0 && L.nf == 0) {  // no unselected vertex: cannot happen for K <= n
      if (G.bi == 0 && threadIdx.x == 0) g_or(&x->err, 2u);
      return;
    }
    just_rebuilt = true;
  }
  if ((a.prof & 2u) && lane == 0) {
    g_add64(&x->work[0], ptiles);
    g_add64(&x->work[1], pcols);
  }
  if (G.bi == 0 && threadIdx.x == 0) {
    c.st->s = s;
    c.st->evals = evals;
    c.st->bulk_rounds = ev_round;
    for (int i = 0; i < PClock::kPhases; ++i) x->prof[i] = clk.acc[i];
    x->prof[12] = clk.barriers;
    x->prof[13] = clk.rounds;
    x->prof[14] = ((uint64_t)clk.bulks << 32) | clk.rebuilds;
    x->prof[15] = clk.ahead;
  }
}

// Many selections in one launch, each with its own scratch.  With `first`
// (prefix sums of workgroups per selection, njobs + 1 entries, every
// selection at least one workgroup), selection j runs on workgroups
// first[j] .. first[j+1]-1.  Otherwise the grid is split into groups of
// group_blocks workgroups (trailing workgroups that make no whole group
// return at once) and group g runs the selections g, g + groups, ... one
// after the other.
__global__ void __launch_bounds__(kPBlock, 2) k_celf_persistent(const PCelfJob* __restrict__ jobs, uint32_t njobs,
                                                            uint32_t group_blocks,
                                                            const uint32_t* __restrict__ first) {
  __shared__ PoolLds L;
  uint32_t j0, step;
  Grp G;
  if (first) {
    if (blockIdx.x >= first[njobs]) return;
    uint32_t lo = 0, hi = njobs;  // last j with first[j] <= blockIdx.x
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (first[mid] <= blockIdx.x)
        lo = mid;
      else
        hi = mid;
    }
    G = Grp{first[lo + 1] - first[lo], blockIdx.x - first[lo]};
    j0 = lo;
    step = njobs;  // this selection only
  } else {
    const uint32_t groups = gridDim.x / group_blocks;
    j0 = blockIdx.x / group_blocks;
    if (j0 >= groups) return;
    G = Grp{group_blocks, blockIdx.x % group_blocks};
    step = groups;
  }
  // one call site, the description read in place (its fields stay scalar)
  for (uint32_t j = j0; j < njobs; j += step) {
    run_celf(jobs[j], G, L);
    __syncthreads();
  }
}

// ---- host side --------------------------------------------------------------

uint64_t pcelf_scratch_bytes() { return sizeof(PCelfScratch); }
uint64_t pcelf_prof_offset() { return offsetof(PCelfScratch, prof); }
uint64_t pcelf_work_offset() { return offsetof(PCelfScratch, work); }
uint64_t pcelf_err_offset() { return offsetof(PCelfScratch, err); }

// Workgroups of the persistent grid on `device`: two per compute unit, or
// one where occupancy allows only one (0: the kernel cannot run there).
uint32_t pcelf_grid(int device) {
  int cus = 0, per = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_celf_persistent, kPBlock, 0) != hipSuccess || per < 1)
    return 0;
  return (uint32_t)cus * (uint32_t)std::min(per, 2);
}

static_assert(sizeof(PCelfJob) <= 512, "the host keeps one description in 512 bytes");
uint64_t pcelf_job_bytes() { return sizeof(PCelfJob); }

// Candidates of a step's first round: `round0` if set, else 16, or fewer
// when 16 would exceed one tile per wavefront of the group.
static uint32_t pcelf_w0(const CelfView& c, uint32_t group_blocks, uint32_t round0) {
  const uint32_t waves = group_blocks * (kPBlock / 64);
  return round0 ? std::min(kMaxCand, round0) : std::max(1u, std::min(16u, (waves + c.m.ntiles - 1) / c.m.ntiles));
}

void pcelf_fill_job(void* host_job, const CelfView& c, void* scratch, uint32_t* blist, uint32_t group_blocks,
                    uint32_t round0, uint32_t prof) {
  PCelfJob* j = static_cast<PCelfJob*>(host_job);
  j->c = c;
  j->x = static_cast<PCelfScratch*>(scratch);
  j->blist = blist;
  j->w0 = pcelf_w0(c, group_blocks, round0);
  j->prof = prof;
}

hipError_t launch_celf_persistent(const void* jobs, uint32_t njobs, uint32_t grid, uint32_t group_blocks,
                                  const uint32_t* first, hipStream_t st) {
  // An ordinary launch on the caller's stream: the grid is at most two
  // workgroups per compute unit, within the kernel's occupancy, so every
  // workgroup becomes resident once the kernels already running drain (the
  // caller orders the context's other streams around it).  A cooperative
  // launch would add nothing the kernel uses (its barriers are its own) and
  // routes the kernel through a separate device queue.
  const PCelfJob* j = static_cast<const PCelfJob*>(jobs);
  hipLaunchKernelGGL(k_celf_persistent, dim3(grid), dim3(kPBlock), 0, st, j, njobs, group_blocks, first);
  return hipGetLastError();
}

}  // namespace infuse
