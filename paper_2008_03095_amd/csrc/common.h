// Internal definitions shared by the gfx950 kernels and the host runtime.
//
// Memo layout (vertex-major, Section III-C).  One int32 word per (vertex,
// simulation) pair, rows of Rs = roundup(R, 256) words:
//   M[v][q] <  0 : v is the smallest vertex of its component in simulation
//                  column q, and -M[v][q] is the component size;
//   M[v][q] >= 0 : M[v][q] is the smallest vertex of v's component.
// So the label array and the size array of the paper (both n x R, sizes
// indexed by label, rows of non-labels unused) share one allocation: the
// size array's used rows are exactly the label array's redundant entries.
//
// Column order.  Column q holds simulation inv[q]; columns are sorted by
// ascending X_r.  Since (h ^ X) < T <= 2^k forces X >> k == h >> k, an edge
// can only be live in the few columns whose X shares its top 32-k bits:
// a 256-column tile is skipped for an edge with one range test.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace infuse {

constexpr int kWave = 64;
constexpr int kTile = 256;        // columns per tile: 64 lanes x 4 columns
constexpr int kPerLane = 4;
constexpr uint32_t kInvalid = 0xFFFFFFFFu;

// MurmurHash3 32-bit finaliser (Appleby, public domain).
__host__ __device__ inline uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

// Key of the unordered pair {u, v} (Eq. 1 hashes min || max): min * n + max
// in 64 bits, folded to 32 bits as lo ^ fmix32(hi) (identity below 2^32).
__host__ __device__ inline uint32_t edge_key32(uint32_t u, uint32_t v, uint32_t n) {
  uint64_t lo = u < v ? u : v, hi = u < v ? v : u;
  uint64_t key = lo * (uint64_t)n + hi;
  return (uint32_t)key ^ fmix32((uint32_t)(key >> 32));
}

// Key of the arc u -> v of a directed graph (an arc is its own edge): the
// ordered pair u * n + v, folded like edge_key32 (equal to it when u < v).
__host__ __device__ inline uint32_t arc_key32(uint32_t u, uint32_t v, uint32_t n) {
  const uint64_t key = (uint64_t)u * n + v;
  return (uint32_t)key ^ fmix32((uint32_t)(key >> 32));
}

// Bit length of t (0 for t = 0): the smallest k with t < 2^k.  With
// tm1 = T - 1 a live edge needs (h ^ X) <= tm1, hence (h ^ X) >> k == 0.
__host__ __device__ inline uint32_t bitlen32(uint32_t t) {
#ifdef __HIP_DEVICE_COMPILE__
  return t ? 32u - (uint32_t)__clz((int)t) : 0u;
#else
  return t ? 32u - (uint32_t)__builtin_clz(t) : 0u;
#endif
}

// Per-graph device view.  Offsets are 32-bit (nnz < 2^32).
struct GraphView {
  uint32_t n;
  uint32_t nnz;
  const uint32_t* row_ptr;  // [n+1]
  const uint32_t* col;      // [nnz] ascending per row
  const uint32_t* src;      // [nnz] the row of each slot
  const uint32_t* split;    // [n]  first slot of row v whose neighbour is > v
  const uint32_t* tm1;      // [nnz] per-slot T-1, or nullptr (uniform p)
  const uint32_t* hubs;     // [nhubs] vertices with more than kWave device neighbours
  const uint2* hub_piece;   // [hub_pieces] {hub vertex, first slot} of each kHubPiece-slot
                            // piece of a hub's smaller neighbours
  uint32_t nhubs;
  uint32_t hub_pieces;      // entries of hub_piece
  uint32_t directed;        // 1: col holds out-arcs, each hashed from its ordered pair
};

// Per-memo device view.
struct MemoView {
  uint32_t n;
  uint32_t R;
  uint32_t Rs;          // row stride, multiple of kTile
  uint32_t ntiles;      // Rs / kTile
  uint32_t mwords;      // 32-bit mask words per vertex: ceil(ntiles / 32)
  uint32_t tm1;         // uniform mode: T - 1
  uint32_t kshift;      // uniform mode: bitlen(tm1)
  uint32_t never_live;  // uniform mode with T = 0
  const uint2* edges;   // [nnz] {neighbour, h_e}
  const uint32_t* xs;   // [Rs] X of column q (ascending for q < R)
  int32_t* M;           // [n][Rs]; only tiles with their tmask bit are written
  uint32_t* tmask;      // [n][mwords]  tile may hold a non-singleton column
                        //              (clear: v is a singleton in every column
                        //              of the tile and its M words are stale)
  uint32_t* lmask;      // [n][mwords]  tile has a column with two or more
                        //              live smaller neighbours (needs k_link)
  int64_t* g0;          // [n]
  // work lists built from the masks by k_lists, entries v * ntiles + t,
  // split into kSubLists sub-lists by vertex range (sub-list j holds the
  // vertices [j * ceil(n / kSubLists), (j + 1) * ceil(n / kSubLists))):
  uint32_t* tlist;      // tiles with a candidate edge (k_flatten, k_gain0)
  uint32_t* llist;      // tiles with a column of two or more live smaller
                        // neighbours (k_link)
  uint32_t* counts;     // [2 * j] = |tlist_j|, [2 * j + 1] = |llist_j|
  uint32_t list_cap;
  // work counts of the construction (kWork* below), or nullptr when not
  // counting (they cost atomics: only while profiling at level 4)
  unsigned long long* work;
};

// Indices of MemoView::work.
enum : uint32_t {
  kWorkLivePairs = 0,    // live (edge, column) pairs: every live edge-sample, seen from its larger end
  kWorkUnions = 1,       // union attempts of the link kernels
  kWorkRewrites = 2,     // member entries k_flatten re-pointed at their root
  kWorkCountAtomics = 3, // root decrements of k_count made in device memory (the others are summed in LDS)
  kWorkRowTiles = 4,     // tiles written by k_hook_rows
  kWorkHubTiles = 5,     // tiles written by k_hook_hubs
  kWorkGathers = 6,      // root-size gathers of k_gain0 (member columns)
  kWorkHubLinkWaves = 7, // k_link_hubs wavefronts with a union tile
  kWorkCounts = 8
};

// Memo entry of v in column q (see MemoView::M): -1 where v's tile has no
// candidate edge, without trusting the unwritten word.  The row word is
// loaded unconditionally so both loads issue together.
__device__ inline int32_t memo_entry(const MemoView& m, uint32_t v, uint32_t q) {
  const uint32_t t = q / kTile;
  const int32_t val = m.M[(uint64_t)v * m.Rs + q];
  const bool on = (m.tmask[(uint64_t)v * m.mwords + (t >> 5)] >> (t & 31)) & 1u;
  return on ? val : -1;
}

// Memo constructions of many graphs in one launch per phase (batching):
// per graph its views and launch shapes, and per phase the prefix sums of
// the workgroups each graph takes (a workgroup finds its graph by binary
// search, then runs the single-graph code on its share).
enum : uint32_t {
  kBpPrep = 0,   // X sort (R <= 4096), edge hashes, mask and counter clearing
  kBpHookRows,
  kBpHookHubs,
  kBpLists,
  kBpLink,
  kBpLinkHubs,
  kBpFlatten,
  kBpCount,
  kBpGain0,
  kBatchPhases
};

struct BuildJob {
  GraphView g;
  MemoView m;
  uint2* edges;          // writable views of the sampler arrays (m.edges, m.xs)
  uint32_t* xs;
  uint32_t* inv;
  uint32_t* pos;
  uint32_t seed;
  uint32_t sort_blocks;  // prep: 1 when the X sort runs here, 0 when done before
  uint32_t hash_blocks;  // prep: edge-hash workgroups after the sort's
  uint32_t hub_chunk;    // hook_hubs: tiles per wavefront
  uint32_t hub_wpv;      // hook_hubs: wavefronts per hub vertex
  uint32_t count_bv;     // count: vertices per workgroup
  uint32_t fill_words;   // prep: u32 words cleared from m.tmask on (both mask arrays)
};

struct BuildBatch {
  const BuildJob* jobs;
  const uint32_t* first;  // [kBatchPhases][njobs + 1] workgroup prefix sums
  uint32_t njobs;
};

// The graph of workgroup `block` in `phase`, its index among that graph's
// workgroups and their number.
__device__ inline uint32_t batch_job(const BuildBatch& b, uint32_t phase, uint32_t block, uint32_t& local,
                                     uint32_t& nblk) {
  const uint32_t* f = b.first + (uint64_t)phase * (b.njobs + 1);
  uint32_t lo = 0, hi = b.njobs;  // the last lo with f[lo] <= block
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (f[mid] <= block) lo = mid;
    else hi = mid;
  }
  local = block - f[lo];
  nblk = f[lo + 1] - f[lo];
  return lo;
}

constexpr uint32_t kHubPiece = 256;  // smaller neighbours of a hub per union wavefront
constexpr uint32_t kSubLists = 256;
constexpr uint32_t kListBlocks = 8192;  // fixed grid of the list kernels (multiple of kSubLists)

// Capacity of one sub-list: it holds the tiles of at most ceil(n / kSubLists)
// vertices, each listed at most once.
inline uint32_t list_capacity(uint32_t n, uint32_t ntiles) {
  return (uint32_t)((uint64_t)((n + kSubLists - 1) / kSubLists) * ntiles);
}

struct CelfState {
  uint32_t s;          // |S|
  uint32_t need_bulk;
  uint32_t ticket1, ticket2, ticket3;
  uint32_t ncand;
  uint64_t next_key;   // (W+1)-th largest key when the candidates were chosen
  uint64_t kstar;
  uint64_t bulk_best;
  uint64_t evals;
  uint64_t bulk_rounds;
};

struct CelfView {
  MemoView m;
  uint32_t K;
  uint32_t W;          // candidates per round (<= 64)
  uint32_t B;          // id bits of the key
  uint32_t cwords;     // Rs / 32
  uint64_t* key;       // [n]
  uint32_t* iter;      // [n]
  uint32_t* cov;       // [n][cwords]
  uint64_t* lists;     // [topw blocks][W+1]
  uint32_t* cand;      // [W]
  uint64_t* candgain;  // [W]
  uint32_t* seeds;     // [K]
  int64_t* marginal;   // [K]
  CelfState* st;
};

// One selection of a batched call (im_batch_select): its set-up as
// workgroup ranges of one launch, and where its results go in the packed
// record array that is downloaded once.
struct CelfBatchJob {
  CelfView v;
  uint32_t* pscratch;      // state of the persistent kernel, cleared
  const uint32_t* perr;    // its error flag (inside pscratch)
  uint32_t scratch_words;  // u32 words of pscratch
  uint32_t cov_blocks;     // workgroups clearing the coverage bits
  uint32_t init_blocks;    // workgroups setting keys and stamps (256 vertices each)
  uint32_t rec_off;        // byte offset of the record: error flag (8 B), CelfState,
                           // seeds (K x u32, padded to 8 B), marginal counts (K x i64)
};

inline uint32_t round_up(uint32_t x, uint32_t m) { return (x + m - 1) / m * m; }

}  // namespace infuse
