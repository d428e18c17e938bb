// Host-side objects behind the opaque handles of include/infuse.h.
#pragma once

#include <atomic>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/infuse.h"
#include "arena.h"
#include "common.h"

struct im_graph;

namespace infuse {

struct PendingEvent {
  std::string name;
  hipEvent_t a, b;
};

// One memo: sampler state and the n x Rs label/size words for (p, R, s).
struct Memo {
  uint64_t tkey = 0;  // threshold floor(p * 2^32) (0 for per-slot p graphs)
  uint32_t R = 0, seed = 0;
  uint32_t Rs = 0, ntiles = 0, mwords = 0;
  uint32_t tm1 = 0, kshift = 0, never_live = 0;
  void* base = nullptr;  // one allocation holding every array below
  size_t bytes = 0;
  uint2* edges = nullptr;
  uint32_t* xs = nullptr;
  uint32_t* inv = nullptr;
  uint32_t* pos = nullptr;
  uint64_t* scratch = nullptr;
  int32_t* M = nullptr;
  uint32_t* tmask = nullptr;
  uint32_t* lmask = nullptr;
  int64_t* g0 = nullptr;
  uint32_t* tlist = nullptr;
  uint32_t* llist = nullptr;
  uint32_t* counts = nullptr;
  unsigned long long* work = nullptr;  // [kWorkCounts], right after counts
  bool counted = false;                // work holds the counts of the construction
  uint32_t list_cap = 0;
  uint64_t last_use = 0;
  int pins = 0;
  // recorded after construction; the memos built by one batched launch
  // share it (each record is a marker the command processor handles in
  // turn: 64 of them took 0.35 ms), and the last of them destroys it
  std::shared_ptr<ihipEvent_t> ready;
  hipEvent_t fork_ev = nullptr;   // hub rows run on the context's side stream
  hipEvent_t join_ev = nullptr;
  MemoView view(const im_graph* g) const;
  hipEvent_t ready_ev() const { return ready.get(); }
};

// A completion event for Memo::ready, recorded on `st` (empty when no event
// can be created).
std::shared_ptr<ihipEvent_t> record_ready(hipStream_t st);

struct CelfBuffers {
  void* base = nullptr;
  size_t bytes = 0;
  CelfView v;
  void* pscratch = nullptr;  // state of the persistent kernel
  void* pjob = nullptr;      // its description of this selection (device copy of hjob)
  alignas(16) unsigned char hjob[512];
  uint32_t* blist = nullptr;  // [n] persistent kernel: bulk candidates
  bool persistent = false;   // enqueued as one persistent kernel
};

im_status fail(im_status s, const char* fmt, ...);
// A pinned host buffer of at least `bytes` from the context's pool (its size
// in *cap), or nullptr when no pinned memory can be had (the caller then
// copies through pageable memory).  Give it back once the copies that use
// it have completed; the pool is freed with the context.
void* pinned_take(im_ctx* c, size_t bytes, size_t* cap);
void pinned_give(im_ctx* c, void* p, size_t cap);
im_status ctx_alloc(im_ctx* c, size_t bytes, void** out);
void ctx_free(im_ctx* c, void* p);
void memo_destroy(im_graph* g, Memo* m);
uint64_t memo_bytes(const im_graph* g, uint32_t R);
Memo* memo_find(im_graph* g, double p, uint32_t R, uint32_t seed);
im_status memo_alloc(im_graph* g, double p, uint32_t R, uint32_t seed, Memo** out);
uint32_t hub_chunk_tiles(const im_ctx* c);
uint32_t pcelf_prof_bits(const im_ctx* c);
bool memo_matches(const im_graph* g, const Memo* m, double p, uint32_t R, uint32_t seed);
im_status memo_build(im_graph* g, double p, uint32_t R, uint32_t seed, hipStream_t st, Memo** out);
im_status memo_acquire(im_graph* g, Memo** out);
void memo_release(im_graph* g, Memo* m);
im_status check_params(const im_graph* g, double p, uint32_t R);
uint32_t key_bits(uint32_t n);
im_status celf_alloc(im_graph* g, const Memo* m, uint32_t K, uint32_t W, CelfBuffers* cb);
// Enqueues a selection: the persistent kernel (when the context's mode and
// persistent_ok allow it; it waits for and holds back every other stream of
// the context) or the per-step kernels, which run beside other work.
void celf_enqueue(im_ctx* c, CelfBuffers* cb, hipStream_t st, bool persistent_ok = true);
bool celf_launch_persistent(im_ctx* c, const void* jobs, uint32_t njobs, uint32_t group_blocks,
                            const uint32_t* first, hipStream_t st);
void celf_enqueue_steps(im_ctx* c, CelfBuffers* cb, hipStream_t st);
im_status celf_collect(im_ctx* c, CelfBuffers* cb, hipStream_t st, uint32_t* seeds,
                       int64_t* marginal, int64_t* cover, uint64_t* evals);
// The checks and totals of a finished selection from its downloaded error
// flag, state and marginal counts (celf_collect, or a batched download).
im_status celf_finish(im_ctx* c, const CelfBuffers* cb, uint32_t perr, const CelfState& hs,
                      const int64_t* marginal, int64_t* cover, uint64_t* evals);
im_status normalize_set(const im_graph* g, const uint32_t* S, uint32_t len, std::vector<uint32_t>* out);
// Enqueues sigma(S) into a scratch block of its own (the count at byte 0,
// the seed ids from byte 256).  With `staged` (pinned host memory laid out
// the same way, the count zeroed), one upload sets both; otherwise the count
// is cleared and S.data() uploaded.  The host memory must stay valid until
// the stream has passed the upload.
im_status sigma_enqueue(im_graph* g, Memo* m, const std::vector<uint32_t>& S, hipStream_t st,
                        void** scratch, unsigned long long** dev_out, const void* staged = nullptr);

// noalloc.hip: device address of the per-device scratch array of the
// allocation-free sigma call (looked up once per device), or nullptr.
void* noalloc_scratch_setup(int device);

// Records HIP events around a launch on `st` when profiling is on.
class KTimer {
 public:
  KTimer(im_ctx* c, const char* name, hipStream_t st, int level = 2);
  ~KTimer();

 private:
  im_ctx* c_;
  const char* name_;
  hipStream_t st_;
  hipEvent_t a_ = nullptr, b_ = nullptr;
  bool on_ = false;
};

}  // namespace infuse

struct im_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipStream_t aux = nullptr;  // side stream for work that overlaps the main stream's
  std::vector<hipStream_t> bstreams;  // memo construction of batched graphs (created on first use)
  // launched CELF graphs, destroyed once their completion event has fired
  struct GraphRun {
    hipGraphExec_t exec;
    hipGraph_t graph;
    hipEvent_t done;
  };
  std::vector<GraphRun> graph_runs;
  std::vector<hipEvent_t> bevents;
  im_allocator alloc = {nullptr, nullptr, nullptr};
  bool has_alloc = false;
  uint64_t budget = 0;
  uint64_t in_use = 0;
  infuse::Arena arena;     // used when budget > 0 and the reservation succeeded
  bool arena_tried = false;
  uint64_t use_clock = 0;
  uint64_t evictions = 0;
  uint64_t last_bulk_rounds = 0;
  im_tuning tune = {};
  int profiling = 0;  // 0 off, 1 per-build kernels, 2 also CELF rounds
  std::vector<infuse::PendingEvent> pending;
  std::map<std::string, std::pair<uint64_t, double>> kstats;
  std::vector<im_graph*> graphs;
  std::unordered_map<void*, size_t> sizes;
  std::recursive_mutex mu;
  // serving loop hook: number of queued queries that want memo m of graph g
  // (evictions prefer memos nobody waits for)
  uint32_t (*memo_demand)(void* user, const im_graph* g, const infuse::Memo* m) = nullptr;
  void* memo_demand_user = nullptr;
  // persistent CELF: workgroups of its grid (0: unavailable), and the
  // completion of the last launch enqueued
  uint32_t coop_grid = 0;
  hipEvent_t coop_done = nullptr;
  bool coop_pending = false;
  hipStream_t coop_stream = nullptr;
  // streams of this context besides stream, aux and bstreams (a server's
  // slots): a persistent launch is fenced against every one of them
  std::vector<hipStream_t> peers;
  std::vector<hipEvent_t> fence_ev;  // one per fenced stream, reused
  // pinned host buffers {address, bytes} for the small copies of the
  // synchronous calls (a selection's results, a seed set and its count):
  // copies from pageable memory are staged by the host, one at a time
  std::vector<std::pair<void*, size_t>> pinned;
};

struct im_graph {
  im_ctx* ctx = nullptr;
  uint32_t n = 0;
  uint64_t nnz_in = 0;  // slots given by the caller
  uint32_t nnz = 0;     // slots on the device (per-slot p: T = 0 slots dropped)
  bool per_edge = false;
  bool directed = false;  // out-arc CSR: only the memo-free spread applies
  void* gbuf = nullptr;
  uint32_t* row_ptr = nullptr;
  uint32_t* col = nullptr;
  uint32_t* src = nullptr;  // row of each slot (the edge hashes take one thread per slot)
  uint32_t* split = nullptr;
  uint32_t* tm1 = nullptr;
  uint32_t* hubs = nullptr;  // vertices with more than kWave device neighbours
  uint2* hub_piece = nullptr;  // {hub, first slot} of every 64-slot piece of their smaller neighbours
  uint32_t nhubs = 0;
  uint32_t hub_pieces = 0;
  uint32_t nlong = 0;  // vertices with more than kSplitArcs device arcs (split by the memo-free search)
  double p = 0.0;
  uint32_t R = 0, seed = 0;
  bool params_set = false;
  std::vector<infuse::Memo*> memos;
  // events: [0] build start, [1] sampler ready, [2] components done,
  // [3] gains done, [4] CELF start, [5] CELF end
  hipEvent_t ev[6] = {};
  bool timed_build = false;
  double phase_ms[4] = {0, 0, 0, 0};
  uint64_t last_evals = 0;
  uint64_t last_search[4] = {0, 0, 0, 0};  // memo-free searches: levels, items, arcs, live pairs
  uint32_t spread_depth = 0;                // levels of the last memo-free spread (first-group guess)
  infuse::GraphView view() const;
};
