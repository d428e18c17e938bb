// Host runtime behind the C ABI of include/infuse.h: contexts, graph upload
// and validation, memo construction and caching, CELF selection, sigma
// queries, label export and per-kernel timing.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/infuse.h"
#include "launch.h"
#include "runtime.h"

using namespace infuse;

infuse::GraphView im_graph::view() const {
  infuse::GraphView v;
  v.n = n;
  v.nnz = nnz;
  v.row_ptr = row_ptr;
  v.col = col;
  v.src = src;
  v.split = split;
  v.tm1 = per_edge ? tm1 : nullptr;
  v.hubs = hubs;
  v.hub_piece = hub_piece;
  v.nhubs = nhubs;
  v.hub_pieces = hub_pieces;
  v.directed = directed ? 1u : 0u;
  return v;
}

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

static thread_local std::string g_err;

namespace infuse {
im_status fail(im_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}
}  // namespace infuse

extern "C" const char* im_last_error(void) { return g_err.c_str(); }
extern "C" const char* im_version(void) { return "infuse-mi355x 0.1 (gfx950)"; }

// ---------------------------------------------------------------------------
// allocation (budgeted, with LRU eviction of unpinned memos)
// ---------------------------------------------------------------------------

namespace infuse {

static void raw_free(im_ctx* c, void* p) {
  if (!p) return;
  if (c->has_alloc) c->alloc.free(c->alloc.user, p, (void*)c->stream);
  else (void)hipFree(p);
}

static void* raw_alloc(im_ctx* c, size_t bytes) {
  void* p = nullptr;
  if (c->has_alloc) {
    p = c->alloc.alloc(c->alloc.user, bytes, (void*)c->stream);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
  }
  return p;
}

// Evicts one unpinned memo: the least recently used among those no queued
// serving query wants, else the least wanted, least recently used one.
static bool evict_one(im_ctx* c) {
  Memo* victim = nullptr;
  im_graph* owner = nullptr;
  uint32_t vd = 0;
  for (im_graph* g : c->graphs)
    for (Memo* m : g->memos) {
      if (m->pins != 0) continue;
      const uint32_t d = c->memo_demand ? c->memo_demand(c->memo_demand_user, g, m) : 0;
      if (!victim || d < vd || (d == vd && m->last_use < victim->last_use)) {
        victim = m;
        owner = g;
        vd = d;
      }
    }
  if (!victim) return false;
  memo_destroy(owner, victim);
  c->evictions++;
  return true;
}

im_status ctx_alloc(im_ctx* c, size_t bytes, void** out) {
  *out = nullptr;
  if (bytes == 0) bytes = 256;
  bytes = (bytes + 255) & ~(size_t)255;
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  if (c->budget && bytes > c->budget)
    return fail(IM_ERR_BUDGET, "request of %zu bytes exceeds the context budget of %llu bytes", bytes,
                (unsigned long long)c->budget);
  while (c->budget && c->in_use + bytes > c->budget)
    if (!evict_one(c))
      return fail(IM_ERR_BUDGET, "budget exhausted: %llu in use, %zu requested, budget %llu",
                  (unsigned long long)c->in_use, bytes, (unsigned long long)c->budget);
  if (c->budget && !c->arena_tried) {
    // one reservation of the whole budget, carved up by the arena
    c->arena_tried = true;
    void* b = raw_alloc(c, c->budget);
    if (b) c->arena.reset(b, c->budget);
  }
  void* p = nullptr;
  if (c->arena.base) {
    p = c->arena.take(bytes);
    while (!p && evict_one(c)) p = c->arena.take(bytes);
    if (!p)
      return fail(IM_ERR_BUDGET, "no free range of %zu bytes in the context budget (%llu in use)", bytes,
                  (unsigned long long)c->in_use);
  } else {
    p = raw_alloc(c, bytes);
    while (!p && evict_one(c)) p = raw_alloc(c, bytes);
  }
  if (!p) return fail(IM_ERR_OUT_OF_MEMORY, "device allocation of %zu bytes failed", bytes);
  c->in_use += bytes;
  c->sizes[p] = bytes;
  *out = p;
  return IM_OK;
}

void ctx_free(im_ctx* c, void* p) {
  if (!p) return;
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  auto it = c->sizes.find(p);
  size_t bytes = 0;
  if (it != c->sizes.end()) {
    bytes = it->second;
    c->in_use -= bytes;
    c->sizes.erase(it);
  }
  const char* q = static_cast<const char*>(p);
  if (c->arena.base && q >= c->arena.base && q < c->arena.base + c->arena.size)
    c->arena.give(p, bytes);
  else
    raw_free(c, p);
}

void* pinned_take(im_ctx* c, size_t bytes, size_t* cap) {
  {
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    for (size_t i = 0; i < c->pinned.size(); ++i)
      if (c->pinned[i].second >= bytes) {
        void* p = c->pinned[i].first;
        *cap = c->pinned[i].second;
        c->pinned.erase(c->pinned.begin() + (ptrdiff_t)i);
        return p;
      }
  }
  const size_t want = std::max<size_t>((bytes + 4095) & ~(size_t)4095, 64 << 10);
  void* p = nullptr;
  if (hipHostMalloc(&p, want, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  *cap = want;
  return p;
}

void pinned_give(im_ctx* c, void* p, size_t cap) {
  if (!p) return;
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  c->pinned.emplace_back(p, cap);
}

// ---------------------------------------------------------------------------
// kernel timing
// ---------------------------------------------------------------------------

KTimer::KTimer(im_ctx* c, const char* name, hipStream_t st, int level)
    : c_(c), name_(name), st_(st), on_(c->profiling >= level) {
  if (!on_) return;
  (void)hipEventCreate(&a_);
  (void)hipEventCreate(&b_);
  (void)hipEventRecord(a_, st_);
}

KTimer::~KTimer() {
  if (!on_) return;
  (void)hipEventRecord(b_, st_);
  std::lock_guard<std::recursive_mutex> lk(c_->mu);
  c_->pending.push_back({name_, a_, b_});
}

static void resolve_pending(im_ctx* c) {
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  for (auto& p : c->pending) {
    (void)hipEventSynchronize(p.b);
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      auto& s = c->kstats[p.name];
      s.first += 1;
      s.second += ms;
    }
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  c->pending.clear();
}

// ---------------------------------------------------------------------------
// memo
// ---------------------------------------------------------------------------

static uint64_t thr_of(double p) {
  if (!(p > 0.0)) return 0;
  if (p >= 1.0) return 1ull << 32;
  return (uint64_t)std::floor(p * 4294967296.0);
}

MemoView Memo::view(const im_graph* g) const {
  MemoView v;
  v.n = g->n;
  v.R = R;
  v.Rs = Rs;
  v.ntiles = ntiles;
  v.mwords = mwords;
  v.tm1 = tm1;
  v.kshift = kshift;
  v.never_live = never_live;
  v.edges = edges;
  v.xs = xs;
  v.M = M;
  v.tmask = tmask;
  v.lmask = lmask;
  v.g0 = g0;
  v.tlist = tlist;
  v.llist = llist;
  v.counts = counts;
  v.list_cap = list_cap;
  v.work = nullptr;
  return v;
}

std::shared_ptr<ihipEvent_t> record_ready(hipStream_t st) {
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return {};
  (void)hipEventRecord(e, st);
  return std::shared_ptr<ihipEvent_t>(e, [](hipEvent_t x) { (void)hipEventDestroy(x); });
}

void memo_destroy(im_graph* g, Memo* m) {
  auto& v = g->memos;
  v.erase(std::remove(v.begin(), v.end(), m), v.end());
  // the memory may next be used from another stream: construction must be over
  // (queries using the memo hold pins, released only after they completed)
  if (m->ready) (void)hipEventSynchronize(m->ready_ev());
  m->ready.reset();
  if (m->fork_ev) (void)hipEventDestroy(m->fork_ev);
  if (m->join_ev) (void)hipEventDestroy(m->join_ev);
  ctx_free(g->ctx, m->base);
  delete m;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

uint64_t memo_bytes(const im_graph* g, uint32_t R) {
  const uint32_t Rs = round_up(R, kTile);
  const uint32_t ntiles = Rs / kTile;
  const uint32_t mwords = (ntiles + 31) / 32;
  size_t b = 0;
  b += align256((size_t)g->nnz * sizeof(uint2));
  b += align256((size_t)Rs * 4) * 2 + align256((size_t)R * 4);
  b += align256((size_t)x_sort_scratch_elems(R) * 8);
  b += align256((size_t)g->n * Rs * 4);
  b += align256((size_t)g->n * mwords * 4) * 2;
  b += align256((size_t)g->n * 8);
  b += align256((size_t)list_capacity(g->n, ntiles) * kSubLists * 4) * 2;
  b += align256((size_t)kSubLists * 2 * 4 + kWorkCounts * 8);
  return b;
}

bool memo_matches(const im_graph* g, const Memo* m, double p, uint32_t R, uint32_t seed) {
  return m->R == R && m->seed == seed && m->tkey == (g->per_edge ? 0 : thr_of(p));
}

Memo* memo_find(im_graph* g, double p, uint32_t R, uint32_t seed) {
  const uint64_t pb = g->per_edge ? 0 : thr_of(p);
  for (Memo* m : g->memos)
    if (m->tkey == pb && m->R == R && m->seed == seed) return m;
  return nullptr;
}

// Tiles per hook_hubs wavefront from the context's cc_chunk (columns).
// Profiling bits of a persistent CELF launch: the phase clock from level 3,
// the work counts (listed tiles, gathers) at level 4.
uint32_t pcelf_prof_bits(const im_ctx* c) { return (c->profiling >= 3 ? 1u : 0u) | (c->profiling >= 4 ? 2u : 0u); }

uint32_t hub_chunk_tiles(const im_ctx* c) { return std::max(1u, std::min(32u, c->tune.cc_chunk / kTile)); }

// Allocates the memo of (p, R, seed), registers it with the graph and
// returns it pinned; nothing is enqueued.
im_status memo_alloc(im_graph* g, double p, uint32_t R, uint32_t seed, Memo** out) {
  if (g->directed)
    return fail(IM_ERR_INVALID_ARG,
                "directed graph: components do not give reachability; use im_estimate_sigma_direct");
  im_ctx* c = g->ctx;
  Memo* m = new Memo();
  m->tkey = g->per_edge ? 0 : thr_of(p);
  m->R = R;
  m->seed = seed;
  m->Rs = round_up(R, kTile);
  m->ntiles = m->Rs / kTile;
  m->mwords = (m->ntiles + 31) / 32;
  const uint64_t T = thr_of(p);
  m->never_live = (!g->per_edge && T == 0) ? 1u : 0u;
  m->tm1 = (g->per_edge || T == 0) ? 0u : (uint32_t)(T - 1);
  m->kshift = bitlen32(m->tm1);
  m->counted = false;
  if (hipEventCreateWithFlags(&m->fork_ev, hipEventDisableTiming) != hipSuccess) m->fork_ev = nullptr;
  if (hipEventCreateWithFlags(&m->join_ev, hipEventDisableTiming) != hipSuccess) m->join_ev = nullptr;
  m->bytes = memo_bytes(g, R);
  void* base = nullptr;
  im_status s = ctx_alloc(c, m->bytes, &base);
  if (s != IM_OK) {
    if (m->fork_ev) (void)hipEventDestroy(m->fork_ev);
    if (m->join_ev) (void)hipEventDestroy(m->join_ev);
    delete m;
    return s;
  }
  m->base = base;
  char* p8 = static_cast<char*>(base);
  auto take = [&](size_t bytes) {
    char* r = p8;
    p8 += align256(bytes);
    return r;
  };
  m->edges = reinterpret_cast<uint2*>(take((size_t)g->nnz * sizeof(uint2)));
  m->xs = reinterpret_cast<uint32_t*>(take((size_t)m->Rs * 4));
  m->inv = reinterpret_cast<uint32_t*>(take((size_t)m->Rs * 4));
  m->pos = reinterpret_cast<uint32_t*>(take((size_t)R * 4));
  m->scratch = reinterpret_cast<uint64_t*>(take((size_t)x_sort_scratch_elems(R) * 8));
  m->M = reinterpret_cast<int32_t*>(take((size_t)g->n * m->Rs * 4));
  // the two mask arrays are adjacent (one fill clears both)
  m->tmask = reinterpret_cast<uint32_t*>(take((size_t)g->n * m->mwords * 4));
  m->lmask = reinterpret_cast<uint32_t*>(take((size_t)g->n * m->mwords * 4));
  m->g0 = reinterpret_cast<int64_t*>(take((size_t)g->n * 8));
  m->list_cap = list_capacity(g->n, m->ntiles);
  m->tlist = reinterpret_cast<uint32_t*>(take((size_t)m->list_cap * kSubLists * 4));
  m->llist = reinterpret_cast<uint32_t*>(take((size_t)m->list_cap * kSubLists * 4));
  m->counts = reinterpret_cast<uint32_t*>(take((size_t)kSubLists * 2 * 4 + kWorkCounts * 8));
  m->work = reinterpret_cast<unsigned long long*>(m->counts + 2 * kSubLists);
  {
    // returned pinned: nothing may evict it before the caller is done with it
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    m->pins = 1;
    g->memos.push_back(m);
    m->last_use = ++c->use_clock;
  }
  *out = m;
  return IM_OK;
}

// Allocates the memo and enqueues its construction on `st`.
im_status memo_build(im_graph* g, double p, uint32_t R, uint32_t seed, hipStream_t st, Memo** out) {
  Memo* m = nullptr;
  im_status s = memo_alloc(g, p, R, seed, &m);
  if (s != IM_OK) return s;
  im_ctx* c = g->ctx;
  MemoView mv = m->view(g);
  m->counted = c->profiling >= 4;
  if (m->counted) {
    mv.work = m->work;
    launch_fill_u32(reinterpret_cast<uint32_t*>(m->work), 2 * kWorkCounts, 0u, st);
  }
  const uint32_t chunk_tiles = hub_chunk_tiles(c);
  const bool timed = g->ev[0] != nullptr && st == c->stream;
  if (timed) (void)hipEventRecord(g->ev[0], st);
  // the sample values are sorted on the side stream while the edges are
  // hashed and the masks cleared (only for the context stream, as below)
  const bool side = c->aux && m->fork_ev && m->join_ev && st == c->stream;
  if (side) {
    (void)hipEventRecord(m->fork_ev, st);
    (void)hipStreamWaitEvent(c->aux, m->fork_ev, 0);
  }
  {
    hipStream_t xs = side ? c->aux : st;
    KTimer t(c, "x_sort", xs);
    launch_x_sort(seed, R, m->Rs, m->scratch, m->xs, m->inv, m->pos, xs);
  }
  if (side) (void)hipEventRecord(m->join_ev, c->aux);
  {
    KTimer t(c, "edge_hash", st);
    launch_edge_hash(g->view(), seed, m->edges, st);
  }
  // hub vertices' mask words are or-ed into; k_lists writes every count
  launch_fill_u32(m->tmask, (uint64_t)(reinterpret_cast<char*>(m->lmask) - reinterpret_cast<char*>(m->tmask)) / 4 +
                                (uint64_t)g->n * m->mwords, 0u, st);
  if (side) (void)hipStreamWaitEvent(st, m->join_ev, 0);
  if (timed) (void)hipEventRecord(g->ev[1], st);
  // hub rows (few, long, latency-bound wavefronts) run on the side stream
  // next to the bandwidth-bound light rows; the two write disjoint rows
  // (only for the context stream: other streams, such as the batch streams,
  // already run several constructions side by side)
  const bool fork = g->nhubs && c->aux && m->fork_ev && m->join_ev && st == c->stream;
  if (fork) {
    (void)hipEventRecord(m->fork_ev, st);
    (void)hipStreamWaitEvent(c->aux, m->fork_ev, 0);
    {
      KTimer t(c, "hook_hubs", c->aux);
      launch_hook_hubs(g->view(), mv, chunk_tiles, c->aux);
    }
    (void)hipEventRecord(m->join_ev, c->aux);
  }
  {
    KTimer t(c, "hook", st);
    launch_hook_rows(g->view(), mv, st);
  }
  if (fork) {
    (void)hipStreamWaitEvent(st, m->join_ev, 0);
  } else if (g->nhubs) {
    KTimer t(c, "hook_hubs", st);
    launch_hook_hubs(g->view(), mv, chunk_tiles, st);
  }
  {
    KTimer t(c, "lists", st);
    launch_lists(mv, st);
  }
  // unions of hub vertices, one wavefront per (hub, tile, 64 smaller
  // neighbours), on the side stream next to the light vertices' unions (both
  // write the memo only by atomics)
  const bool fork2 = g->hub_pieces && c->aux && m->fork_ev && m->join_ev && st == c->stream;
  if (fork2) {
    (void)hipEventRecord(m->fork_ev, st);
    (void)hipStreamWaitEvent(c->aux, m->fork_ev, 0);
    {
      KTimer t(c, "link_hubs", c->aux);
      launch_link_hubs(g->view(), mv, c->aux);
    }
    (void)hipEventRecord(m->join_ev, c->aux);
  }
  {
    KTimer t(c, "link", st);
    launch_link(g->view(), mv, c->tune.list_blocks, st);
  }
  if (fork2) {
    (void)hipStreamWaitEvent(st, m->join_ev, 0);
  } else if (g->hub_pieces) {
    KTimer t(c, "link_hubs", st);
    launch_link_hubs(g->view(), mv, st);
  }
  {
    KTimer t(c, "flatten", st);
    launch_flatten(mv, c->tune.list_blocks, st);
  }
  {
    KTimer t(c, "count", st);
    launch_count(mv, st);
  }
  if (timed) (void)hipEventRecord(g->ev[2], st);
  {
    KTimer t(c, "gain0", st);
    launch_gain0(mv, c->tune.list_blocks, st);
  }
  if (timed) (void)hipEventRecord(g->ev[3], st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    memo_destroy(g, m);
    return fail(IM_ERR_DEVICE, "memo kernels failed to launch: %s", hipGetErrorString(e));
  }
  m->ready = record_ready(st);
  g->timed_build = timed;
  *out = m;
  return IM_OK;
}

// Finds or builds the memo of the graph's current parameters and pins it.
im_status memo_acquire(im_graph* g, Memo** out) {
  if (!g->params_set) return fail(IM_ERR_INVALID_ARG, "im_set_params has not been called");
  im_ctx* c = g->ctx;
  Memo* m = nullptr;
  {
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    m = memo_find(g, g->p, g->R, g->seed);
    if (m) {
      m->pins++;  // pinned before anything else may evict it
      m->last_use = ++c->use_clock;
    }
  }
  if (!m) {
    im_status s = memo_build(g, g->p, g->R, g->seed, c->stream, &m);  // returned pinned
    if (s != IM_OK) return s;
  } else {
    g->timed_build = false;
    if (m->ready) (void)hipStreamWaitEvent(c->stream, m->ready_ev(), 0);
  }
  *out = m;
  return IM_OK;
}

void memo_release(im_graph* g, Memo* m) {
  std::lock_guard<std::recursive_mutex> lk(g->ctx->mu);
  m->pins--;
}


// ---------------------------------------------------------------------------
// CELF selection on a memo
// ---------------------------------------------------------------------------

uint32_t key_bits(uint32_t n) { return bitlen32(n); }

im_status celf_alloc(im_graph* g, const Memo* m, uint32_t K, uint32_t W, CelfBuffers* cb) {
  im_ctx* c = g->ctx;
  const uint32_t n = g->n;
  const uint32_t cwords = m->Rs / 32;
  const uint32_t tb = celf_topw_blocks(n);
  // the last top-W block merges tb * (W + 1) keys held in registers (at most
  // 8192); the width only changes how many candidates a round evaluates
  const uint32_t wmax = 8192 / tb;
  if (wmax < 2) return fail(IM_ERR_INVALID_ARG, "graph too large for on-device CELF (n > 2^22)");
  W = std::max(1u, std::min(W, wmax - 1));
  size_t b = 0;
  b += align256((size_t)n * 8);
  b += align256((size_t)n * 4);
  b += align256((size_t)n * cwords * 4);
  b += align256((size_t)tb * (W + 1) * 8);
  b += align256((size_t)W * 4) + align256((size_t)W * 8);
  b += align256((size_t)std::max(K, 1u) * 4) + align256((size_t)std::max(K, 1u) * 8);
  b += align256(sizeof(CelfState));
  b += align256(pcelf_scratch_bytes()) + align256(pcelf_job_bytes());
  b += align256((size_t)n * 4);
  void* base = nullptr;
  im_status s = ctx_alloc(c, b, &base);
  if (s != IM_OK) return s;
  cb->base = base;
  cb->bytes = b;
  char* p8 = static_cast<char*>(base);
  auto take = [&](size_t bytes) {
    char* r = p8;
    p8 += align256(bytes);
    return r;
  };
  CelfView& v = cb->v;
  v.m = m->view(g);
  v.K = K;
  v.W = W;
  v.B = key_bits(n);
  v.cwords = cwords;
  v.key = reinterpret_cast<uint64_t*>(take((size_t)n * 8));
  v.iter = reinterpret_cast<uint32_t*>(take((size_t)n * 4));
  v.cov = reinterpret_cast<uint32_t*>(take((size_t)n * cwords * 4));
  v.lists = reinterpret_cast<uint64_t*>(take((size_t)tb * (W + 1) * 8));
  v.cand = reinterpret_cast<uint32_t*>(take((size_t)W * 4));
  v.candgain = reinterpret_cast<uint64_t*>(take((size_t)W * 8));
  v.seeds = reinterpret_cast<uint32_t*>(take((size_t)std::max(K, 1u) * 4));
  v.marginal = reinterpret_cast<int64_t*>(take((size_t)std::max(K, 1u) * 8));
  v.st = reinterpret_cast<CelfState*>(take(sizeof(CelfState)));
  cb->pscratch = take(pcelf_scratch_bytes());
  cb->pjob = take(pcelf_job_bytes());
  cb->blist = reinterpret_cast<uint32_t*>(take((size_t)n * 4));
  cb->persistent = false;
  return IM_OK;
}

// Clears the coverage bitmap (the words of listed tiles: the others are
// never read) and the state of a selection, and with `job` writes the
// persistent kernel's description, in one launch.
static void celf_prepare(CelfBuffers* cb, const void* job, hipStream_t st) {
  launch_celf_setup(cb->v, static_cast<uint32_t*>(cb->pscratch), (uint32_t)(pcelf_scratch_bytes() / 4), job,
                    cb->pjob, st);
}

// One persistent launch over `njobs` selections (device descriptions).
// Returns false when the device cannot run it.
bool celf_launch_persistent(im_ctx* c, const void* jobs, uint32_t njobs, uint32_t group_blocks,
                            const uint32_t* first, hipStream_t st) {
  // The grid waits at barriers for all of its workgroups, so all of them must
  // become resident: no other kernel of this context may hold the device's
  // resources meanwhile (a server's slots keep feeding kernels; a late
  // workgroup could wait behind them until the barrier gives up).  The
  // launch waits for the work already enqueued on every other stream of the
  // context, and their later work waits for the launch.  This also keeps
  // two persistent grids apart.
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  std::vector<hipStream_t> others;
  auto add = [&](hipStream_t o) {
    if (o && o != st && std::find(others.begin(), others.end(), o) == others.end()) others.push_back(o);
  };
  add(c->stream);
  add(c->aux);
  for (hipStream_t o : c->bstreams) add(o);
  for (hipStream_t o : c->peers) add(o);
  while (c->fence_ev.size() < others.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return false;
    c->fence_ev.push_back(e);
  }
  for (size_t i = 0; i < others.size(); ++i) {
    if (hipEventRecord(c->fence_ev[i], others[i]) != hipSuccess ||
        hipStreamWaitEvent(st, c->fence_ev[i], 0) != hipSuccess)
      return false;
  }
  if (c->coop_pending && c->coop_stream != st) (void)hipStreamWaitEvent(st, c->coop_done, 0);
  hipError_t e;
  {
    KTimer t(c, "celf", st, 1);
    e = launch_celf_persistent(jobs, njobs, c->coop_grid, group_blocks, first, st);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  (void)hipEventRecord(c->coop_done, st);
  for (hipStream_t o : others) (void)hipStreamWaitEvent(o, c->coop_done, 0);
  c->coop_pending = true;
  c->coop_stream = st;
  return true;
}

void celf_enqueue(im_ctx* c, CelfBuffers* cb, hipStream_t st, bool persistent_ok) {
  const bool persistent = persistent_ok && c->tune.celf_mode == 1 && c->coop_grid;
  if (persistent)
    pcelf_fill_job(cb->hjob, cb->v, cb->pscratch, cb->blist, c->coop_grid, c->tune.celf_round0,
                   pcelf_prof_bits(c));
  celf_prepare(cb, persistent ? cb->hjob : nullptr, st);
  if (persistent) {
    if (celf_launch_persistent(c, cb->pjob, 1, c->coop_grid, nullptr, st)) {
      cb->persistent = true;
      return;
    }
    (void)hipGetLastError();  // not launchable here: run the per-step kernels
  }
  celf_enqueue_steps(c, cb, st);
}

// The per-step kernels (three launches per greedy step).  With use_graphs
// the K steps are captured into one graph (kernel nodes only) and launched
// once.
static void celf_steps_direct(im_ctx* c, CelfBuffers* cb, hipStream_t st);

// Destroys the launched CELF graphs that have completed (all of them when
// `wait`).
static void sweep_graph_runs(im_ctx* c, bool wait) {
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  auto& v = c->graph_runs;
  for (size_t i = 0; i < v.size();) {
    if (wait) (void)hipEventSynchronize(v[i].done);
    if (hipEventQuery(v[i].done) != hipSuccess) {
      ++i;
      continue;
    }
    (void)hipGraphExecDestroy(v[i].exec);
    (void)hipGraphDestroy(v[i].graph);
    (void)hipEventDestroy(v[i].done);
    v[i] = v.back();
    v.pop_back();
  }
}

void celf_enqueue_steps(im_ctx* c, CelfBuffers* cb, hipStream_t st) {
  sweep_graph_runs(c, false);
  if (c->tune.use_graphs && c->profiling < 3) {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;
    bool ok = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
      celf_steps_direct(c, cb, st);
      ok = hipStreamEndCapture(st, &graph) == hipSuccess && graph;
    }
    if (ok) ok = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
    if (ok) ok = hipEventCreateWithFlags(&done, hipEventDisableTiming) == hipSuccess;
    if (ok) ok = hipGraphLaunch(exec, st) == hipSuccess && hipEventRecord(done, st) == hipSuccess;
    if (ok) {
      std::lock_guard<std::recursive_mutex> lk(c->mu);
      c->graph_runs.push_back({exec, graph, done});
      return;
    }
    (void)hipGetLastError();  // capture not possible here: launch directly
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (done) (void)hipEventDestroy(done);
  }
  celf_steps_direct(c, cb, st);
}

static void celf_steps_direct(im_ctx* c, CelfBuffers* cb, hipStream_t st) {
  const CelfView& v = cb->v;
  const uint32_t bulk_blocks = std::max(1u, std::min(2048u, v.m.n));
  for (uint32_t k = 0; k < v.K; ++k) {
    {
      KTimer t(c, "celf_topw", st, 3);
      launch_celf_topw(v, st);
    }
    {
      KTimer t(c, "celf_eval", st, 3);
      launch_celf_eval(v, st);
    }
    {
      KTimer t(c, "celf_bulk", st, 3);
      launch_celf_bulk(v, bulk_blocks, st);
    }
  }
}

im_status celf_collect(im_ctx* c, CelfBuffers* cb, hipStream_t st, uint32_t* seeds,
                       int64_t* marginal, int64_t* cover, uint64_t* evals) {
  const CelfView& v = cb->v;
  // seeds, marginals, the state and the persistent kernel's scratch (its
  // error word first; cleared at set-up, so 0 for the per-step kernels) lie
  // in this order in one allocation: one copy into a pinned record, one wait
  const char* d0 = reinterpret_cast<const char*>(v.seeds);
  const size_t o_marg = reinterpret_cast<const char*>(v.marginal) - d0,
               o_st = reinterpret_cast<const char*>(v.st) - d0,
               o_err = static_cast<const char*>(cb->pscratch) + pcelf_err_offset() - d0,
               span = o_err + sizeof(uint32_t);
  size_t cap = 0;
  char* h = static_cast<char*>(pinned_take(c, span, &cap));
  std::vector<char> pageable;
  if (!h) {
    pageable.resize(span);
    h = pageable.data();
  }
  hipError_t e = hipMemcpyAsync(h, d0, span, hipMemcpyDeviceToHost, st);
  const hipError_t es = hipStreamSynchronize(st);  // also when the copy failed: h is reused
  if (e == hipSuccess) e = es;
  im_status s;
  if (e != hipSuccess) {
    s = fail(IM_ERR_DEVICE, "CELF failed on the device: %s", hipGetErrorString(e));
  } else {
    uint32_t perr;
    CelfState hs;
    std::memcpy(&perr, h + o_err, sizeof(perr));
    std::memcpy(&hs, h + o_st, sizeof(hs));
    std::memcpy(seeds, h, (size_t)v.K * 4);
    std::memcpy(marginal, h + o_marg, (size_t)v.K * 8);
    s = celf_finish(c, cb, perr, hs, marginal, cover, evals);
  }
  if (pageable.empty()) pinned_give(c, h, cap);
  return s;
}

im_status celf_finish(im_ctx* c, const CelfBuffers* cb, uint32_t perr, const CelfState& hs,
                      const int64_t* marginal, int64_t* cover, uint64_t* evals) {
  const CelfView& v = cb->v;
  if (perr) return fail(IM_ERR_DEVICE, "persistent CELF kernel aborted (code %u)", perr);
  if (cb->persistent && c->profiling >= 3) {
    // phase clock of the persistent kernel: ticks of 10 ns per phase
    uint64_t pr[16];
    if (hipMemcpy(pr, static_cast<char*>(cb->pscratch) + pcelf_prof_offset(), sizeof(pr),
                  hipMemcpyDeviceToHost) == hipSuccess) {
      std::lock_guard<std::recursive_mutex> lk(c->mu);
      const char* names[10] = {"celf.barrier", "celf.eval",    "celf.commit", "celf.restale", "celf.prep",
                               "celf.post",    "celf.rebuild", "celf.bulk",   "celf.sort",    "celf.move"};
      const uint64_t counts[10] = {pr[12], pr[13], v.K, v.K, pr[13], pr[13], pr[14] & 0xFFFFFFFFu, pr[14] >> 32,
                                   v.K, v.K};
      for (int i = 0; i < 10; ++i) {
        auto& e = c->kstats[names[i]];
        e.first += counts[i];
        e.second += pr[i] * 1e-5;
      }
      c->kstats["celf.lookahead_commits"].first += pr[15];  // steps decided without a round
    }
    uint64_t wk[2];
    if (c->profiling >= 4 &&
        hipMemcpy(wk, static_cast<char*>(cb->pscratch) + pcelf_work_offset(), sizeof(wk), hipMemcpyDeviceToHost) ==
            hipSuccess) {
      std::lock_guard<std::recursive_mutex> lk(c->mu);
      c->kstats["celf.listed_tiles"].first += wk[0];  // listed (candidate, tile) pairs evaluated
      c->kstats["celf.gathers"].first += wk[1];       // their non-singleton columns
    }
  }
  if (hs.s != v.K) return fail(IM_ERR_DEVICE, "CELF committed %u of %u seeds", hs.s, v.K);
  int64_t tot = 0;
  for (uint32_t i = 0; i < v.K; ++i) tot += marginal[i];
  if (cover) *cover = tot;
  if (evals) *evals = hs.evals;
  c->last_bulk_rounds = hs.bulk_rounds;
  return IM_OK;
}

}  // namespace infuse

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------

extern "C" im_status im_ctx_create(int device, void* stream, const im_allocator* alloc,
                                   uint64_t hbm_budget, im_ctx** out) {
  if (!out) return fail(IM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
    return fail(IM_ERR_DEVICE, "device %d not available (%d devices)", device, count);
  if (hipSetDevice(device) != hipSuccess) return fail(IM_ERR_DEVICE, "hipSetDevice(%d) failed", device);
  // scratch of im_estimate_sigma_noalloc on this device (a failed lookup is
  // retried, and reported, by that call)
  (void)noalloc_scratch_setup(device);
  if (alloc && (!alloc->alloc || !alloc->free))
    return fail(IM_ERR_INVALID_ARG, "allocator needs both alloc and free");
  im_ctx* c = new im_ctx();
  c->device = device;
  c->budget = hbm_budget;
  if (alloc) {
    c->alloc = *alloc;
    c->has_alloc = true;
  }
  if (stream) {
    c->stream = static_cast<hipStream_t>(stream);
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return fail(IM_ERR_DEVICE, "stream creation failed");
    }
    c->own_stream = true;
  }
  if (hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking) != hipSuccess) c->aux = nullptr;
  c->tune.cc_chunk = 256;
  c->tune.celf_width = 16;
  c->tune.use_graphs = 0;
  c->tune.list_blocks = kListBlocks;
  c->coop_grid = pcelf_grid(device);
  c->tune.celf_mode = c->coop_grid ? 1 : 2;
  if (c->coop_grid && hipEventCreateWithFlags(&c->coop_done, hipEventDisableTiming) != hipSuccess) {
    c->coop_grid = 0;
    c->tune.celf_mode = 2;
  }
  *out = c;
  return IM_OK;
}

extern "C" void im_ctx_destroy(im_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  resolve_pending(c);
  while (!c->graphs.empty()) im_graph_free(c->graphs.back());
  sweep_graph_runs(c, true);
  if (c->arena.base) raw_free(c, c->arena.base);
  for (hipStream_t b : c->bstreams) {
    (void)hipStreamSynchronize(b);
    (void)hipStreamDestroy(b);
  }
  for (hipEvent_t e : c->bevents) (void)hipEventDestroy(e);
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  if (c->aux) {
    (void)hipStreamSynchronize(c->aux);
    (void)hipStreamDestroy(c->aux);
  }
  if (c->coop_done) (void)hipEventDestroy(c->coop_done);
  for (hipEvent_t e : c->fence_ev) (void)hipEventDestroy(e);
  for (auto& b : c->pinned) (void)hipHostFree(b.first);
  delete c;
}

extern "C" uint64_t im_ctx_bytes_in_use(const im_ctx* c) { return c ? c->in_use : 0; }

extern "C" im_status im_set_tuning(im_ctx* c, const im_tuning* t) {
  if (!c || !t) return fail(IM_ERR_INVALID_ARG, "NULL argument");
  if (t->cc_chunk) {
    const uint32_t tiles = t->cc_chunk / kTile;
    if (t->cc_chunk % kTile || tiles == 0 || tiles > 32 || (tiles & (tiles - 1)))
      return fail(IM_ERR_INVALID_ARG, "cc_chunk must be 256 * 2^k with 2^k <= 32");
    c->tune.cc_chunk = t->cc_chunk;
  }
  if (t->celf_width) {
    if (t->celf_width > 64) return fail(IM_ERR_INVALID_ARG, "celf_width must be <= 64");
    c->tune.celf_width = t->celf_width;
  }
  if (t->use_graphs) c->tune.use_graphs = t->use_graphs == 1 ? 1 : 0;
  if (t->celf_mode) {
    if (t->celf_mode > 2) return fail(IM_ERR_INVALID_ARG, "celf_mode must be 1 or 2");
    if (t->celf_mode == 1 && !c->coop_grid)
      return fail(IM_ERR_INVALID_ARG, "the device cannot run the persistent CELF kernel");
    c->tune.celf_mode = t->celf_mode;
  }
  if (t->celf_round0 != 0xFFFFFFFFu) {
    if (t->celf_round0 > 1024) return fail(IM_ERR_INVALID_ARG, "celf_round0 must be <= 1024");
    c->tune.celf_round0 = t->celf_round0;
  }
  if (t->list_blocks) {
    if (t->list_blocks < 256 || t->list_blocks > 65536)
      return fail(IM_ERR_INVALID_ARG, "list_blocks must be in 256 .. 65536");
    c->tune.list_blocks = t->list_blocks;
  }
  return IM_OK;
}

extern "C" im_status im_get_tuning(const im_ctx* c, im_tuning* t) {
  if (!c || !t) return fail(IM_ERR_INVALID_ARG, "NULL argument");
  *t = c->tune;
  return IM_OK;
}

extern "C" im_status im_set_profiling(im_ctx* c, int level) {
  if (!c) return fail(IM_ERR_INVALID_ARG, "NULL context");
  if (level < 0 || level > 4) return fail(IM_ERR_INVALID_ARG, "profiling level must be 0 to 4");
  c->profiling = level;
  return IM_OK;
}

extern "C" im_status im_reset_kernel_stats(im_ctx* c) {
  if (!c) return fail(IM_ERR_INVALID_ARG, "NULL context");
  resolve_pending(c);
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  c->kstats.clear();
  return IM_OK;
}

extern "C" im_status im_kernel_stats(im_ctx* c, const char* kernel, uint64_t* launches,
                                     double* total_ms) {
  if (!c || !kernel) return fail(IM_ERR_INVALID_ARG, "NULL argument");
  resolve_pending(c);
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  auto it = c->kstats.find(kernel);
  if (launches) *launches = it == c->kstats.end() ? 0 : it->second.first;
  if (total_ms) *total_ms = it == c->kstats.end() ? 0.0 : it->second.second;
  return IM_OK;
}

// ---------------------------------------------------------------------------
// graph
// ---------------------------------------------------------------------------

static im_status validate_csr(uint32_t n, uint64_t nnz, const uint64_t* rp, const uint32_t* col,
                              const double* p_slot, bool directed) {
  if (n == 0) return fail(IM_ERR_INVALID_GRAPH, "n must be >= 1");
  if (n >= (1u << 31)) return fail(IM_ERR_INVALID_GRAPH, "n must be < 2^31");
  if (nnz >= (1ull << 32)) return fail(IM_ERR_INVALID_GRAPH, "nnz must be < 2^32");
  if (!rp || (nnz && !col)) return fail(IM_ERR_INVALID_GRAPH, "NULL CSR array");
  if (rp[0] != 0 || rp[n] != nnz) return fail(IM_ERR_INVALID_GRAPH, "row_ptr must start at 0 and end at nnz");
  for (uint32_t u = 0; u < n; ++u) {
    if (rp[u + 1] < rp[u]) return fail(IM_ERR_INVALID_GRAPH, "row_ptr decreases at row %u", u);
    for (uint64_t j = rp[u]; j < rp[u + 1]; ++j) {
      const uint32_t v = col[j];
      if (v >= n) return fail(IM_ERR_INVALID_GRAPH, "neighbour id %u >= n in row %u", v, u);
      if (v == u) return fail(IM_ERR_INVALID_GRAPH, "self-loop at vertex %u", u);
      if (j > rp[u] && col[j - 1] >= v)
        return fail(IM_ERR_INVALID_GRAPH, "row %u is not strictly increasing", u);
      if (p_slot && (!(p_slot[j] >= 0.0) || !(p_slot[j] <= 1.0)))
        return fail(IM_ERR_INVALID_GRAPH, "p_slot[%llu] outside [0,1]", (unsigned long long)j);
      if (directed) continue;
      // symmetric: (v, u) must exist with the same probability
      const uint32_t* b = col + rp[v];
      const uint32_t* e = col + rp[v + 1];
      const uint32_t* f = std::lower_bound(b, e, u);
      if (f == e || *f != u) return fail(IM_ERR_INVALID_GRAPH, "edge (%u,%u) has no reverse", u, v);
      if (p_slot && p_slot[rp[v] + (f - b)] != p_slot[j])
        return fail(IM_ERR_INVALID_GRAPH, "p_slot differs between (%u,%u) and its reverse", u, v);
    }
  }
  return IM_OK;
}

static im_status load_graph(im_ctx* c, uint32_t n, uint64_t nnz, const uint64_t* row_ptr,
                            const uint32_t* col_idx, const double* p_slot, bool directed, im_graph** out) {
  if (!c || !out) return fail(IM_ERR_INVALID_ARG, "NULL argument");
  *out = nullptr;
  im_status s = validate_csr(n, nnz, row_ptr, col_idx, p_slot, directed);
  if (s != IM_OK) return s;
  // device CSR: with per-slot p, slots with T = 0 are never live and are
  // dropped; the rest keep T - 1 per slot
  std::vector<uint32_t> rp(n + 1), col, split(n), tm1;
  col.reserve(nnz);
  if (p_slot) tm1.reserve(nnz);
  for (uint32_t u = 0; u < n; ++u) {
    rp[u] = (uint32_t)col.size();
    for (uint64_t j = row_ptr[u]; j < row_ptr[u + 1]; ++j) {
      if (p_slot) {
        const uint64_t T = thr_of(p_slot[j]);
        if (T == 0) continue;
        tm1.push_back((uint32_t)(T - 1));
      }
      col.push_back(col_idx[j]);
    }
    split[u] = (uint32_t)(std::lower_bound(col.begin() + rp[u], col.end(), u) - col.begin());
  }
  rp[n] = (uint32_t)col.size();
  std::vector<uint32_t> src(col.size());
  for (uint32_t u = 0; u < n; ++u)
    for (uint32_t j = rp[u]; j < rp[u + 1]; ++j) src[j] = u;
  std::vector<uint32_t> hubs;
  std::vector<uint2> hub_piece;
  for (uint32_t u = 0; u < n; ++u)
    if (rp[u + 1] - rp[u] > (uint32_t)kWave) {
      hubs.push_back(u);
      for (uint32_t j = rp[u]; j < split[u]; j += kHubPiece) hub_piece.push_back(make_uint2(u, j));
    }
  im_graph* g = new im_graph();
  g->ctx = c;
  g->n = n;
  g->nnz_in = nnz;
  g->nnz = rp[n];
  g->per_edge = p_slot != nullptr;
  g->directed = directed;
  const size_t b_rp = align256((size_t)(n + 1) * 4), b_col = align256((size_t)g->nnz * 4 + 4);
  const size_t b_split = align256((size_t)n * 4), b_tm1 = p_slot ? align256((size_t)g->nnz * 4 + 4) : 0;
  const size_t b_hubs = align256((size_t)hubs.size() * 4 + 4);
  const size_t b_poff = align256((size_t)hub_piece.size() * 8 + 8);
  g->nhubs = (uint32_t)hubs.size();
  g->hub_pieces = (uint32_t)hub_piece.size();
  for (uint32_t u = 0; u < n; ++u) g->nlong += rp[u + 1] - rp[u] > kSplitArcs;
  void* base = nullptr;
  s = ctx_alloc(c, b_rp + b_col + b_split + b_tm1 + b_hubs + b_poff + b_col, &base);
  if (s != IM_OK) {
    delete g;
    return s;
  }
  g->gbuf = base;
  char* p8 = static_cast<char*>(base);
  g->row_ptr = reinterpret_cast<uint32_t*>(p8);
  g->col = reinterpret_cast<uint32_t*>(p8 + b_rp);
  g->split = reinterpret_cast<uint32_t*>(p8 + b_rp + b_col);
  g->tm1 = p_slot ? reinterpret_cast<uint32_t*>(p8 + b_rp + b_col + b_split) : nullptr;
  g->hubs = reinterpret_cast<uint32_t*>(p8 + b_rp + b_col + b_split + b_tm1);
  g->hub_piece = reinterpret_cast<uint2*>(p8 + b_rp + b_col + b_split + b_tm1 + b_hubs);
  g->src = reinterpret_cast<uint32_t*>(p8 + b_rp + b_col + b_split + b_tm1 + b_hubs + b_poff);
  hipError_t e = hipMemcpyAsync(g->row_ptr, rp.data(), (size_t)(n + 1) * 4, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess && g->nnz)
    e = hipMemcpyAsync(g->col, col.data(), (size_t)g->nnz * 4, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess && g->nnz)
    e = hipMemcpyAsync(g->src, src.data(), (size_t)g->nnz * 4, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(g->split, split.data(), (size_t)n * 4, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess && p_slot && g->nnz)
    e = hipMemcpyAsync(g->tm1, tm1.data(), (size_t)g->nnz * 4, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess && g->nhubs)
    e = hipMemcpyAsync(g->hubs, hubs.data(), (size_t)g->nhubs * 4, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess && g->hub_pieces)
    e = hipMemcpyAsync(g->hub_piece, hub_piece.data(), hub_piece.size() * 8, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    ctx_free(c, base);
    delete g;
    return fail(IM_ERR_DEVICE, "graph upload failed: %s", hipGetErrorString(e));
  }
  for (int i = 0; i < 6; ++i) (void)hipEventCreate(&g->ev[i]);
  {
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    c->graphs.push_back(g);
  }
  *out = g;
  return IM_OK;
}

extern "C" im_status im_graph_load_csr(im_ctx* c, uint32_t n, uint64_t nnz, const uint64_t* row_ptr,
                                       const uint32_t* col_idx, const double* p_slot, im_graph** out) {
  return load_graph(c, n, nnz, row_ptr, col_idx, p_slot, false, out);
}

extern "C" im_status im_graph_load_arcs(im_ctx* c, uint32_t n, uint64_t nnz, const uint64_t* row_ptr,
                                        const uint32_t* col_idx, const double* p_slot, im_graph** out) {
  return load_graph(c, n, nnz, row_ptr, col_idx, p_slot, true, out);
}

extern "C" void im_graph_free(im_graph* g) {
  if (!g) return;
  im_ctx* c = g->ctx;
  (void)hipStreamSynchronize(c->stream);
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  while (!g->memos.empty()) memo_destroy(g, g->memos.back());
  ctx_free(c, g->gbuf);
  for (int i = 0; i < 6; ++i)
    if (g->ev[i]) (void)hipEventDestroy(g->ev[i]);
  auto& v = c->graphs;
  v.erase(std::remove(v.begin(), v.end(), g), v.end());
  delete g;
}

extern "C" uint32_t im_graph_n(const im_graph* g) { return g ? g->n : 0; }
extern "C" uint64_t im_graph_nnz(const im_graph* g) { return g ? g->nnz_in : 0; }

im_status infuse::check_params(const im_graph* g, double p, uint32_t R) {
  if (R == 0) return fail(IM_ERR_INVALID_ARG, "R must be >= 1");
  if (R > (1u << 24)) return fail(IM_ERR_INVALID_ARG, "R must be <= 2^24");
  if (!(p >= 0.0) || !(p <= 1.0)) return fail(IM_ERR_INVALID_ARG, "p must be in [0,1]");
  // keys pack gain (<= n*R) above bitlen(n) id bits in 64 bits
  const unsigned __int128 lim = (unsigned __int128)g->n * R << key_bits(g->n);
  if (lim >> 64) return fail(IM_ERR_INVALID_ARG, "n*R too large for 64-bit CELF keys");
  const unsigned __int128 words = (unsigned __int128)g->n * round_up(R, kTile);
  if (words >> 40) return fail(IM_ERR_INVALID_ARG, "memo larger than 4 TiB");
  // work-list entries are v * ntiles + t in 32 bits
  if ((uint64_t)g->n * (round_up(R, kTile) / kTile) >= (1ull << 32))
    return fail(IM_ERR_INVALID_ARG, "n * ceil(R / 256) must be below 2^32");
  return IM_OK;
}

extern "C" im_status im_set_params(im_graph* g, double p, uint32_t R, uint32_t hash_seed) {
  if (!g) return fail(IM_ERR_INVALID_ARG, "NULL graph");
  im_status s = check_params(g, p, R);
  if (s != IM_OK) return s;
  g->p = p;
  g->R = R;
  g->seed = hash_seed;
  g->params_set = true;
  return IM_OK;
}

// Phase times of the last construction, once its events completed.
static void read_build_phases(im_graph* g) {
  if (!g->timed_build) return;
  float a = 0, b = 0, c = 0;
  (void)hipEventElapsedTime(&a, g->ev[0], g->ev[1]);
  (void)hipEventElapsedTime(&b, g->ev[1], g->ev[2]);
  (void)hipEventElapsedTime(&c, g->ev[2], g->ev[3]);
  g->phase_ms[0] = a;
  g->phase_ms[1] = b;
  g->phase_ms[2] = c;
  g->timed_build = false;
}

extern "C" im_status im_build_memo(im_graph* g) {
  if (!g) return fail(IM_ERR_INVALID_ARG, "NULL graph");
  Memo* m = nullptr;
  im_status s = memo_acquire(g, &m);
  if (s != IM_OK) return s;
  hipError_t e = hipStreamSynchronize(g->ctx->stream);
  if (e == hipSuccess) read_build_phases(g);
  memo_release(g, m);
  if (e != hipSuccess) return fail(IM_ERR_DEVICE, "memo construction failed: %s", hipGetErrorString(e));
  return IM_OK;
}

extern "C" im_status im_drop_memo(im_graph* g) {
  if (!g) return fail(IM_ERR_INVALID_ARG, "NULL graph");
  (void)hipStreamSynchronize(g->ctx->stream);
  std::lock_guard<std::recursive_mutex> lk(g->ctx->mu);
  std::vector<Memo*> keep;
  for (Memo* m : std::vector<Memo*>(g->memos))
    if (m->pins == 0) memo_destroy(g, m);
  return IM_OK;
}

extern "C" im_status im_select_seeds(im_graph* g, uint32_t K, uint32_t* seeds, int64_t* marginal,
                                     int64_t* cover_count) {
  if (!g) return fail(IM_ERR_INVALID_ARG, "NULL graph");
  if (K > g->n) return fail(IM_ERR_INVALID_ARG, "K = %u exceeds n = %u", K, g->n);
  if (K && (!seeds || !marginal)) return fail(IM_ERR_INVALID_ARG, "NULL output array");
  if (K == 0) {
    if (cover_count) *cover_count = 0;
    return IM_OK;
  }
  im_ctx* c = g->ctx;
  Memo* m = nullptr;
  im_status s = memo_acquire(g, &m);
  if (s != IM_OK) return s;
  CelfBuffers cb;
  s = celf_alloc(g, m, K, c->tune.celf_width, &cb);
  if (s != IM_OK) {
    memo_release(g, m);
    return s;
  }
  (void)hipEventRecord(g->ev[4], c->stream);
  celf_enqueue(c, &cb, c->stream);
  (void)hipEventRecord(g->ev[5], c->stream);
  std::vector<uint32_t> hs(K);
  std::vector<int64_t> hm(K);
  int64_t cover = 0;
  uint64_t evals = 0;
  s = celf_collect(c, &cb, c->stream, hs.data(), hm.data(), &cover, &evals);
  if (s == IM_OK) {
    float ms = 0;
    (void)hipEventElapsedTime(&ms, g->ev[4], g->ev[5]);
    g->phase_ms[3] = ms;
    read_build_phases(g);
    g->last_evals = evals;
    std::memcpy(seeds, hs.data(), (size_t)K * 4);
    std::memcpy(marginal, hm.data(), (size_t)K * 8);
    if (cover_count) *cover_count = cover;
  }
  ctx_free(c, cb.base);
  memo_release(g, m);
  return s;
}

// Dedups S; returns IM_ERR_INVALID_ARG for an id >= n.
im_status infuse::normalize_set(const im_graph* g, const uint32_t* S, uint32_t len, std::vector<uint32_t>* out) {
  out->assign(S, S + len);
  for (uint32_t x : *out)
    if (x >= g->n) return fail(IM_ERR_INVALID_ARG, "seed id %u >= n = %u", x, g->n);
  std::sort(out->begin(), out->end());
  out->erase(std::unique(out->begin(), out->end()), out->end());
  return IM_OK;
}

im_status infuse::sigma_enqueue(im_graph* g, Memo* m, const std::vector<uint32_t>& S, hipStream_t st,
                        void** scratch, unsigned long long** dev_out, const void* staged) {
  im_ctx* c = g->ctx;
  const uint32_t len = (uint32_t)S.size();
  const bool pair = len <= sigma_pair_max();
  const uint32_t cwords = m->Rs / 32;
  size_t b = align256(8) + align256((size_t)len * 4);
  if (!pair) b += align256((size_t)g->n * cwords * 4);
  void* base = nullptr;
  im_status s = ctx_alloc(c, b, &base);
  if (s != IM_OK) return s;
  char* p8 = static_cast<char*>(base);
  auto* out = reinterpret_cast<unsigned long long*>(p8);
  auto* dS = reinterpret_cast<uint32_t*>(p8 + align256(8));
  uint32_t* bm = pair ? nullptr : reinterpret_cast<uint32_t*>(p8 + align256(8) + align256((size_t)len * 4));
  if (staged) {
    (void)hipMemcpyAsync(base, staged, align256(8) + (size_t)len * 4, hipMemcpyHostToDevice, st);
  } else {
    launch_fill_u32(reinterpret_cast<uint32_t*>(out), 2, 0u, st);
    if (len) (void)hipMemcpyAsync(dS, S.data(), (size_t)len * 4, hipMemcpyHostToDevice, st);
  }
  const MemoView mv = m->view(g);
  {
    KTimer t(c, "sigma", st);
    if (pair) {
      if (len) launch_sigma_pair(mv, dS, len, out, st);
    } else {
      launch_fill_u32(bm, (uint64_t)g->n * cwords, 0u, st);
      launch_sigma_bitmap(mv, dS, len, bm, cwords, out, st);
    }
  }
  *scratch = base;
  *dev_out = out;
  return IM_OK;
}

extern "C" im_status im_estimate_sigma(im_graph* g, const uint32_t* S, uint32_t s_len, int64_t* count,
                                       double* sigma) {
  if (!g) return fail(IM_ERR_INVALID_ARG, "NULL graph");
  if (s_len && !S) return fail(IM_ERR_INVALID_ARG, "NULL seed array");
  std::vector<uint32_t> set;
  im_status s = normalize_set(g, S, s_len, &set);
  if (s != IM_OK) return s;
  if (!g->params_set) return fail(IM_ERR_INVALID_ARG, "im_set_params has not been called");
  if (set.empty()) {
    if (count) *count = 0;
    if (sigma) *sigma = 0.0;
    return IM_OK;
  }
  im_ctx* c = g->ctx;
  Memo* m = nullptr;
  s = memo_acquire(g, &m);
  if (s != IM_OK) return s;
  void* scratch = nullptr;
  unsigned long long* dout = nullptr;
  // pinned staging laid out as the device block: the count (zero) at 0, the
  // seed ids from byte 256
  size_t cap = 0;
  char* hp = static_cast<char*>(pinned_take(c, 256 + set.size() * 4, &cap));
  if (hp) {
    std::memset(hp, 0, 256);
    std::memcpy(hp + 256, set.data(), set.size() * 4);
  }
  s = sigma_enqueue(g, m, set, c->stream, &scratch, &dout, hp);
  if (s == IM_OK) {
    unsigned long long hpg = 0;
    unsigned long long* h = hp ? reinterpret_cast<unsigned long long*>(hp) : &hpg;
    hipError_t e = hipMemcpyAsync(h, dout, 8, hipMemcpyDeviceToHost, c->stream);
    const hipError_t es = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = es;
    if (e != hipSuccess) {
      s = fail(IM_ERR_DEVICE, "sigma failed: %s", hipGetErrorString(e));
    } else {
      if (count) *count = (int64_t)*h;
      if (sigma) *sigma = (double)*h / (double)g->R;
    }
    ctx_free(c, scratch);
  } else {
    (void)hipStreamSynchronize(c->stream);  // an upload from hp may be queued
  }
  pinned_give(c, hp, cap);
  memo_release(g, m);
  return s;
}

// The levels of a search, enqueued in groups: each level reads its
// frontier size on the device (an empty frontier makes the rest no-ops) and
// the host looks at it once per group.  The first group has `first` levels
// (a caller's guess of the depth, 8 to 64: a surplus level costs two empty
// launches, a missing one a host round trip), the later ones 8.  The
// seed kernel has set the list sizes of level 1; frontier sets fa / fb and
// lists la / lb alternate.
static hipError_t bfs_levels(im_ctx* c, const GraphView& gv, const MemoView& mv, BfsView bv, uint64_t* fa,
                             uint64_t* fb, uint32_t* la, uint32_t* lb, hipStream_t st, uint32_t* levels,
                             uint32_t first = 8) {
  hipError_t e = hipSuccess;
  for (uint32_t level = 1, group = std::min(std::max(first, 8u), 64u);; group = 8) {
    for (uint32_t k = 0; k < group; ++k, ++level) {
      bv.F = fa;
      bv.N = fb;
      bv.cur = la;
      bv.next = lb;
      {
        KTimer t(c, "bfs_level", st, 1);
        launch_bfs_level(gv, mv, bv, level, st);
      }
      launch_bfs_compact(bv, level, st);
      std::swap(fa, fb);
      std::swap(la, lb);
    }
    uint32_t h = 0;
    e = hipMemcpyAsync(&h, bv.lcount + level % 3, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess || h == 0) break;
  }
  uint32_t lv = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&lv, bv.levels, 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (levels) *levels = lv;
  return e;
}

extern "C" im_status im_estimate_sigma_direct(im_graph* g, const uint32_t* S, uint32_t s_len, int64_t* count,
                                              double* sigma, uint32_t* levels) {
  if (!g) return fail(IM_ERR_INVALID_ARG, "NULL graph");
  if (s_len && !S) return fail(IM_ERR_INVALID_ARG, "NULL seed array");
  std::vector<uint32_t> set;
  im_status s = normalize_set(g, S, s_len, &set);
  if (s != IM_OK) return s;
  if (!g->params_set) return fail(IM_ERR_INVALID_ARG, "im_set_params has not been called");
  if (levels) *levels = 0;
  if (set.empty()) {
    if (count) *count = 0;
    if (sigma) *sigma = 0.0;
    return IM_OK;
  }
  im_ctx* c = g->ctx;
  hipStream_t st = c->stream;
  const uint32_t n = g->n, R = g->R, Rs = round_up(R, kTile), ntiles = Rs / kTile, len = (uint32_t)set.size();
  const uint64_t T = thr_of(g->p);
  const uint64_t words = (uint64_t)n * ntiles * 4;
  // one allocation: sampler state, visited and two frontier bitsets, two
  // frontier lists, the next frontier's bitmap, counters, S
  const size_t b_edges = align256((size_t)g->nnz * 8), b_x = align256((size_t)Rs * 4);
  const size_t b_pos = align256((size_t)R * 4), b_scr = align256((size_t)x_sort_scratch_elems(R) * 8);
  if ((uint64_t)n * ntiles > UINT32_MAX) return fail(IM_ERR_INVALID_ARG, "n * ceil(R / 256) exceeds 2^32 - 1");
  // long rows are split into kPieces entries when item ids leave room for the piece
  const uint32_t pieces = (uint64_t)n * ntiles <= (1ull << kPieceShift) && g->nlong ? kPieces : 1u;
  const uint64_t entries = ((uint64_t)n + (uint64_t)(pieces - 1) * g->nlong) * ntiles;
  const size_t b_bits = align256((size_t)words * 8), b_list = align256((size_t)entries * 4);
  const size_t b_nb = align256(((size_t)n * ntiles + 63) / 64 * 8), b_hm = pieces > 1 ? b_nb : 0;
  // cnt: [0..2] list sizes, [3] levels; then the count slots and the work counts
  const size_t o_counts = 64, o_stats = align256(o_counts + kCountSlots * 8);
  const size_t b_cnt = align256(o_stats + kCountSlots * 24), b_S = align256((size_t)len * 4);
  const size_t total = b_edges + 2 * b_x + b_pos + b_scr + 3 * b_bits + 2 * b_list + b_nb + b_cnt + b_S + b_hm;
  void* base = nullptr;
  s = ctx_alloc(c, total, &base);
  if (s != IM_OK) return s;
  char* p8 = static_cast<char*>(base);
  auto take = [&](size_t bytes) {
    char* r = p8;
    p8 += bytes;
    return r;
  };
  MemoView mv = {};
  mv.n = n;
  mv.R = R;
  mv.Rs = Rs;
  mv.ntiles = ntiles;
  mv.never_live = (!g->per_edge && T == 0) ? 1u : 0u;
  mv.tm1 = (g->per_edge || T == 0) ? 0u : (uint32_t)(T - 1);
  mv.kshift = bitlen32(mv.tm1);
  uint2* edges = reinterpret_cast<uint2*>(take(b_edges));
  uint32_t* xs = reinterpret_cast<uint32_t*>(take(b_x));
  uint32_t* inv = reinterpret_cast<uint32_t*>(take(b_x));
  uint32_t* pos = reinterpret_cast<uint32_t*>(take(b_pos));
  uint64_t* scr = reinterpret_cast<uint64_t*>(take(b_scr));
  uint64_t* V = reinterpret_cast<uint64_t*>(take(b_bits));
  uint64_t* A = reinterpret_cast<uint64_t*>(take(b_bits));
  uint64_t* B = reinterpret_cast<uint64_t*>(take(b_bits));
  uint32_t* L0 = reinterpret_cast<uint32_t*>(take(b_list));
  uint32_t* L1 = reinterpret_cast<uint32_t*>(take(b_list));
  uint64_t* nbits = reinterpret_cast<uint64_t*>(take(b_nb));
  uint32_t* cnt = reinterpret_cast<uint32_t*>(take(b_cnt));
  uint32_t* dS = reinterpret_cast<uint32_t*>(take(b_S));
  uint64_t* hubmask = pieces > 1 ? reinterpret_cast<uint64_t*>(take(b_hm)) : nullptr;
  unsigned long long* counts = reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(cnt) + o_counts);
  unsigned long long* wstats = reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(cnt) + o_stats);
  mv.edges = edges;
  mv.xs = xs;
  const GraphView gv = g->view();
  launch_edge_hash(gv, g->seed, edges, st);
  launch_x_sort(g->seed, R, Rs, scr, xs, inv, pos, st);
  launch_fill_u32(reinterpret_cast<uint32_t*>(V), (uint64_t)(3 * b_bits + 2 * b_list + b_nb + b_cnt) / 4, 0u, st);
  hipError_t e = hipMemcpyAsync(dS, set.data(), (size_t)len * 4, hipMemcpyHostToDevice, st);
  BfsView bv = {};
  bv.n = n;
  bv.gn = n;
  bv.ntiles = ntiles;
  bv.V = V;
  bv.N = A;
  bv.next = L0;
  bv.lcount = cnt;
  bv.levels = cnt + 3;
  bv.nbits = nbits;
  bv.counts = counts;
  bv.stats = c->profiling >= 1 ? wstats : nullptr;  // work counts cost atomics: kept while profiling
  bv.pieces = pieces;
  bv.hubmask = hubmask;
  uint32_t nlev = 0;
  {
    KTimer t(c, "sigma_direct", st);
    if (hubmask) launch_bfs_hubmask(gv, bv, hubmask, st);
    launch_bfs_seed(gv, mv, bv, dS, len, st);  // the seeds: visited, and the first frontier in A / L0
    if (e == hipSuccess) e = bfs_levels(c, gv, mv, bv, A, B, L0, L1, st, &nlev, g->spread_depth + 2);
  }
  std::vector<unsigned long long> hb(b_cnt / 8);
  if (e == hipSuccess) e = hipMemcpyAsync(hb.data(), cnt, b_cnt, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  const unsigned long long* hc = hb.data() + o_counts / 8;
  const unsigned long long* hs = hb.data() + o_stats / 8;
  ctx_free(c, base);
  if (e != hipSuccess) return fail(IM_ERR_DEVICE, "memo-free sigma failed: %s", hipGetErrorString(e));
  unsigned long long h = 0;
  for (uint32_t k = 0; k < kCountSlots; ++k) h += hc[k];
  g->last_search[0] = nlev;
  g->spread_depth = nlev;
  for (int k = 1; k < 4; ++k) g->last_search[k] = 0;
  for (uint32_t k = 0; k < kCountSlots; ++k)
    for (int j = 0; j < 3; ++j) g->last_search[1 + j] += hs[k * 3 + j];
  if (count) *count = (int64_t)h;
  if (sigma) *sigma = (double)h / (double)R;
  if (levels) *levels = nlev;
  return IM_OK;
}

// Greedy selection without a memo.  The gains are spreads over uncovered
// vertices, computed by the level-synchronous search: a batch of candidates
// is searched side by side as copies of the graph, each copy's visited set
// starting from the covered set R_r(S) of every sample, so a copy's new bits
// are the candidate's gain.  The lazy queue (on the host) commits the largest
// key when it is fresh, ties to the smaller id, and otherwise re-evaluates
// the largest stale keys that still rank above the best fresh one (no other
// can win this step), as many as fit side by side; every key starts
// unevaluated.  A commit grows the covered set by one more search.
extern "C" im_status im_select_seeds_direct(im_graph* g, uint32_t K, uint32_t* seeds, int64_t* marginal,
                                            int64_t* cover_count) {
  if (!g) return fail(IM_ERR_INVALID_ARG, "NULL graph");
  if (!g->params_set) return fail(IM_ERR_INVALID_ARG, "im_set_params has not been called");
  if (K > g->n) return fail(IM_ERR_INVALID_ARG, "K = %u exceeds n = %u", K, g->n);
  if (K && (!seeds || !marginal)) return fail(IM_ERR_INVALID_ARG, "NULL output array");
  if (cover_count) *cover_count = 0;
  if (K == 0) return IM_OK;
  im_ctx* c = g->ctx;
  hipStream_t st = c->stream;
  const uint32_t n = g->n, R = g->R, Rs = round_up(R, kTile), ntiles = Rs / kTile;
  const uint64_t T = thr_of(g->p);
  const uint64_t words = (uint64_t)n * ntiles * 4;  // u64 words of one copy's bit sets
  // list entries per copy: one per item, kPieces for an item of a long row (split when ids leave room)
  const uint64_t entries_max = ((uint64_t)n + (uint64_t)(kPieces - 1) * g->nlong) * ntiles;
  const uint64_t per_copy = 3 * words * 8 + 2 * entries_max * 4 + (uint64_t)n * ntiles / 4 + 1;
  const uint64_t copy_budget = 8ull << 30;
  if ((uint64_t)n * ntiles > UINT32_MAX) return fail(IM_ERR_INVALID_ARG, "n * ceil(R / 256) exceeds 2^32 - 1");
  // copies * n * ntiles level items must fit in 32 bits
  const uint32_t copies = (uint32_t)std::max<uint64_t>(
      1, std::min<uint64_t>({1024, n, copy_budget / per_copy, (uint64_t)UINT32_MAX / ((uint64_t)n * ntiles)}));
  const size_t b_edges = align256((size_t)g->nnz * 8), b_x = align256((size_t)Rs * 4);
  const size_t b_pos = align256((size_t)R * 4), b_scr = align256((size_t)x_sort_scratch_elems(R) * 8);
  const size_t b_one = align256((size_t)words * 8), b_many = align256((size_t)words * 8 * copies);
  // lc: [0..2] list sizes, [3] levels; then the work counts and the count slots of each copy
  const size_t o_stats = 64, o_counts = align256(o_stats + kCountSlots * 24);
  const uint32_t pieces = (uint64_t)n * ntiles * copies <= (1ull << kPieceShift) && g->nlong ? kPieces : 1u;
  const uint64_t entries = ((uint64_t)n + (uint64_t)(pieces - 1) * g->nlong) * ntiles * copies;
  const size_t b_list = align256((size_t)entries * 4), b_cnt = align256(o_counts + (size_t)copies * kCountSlots * 8);
  const size_t b_nb = align256(((size_t)n * ntiles * copies + 63) / 64 * 8), b_S = align256((size_t)copies * 4);
  const size_t b_hm = pieces > 1 ? b_nb : 0;
  const size_t total = b_edges + 2 * b_x + b_pos + b_scr + b_one + 3 * b_many + 2 * b_list + b_nb + b_cnt + b_S + b_hm;
  void* base = nullptr;
  im_status s = ctx_alloc(c, total, &base);
  if (s != IM_OK) return s;
  char* p8 = static_cast<char*>(base);
  auto take = [&](size_t bytes) {
    char* r = p8;
    p8 += bytes;
    return r;
  };
  MemoView mv = {};
  mv.n = n;
  mv.R = R;
  mv.Rs = Rs;
  mv.ntiles = ntiles;
  mv.never_live = (!g->per_edge && T == 0) ? 1u : 0u;
  mv.tm1 = (g->per_edge || T == 0) ? 0u : (uint32_t)(T - 1);
  mv.kshift = bitlen32(mv.tm1);
  uint2* edges = reinterpret_cast<uint2*>(take(b_edges));
  uint32_t* xs = reinterpret_cast<uint32_t*>(take(b_x));
  uint32_t* inv = reinterpret_cast<uint32_t*>(take(b_x));
  uint32_t* pos = reinterpret_cast<uint32_t*>(take(b_pos));
  uint64_t* scr = reinterpret_cast<uint64_t*>(take(b_scr));
  uint64_t* Vs = reinterpret_cast<uint64_t*>(take(b_one));  // covered: R_r(S), one copy
  uint64_t* V = reinterpret_cast<uint64_t*>(take(b_many));
  uint64_t* A = reinterpret_cast<uint64_t*>(take(b_many));
  uint64_t* B = reinterpret_cast<uint64_t*>(take(b_many));
  uint32_t* L0 = reinterpret_cast<uint32_t*>(take(b_list));
  uint32_t* L1 = reinterpret_cast<uint32_t*>(take(b_list));
  uint64_t* nbits = reinterpret_cast<uint64_t*>(take(b_nb));
  uint32_t* lc = reinterpret_cast<uint32_t*>(take(b_cnt));
  unsigned long long* wstats = reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(lc) + o_stats);
  unsigned long long* counts = reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(lc) + o_counts);
  uint32_t* dS = reinterpret_cast<uint32_t*>(take(b_S));
  uint64_t* hubmask = pieces > 1 ? reinterpret_cast<uint64_t*>(take(b_hm)) : nullptr;
  mv.edges = edges;
  mv.xs = xs;
  const GraphView gv = g->view();
  launch_edge_hash(gv, g->seed, edges, st);
  launch_x_sort(g->seed, R, Rs, scr, xs, inv, pos, st);
  launch_fill_u32(reinterpret_cast<uint32_t*>(Vs), words * 2, 0u, st);
  if (hubmask) {  // over the items of every copy
    BfsView hv = {};
    hv.n = n * copies;
    hv.gn = n;
    hv.ntiles = ntiles;
    launch_bfs_hubmask(gv, hv, hubmask, st);
  }
  // the frontier sets and the bitmap start zero and every search leaves them zero
  launch_fill_u32(reinterpret_cast<uint32_t*>(A), words * 2 * copies, 0u, st);
  launch_fill_u32(reinterpret_cast<uint32_t*>(B), words * 2 * copies, 0u, st);
  launch_fill_u32(reinterpret_cast<uint32_t*>(nbits), b_nb / 4, 0u, st);
  launch_fill_u32(reinterpret_cast<uint32_t*>(wstats), kCountSlots * 3 * 2, 0u, st);
  uint64_t total_levels = 0;
  hipError_t e = hipSuccess;
  std::vector<uint32_t> hsrc(copies);
  std::vector<unsigned long long> hcnt((size_t)copies * kCountSlots);
  // searches from the sources src[c] of copies 0 .. nc-1, each over the
  // visited set Vv (nc copies); counts[c] receives copy c's new bits
  uint32_t depth[2] = {0, 0};  // levels of the last batch search and of the last commit search
  auto search = [&](uint64_t* Vv, uint32_t nc) {
    launch_fill_u32(reinterpret_cast<uint32_t*>(counts), (uint64_t)nc * kCountSlots * 2, 0u, st);
    launch_fill_u32(lc, 4, 0u, st);  // list sizes and level count
    if (e == hipSuccess) e = hipMemcpyAsync(dS, hsrc.data(), (size_t)nc * 4, hipMemcpyHostToDevice, st);
    BfsView bv = {};
    bv.n = n * nc;
    bv.gn = n;
    bv.ntiles = ntiles;
    bv.V = Vv;
    bv.N = A;
    bv.next = L0;
    bv.lcount = lc;
    bv.levels = lc + 3;
    bv.nbits = nbits;
    bv.counts = counts;
    bv.stats = c->profiling >= 1 ? wstats : nullptr;
    bv.pieces = pieces;
    bv.hubmask = hubmask;
    launch_bfs_seed(gv, mv, bv, dS, nc, st);
    uint32_t lv = 0;
    uint32_t& d = depth[Vv == Vs ? 1 : 0];
    if (e == hipSuccess) e = bfs_levels(c, gv, mv, bv, A, B, L0, L1, st, &lv, d + 2);
    d = lv;
    total_levels += lv;
  };
  std::vector<int64_t> key(n, INT64_MAX), when(n, -1);
  std::vector<uint8_t> chosen(n, 0);
  std::vector<uint32_t> order;
  int64_t cover = 0;
  uint64_t evals = 0;
  {
    KTimer t(c, "select_direct", st);
    uint32_t step = 0, rounds = 0;  // evaluation rounds of this step
    auto before = [&](uint32_t a, uint32_t b) { return key[a] != key[b] ? key[a] > key[b] : a < b; };
    while (e == hipSuccess && step < K) {
      uint32_t top = kInvalid;
      for (uint32_t v = 0; v < n; ++v)
        if (!chosen[v] && (top == kInvalid || before(v, top))) top = v;
      if (when[top] == (int64_t)step) {  // fresh: the exact maximiser
        hsrc[0] = top;
        search(Vs, 1);
        seeds[step] = top;
        marginal[step] = key[top];
        cover += key[top];
        chosen[top] = 1;
        ++step;
        rounds = 0;
        continue;
      }
      // the largest stale keys above the best fresh one, as many as fit side by side
      uint32_t best_fresh = kInvalid;
      for (uint32_t v = 0; v < n; ++v)
        if (!chosen[v] && when[v] == (int64_t)step && (best_fresh == kInvalid || before(v, best_fresh))) best_fresh = v;
      order.clear();
      for (uint32_t v = 0; v < n; ++v)
        if (!chosen[v] && when[v] != (int64_t)step && (best_fresh == kInvalid || before(v, best_fresh)))
          order.push_back(v);
      // never-evaluated keys fill whole batches; re-evaluations start at 64
      // candidates per step and double with every further round
      const uint32_t room = key[top] == INT64_MAX ? copies : std::min<uint32_t>(copies, 64u << std::min(rounds, 10u));
      ++rounds;
      const uint32_t nc = std::min<uint32_t>(room, (uint32_t)order.size());
      std::partial_sort(order.begin(), order.begin() + nc, order.end(), before);
      for (uint32_t i = 0; i < nc; ++i) hsrc[i] = i * n + order[i];
      launch_bfs_replicate(Vs, V, words, nc, st);
      search(V, nc);
      if (e == hipSuccess)
        e = hipMemcpyAsync(hcnt.data(), counts, (size_t)nc * kCountSlots * 8, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      for (uint32_t i = 0; i < nc && e == hipSuccess; ++i) {
        int64_t gain = 0;  // bits of the copy beyond the covered set
        for (uint32_t k = 0; k < kCountSlots; ++k) gain += (int64_t)hcnt[(size_t)i * kCountSlots + k];
        key[order[i]] = gain;
        when[order[i]] = step;
      }
      evals += nc;
    }
  }
  std::vector<unsigned long long> hw(kCountSlots * 3);
  if (e == hipSuccess) e = hipMemcpyAsync(hw.data(), wstats, hw.size() * 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  ctx_free(c, base);
  if (e != hipSuccess) return fail(IM_ERR_DEVICE, "memo-free selection failed: %s", hipGetErrorString(e));
  if (cover_count) *cover_count = cover;
  g->last_evals = evals;
  g->last_search[0] = total_levels;
  for (int k = 1; k < 4; ++k) g->last_search[k] = 0;
  for (uint32_t k = 0; k < kCountSlots; ++k)
    for (int j = 0; j < 3; ++j) g->last_search[1 + j] += hw[k * 3 + j];
  return IM_OK;
}

extern "C" im_status im_last_search_stats(const im_graph* g, uint64_t* out4) {
  if (!g || !out4) return fail(IM_ERR_INVALID_ARG, "NULL argument");
  for (int k = 0; k < 4; ++k) out4[k] = g->last_search[k];
  return IM_OK;
}

static im_status export_range(im_graph* g, int32_t* host, uint64_t first, uint32_t cnt, int mode) {
  if (!g) return fail(IM_ERR_INVALID_ARG, "NULL graph");
  if (!g->params_set) return fail(IM_ERR_INVALID_ARG, "im_set_params has not been called");
  if (first > g->R || cnt > g->R - first) return fail(IM_ERR_INVALID_ARG, "sample range exceeds R");
  if (cnt == 0) return IM_OK;
  if (!host) return fail(IM_ERR_INVALID_ARG, "NULL output");
  im_ctx* c = g->ctx;
  Memo* m = nullptr;
  im_status s = memo_acquire(g, &m);
  if (s != IM_OK) return s;
  const uint64_t max_words = 64ull << 20;  // staging chunk: 256 MiB
  uint32_t vchunk = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(g->n, max_words / cnt));
  void* buf = nullptr;
  s = ctx_alloc(c, (size_t)vchunk * cnt * 4, &buf);
  if (s != IM_OK) {
    memo_release(g, m);
    return s;
  }
  const MemoView mv = m->view(g);
  for (uint32_t v0 = 0; v0 < g->n && s == IM_OK; v0 += vchunk) {
    const uint32_t nv = std::min(vchunk, g->n - v0);
    launch_export(mv, m->pos, (uint32_t)first, cnt, v0, nv, mode, static_cast<int32_t*>(buf), c->stream);
    hipError_t e = hipMemcpyAsync(host + (uint64_t)v0 * cnt, buf, (size_t)nv * cnt * 4,
                                  hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) s = fail(IM_ERR_DEVICE, "export failed: %s", hipGetErrorString(e));
  }
  ctx_free(c, buf);
  memo_release(g, m);
  return s;
}

extern "C" im_status im_copy_labels(im_graph* g, int32_t* host, uint64_t first, uint32_t n_samples) {
  return export_range(g, host, first, n_samples, 0);
}

extern "C" im_status im_copy_sizes(im_graph* g, int32_t* host, uint64_t first, uint32_t n_samples) {
  return export_range(g, host, first, n_samples, 1);
}

extern "C" im_status im_copy_gains0(im_graph* g, int64_t* host) {
  if (!g || !host) return fail(IM_ERR_INVALID_ARG, "NULL argument");
  Memo* m = nullptr;
  im_status s = memo_acquire(g, &m);
  if (s != IM_OK) return s;
  hipError_t e = hipMemcpyAsync(host, m->g0, (size_t)g->n * 8, hipMemcpyDeviceToHost, g->ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(g->ctx->stream);
  memo_release(g, m);
  if (e != hipSuccess) return fail(IM_ERR_DEVICE, "copy failed: %s", hipGetErrorString(e));
  return IM_OK;
}

extern "C" im_status im_last_phase_ms(const im_graph* g, double* ms4) {
  if (!g || !ms4) return fail(IM_ERR_INVALID_ARG, "NULL argument");
  for (int i = 0; i < 4; ++i) ms4[i] = g->phase_ms[i];
  return IM_OK;
}

extern "C" uint64_t im_last_celf_evals(const im_graph* g) { return g ? g->last_evals : 0; }

extern "C" im_status im_memo_work(im_graph* g, uint64_t* out, uint32_t n_out) {
  if (!g || (n_out && !out)) return fail(IM_ERR_INVALID_ARG, "NULL argument");
  if (!g->params_set) return fail(IM_ERR_INVALID_ARG, "im_set_params has not been called");
  im_ctx* c = g->ctx;
  Memo* m = nullptr;
  {
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    m = memo_find(g, g->p, g->R, g->seed);
    if (m) m->pins++;
  }
  if (!m) return fail(IM_ERR_INVALID_ARG, "no resident memo for the current parameters");
  if (!m->counted) {
    memo_release(g, m);
    return fail(IM_ERR_INVALID_ARG, "the memo was built without work counting (profiling level 4)");
  }
  unsigned long long h[kWorkCounts];
  if (m->ready) (void)hipStreamWaitEvent(c->stream, m->ready_ev(), 0);
  hipError_t e = hipMemcpyAsync(h, m->work, sizeof(h), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  memo_release(g, m);
  if (e != hipSuccess) return fail(IM_ERR_DEVICE, "work count copy failed: %s", hipGetErrorString(e));
  for (uint32_t k = 0; k < n_out; ++k) out[k] = k < kWorkCounts ? h[k] : 0;
  return IM_OK;
}

extern "C" im_status im_memo_stats(im_graph* g, uint64_t* out4) {
  if (!g || !out4) return fail(IM_ERR_INVALID_ARG, "NULL argument");
  Memo* m = nullptr;
  im_status s = memo_acquire(g, &m);
  if (s != IM_OK) return s;
  std::vector<uint32_t> counts(kSubLists * 2);
  hipError_t e = hipMemcpyAsync(counts.data(), m->counts, counts.size() * 4, hipMemcpyDeviceToHost, g->ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(g->ctx->stream);
  if (e == hipSuccess) {
    uint64_t t = 0, l = 0;
    for (uint32_t j = 0; j < kSubLists; ++j) {
      t += counts[2 * j];
      l += counts[2 * j + 1];
    }
    out4[0] = t;
    out4[1] = l;
    out4[2] = g->nhubs;
    out4[3] = m->bytes;
  }
  memo_release(g, m);
  if (e != hipSuccess) return fail(IM_ERR_DEVICE, "memo statistics copy failed: %s", hipGetErrorString(e));
  return IM_OK;
}
