// Serving loop: admission by device-memory budget, resident graphs and memos
// keyed by (graph, p, R, s), and overlapping queries on per-slot streams.
//
// One worker thread owns the device side.  Each pass it (1) retires slots
// whose completion event fired, (2) admits queued queries into free slots in
// arrival order: it finds or builds the memo on the slot's stream (waiting on
// the memo's ready event when another slot is still building it), pins it,
// enqueues the sigma or CELF kernels and the result copies, and records a
// completion event.  A query whose memory does not fit waits while other
// queries run (their memos are pinned); with nothing running it is rejected.
// Queries that arrive while others run are admitted as soon as a slot and
// memory free up, so their kernels overlap on the device.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/infuse.h"
#include "launch.h"
#include "runtime.h"

using namespace infuse;
using Clock = std::chrono::steady_clock;

namespace {

enum TState { QUEUED, RUNNING, DONE };

struct Ticket {
  uint64_t id = 0;
  im_graph* g = nullptr;
  int kind = 0;
  uint32_t K = 0;
  double p = 0;
  uint32_t R = 0, seed = 0;
  std::vector<uint32_t> S;
  TState state = QUEUED;
  bool cancel = false;
  im_result res = {};
  std::vector<uint32_t> seeds;
  std::vector<int64_t> marginal;
  Clock::time_point t_submit, t_admit;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  Ticket* t = nullptr;
  Memo* m = nullptr;
  void* scratch = nullptr;  // device scratch of the query (CELF buffers / sigma)
  // pinned host landing area for results
  void* host = nullptr;
  size_t host_bytes = 0;
};

}  // namespace

struct im_server {
  im_ctx* ctx = nullptr;
  std::vector<Slot> slots;
  std::deque<Ticket*> queue;
  std::map<uint64_t, std::unique_ptr<Ticket>> tickets;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::thread worker;
  bool stop = false;
  uint64_t next_id = 1;
  uint64_t admitted = 0, completed = 0, rejected = 0, hits = 0, builds = 0, peak = 0;
  uint64_t persistent_min_words = 0;  // selections on smaller memos run the per-step kernels
  uint32_t busy = 0;
};

static bool ensure_host(Slot& s, size_t bytes) {
  if (s.host_bytes >= bytes) return true;
  if (s.host) (void)hipHostFree(s.host);
  s.host = nullptr;
  s.host_bytes = 0;
  if (hipHostMalloc(&s.host, bytes, hipHostMallocDefault) != hipSuccess) return false;
  s.host_bytes = bytes;
  return true;
}

static void finish(im_server* sv, Ticket* t, im_status st) {
  t->res.status = st;
  t->res.latency_ms = std::chrono::duration<double, std::milli>(Clock::now() - t->t_submit).count();
  if (t->cancel && st == IM_OK) t->res.status = IM_ERR_CANCELLED;
  t->state = DONE;
  sv->completed++;
  sv->cv_done.notify_all();
}

// Retires a slot whose completion event fired (server lock held).
static void retire(im_server* sv, Slot& s) {
  Ticket* t = s.t;
  im_status st = IM_OK;
  if (hipEventSynchronize(s.done) != hipSuccess) st = IM_ERR_DEVICE;
  if (st == IM_OK) {
    if (t->kind == 0) {
      const uint64_t cnt = *static_cast<uint64_t*>(s.host);
      t->res.count = (int64_t)cnt;
      t->res.sigma = (double)cnt / (double)t->R;
    } else {
      char* h = static_cast<char*>(s.host);
      CelfState cs;
      std::memcpy(&cs, h, sizeof(cs));
      t->seeds.assign(reinterpret_cast<uint32_t*>(h + 256), reinterpret_cast<uint32_t*>(h + 256) + t->K);
      const size_t off = 256 + ((size_t)t->K * 4 + 255) / 256 * 256;
      t->marginal.assign(reinterpret_cast<int64_t*>(h + off), reinterpret_cast<int64_t*>(h + off) + t->K);
      int64_t tot = 0;
      for (int64_t x : t->marginal) tot += x;
      t->res.count = tot;
      t->res.sigma = (double)tot / (double)t->R;
      if (cs.s != t->K) st = IM_ERR_DEVICE;
    }
  }
  ctx_free(sv->ctx, s.scratch);
  s.scratch = nullptr;
  memo_release(t->g, s.m);
  s.m = nullptr;
  s.t = nullptr;
  sv->busy--;
  finish(sv, t, st);
}

// Tries to start ticket t on slot s.  Returns false when it must wait for
// memory held by running queries.
static bool admit(im_server* sv, Slot& s, Ticket* t) {
  im_ctx* c = sv->ctx;
  im_graph* g = t->g;
  Memo* m = nullptr;
  bool hit = false;
  {
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    m = memo_find(g, t->p, t->R, t->seed);
    if (m) {
      m->pins++;  // pinned before anything else may evict it
      m->last_use = ++c->use_clock;
      hit = true;
    }
  }
  im_status st = IM_OK;
  if (!m) {
    st = memo_build(g, t->p, t->R, t->seed, s.stream, &m);  // returned pinned
    if (st == IM_OK) sv->builds++;
  } else if (m->ready) {
    (void)hipStreamWaitEvent(s.stream, m->ready_ev(), 0);
  }
  if (st == IM_OK) {
    if (t->kind == 0) {
      unsigned long long* dout = nullptr;
      st = sigma_enqueue(g, m, t->S, s.stream, &s.scratch, &dout);
      if (st == IM_OK) {
        if (!ensure_host(s, 256)) st = fail(IM_ERR_OUT_OF_MEMORY, "pinned host allocation failed");
        else (void)hipMemcpyAsync(s.host, dout, 8, hipMemcpyDeviceToHost, s.stream);
      }
    } else {
      CelfBuffers cb;
      st = celf_alloc(g, m, t->K, c->tune.celf_width, &cb);
      if (st == IM_OK) {
        s.scratch = cb.base;
        const uint64_t words = (uint64_t)g->n * m->Rs;
        celf_enqueue(c, &cb, s.stream, words >= sv->persistent_min_words);
        const size_t off = 256 + ((size_t)t->K * 4 + 255) / 256 * 256;
        if (!ensure_host(s, off + (size_t)t->K * 8)) {
          st = fail(IM_ERR_OUT_OF_MEMORY, "pinned host allocation failed");
        } else {
          char* h = static_cast<char*>(s.host);
          (void)hipMemcpyAsync(h, cb.v.st, sizeof(CelfState), hipMemcpyDeviceToHost, s.stream);
          (void)hipMemcpyAsync(h + 256, cb.v.seeds, (size_t)t->K * 4, hipMemcpyDeviceToHost, s.stream);
          (void)hipMemcpyAsync(h + off, cb.v.marginal, (size_t)t->K * 8, hipMemcpyDeviceToHost, s.stream);
        }
      }
    }
  }
  if (st != IM_OK) {
    // undo: nothing of this query may stay enqueued without a waiter
    (void)hipStreamSynchronize(s.stream);
    if (s.scratch) ctx_free(c, s.scratch);
    s.scratch = nullptr;
    if (m) memo_release(g, m);
    if ((st == IM_ERR_BUDGET || st == IM_ERR_OUT_OF_MEMORY) && sv->busy > 0) return false;
    t->t_admit = Clock::now();
    sv->rejected++;
    finish(sv, t, st);
    return true;
  }
  (void)hipEventRecord(s.done, s.stream);
  s.t = t;
  s.m = m;
  t->state = RUNNING;
  t->t_admit = Clock::now();
  t->res.queue_ms = std::chrono::duration<double, std::milli>(t->t_admit - t->t_submit).count();
  t->res.memo_hit = hit ? 1u : 0u;
  if (hit) sv->hits++;
  sv->admitted++;
  sv->busy++;
  if (sv->busy > sv->peak) sv->peak = sv->busy;
  return true;
}

// Queued queries wanting the memo (g, m's parameters).  Called during
// evictions: from the worker, which holds the server lock, or from a direct
// call on another thread, which takes it.
static uint32_t memo_demand(void* user, const im_graph* g, const Memo* m) {
  im_server* sv = static_cast<im_server*>(user);
  std::unique_lock<std::mutex> lk(sv->mu, std::defer_lock);
  if (std::this_thread::get_id() != sv->worker.get_id()) lk.lock();
  uint32_t d = 0;
  for (const Ticket* t : sv->queue)
    if (t->g == g && memo_matches(g, m, t->p, t->R, t->seed)) ++d;
  return d;
}

// Index of the queued ticket to admit next.  Unless the head has waited
// longer than kMaxBypassMs: among the next kLookahead tickets, the first
// whose memo is resident; if none is, the first ticket of the parameter set
// (graph, p, R, s) that most of them share, so that one construction serves
// as many queued queries as possible.  Otherwise the head.
constexpr size_t kLookahead = 256;
constexpr double kMaxBypassMs = 100.0;

static size_t pick_next(im_server* sv) {
  Ticket* head = sv->queue.front();
  const double waited = std::chrono::duration<double, std::milli>(Clock::now() - head->t_submit).count();
  if (waited > kMaxBypassMs) return 0;
  std::lock_guard<std::recursive_mutex> lk(sv->ctx->mu);
  const size_t lim = std::min(kLookahead, sv->queue.size());
  for (size_t i = 0; i < lim; ++i) {
    Ticket* t = sv->queue[i];
    if (!t->cancel && memo_find(t->g, t->p, t->R, t->seed)) return i;
  }
  size_t best = 0, best_n = 0;
  for (size_t i = 0; i < lim; ++i) {
    const Ticket* t = sv->queue[i];
    if (t->cancel) continue;
    size_t same = 0;
    for (size_t j = i; j < lim; ++j) {
      const Ticket* u = sv->queue[j];
      same += (u->g == t->g && u->R == t->R && u->seed == t->seed && u->p == t->p) ? 1 : 0;
    }
    if (same > best_n) {
      best_n = same;
      best = i;
    }
  }
  return best;
}

static void worker_main(im_server* sv) {
  (void)hipSetDevice(sv->ctx->device);
  std::unique_lock<std::mutex> lk(sv->mu);
  while (true) {
    bool progress = false;
    for (Slot& s : sv->slots)
      if (s.t && hipEventQuery(s.done) == hipSuccess) {
        retire(sv, s);
        progress = true;
      }
    while (!sv->queue.empty()) {
      Ticket* h = sv->queue.front();
      if (h->cancel) {
        sv->queue.pop_front();
        finish(sv, h, IM_ERR_CANCELLED);
        progress = true;
        continue;
      }
      Slot* free_slot = nullptr;
      for (Slot& s : sv->slots)
        if (!s.t) {
          free_slot = &s;
          break;
        }
      if (!free_slot) break;
      const size_t i = pick_next(sv);
      Ticket* t = sv->queue[i];
      sv->queue.erase(sv->queue.begin() + (std::ptrdiff_t)i);
      if (!admit(sv, *free_slot, t)) {  // waits for memory
        sv->queue.insert(sv->queue.begin() + (std::ptrdiff_t)i, t);
        break;
      }
      progress = true;
    }
    if (sv->stop && sv->queue.empty() && sv->busy == 0) break;
    if (!progress) {
      if (sv->busy) sv->cv_work.wait_for(lk, std::chrono::microseconds(50));
      else sv->cv_work.wait_for(lk, std::chrono::milliseconds(5));
    }
  }
}

extern "C" im_status im_server_create(im_ctx* c, const im_server_config* cfg, im_server** out) {
  if (!c || !out) return fail(IM_ERR_INVALID_ARG, "NULL argument");
  *out = nullptr;
  const uint32_t n = cfg && cfg->slots ? cfg->slots : 4;
  if (n > 64) return fail(IM_ERR_INVALID_ARG, "at most 64 slots");
  im_server* sv = new im_server();
  sv->ctx = c;
  if (cfg)
    sv->persistent_min_words = cfg->persistent_min_mwords == 0xFFFFFFFFu ? ~0ull
                                                                        : (uint64_t)cfg->persistent_min_mwords << 20;
  sv->slots.resize(n);
  for (Slot& s : sv->slots) {
    if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess) {
      for (Slot& x : sv->slots) {
        if (x.stream) (void)hipStreamDestroy(x.stream);
        if (x.done) (void)hipEventDestroy(x.done);
      }
      delete sv;
      return fail(IM_ERR_DEVICE, "stream/event creation failed");
    }
  }
  // work the context enqueued before (graph uploads) precedes every slot
  (void)hipStreamSynchronize(c->stream);
  {
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    c->memo_demand = memo_demand;
    c->memo_demand_user = sv;
    for (Slot& s : sv->slots) c->peers.push_back(s.stream);  // fenced by persistent launches
  }
  sv->worker = std::thread(worker_main, sv);
  *out = sv;
  return IM_OK;
}

extern "C" im_status im_server_submit(im_server* sv, im_graph* g, const im_query* q, uint64_t* ticket) {
  if (!sv || !g || !q || !ticket) return fail(IM_ERR_INVALID_ARG, "NULL argument");
  if (g->ctx != sv->ctx) return fail(IM_ERR_INVALID_ARG, "graph belongs to another context");
  if (q->kind != 0 && q->kind != 1) return fail(IM_ERR_INVALID_ARG, "unknown query kind %d", q->kind);
  if (g->directed) return fail(IM_ERR_INVALID_ARG, "directed graph: the server answers from memos");
  im_status st = check_params(g, q->p, q->R);
  if (st != IM_OK) return st;
  auto t = std::make_unique<Ticket>();
  t->g = g;
  t->kind = q->kind;
  t->K = q->K;
  t->p = q->p;
  t->R = q->R;
  t->seed = q->hash_seed;
  if (q->kind == 1) {
    if (q->K == 0 || q->K > g->n) return fail(IM_ERR_INVALID_ARG, "K must be in 1..n");
  } else {
    if (q->s_len && !q->S) return fail(IM_ERR_INVALID_ARG, "NULL seed array");
    st = normalize_set(g, q->S, q->s_len, &t->S);
    if (st != IM_OK) return st;
  }
  t->t_submit = Clock::now();
  std::lock_guard<std::mutex> lk(sv->mu);
  t->id = sv->next_id++;
  *ticket = t->id;
  Ticket* raw = t.get();
  sv->tickets[t->id] = std::move(t);
  if (raw->kind == 0 && raw->S.empty()) {
    raw->t_admit = raw->t_submit;
    finish(sv, raw, IM_OK);
    return IM_OK;
  }
  sv->queue.push_back(raw);
  sv->cv_work.notify_one();
  return IM_OK;
}

extern "C" im_status im_server_poll(im_server* sv, uint64_t ticket, uint32_t wait_ms, im_result* res,
                                    uint32_t* seeds, int64_t* marginal) {
  if (!sv) return fail(IM_ERR_INVALID_ARG, "NULL server");
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->tickets.find(ticket);
  if (it == sv->tickets.end()) return fail(IM_ERR_NOT_FOUND, "unknown ticket %llu", (unsigned long long)ticket);
  Ticket* t = it->second.get();
  if (t->state != DONE && wait_ms)
    sv->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return t->state == DONE; });
  if (t->state != DONE) return IM_ERR_NOT_READY;
  if (res) *res = t->res;
  if (t->kind == 1 && t->res.status == IM_OK) {
    if (seeds) std::memcpy(seeds, t->seeds.data(), t->seeds.size() * 4);
    if (marginal) std::memcpy(marginal, t->marginal.data(), t->marginal.size() * 8);
  }
  const im_status st = t->res.status == IM_ERR_CANCELLED ? IM_ERR_CANCELLED : IM_OK;
  sv->tickets.erase(it);
  return st;
}

extern "C" im_status im_server_cancel(im_server* sv, uint64_t ticket) {
  if (!sv) return fail(IM_ERR_INVALID_ARG, "NULL server");
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->tickets.find(ticket);
  if (it == sv->tickets.end()) return fail(IM_ERR_NOT_FOUND, "unknown ticket %llu", (unsigned long long)ticket);
  it->second->cancel = true;
  sv->cv_work.notify_one();
  return IM_OK;
}

extern "C" im_status im_server_drain(im_server* sv) {
  if (!sv) return fail(IM_ERR_INVALID_ARG, "NULL server");
  std::unique_lock<std::mutex> lk(sv->mu);
  while (!sv->queue.empty() || sv->busy) sv->cv_done.wait_for(lk, std::chrono::milliseconds(5));
  return IM_OK;
}

extern "C" im_status im_server_stats(im_server* sv, uint64_t* out7) {
  if (!sv || !out7) return fail(IM_ERR_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(sv->mu);
  out7[0] = sv->admitted;
  out7[1] = sv->completed;
  out7[2] = sv->rejected;
  out7[3] = sv->hits;
  out7[4] = sv->builds;
  out7[5] = sv->ctx->evictions;
  out7[6] = sv->peak;
  return IM_OK;
}

extern "C" void im_server_destroy(im_server* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    for (Ticket* t : sv->queue) t->cancel = true;
    sv->stop = true;
    sv->cv_work.notify_one();
  }
  sv->worker.join();
  {
    std::lock_guard<std::recursive_mutex> lk(sv->ctx->mu);
    if (sv->ctx->memo_demand_user == sv) {
      sv->ctx->memo_demand = nullptr;
      sv->ctx->memo_demand_user = nullptr;
    }
    auto& pe = sv->ctx->peers;
    for (Slot& s : sv->slots) pe.erase(std::remove(pe.begin(), pe.end(), s.stream), pe.end());
  }
  for (Slot& s : sv->slots) {
    if (s.host) (void)hipHostFree(s.host);
    (void)hipStreamDestroy(s.stream);
    (void)hipEventDestroy(s.done);
  }
  delete sv;
}
