// Many graphs per call (im_batch_select).  The memos of graphs that are not
// resident are built on kBatchStreams streams at once (the kernels of small
// graphs overlap on the device), then every selection runs in one launch of
// the persistent CELF kernel, which gives each graph its own group of
// workgroups, sized by the graph's memo; one synchronisation at the end.
#include <algorithm>
#include <cstring>
#include <vector>

#include "../../include/infuse.h"
#include "launch.h"
#include "runtime.h"

using namespace infuse;

static constexpr uint32_t kBatchStreams = 4;

static bool batch_streams(im_ctx* c) {
  if (!c->bstreams.empty()) return true;
  for (uint32_t i = 0; i < kBatchStreams; ++i) {
    hipStream_t s = nullptr;
    hipEvent_t e = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return false;
    c->bstreams.push_back(s);
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return false;
    c->bevents.push_back(e);
  }
  return true;
}

extern "C" im_status im_batch_select(im_ctx* c, uint32_t ng, im_graph* const* graphs, const uint32_t* K,
                                     uint32_t* const* seeds, int64_t* const* marginal, int64_t* cover) {
  if (!c || (ng && (!graphs || !K || !seeds || !marginal))) return fail(IM_ERR_INVALID_ARG, "NULL argument");
  for (uint32_t i = 0; i < ng; ++i) {
    if (!graphs[i] || graphs[i]->ctx != c) return fail(IM_ERR_INVALID_ARG, "graph %u is not of this context", i);
    if (K[i] > graphs[i]->n) return fail(IM_ERR_INVALID_ARG, "K[%u] exceeds n", i);
    if (!graphs[i]->params_set) return fail(IM_ERR_INVALID_ARG, "graph %u has no parameters", i);
    if (graphs[i]->directed) return fail(IM_ERR_INVALID_ARG, "graph %u is directed: no memo selection", i);
  }
  std::vector<Memo*> memos(ng, nullptr);
  std::vector<CelfBuffers> cbs(ng);
  im_status st = IM_OK;
  // memos: resident ones are pinned, missing ones built round-robin on the
  // batch streams; the context stream then waits for every batch stream
  const bool multi = ng > 1 && batch_streams(c);
  std::vector<bool> used(kBatchStreams, false);
  for (uint32_t i = 0; i < ng && st == IM_OK; ++i) {
    im_graph* g = graphs[i];
    {
      std::lock_guard<std::recursive_mutex> lk(c->mu);
      Memo* m = memo_find(g, g->p, g->R, g->seed);
      if (m) {
        m->pins++;
        m->last_use = ++c->use_clock;
        memos[i] = m;
      }
    }
    if (memos[i]) {
      if (memos[i]->ready_ev) (void)hipStreamWaitEvent(c->stream, memos[i]->ready_ev, 0);
      continue;
    }
    const uint32_t b = i % kBatchStreams;
    hipStream_t bs = multi ? c->bstreams[b] : c->stream;
    if (multi && !used[b]) {  // batch streams start after the context stream's earlier work
      (void)hipEventRecord(c->bevents[b], c->stream);
      (void)hipStreamWaitEvent(bs, c->bevents[b], 0);
      used[b] = true;
    }
    st = memo_build(g, g->p, g->R, g->seed, bs, &memos[i]);  // returned pinned
  }
  if (multi)
    for (uint32_t b = 0; b < kBatchStreams; ++b)
      if (used[b]) {
        (void)hipEventRecord(c->bevents[b], c->bstreams[b]);
        (void)hipStreamWaitEvent(c->stream, c->bevents[b], 0);
      }
  for (uint32_t i = 0; i < ng && st == IM_OK; ++i)
    if (K[i]) st = celf_alloc(graphs[i], memos[i], K[i], c->tune.celf_width, &cbs[i]);
  void* djobs = nullptr;
  std::vector<unsigned char> hjobs;
  if (st == IM_OK) {
    std::vector<uint32_t> sel;
    for (uint32_t i = 0; i < ng; ++i)
      if (K[i]) {
        celf_prepare(&cbs[i], c->stream);
        sel.push_back(i);
      }
    bool launched = false;
    if (!sel.empty() && c->tune.celf_mode == 1 && c->coop_grid) {
      const uint32_t nj = (uint32_t)sel.size(), grid = c->coop_grid;
      // workgroups per selection: one each, the rest in proportion to the
      // memo words (n * ntiles); with more selections than workgroups, one
      // workgroup each, taking selections in turn
      std::vector<uint32_t> first(nj + 1, 0);
      const bool shaped = nj <= grid;
      if (shaped) {
        double wsum = 0;
        for (uint32_t i : sel) wsum += (double)cbs[i].v.m.n * cbs[i].v.m.ntiles;
        for (uint32_t k = 0; k < nj; ++k) {
          const CelfView& v = cbs[sel[k]].v;
          const uint32_t extra = (uint32_t)((double)(grid - nj) * ((double)v.m.n * v.m.ntiles) / wsum);
          first[k + 1] = first[k] + 1 + extra;
        }
      }
      const size_t jb = pcelf_job_bytes();
      const size_t fb = (nj + 1) * sizeof(uint32_t);
      hjobs.resize(jb * nj + fb);
      for (uint32_t k = 0; k < nj; ++k) {
        CelfBuffers& cb = cbs[sel[k]];
        const uint32_t gb = shaped ? first[k + 1] - first[k] : 1;
        pcelf_fill_job(hjobs.data() + k * jb, cb.v, cb.pscratch, cb.blist, gb, c->tune.celf_round0,
                       c->profiling >= 2);
      }
      std::memcpy(hjobs.data() + jb * nj, first.data(), fb);
      if (ctx_alloc(c, hjobs.size(), &djobs) == IM_OK &&
          hipMemcpyAsync(djobs, hjobs.data(), hjobs.size(), hipMemcpyHostToDevice, c->stream) == hipSuccess &&
          celf_launch_persistent(c, djobs, nj, 1,
                                 shaped ? reinterpret_cast<const uint32_t*>(static_cast<char*>(djobs) + jb * nj)
                                        : nullptr,
                                 c->stream)) {
        launched = true;
        for (uint32_t i : sel) cbs[i].persistent = true;
      }
      (void)hipGetLastError();
    }
    if (!launched)
      for (uint32_t i : sel) celf_enqueue_steps(c, &cbs[i], c->stream);
    for (uint32_t i = 0; i < ng && st == IM_OK; ++i) {
      if (!K[i]) {
        if (cover) cover[i] = 0;
        continue;
      }
      int64_t cv = 0;
      uint64_t ev = 0;
      st = celf_collect(c, &cbs[i], c->stream, seeds[i], marginal[i], &cv, &ev);
      if (cover) cover[i] = cv;
      graphs[i]->last_evals = ev;
    }
  }
  if (st != IM_OK) (void)hipStreamSynchronize(c->stream);
  if (djobs) ctx_free(c, djobs);
  for (uint32_t i = 0; i < ng; ++i) {
    if (cbs[i].base) ctx_free(c, cbs[i].base);
    if (memos[i]) memo_release(graphs[i], memos[i]);
  }
  return st;
}
