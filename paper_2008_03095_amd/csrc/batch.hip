// Many graphs per call (im_batch_select).  The memos of the graphs that are
// not resident are built together: one launch per labelling phase (set-up,
// hook of light rows, hook of hubs, work lists, unions of light rows and of
// hubs, flatten, count, initial gains) over all of them, each launch's
// workgroups split among the graphs by prefix sums of per-graph shapes.
// Then every selection runs in one launch of the persistent CELF kernel,
// which gives each graph its own group of workgroups, sized by the graph's
// memo; one synchronisation at the end.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/infuse.h"
#include "launch.h"
#include "runtime.h"

using namespace infuse;

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static const char* const kPhaseNames[kBatchPhases] = {"batch.prep",  "batch.hook",    "batch.hook_hubs",
                                                      "batch.lists", "batch.link",    "batch.link_hubs",
                                                      "batch.flatten", "batch.count", "batch.gain0"};

// Allocates and builds the memos of graphs[todo[k]] (returned pinned in
// memos[]) with one launch per phase on the context stream.  *djobs receives
// the device copy of the job descriptions, to be freed once the stream has
// passed the launches.  On failure no memo of this call stays registered.
static im_status batch_build(im_ctx* c, im_graph* const* graphs, const std::vector<uint32_t>& todo,
                             std::vector<Memo*>& memos, void** djobs) {
  hipStream_t st = c->stream;
  const uint32_t nj = (uint32_t)todo.size();
  im_status s = IM_OK;
  uint32_t made = 0;
  for (; made < nj && s == IM_OK; ++made) {
    im_graph* g = graphs[todo[made]];
    s = memo_alloc(g, g->p, g->R, g->seed, &memos[todo[made]]);
    if (s != IM_OK) break;
  }
  auto undo = [&]() {
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    for (uint32_t k = 0; k < made; ++k) {
      Memo*& m = memos[todo[k]];
      if (m) memo_destroy(graphs[todo[k]], m);
      m = nullptr;
    }
  };
  if (s != IM_OK) {
    undo();
    return s;
  }
  std::vector<BuildJob> jobs(nj);
  std::vector<uint32_t> first((size_t)kBatchPhases * (nj + 1), 0);
  uint64_t total[kBatchPhases] = {};
  const uint32_t chunk_tiles = hub_chunk_tiles(c);
  for (uint32_t k = 0; k < nj; ++k) {
    im_graph* g = graphs[todo[k]];
    Memo* m = memos[todo[k]];
    const GraphView gv = g->view();
    BuildJob& J = jobs[k];
    J.g = gv;
    J.m = m->view(g);
    J.edges = m->edges;
    J.xs = m->xs;
    J.inv = m->inv;
    J.pos = m->pos;
    J.seed = m->seed;
    uint32_t blocks[kBatchPhases] = {};
    build_job_shape(gv, J.m, chunk_tiles, c->tune.list_blocks, &J, blocks);
    // X of a large R is sorted by the single-graph kernels beforehand
    J.sort_blocks = m->R <= x_sort_single_max() ? 1u : 0u;
    if (!J.sort_blocks) launch_x_sort(m->seed, m->R, m->Rs, m->scratch, m->xs, m->inv, m->pos, st);
    J.hash_blocks = std::max(1u, std::min(65536u, (g->nnz + 255) / 256));
    J.fill_words = (uint32_t)((reinterpret_cast<char*>(m->lmask) - reinterpret_cast<char*>(m->tmask)) / 4 +
                              (uint64_t)g->n * m->mwords);
    const uint32_t fill_blocks = std::min(4096u, (J.fill_words + 2047) / 2048);
    blocks[kBpPrep] = J.sort_blocks + J.hash_blocks + fill_blocks;
    for (uint32_t ph = 0; ph < kBatchPhases; ++ph) {
      total[ph] += blocks[ph];
      if (total[ph] > 0x7FFFFFFFull) {
        undo();
        return fail(IM_ERR_INVALID_ARG, "batched construction: more than 2^31 workgroups in one phase");
      }
      first[(size_t)ph * (nj + 1) + k + 1] = (uint32_t)total[ph];
    }
  }
  const size_t jb = (sizeof(BuildJob) * nj + 255) / 256 * 256;
  s = ctx_alloc(c, jb + first.size() * 4, djobs);
  if (s != IM_OK) {
    undo();
    return s;
  }
  char* d = static_cast<char*>(*djobs);
  if (hipMemcpyAsync(d, jobs.data(), sizeof(BuildJob) * nj, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(d + jb, first.data(), first.size() * 4, hipMemcpyHostToDevice, st) != hipSuccess) {
    undo();
    return fail(IM_ERR_DEVICE, "batched construction: job upload failed");
  }
  BuildBatch b;
  b.jobs = reinterpret_cast<const BuildJob*>(d);
  b.first = reinterpret_cast<const uint32_t*>(d + jb);
  b.njobs = nj;
  {
    KTimer t(c, kPhaseNames[kBpPrep], st);
    launch_prep_batch(b, (uint32_t)total[kBpPrep], st);
  }
  for (uint32_t ph = kBpHookRows; ph < kBatchPhases; ++ph) {
    KTimer t(c, kPhaseNames[ph], st);
    launch_build_batch(b, ph, (uint32_t)total[ph], st);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(st);
    undo();
    return fail(IM_ERR_DEVICE, "batched construction failed to launch: %s", hipGetErrorString(e));
  }
  const std::shared_ptr<ihipEvent_t> ready = record_ready(st);
  for (uint32_t k = 0; k < nj; ++k) {
    memos[todo[k]]->ready = ready;
    graphs[todo[k]]->timed_build = false;
  }
  return IM_OK;
}

extern "C" im_status im_batch_select(im_ctx* c, uint32_t ng, im_graph* const* graphs, const uint32_t* K,
                                     uint32_t* const* seeds, int64_t* const* marginal, int64_t* cover) {
  if (!c || (ng && (!graphs || !K || !seeds || !marginal))) return fail(IM_ERR_INVALID_ARG, "NULL argument");
  for (uint32_t i = 0; i < ng; ++i) {
    if (!graphs[i] || graphs[i]->ctx != c) return fail(IM_ERR_INVALID_ARG, "graph %u is not of this context", i);
    if (K[i] > graphs[i]->n) return fail(IM_ERR_INVALID_ARG, "K[%u] exceeds n", i);
    if (!graphs[i]->params_set) return fail(IM_ERR_INVALID_ARG, "graph %u has no parameters", i);
    if (graphs[i]->directed) return fail(IM_ERR_INVALID_ARG, "graph %u is directed: no memo selection", i);
    for (uint32_t k = 0; k < i; ++k)
      if (graphs[k] == graphs[i]) return fail(IM_ERR_INVALID_ARG, "graph %u appears twice", i);
  }
  std::vector<Memo*> memos(ng, nullptr);
  std::vector<CelfBuffers> cbs(ng);
  im_status st = IM_OK;
  // memos: resident ones are pinned (the context stream waits for their
  // construction), missing ones built together
  std::vector<uint32_t> todo;
  for (uint32_t i = 0; i < ng; ++i) {
    im_graph* g = graphs[i];
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    Memo* m = memo_find(g, g->p, g->R, g->seed);
    if (m) {
      m->pins++;
      m->last_use = ++c->use_clock;
      memos[i] = m;
      if (m->ready) (void)hipStreamWaitEvent(c->stream, m->ready_ev(), 0);
    } else {
      todo.push_back(i);
    }
  }
  void* dbuild = nullptr;
  if (!todo.empty()) st = batch_build(c, graphs, todo, memos, &dbuild);
  for (uint32_t i = 0; i < ng && st == IM_OK; ++i)
    if (K[i]) st = celf_alloc(graphs[i], memos[i], K[i], c->tune.celf_width, &cbs[i]);
  // the selections: set up in one launch, run in one persistent launch (or
  // the per-step kernels), their results packed by one launch and
  // downloaded with one copy; the descriptions of all launches go up in one
  // copy
  void* djobs = nullptr;
  unsigned char* hb = nullptr;  // host side of the selections' block
  size_t hcap = 0;              // its pinned size (0: pageable or none)
  std::vector<uint32_t> sel;
  for (uint32_t i = 0; i < ng && st == IM_OK; ++i)
    if (K[i]) sel.push_back(i);
  if (st == IM_OK && !sel.empty()) {
    const uint32_t nj = (uint32_t)sel.size();
    std::vector<CelfBatchJob> bj(nj);
    std::vector<uint32_t> pfirst(nj + 1, 0);
    uint64_t rec_bytes = 0;
    for (uint32_t k = 0; k < nj; ++k) {
      CelfBuffers& cb = cbs[sel[k]];
      CelfBatchJob& J = bj[k];
      J.v = cb.v;
      J.pscratch = static_cast<uint32_t*>(cb.pscratch);
      J.perr = reinterpret_cast<const uint32_t*>(static_cast<char*>(cb.pscratch) + pcelf_err_offset());
      J.scratch_words = (uint32_t)(pcelf_scratch_bytes() / 4);
      const uint64_t cw = (uint64_t)cb.v.m.n * cb.v.cwords;
      J.cov_blocks = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(1024, (cw + 4095) / 4096));
      J.init_blocks = (cb.v.m.n + 255) / 256;
      J.rec_off = (uint32_t)rec_bytes;
      rec_bytes += 8 + sizeof(CelfState) + (((uint64_t)cb.v.K * 4 + 7) & ~7ull) + (uint64_t)cb.v.K * 8;
      const uint64_t f = (uint64_t)pfirst[k] + J.cov_blocks + J.init_blocks + 1;
      if (f > 0x7FFFFFFFull || rec_bytes > 0xFFFFFFFFull) {
        st = fail(IM_ERR_INVALID_ARG, "batched selection: too many selections for one call");
        break;
      }
      pfirst[k + 1] = (uint32_t)f;
    }
    const bool coop = c->tune.celf_mode == 1 && c->coop_grid;
    // workgroups of the persistent launch per selection: one each, the rest
    // in proportion to the square root of the memo words (n * ntiles): the
    // longest selection sets the launch's time, and a small graph's
    // selection is not proportionally shorter (its evaluations are rounds
    // of dependent loads whatever their number); with more selections than
    // workgroups, one workgroup each, taking selections in turn
    const uint32_t grid = c->coop_grid;
    std::vector<uint32_t> first(nj + 1, 0);
    const bool shaped = coop && nj <= grid;
    if (shaped) {
      double wsum = 0;
      for (uint32_t i : sel) wsum += std::sqrt((double)cbs[i].v.m.n * cbs[i].v.m.ntiles);
      for (uint32_t k = 0; k < nj; ++k) {
        const CelfView& v = cbs[sel[k]].v;
        const uint32_t extra = (uint32_t)((double)(grid - nj) * std::sqrt((double)v.m.n * v.m.ntiles) / wsum);
        first[k + 1] = first[k] + 1 + extra;
      }
    }
    // one device block: prepare jobs | their prefix | persistent jobs | their
    // prefix | packed records
    const size_t jb = pcelf_job_bytes();
    const size_t o_pf = align256(sizeof(CelfBatchJob) * nj);
    const size_t o_pj = o_pf + align256((nj + 1) * 4);
    const size_t o_fi = o_pj + (coop ? align256(jb * nj) : 0);
    const size_t o_rec = o_fi + (coop ? align256((nj + 1) * 4) : 0);
    // host side of the block: pinned when possible (one upload of the jobs,
    // one download of the records), else pageable
    std::vector<unsigned char> pg;
    if (st == IM_OK) {
      hb = static_cast<unsigned char*>(pinned_take(c, o_rec + rec_bytes, &hcap));
      if (!hb) {
        pg.resize(o_rec + rec_bytes);
        hb = pg.data();
      }
      std::memset(hb, 0, o_rec);
      unsigned char* up = hb;
      std::memcpy(up, bj.data(), sizeof(CelfBatchJob) * nj);
      std::memcpy(up + o_pf, pfirst.data(), (nj + 1) * 4);
      if (coop) {
        for (uint32_t k = 0; k < nj; ++k) {
          CelfBuffers& cb = cbs[sel[k]];
          const uint32_t gb = shaped ? first[k + 1] - first[k] : 1;
          pcelf_fill_job(up + o_pj + k * jb, cb.v, cb.pscratch, cb.blist, gb, c->tune.celf_round0,
                         pcelf_prof_bits(c));
        }
        std::memcpy(up + o_fi, first.data(), (nj + 1) * 4);
      }
      st = ctx_alloc(c, o_rec + rec_bytes, &djobs);
    }
    if (st == IM_OK) {
      char* d = static_cast<char*>(djobs);
      const CelfBatchJob* dbj = reinterpret_cast<const CelfBatchJob*>(d);
      if (hipMemcpyAsync(d, hb, o_rec, hipMemcpyHostToDevice, c->stream) != hipSuccess) {
        st = fail(IM_ERR_DEVICE, "batched selection: upload failed");
      } else {
        launch_celf_prepare_batch(dbj, reinterpret_cast<const uint32_t*>(d + o_pf), nj, pfirst[nj], c->stream);
        bool launched = false;
        if (coop && celf_launch_persistent(c, d + o_pj, nj, 1,
                                           shaped ? reinterpret_cast<const uint32_t*>(d + o_fi) : nullptr,
                                           c->stream)) {
          launched = true;
          for (uint32_t i : sel) cbs[i].persistent = true;
        }
        (void)hipGetLastError();
        if (!launched)
          for (uint32_t i : sel) celf_enqueue_steps(c, &cbs[i], c->stream);
        launch_celf_collect_batch(dbj, nj, reinterpret_cast<unsigned char*>(d + o_rec), c->stream);
        if (hipMemcpyAsync(hb + o_rec, d + o_rec, rec_bytes, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess) {
          hipError_t e = hipGetLastError();
          st = fail(IM_ERR_DEVICE, "batched selection failed on the device: %s", hipGetErrorString(e));
        }
      }
    }
    for (uint32_t k = 0; k < nj && st == IM_OK; ++k) {
      const uint32_t i = sel[k];
      const unsigned char* r = hb + o_rec + bj[k].rec_off;
      const uint32_t Ki = K[i];
      uint32_t perr;
      CelfState hs;
      std::memcpy(&perr, r, 4);
      std::memcpy(&hs, r + 8, sizeof(CelfState));
      std::memcpy(seeds[i], r + 8 + sizeof(CelfState), (size_t)Ki * 4);
      std::memcpy(marginal[i], r + 8 + sizeof(CelfState) + (((uint64_t)Ki * 4 + 7) & ~7ull), (size_t)Ki * 8);
      int64_t cv = 0;
      uint64_t ev = 0;
      st = celf_finish(c, &cbs[i], perr, hs, marginal[i], &cv, &ev);
      if (cover) cover[i] = cv;
      graphs[i]->last_evals = ev;
    }
  }
  for (uint32_t i = 0; i < ng && st == IM_OK; ++i)
    if (!K[i] && cover) cover[i] = 0;
  if (st != IM_OK) (void)hipStreamSynchronize(c->stream);
  if (hcap) pinned_give(c, hb, hcap);
  if (djobs) ctx_free(c, djobs);
  if (dbuild) ctx_free(c, dbuild);
  for (uint32_t i = 0; i < ng; ++i) {
    if (cbs[i].base) ctx_free(c, cbs[i].base);
    if (memos[i]) memo_release(graphs[i], memos[i]);
  }
  return st;
}
