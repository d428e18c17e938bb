// Many graphs per call (im_batch_select): every memo construction and every
// CELF step of all graphs is enqueued back to back on the context stream with
// a single synchronisation at the end.
#include <algorithm>
#include <vector>

#include "../../include/infuse.h"
#include "launch.h"
#include "runtime.h"

using namespace infuse;

extern "C" im_status im_batch_select(im_ctx* c, uint32_t ng, im_graph* const* graphs, const uint32_t* K,
                                     uint32_t* const* seeds, int64_t* const* marginal, int64_t* cover) {
  if (!c || (ng && (!graphs || !K || !seeds || !marginal))) return fail(IM_ERR_INVALID_ARG, "NULL argument");
  for (uint32_t i = 0; i < ng; ++i) {
    if (!graphs[i] || graphs[i]->ctx != c) return fail(IM_ERR_INVALID_ARG, "graph %u is not of this context", i);
    if (K[i] > graphs[i]->n) return fail(IM_ERR_INVALID_ARG, "K[%u] exceeds n", i);
    if (!graphs[i]->params_set) return fail(IM_ERR_INVALID_ARG, "graph %u has no parameters", i);
  }
  std::vector<Memo*> memos(ng, nullptr);
  std::vector<CelfBuffers> cbs(ng);
  im_status st = IM_OK;
  for (uint32_t i = 0; i < ng && st == IM_OK; ++i) st = memo_acquire(graphs[i], &memos[i]);
  for (uint32_t i = 0; i < ng && st == IM_OK; ++i)
    if (K[i]) st = celf_alloc(graphs[i], memos[i], K[i], c->tune.celf_width, &cbs[i]);
  if (st == IM_OK) {
    for (uint32_t i = 0; i < ng; ++i)
      if (K[i]) celf_enqueue(c, &cbs[i], c->stream);
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
  for (uint32_t i = 0; i < ng; ++i) {
    if (cbs[i].base) ctx_free(c, cbs[i].base);
    if (memos[i]) memo_release(graphs[i], memos[i]);
  }
  return st;
}
