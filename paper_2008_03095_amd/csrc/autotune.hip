// Autotuner (im_autotune): picks launch shapes for a graph by timing cold
// selections.  The knobs change only how the work is spread over the device
// (simulations per hub wavefront, workgroups of the list-walking kernels,
// candidates of a CELF step's first round), never the result, which the
// tuner checks.
#include <chrono>
#include <cstring>
#include <vector>

#include "../../include/infuse.h"
#include "runtime.h"

using namespace infuse;

extern "C" im_status im_autotune(im_graph* g, uint32_t K, uint32_t reps, im_tuning* best) {
  if (!g || !best) return fail(IM_ERR_INVALID_ARG, "NULL argument");
  if (!g->params_set) return fail(IM_ERR_INVALID_ARG, "im_set_params has not been called");
  if (g->directed) return fail(IM_ERR_INVALID_ARG, "directed graph: no memo selection to tune");
  if (K == 0 || K > g->n) return fail(IM_ERR_INVALID_ARG, "K must be in 1..n");
  if (reps == 0) reps = 1;
  im_ctx* c = g->ctx;
  const im_tuning saved = c->tune;
  const uint32_t chunks[] = {256, 512, 1024};
  const uint32_t lists[] = {2048, 8192, 32768};
  const uint32_t round0s[] = {8, 16, 32};
  std::vector<uint32_t> seeds(K), ref;
  std::vector<int64_t> marg(K);
  double best_ms = 1e300;
  im_tuning pick = saved;
  for (uint32_t ch : chunks)
    for (uint32_t lb : lists)
    for (uint32_t r0 : round0s) {
      if (c->tune.celf_mode != 1 && r0 != round0s[0]) continue;  // round0 only shapes the persistent kernel
      im_tuning t = saved;
      t.cc_chunk = ch;
      t.list_blocks = lb;
      t.celf_round0 = r0;
      c->tune = t;
      double ms = 1e300;
      for (uint32_t i = 0; i < reps; ++i) {
        im_status s = im_drop_memo(g);
        int64_t cover = 0;
        const auto t0 = std::chrono::steady_clock::now();
        if (s == IM_OK) s = im_select_seeds(g, K, seeds.data(), marg.data(), &cover);
        const auto t1 = std::chrono::steady_clock::now();
        if (s != IM_OK) {
          c->tune = saved;
          return s;
        }
        ms = std::min(ms, std::chrono::duration<double, std::milli>(t1 - t0).count());
        if (ref.empty()) {
          ref = seeds;
        } else if (ref != seeds) {
          c->tune = saved;
          return fail(IM_ERR_DEVICE, "selections differ between launch shapes");
        }
      }
      if (ms < best_ms) {
        best_ms = ms;
        pick = t;
      }
    }
  c->tune = pick;
  *best = pick;
  return IM_OK;
}
