// sigma(S) on a resident memo without any device allocation, for callers
// that cannot allocate (code under stream capture, tight serving loops).
//
// The query's scratch (the count, the seed list and, for more than
// sigma_pair_max() seeds, the (root, column) bitmap) lives in one file-scope
// device array per GPU.  Its address on each device is looked up once, when
// a context is created on that device, and kept: host code never passes the
// array's own name to a kernel or a copy.  Every call on a GPU shares that
// GPU's array, so two calls that overlap on one GPU (two host threads, or two
// streams without an ordering between them) race on it.
#include <algorithm>
#include <mutex>

#include "../../include/infuse.h"
#include "launch.h"
#include "runtime.h"

namespace infuse {

constexpr size_t kNoAllocScratchBytes = 16u << 20;  // 16 MiB per device
constexpr int kNoAllocMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static size_t round256(size_t x) { return (x + 255) & ~(size_t)255; }

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kNoAllocMaxDevices] = {};

// Returns the device address of the scratch array on `device`, looked up
// (with that device current) on the first call for the device and kept; or
// nullptr when the lookup fails.  im_ctx_create makes the first call.
void* noalloc_scratch_setup(int device) {
  if (device < 0 || device >= kNoAllocMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return nullptr;
    if (cur != device && hipSetDevice(device) != hipSuccess) return nullptr;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_ptr[device] = p;
  }
  return g_scratch_ptr[device];
}

size_t noalloc_scratch_bytes() { return kNoAllocScratchBytes; }

}  // namespace infuse

using namespace infuse;

extern "C" im_status im_estimate_sigma_noalloc(im_graph* g, const uint32_t* S, uint32_t s_len,
                                               int64_t* count, double* sigma) {
  if (!g) return fail(IM_ERR_INVALID_ARG, "NULL graph");
  if (s_len && !S) return fail(IM_ERR_INVALID_ARG, "NULL seed array");
  for (uint32_t i = 0; i < s_len; ++i)
    if (S[i] >= g->n) return fail(IM_ERR_INVALID_ARG, "seed id %u >= n = %u", S[i], g->n);
  if (!g->params_set) return fail(IM_ERR_INVALID_ARG, "im_set_params has not been called");
  if (g->directed) return fail(IM_ERR_INVALID_ARG, "directed graph: no memo; use im_estimate_sigma_direct");
  im_ctx* c = g->ctx;

  // Seed sets of up to sigma_pair_max() ids are deduplicated here (the
  // pairwise kernel expects distinct ids); larger ones go to the bitmap
  // kernel, whose bitmap gives set semantics by itself.
  uint32_t small[256];
  const uint32_t pair_max = std::min<uint32_t>(sigma_pair_max(), 256);
  const bool pair = s_len <= pair_max;
  uint32_t len = s_len;
  const uint32_t* src = S;
  if (pair) {
    std::copy(S, S + s_len, small);
    std::sort(small, small + s_len);
    len = (uint32_t)(std::unique(small, small + s_len) - small);
    src = small;
  }
  if (len == 0) {
    if (count) *count = 0;
    if (sigma) *sigma = 0.0;
    return IM_OK;
  }

  Memo* m = nullptr;
  {
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    m = memo_find(g, g->p, g->R, g->seed);
    if (m) {
      m->pins++;
      m->last_use = ++c->use_clock;
    }
  }
  if (!m)
    return fail(IM_ERR_INVALID_ARG,
                "no resident memo for the current parameters (this call builds none; call im_build_memo first)");

  const uint32_t cwords = m->Rs / 32;
  const size_t s_off = 256;
  const size_t bm_off = s_off + round256((size_t)len * 4);
  const size_t need = pair ? bm_off : bm_off + (size_t)g->n * cwords * 4;
  if (need > kNoAllocScratchBytes) {
    memo_release(g, m);
    return fail(IM_ERR_INVALID_ARG,
                "the query needs %zu bytes of scratch, more than the %zu available without allocation "
                "(%u seeds on n = %u, R = %u)",
                need, kNoAllocScratchBytes, len, g->n, g->R);
  }
  void* base = noalloc_scratch_setup(c->device);
  if (!base) {
    memo_release(g, m);
    return fail(IM_ERR_DEVICE, "device address of the scratch array unavailable on device %d", c->device);
  }

  char* p8 = static_cast<char*>(base);
  auto* out = reinterpret_cast<unsigned long long*>(p8);
  auto* dS = reinterpret_cast<uint32_t*>(p8 + s_off);
  hipStream_t st = c->stream;
  if (m->ready) (void)hipStreamWaitEvent(st, m->ready_ev(), 0);
  launch_fill_u32(reinterpret_cast<uint32_t*>(out), 2, 0u, st);
  hipError_t e = hipMemcpyAsync(dS, src, (size_t)len * 4, hipMemcpyHostToDevice, st);
  const MemoView mv = m->view(g);
  if (e == hipSuccess) {
    if (pair) {
      launch_sigma_pair(mv, dS, len, out, st);
    } else {
      uint32_t* bm = reinterpret_cast<uint32_t*>(p8 + bm_off);
      launch_fill_u32(bm, (uint64_t)g->n * cwords, 0u, st);
      launch_sigma_bitmap(mv, dS, len, bm, cwords, out, st);
    }
    e = hipGetLastError();
  }
  unsigned long long h = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&h, out, 8, hipMemcpyDeviceToHost, st);
  // also keeps `small` alive until its copy has run
  const hipError_t es = hipStreamSynchronize(st);
  if (e == hipSuccess) e = es;
  memo_release(g, m);
  if (e != hipSuccess) return fail(IM_ERR_DEVICE, "sigma (no allocation) failed: %s", hipGetErrorString(e));
  if (count) *count = (int64_t)h;
  if (sigma) *sigma = (double)h / (double)g->R;
  return IM_OK;
}
