// sigma(S) from the memo (Algorithm 4 over the memo's samples) and the
// label/size export used by callers that want the paper's two n x R arrays.
//
// sigma count = sum over columns of |union_{s in S} C_q(s)| = sum over the
// distinct component labels of the seeds in each column of their sizes.
#include "common.h"

namespace infuse {

constexpr int kSigmaPairMax = 128;  // |S| handled by the pairwise kernel

__device__ inline uint64_t wave_sum_u64q(uint64_t x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off);
  return x;
}

// A workgroup per 16 columns: lane l of the workgroup takes column l % 16
// and the seeds j = l / 16 + 16 k, so the loads of all its (at most 128)
// seeds are issued in one batch per lane (8 seeds) and a launch has R / 16
// workgroups.  Each (seed, column) gets its label and component size; then a
// seed's component counts unless an earlier seed of the list has the same
// label in that column.  S holds distinct ids (the callers deduplicate it),
// so a singleton seed shares its component with no other seed.
constexpr int kSigmaCols = 16;
constexpr int kSigmaBatch = kSigmaPairMax / (256 / kSigmaCols);
__global__ void __launch_bounds__(256) k_sigma_pair(MemoView m, const uint32_t* S, uint32_t len,
                                                    unsigned long long* out) {
  __shared__ uint32_t roots[kSigmaPairMax][kSigmaCols];
  __shared__ int32_t sizes[kSigmaPairMax][kSigmaCols];
  __shared__ unsigned long long part[4];
  constexpr uint32_t kSlots = 256 / kSigmaCols;
  const uint32_t c = threadIdx.x % kSigmaCols, sl = threadIdx.x / kSigmaCols, w = threadIdx.x >> 6;
  const uint32_t q = blockIdx.x * kSigmaCols + c;
  const uint32_t qq = q < m.R ? q : m.R - 1;  // in range; the count skips q >= R
  const uint32_t t = qq / kTile;
  if (sl < len) {  // len <= kSigmaPairMax = kSlots * kSigmaBatch: one batch
    uint32_t s[kSigmaBatch];
    int32_t raw[kSigmaBatch];
    uint32_t tw[kSigmaBatch];
#pragma unroll
    for (int k = 0; k < kSigmaBatch; ++k) {
      s[k] = S[min(sl + kSlots * k, len - 1)];
      raw[k] = m.M[(uint64_t)s[k] * m.Rs + qq];
      tw[k] = m.tmask[(uint64_t)s[k] * m.mwords + (t >> 5)];
    }
    int32_t val[kSigmaBatch], gsz[kSigmaBatch];
#pragma unroll
    for (int k = 0; k < kSigmaBatch; ++k) {
      val[k] = ((tw[k] >> (t & 31)) & 1u) ? raw[k] : -1;
      gsz[k] = m.M[(uint64_t)(val[k] < 0 ? s[k] : (uint32_t)val[k]) * m.Rs + qq];  // issued for every seed
    }
#pragma unroll
    for (int k = 0; k < kSigmaBatch; ++k) {
      const uint32_t j = sl + kSlots * k;
      if (j < len) {
        roots[j][c] = val[k] < 0 ? s[k] : (uint32_t)val[k];
        sizes[j][c] = val[k] == -1 ? 0 : (val[k] < 0 ? -val[k] : -gsz[k]);  // 0 marks a singleton
      }
    }
  }
  __syncthreads();
  uint64_t cnt = 0;
  if (q < m.R) {
    for (uint32_t j = sl; j < len; j += kSlots) {
      const int32_t sz = sizes[j][c];
      if (sz == 0) {  // a singleton seed: its own component, of size 1
        cnt += 1;
        continue;
      }
      const uint32_t r = roots[j][c];
      bool dup = false;
      for (uint32_t i = 0; i < j; ++i)
        if (roots[i][c] == r) {
          dup = true;
          break;
        }
      cnt += dup ? 0 : (uint64_t)sz;
    }
  }
  cnt = wave_sum_u64q(cnt);
  if ((threadIdx.x & 63) == 0) part[w] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long tot = part[0] + part[1] + part[2] + part[3];
    if (tot) atomicAdd(out, tot);
  }
}

// Any |S|: the first seed to set its component's bit in a zeroed
// (label, column) bitmap adds the component size.
__global__ void __launch_bounds__(256) k_sigma_bitmap(MemoView m, const uint32_t* S, uint32_t len,
                                                      uint32_t* bm, uint32_t cwords,
                                                      unsigned long long* out) {
  const uint64_t total = (uint64_t)len * m.R;
  uint64_t cnt = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t j = (uint32_t)(i / m.R), q = (uint32_t)(i % m.R);
    const uint32_t s = S[j];
    const int32_t val = memo_entry(m, s, q);
    const uint32_t root = val < 0 ? s : (uint32_t)val;
    const uint32_t bit = 1u << (q & 31);
    const uint32_t old = atomicOr(&bm[(uint64_t)root * cwords + (q >> 5)], bit);
    if (!(old & bit)) cnt += (uint64_t)(val < 0 ? -val : -m.M[(uint64_t)val * m.Rs + q]);
  }
  cnt = wave_sum_u64q(cnt);
  if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(out, (unsigned long long)cnt);
}

// out[(v - v0) * cnt + i] = label (mode 0) or component size (mode 1) of
// vertex v in simulation r0 + i, for v in [v0, v0 + nv).
__global__ void __launch_bounds__(256) k_export(MemoView m, const uint32_t* pos, uint32_t r0,
                                                uint32_t cnt, uint32_t v0, uint32_t nv, int mode,
                                                int32_t* out) {
  const uint64_t total = (uint64_t)nv * cnt;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t vv = (uint32_t)(i / cnt), k = (uint32_t)(i % cnt);
    const uint32_t v = v0 + vv;
    const uint32_t q = pos[r0 + k];
    const int32_t val = memo_entry(m, v, q);
    int32_t res;
    if (mode == 0) res = val < 0 ? (int32_t)v : val;
    else res = val < 0 ? -val : -m.M[(uint64_t)val * m.Rs + q];
    out[i] = res;
  }
}

uint32_t sigma_pair_max() { return kSigmaPairMax; }

void launch_sigma_pair(const MemoView& m, const uint32_t* S, uint32_t len, unsigned long long* out,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_sigma_pair, dim3((m.R + kSigmaCols - 1) / kSigmaCols), dim3(256), 0, st, m, S, len, out);
}

void launch_sigma_bitmap(const MemoView& m, const uint32_t* S, uint32_t len, uint32_t* bm,
                         uint32_t cwords, unsigned long long* out, hipStream_t st) {
  uint64_t blocks = ((uint64_t)len * m.R + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (!blocks) blocks = 1;
  hipLaunchKernelGGL(k_sigma_bitmap, dim3((uint32_t)blocks), dim3(256), 0, st, m, S, len, bm,
                     cwords, out);
}

void launch_export(const MemoView& m, const uint32_t* pos, uint32_t r0, uint32_t cnt, uint32_t v0,
                   uint32_t nv, int mode, int32_t* out, hipStream_t st) {
  uint64_t blocks = ((uint64_t)nv * cnt + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  if (!blocks) return;
  hipLaunchKernelGGL(k_export, dim3((uint32_t)blocks), dim3(256), 0, st, m, pos, r0, cnt, v0, nv,
                     mode, out);
}

}  // namespace infuse
