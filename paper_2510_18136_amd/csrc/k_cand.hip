// Candidate extraction (threshold + top-K by S/N).
//
// Paper section 2.2: a 6-sigma S/N threshold turns the maximum-S/N maps into
// candidates; section 2.3: post-processing keeps the ten highest-S/N ones.
// Here one candidate is a pixel whose best (DM, width) trial has S/N >= theta.
// Candidates are ordered by S/N descending, then pixel index ascending; the
// first K are returned together with the total count.
//
// Each candidate is encoded as a 64-bit key whose unsigned order is that
// ranking: high word = order-preserving bits of the FP32 S/N, low word =
// ~pixel. Stage 1 compacts keys with one atomic per wave; stage 2 (one
// workgroup) sorts them in LDS when they fit, otherwise it first finds the
// K-th largest key by an 8-bit radix selection and sorts only the top K.
#include "device_common.h"
#include "nsfrb_internal.h"
#include "../../include/nsfrb.h"

namespace nsfrb {

constexpr int kSortCap = 4096;     // keys sorted directly in LDS
constexpr int kSelThreads = 1024;

__device__ __forceinline__ uint32_t ordered_bits(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float unordered_bits(uint32_t o) {
  return __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
}

__global__ void k_cand_zero(int* count) { if (threadIdx.x == 0) { count[0] = 0; } }

__global__ __launch_bounds__(256) void k_cand_compact(const float* __restrict__ best, int n_pix, float theta,
                                                      unsigned long long* __restrict__ keys, int* __restrict__ count) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  bool hit = false;
  float v = 0.f;
  if (p < n_pix) {
    v = best[p];
    hit = __builtin_isfinite(v) && v >= theta;
  }
  const uint64_t m = ballot(hit);
  if (m == 0) return;
  const int leader = __ffsll((long long)m) - 1;
  int base = 0;
  if (lane_id() == leader) base = atomicAdd(count, popc64(m));
  base = __shfl(base, leader);
  if (hit) {
    const int pos = base + lanes_below(m);
    keys[pos] = ((unsigned long long)ordered_bits(v) << 32) | (unsigned long long)(0xffffffffu - (uint32_t)p);
  }
}

// Bitonic sort, descending, of n2 (power of two) keys in LDS.
__device__ void block_sort_desc(unsigned long long* s, int n2) {
  for (int k = 2; k <= n2; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < n2; i += blockDim.x) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const unsigned long long a = s[i], b = s[ixj];
          const bool desc = (i & k) == 0;
          if (desc ? (a < b) : (a > b)) { s[i] = b; s[ixj] = a; }
        }
      }
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(kSelThreads) void k_cand_select(
    const unsigned long long* __restrict__ keys, const int* __restrict__ count, int k_max, int nx,
    const int* __restrict__ best_d, const int* __restrict__ best_w, const int* __restrict__ best_t,
    nsfrb_candidate* __restrict__ out, int* __restrict__ n_out) {
  __shared__ unsigned long long s[kSortCap];
  __shared__ uint32_t hist[256];
  __shared__ unsigned long long prefix_sh, mask_sh;
  __shared__ int need_sh, fill_sh;
  const int n = count[0];
  const int K = n < k_max ? n : k_max;
  int m = n;                                  // keys that go into the LDS sort
  if (n > kSortCap) {
    // radix-select the K-th largest key: fix the key 8 bits at a time from the top
    if (threadIdx.x == 0) { prefix_sh = 0; mask_sh = 0; need_sh = K; }
    __syncthreads();
    for (int shift = 56; shift >= 0; shift -= 8) {
      for (int i = threadIdx.x; i < 256; i += blockDim.x) hist[i] = 0;
      __syncthreads();
      const unsigned long long pre = prefix_sh, msk = mask_sh;
      for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const unsigned long long k = keys[i];
        if ((k & msk) == pre) atomicAdd(&hist[(k >> shift) & 0xff], 1u);
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        int need = need_sh;
        int dsel = 0;
        for (int dg = 255; dg >= 0; --dg) {
          if ((int)hist[dg] >= need) { dsel = dg; break; }
          need -= (int)hist[dg];
        }
        need_sh = need;
        prefix_sh = pre | ((unsigned long long)dsel << shift);
        mask_sh = msk | (0xffull << shift);
      }
      __syncthreads();
    }
    // prefix_sh is now the K-th largest key; gather every key >= it (exactly K)
    const unsigned long long thr = prefix_sh;
    if (threadIdx.x == 0) fill_sh = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const unsigned long long k = keys[i];
      if (k >= thr) { const int pos = atomicAdd(&fill_sh, 1); if (pos < kSortCap) s[pos] = k; }
    }
    __syncthreads();
    m = K;
  } else {
    for (int i = threadIdx.x; i < n; i += blockDim.x) s[i] = keys[i];
  }
  int n2 = 1;
  while (n2 < m) n2 <<= 1;
  for (int i = m + threadIdx.x; i < n2; i += blockDim.x) s[i] = 0ull;
  __syncthreads();
  if (n2 > 1) block_sort_desc(s, n2);
  for (int i = threadIdx.x; i < K; i += blockDim.x) {
    const unsigned long long k = s[i];
    const int p = (int)(0xffffffffu - (uint32_t)(k & 0xffffffffull));
    nsfrb_candidate c;
    c.x = p % nx;
    c.y = p / nx;
    c.dm_index = best_d[p];
    c.width_index = best_w[p];
    c.toa = best_t[p];
    c.snr = unordered_bits((uint32_t)(k >> 32));
    out[i] = c;
  }
  if (threadIdx.x == 0) { n_out[0] = K; n_out[1] = n; }
}

hipError_t launch_candidates(const CandLaunch& a, hipStream_t st) {
  hipLaunchKernelGGL(k_cand_zero, dim3(1), dim3(64), 0, st, a.count);
  hipLaunchKernelGGL(k_cand_compact, dim3((a.n_pix + 255) / 256), dim3(256), 0, st, a.best_snr, a.n_pix,
                     a.theta, a.keys, a.count);
  hipLaunchKernelGGL(k_cand_select, dim3(1), dim3(kSelThreads), 0, st, a.keys, a.count, a.k_max, a.nx,
                     a.best_d, a.best_w, a.best_t, (nsfrb_candidate*)a.out, a.n_out);
  return hipGetLastError();
}

}  // namespace nsfrb
