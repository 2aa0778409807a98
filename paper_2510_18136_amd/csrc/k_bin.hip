// Time binning of a raw cube for the longer search timescales (paper section
// 2.2: the images are also searched binned by 5 and by 75 samples).
// out[t'][s][p] = RN32(x[t' b][s][p] + x[t' b + 1][s][p] + ... + x[t' b + b - 1][s][p]),
// the sum taken in FP64 in that order; t' < n_t / b (a trailing partial bin is
// dropped). One thread per output element, consecutive threads on consecutive
// (s, p), so every read and write is coalesced.
#include <algorithm>

#include "device_common.h"
#include "nsfrb_internal.h"

namespace nsfrb {

template <typename T>
__global__ void k_bin_time(const T* __restrict__ x, long long n_out, long long n_sp, int factor,
                           float* __restrict__ out) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n_out;
       i += (long long)gridDim.x * blockDim.x) {
    const long long tb = i / n_sp, sp = i % n_sp;
    const T* src = x + tb * factor * n_sp + sp;
    double acc = 0.0;
    for (int k = 0; k < factor; ++k) acc += (double)to_f32(src[(long long)k * n_sp]);
    out[i] = (float)acc;
  }
}

// Two binnings from one read, for factors fa < fb with fb a multiple of fa: a
// thread takes one (s, p) series and one group of fb raw samples, g, and writes
// the group's fb / fa bins of factor fa and, when the group is whole, its one bin
// of factor fb. Both sums run over the samples in time order in FP64, so each
// output equals the single-factor kernel's. The last group may be partial: it
// holds the trailing factor-fa bins (t' < n_t / fa) past the last whole group.
template <typename T>
__global__ void k_bin_time_pair(const T* __restrict__ x, long long n_items, long long n_sp, int fa, int na,
                                float* __restrict__ out_a, int fb, int nb, float* __restrict__ out_b) {
  const int per = fb / fa;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n_items;
       i += (long long)gridDim.x * blockDim.x) {
    const long long g = i / n_sp, sp = i % n_sp;
    const T* src = x + g * fb * n_sp + sp;
    const int nj = (int)std::min<long long>(per, (long long)na - g * per);
    double acc_b = 0.0;
    for (int j = 0; j < nj; ++j) {
      double acc_a = 0.0;
      for (int k = 0; k < fa; ++k) {
        const double v = (double)to_f32(src[(long long)(j * fa + k) * n_sp]);
        acc_a += v;
        acc_b += v;
      }
      out_a[(g * per + j) * n_sp + sp] = (float)acc_a;
    }
    if (g < nb) out_b[g * n_sp + sp] = (float)acc_b;
  }
}

hipError_t launch_bin_time_pair(const void* x, int in_dtype, int n_t, int n_sub, int n_pix, int fa, float* out_a,
                                int fb, float* out_b, hipStream_t st) {
  if (fa < 2 || fb <= fa || fb % fa != 0) return hipErrorInvalidValue;
  const int na = n_t / fa, nb = n_t / fb, per = fb / fa;
  const long long n_sp = (long long)n_sub * n_pix, n_items = (long long)((na + per - 1) / per) * n_sp;
  if (n_items == 0) return hipSuccess;
  const unsigned grid = (unsigned)std::min<long long>((n_items + 255) / 256, 65536LL * 4);
  if (in_dtype == DT_F32)
    hipLaunchKernelGGL(k_bin_time_pair<float>, dim3(grid), dim3(256), 0, st, (const float*)x, n_items, n_sp, fa, na,
                       out_a, fb, nb, out_b);
  else if (in_dtype == DT_F16)
    hipLaunchKernelGGL(k_bin_time_pair<_Float16>, dim3(grid), dim3(256), 0, st, (const _Float16*)x, n_items, n_sp,
                       fa, na, out_a, fb, nb, out_b);
  else
    hipLaunchKernelGGL(k_bin_time_pair<bf16_t>, dim3(grid), dim3(256), 0, st, (const bf16_t*)x, n_items, n_sp, fa,
                       na, out_a, fb, nb, out_b);
  return hipGetLastError();
}

hipError_t launch_bin_time(const void* x, int in_dtype, int n_t, int n_sub, int n_pix, int factor, float* out,
                           hipStream_t st) {
  const long long n_sp = (long long)n_sub * n_pix, n_out = (long long)(n_t / factor) * n_sp;
  const unsigned grid = (unsigned)std::min<long long>((n_out + 255) / 256, 65536LL * 4);
  if (in_dtype == DT_F32)
    hipLaunchKernelGGL(k_bin_time<float>, dim3(grid), dim3(256), 0, st, (const float*)x, n_out, n_sp, factor, out);
  else if (in_dtype == DT_F16)
    hipLaunchKernelGGL(k_bin_time<_Float16>, dim3(grid), dim3(256), 0, st, (const _Float16*)x, n_out, n_sp, factor,
                       out);
  else
    hipLaunchKernelGGL(k_bin_time<bf16_t>, dim3(grid), dim3(256), 0, st, (const bf16_t*)x, n_out, n_sp, factor, out);
  return hipGetLastError();
}

}  // namespace nsfrb
