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
