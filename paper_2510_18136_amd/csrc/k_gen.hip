// Synthetic input on the device: Philox4x32-10 Gaussian noise and boxcar
// injections (input generator; holds none of the search's arithmetic).
//
// Philox4x32-10 follows its published definition (Salmon, Moraes, Dror &
// Shaw 2011, "Parallel random numbers: as easy as 1, 2, 3"): ten rounds of
// two 32x32->64 multiplications with the constants 0xD2511F53 and 0xCD9E8D57,
// the key bumped by the Weyl constants 0x9E3779B9 and 0xBB67AE85 between
// rounds. Block i (counter (i, 0, 0, 0)) yields four uniform words, turned
// into two Box-Muller pairs for elements 4i .. 4i+3 of the cube.
#include "device_common.h"
#include "nsfrb_internal.h"

namespace nsfrb {

struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    U4 n;
    n.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
    n.y = (uint32_t)p1;
    n.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
    n.w = (uint32_t)p0;
    c = n;
  }
  return c;
}

__global__ void k_philox_fill(uint32_t* __restrict__ out, long long n_blocks, uint32_t k0, uint32_t k1) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n_blocks;
       i += (long long)gridDim.x * blockDim.x) {
    const U4 r = philox4x32_10(U4{(uint32_t)i, (uint32_t)(i >> 32), 0u, 0u}, k0, k1);
    out[4 * i + 0] = r.x;
    out[4 * i + 1] = r.y;
    out[4 * i + 2] = r.z;
    out[4 * i + 3] = r.w;
  }
}

// uniform in (0, 1): top 23 bits, centred in their interval (exact in FP32,
// so the value never rounds to 1)
__device__ __forceinline__ float unit_open(uint32_t u) { return ((float)(u >> 9) + 0.5f) * (1.0f / 8388608.0f); }

template <typename T>
__global__ void k_noise(T* __restrict__ out, long long n, uint32_t k0, uint32_t k1, float sigma) {
  const long long nb = (n + 3) / 4;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nb;
       i += (long long)gridDim.x * blockDim.x) {
    const U4 r = philox4x32_10(U4{(uint32_t)i, (uint32_t)(i >> 32), 0u, 0u}, k0, k1);
    float v[4];
    const float r0 = sqrtf(-2.0f * logf(unit_open(r.x))), a0 = 6.283185307179586f * unit_open(r.y);
    const float r1 = sqrtf(-2.0f * logf(unit_open(r.z))), a1 = 6.283185307179586f * unit_open(r.w);
    float s0, c0, s1, c1;
    sincosf(a0, &s0, &c0);
    sincosf(a1, &s1, &c1);
    v[0] = r0 * c0; v[1] = r0 * s0; v[2] = r1 * c1; v[3] = r1 * s1;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (4 * i + k < n) out[4 * i + k] = from_f32<T>(sigma * v[k]);
  }
}

template <typename T>
__global__ void k_inject(T* __restrict__ cube, int layout, int n_pix, int n_sub, int n_t, int pixel, int t0,
                         int width, float amp, const int* __restrict__ offsets) {
  const int s = blockIdx.x;
  for (int k = threadIdx.x; k < width; k += blockDim.x) {
    const int t = t0 + offsets[s] + k;
    if (t < 0 || t >= n_t) continue;
    const size_t idx = layout == 0 ? ((size_t)t * n_sub + s) * n_pix + pixel
                                   : ((size_t)pixel * n_sub + s) * n_t + t;
    cube[idx] = from_f32<T>(to_f32(cube[idx]) + amp);
  }
}

// Many boxcars at once: record r (blockIdx.y) adds amp_r to samples
// t0_r + offsets[r][s] ... + width_r - 1 of sub-band s (blockIdx.x) of pixel
// pixel_r of cube cube_r. Records name distinct (cube, pixel) pairs, so no two
// blocks touch the same element.
template <typename T>
__global__ void k_inject_many(T* const* __restrict__ cubes, const BoxcarRec* __restrict__ recs,
                              const int* __restrict__ offsets, int layout, int n_pix, int n_sub, int n_t) {
  const int s = blockIdx.x;
  const BoxcarRec r = recs[blockIdx.y];
  T* cube = cubes[r.cube];
  const int off = offsets[(size_t)blockIdx.y * n_sub + s];
  for (int k = threadIdx.x; k < r.width; k += blockDim.x) {
    const int t = r.t0 + off + k;
    if (t < 0 || t >= n_t) continue;
    const size_t idx = layout == 0 ? ((size_t)t * n_sub + s) * n_pix + r.pixel : ((size_t)r.pixel * n_sub + s) * n_t + t;
    cube[idx] = from_f32<T>(to_f32(cube[idx]) + r.amp);
  }
}

// Broadband or narrowband interference over all pixels: kind 0 adds `amp` to
// sample t0 of every sub-band (a zero-DM spike); kind 1 adds `amp` to samples
// t0 .. t0+len-1 of sub-band s0 (a stripe).
template <typename T>
__global__ void k_inject_rfi(T* __restrict__ cube, int layout, int n_pix, int n_sub, int n_t, int kind, int t0, int len,
                             int s0, float amp) {
  const int nsb = kind == 0 ? n_sub : 1;
  const int nts = kind == 0 ? 1 : len;
  const long long total = (long long)n_pix * nsb * nts;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const int p = (int)(i % n_pix);
    const long long r = i / n_pix;
    const int s = kind == 0 ? (int)(r % nsb) : s0;
    const int t = t0 + (kind == 0 ? 0 : (int)(r % nts));
    if (t < 0 || t >= n_t || s < 0 || s >= n_sub) continue;
    const size_t idx = layout == 0 ? ((size_t)t * n_sub + s) * n_pix + p : ((size_t)p * n_sub + s) * n_t + t;
    cube[idx] = from_f32<T>(to_f32(cube[idx]) + amp);
  }
}

hipError_t launch_inject_rfi(void* cube, int dtype, int layout, int n_pix, int n_sub, int n_t, int kind, int t0, int len,
                             int s0, float amp, hipStream_t st) {
  const long long total = (long long)n_pix * (kind == 0 ? n_sub : len);
  const unsigned blocks = (unsigned)(total < 65536LL * 256 ? (total + 255) / 256 : 65536LL);
  if (dtype == DT_F32) hipLaunchKernelGGL(k_inject_rfi<float>, dim3(blocks ? blocks : 1), dim3(256), 0, st, (float*)cube, layout, n_pix, n_sub, n_t, kind, t0, len, s0, amp);
  else if (dtype == DT_F16) hipLaunchKernelGGL(k_inject_rfi<_Float16>, dim3(blocks ? blocks : 1), dim3(256), 0, st, (_Float16*)cube, layout, n_pix, n_sub, n_t, kind, t0, len, s0, amp);
  else hipLaunchKernelGGL(k_inject_rfi<bf16_t>, dim3(blocks ? blocks : 1), dim3(256), 0, st, (bf16_t*)cube, layout, n_pix, n_sub, n_t, kind, t0, len, s0, amp);
  return hipGetLastError();
}

hipError_t launch_inject_many(void* const* cubes, int dtype, int layout, int n_pix, int n_sub, int n_t,
                              const BoxcarRec* recs, const int* offsets, int n, hipStream_t st) {
  const dim3 grid(n_sub, n);
  if (dtype == DT_F32) hipLaunchKernelGGL(k_inject_many<float>, grid, dim3(256), 0, st, (float* const*)cubes, recs, offsets, layout, n_pix, n_sub, n_t);
  else if (dtype == DT_F16) hipLaunchKernelGGL(k_inject_many<_Float16>, grid, dim3(256), 0, st, (_Float16* const*)cubes, recs, offsets, layout, n_pix, n_sub, n_t);
  else hipLaunchKernelGGL(k_inject_many<bf16_t>, grid, dim3(256), 0, st, (bf16_t* const*)cubes, recs, offsets, layout, n_pix, n_sub, n_t);
  return hipGetLastError();
}

hipError_t launch_philox_fill(uint32_t* out, long long n_blocks, unsigned long long seed, hipStream_t st) {
  const long long blocks = n_blocks < 65536LL * 4 ? (n_blocks + 255) / 256 : 65536LL * 4;
  hipLaunchKernelGGL(k_philox_fill, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(256), 0, st, out, n_blocks,
                     (uint32_t)seed, (uint32_t)(seed >> 32));
  return hipGetLastError();
}

hipError_t launch_noise(void* out, int dtype, long long n, unsigned long long seed, float sigma, hipStream_t st) {
  const long long nb = (n + 3) / 4;
  const unsigned blocks = (unsigned)(nb < 65536LL * 8 ? (nb + 255) / 256 : 65536LL * 8);
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  if (dtype == DT_F32) hipLaunchKernelGGL(k_noise<float>, dim3(blocks ? blocks : 1), dim3(256), 0, st, (float*)out, n, k0, k1, sigma);
  else if (dtype == DT_F16) hipLaunchKernelGGL(k_noise<_Float16>, dim3(blocks ? blocks : 1), dim3(256), 0, st, (_Float16*)out, n, k0, k1, sigma);
  else hipLaunchKernelGGL(k_noise<bf16_t>, dim3(blocks ? blocks : 1), dim3(256), 0, st, (bf16_t*)out, n, k0, k1, sigma);
  return hipGetLastError();
}

hipError_t launch_inject(void* cube, int dtype, int layout, int n_pix, int n_sub, int n_t, int pixel, int t0,
                         int width, float amp, const int* d_offsets, hipStream_t st) {
  if (dtype == DT_F32) hipLaunchKernelGGL(k_inject<float>, dim3(n_sub), dim3(256), 0, st, (float*)cube, layout, n_pix, n_sub, n_t, pixel, t0, width, amp, d_offsets);
  else if (dtype == DT_F16) hipLaunchKernelGGL(k_inject<_Float16>, dim3(n_sub), dim3(256), 0, st, (_Float16*)cube, layout, n_pix, n_sub, n_t, pixel, t0, width, amp, d_offsets);
  else hipLaunchKernelGGL(k_inject<bf16_t>, dim3(n_sub), dim3(256), 0, st, (bf16_t*)cube, layout, n_pix, n_sub, n_t, pixel, t0, width, amp, d_offsets);
  return hipGetLastError();
}

}  // namespace nsfrb
