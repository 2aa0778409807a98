// Device-side helpers shared by the search kernels (gfx950, wave64).
#pragma once
#ifndef __HIPCC_RTC__   // hipRTC provides the HIP device API itself
#include <hip/hip_runtime.h>
#include <stdint.h>
#else
using __hip_internal::uint16_t;
using __hip_internal::uint32_t;
using __hip_internal::uint64_t;
#endif

namespace nsfrb {

constexpr int kWave = 64;

// ---------------------------------------------------------------- dtypes
struct bf16_t { uint16_t bits; };

__device__ __forceinline__ float to_f32(float v) { return v; }
__device__ __forceinline__ float to_f32(_Float16 v) { return (float)v; }
__device__ __forceinline__ float to_f32(bf16_t v) { return __uint_as_float((uint32_t)v.bits << 16); }

// FP32 -> store dtype, round to nearest even.
template <typename T> __device__ __forceinline__ T from_f32(float v);
template <> __device__ __forceinline__ float from_f32<float>(float v) { return v; }
template <> __device__ __forceinline__ _Float16 from_f32<_Float16>(float v) { return (_Float16)v; }
template <> __device__ __forceinline__ bf16_t from_f32<bf16_t>(float v) {
  uint32_t u = __float_as_uint(v);
  bf16_t r;
  if ((u & 0x7fffffffu) > 0x7f800000u) { r.bits = 0x7fc0; return r; }   // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  r.bits = (uint16_t)(u >> 16);
  return r;
}

// ----------------------------------------------------------- wave helpers
__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// Order LDS traffic of one wave (lanes of a wave do not need a barrier).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int popc64(uint64_t m) { return __popcll(m); }

__device__ __forceinline__ int lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// DPP lane moves (GFX9 encodings): quad_perm [1,0,3,2] (lane ^ 1), quad_perm
// [2,3,0,1] (lane ^ 2), row_half_mirror, row_mirror, row_shr:k, row_bcast:15,
// row_bcast:31.
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143;

template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const unsigned long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)u, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ float readlane_f(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ __forceinline__ double readlane_d(double v, int lane) {
  const unsigned long long u = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
  return __longlong_as_double(((unsigned long long)hi << 32) | lo);
}

// Reductions over the whole wave (all 64 lanes active); the result is uniform.
// Rows of 16 lanes are reduced with DPP, then the four row results are read.
__device__ __forceinline__ float wave_min_f(float v) {
  v = fminf(v, dpp_f<kDppXor1>(v));
  v = fminf(v, dpp_f<kDppXor2>(v));
  v = fminf(v, dpp_f<kDppHalfMirror>(v));
  v = fminf(v, dpp_f<kDppMirror>(v));
  return fminf(fminf(readlane_f(v, 0), readlane_f(v, 16)), fminf(readlane_f(v, 32), readlane_f(v, 48)));
}
__device__ __forceinline__ float wave_max_f(float v) {
  v = fmaxf(v, dpp_f<kDppXor1>(v));
  v = fmaxf(v, dpp_f<kDppXor2>(v));
  v = fmaxf(v, dpp_f<kDppHalfMirror>(v));
  v = fmaxf(v, dpp_f<kDppMirror>(v));
  return fmaxf(fmaxf(readlane_f(v, 0), readlane_f(v, 16)), fmaxf(readlane_f(v, 32), readlane_f(v, 48)));
}
__device__ __forceinline__ double wave_min(double v) {
  v = fmin(v, dpp_d<kDppXor1>(v));
  v = fmin(v, dpp_d<kDppXor2>(v));
  v = fmin(v, dpp_d<kDppHalfMirror>(v));
  v = fmin(v, dpp_d<kDppMirror>(v));
  return fmin(fmin(readlane_d(v, 0), readlane_d(v, 16)), fmin(readlane_d(v, 32), readlane_d(v, 48)));
}
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_d<kDppXor1>(v));
  v = fmax(v, dpp_d<kDppXor2>(v));
  v = fmax(v, dpp_d<kDppHalfMirror>(v));
  v = fmax(v, dpp_d<kDppMirror>(v));
  return fmax(fmax(readlane_d(v, 0), readlane_d(v, 16)), fmax(readlane_d(v, 32), readlane_d(v, 48)));
}
__device__ __forceinline__ int wave_sum(int v) {
  v += __builtin_amdgcn_mov_dpp(v, kDppXor1, 0xf, 0xf, false);
  v += __builtin_amdgcn_mov_dpp(v, kDppXor2, 0xf, 0xf, false);
  v += __builtin_amdgcn_mov_dpp(v, kDppHalfMirror, 0xf, 0xf, false);
  v += __builtin_amdgcn_mov_dpp(v, kDppMirror, 0xf, 0xf, false);
  return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16) + __builtin_amdgcn_readlane(v, 32) +
         __builtin_amdgcn_readlane(v, 48);
}
__device__ __forceinline__ int wave_min_i(int v) {
  v = min(v, __builtin_amdgcn_mov_dpp(v, kDppXor1, 0xf, 0xf, false));
  v = min(v, __builtin_amdgcn_mov_dpp(v, kDppXor2, 0xf, 0xf, false));
  v = min(v, __builtin_amdgcn_mov_dpp(v, kDppHalfMirror, 0xf, 0xf, false));
  v = min(v, __builtin_amdgcn_mov_dpp(v, kDppMirror, 0xf, 0xf, false));
  return min(min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
             min(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}
// Inclusive prefix sum over lanes: Hillis-Steele inside rows (row_shr with
// zero fill), then the row totals carried by row_bcast:15 and row_bcast:31.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  int x = (int)v;
  x += __builtin_amdgcn_update_dpp(0, x, kDppRowShr1, 0xf, 0xf, true);
  x += __builtin_amdgcn_update_dpp(0, x, kDppRowShr2, 0xf, 0xf, true);
  x += __builtin_amdgcn_update_dpp(0, x, kDppRowShr4, 0xf, 0xf, true);
  x += __builtin_amdgcn_update_dpp(0, x, kDppRowShr8, 0xf, 0xf, true);
  x += __builtin_amdgcn_update_dpp(0, x, kDppRowBcast15, 0xa, 0xf, false);
  x += __builtin_amdgcn_update_dpp(0, x, kDppRowBcast31, 0xc, 0xf, false);
  return (uint32_t)x;
}

// Value of v held by lane `src` (any lane; ds_bpermute without bounds logic).
__device__ __forceinline__ double lane_read_d(double v, int src) {
  const unsigned long long u = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_ds_bpermute(src << 2, (int)(unsigned)u);
  const unsigned hi = (unsigned)__builtin_amdgcn_ds_bpermute(src << 2, (int)(unsigned)(u >> 32));
  return __longlong_as_double(((unsigned long long)hi << 32) | lo);
}

// Ascending bitonic sort of one value per lane over lanes [0, K), K the
// smallest power of two >= n (at least 2; n <= 64): the merge stages of
// blocks wider than K are skipped, so a few candidates cost a few stages.
// Lanes from K up are left in an unspecified order.
__device__ __forceinline__ double wave_sort_asc(double v, int n) {
  const int l = lane_id();
#pragma unroll
  for (int k = 2; k <= kWave; k <<= 1) {
    if (k > 2 && n <= (k >> 1)) break;             // uniform: lanes [0, k/2) already sorted
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      double o = lane_read_d(v, l ^ j);
      bool up = (l & k) == 0;
      bool lower = (l & j) == 0;
      v = (lower == up) ? fmin(v, o) : fmax(v, o);
    }
  }
  return v;
}

}  // namespace nsfrb
