// De-dispersion, boxcar filtering, S/N and max/argmax over time (search stage).
//
// Paper section 2.2: every pixel's time series is de-dispersed over a grid of
// DM trials with precomputed integer shifts, filtered with boxcars of several
// widths, normalised to S/N, and reduced to the maximum S/N over time and its
// TOA; section 2.3 keeps those S/N and TOA maps for all pixels, widths and DM
// trials.
//
// This file is compiled at plan time with the sample count per lane (kC), the
// store dtype (ST) and the boxcar plan (nsfrb_chain) fixed as constants; the
// generated prologue defines them. DM trials, delays, n_sub and n_t stay
// runtime values.
//
// Layout and work split (gfx950, wave64):
//  * one workgroup of kWaves waves per pixel; the pixel's normalised series
//    z[s][0..n_t) is staged in LDS, one row per sub-band of rs samples; samples
//    at and beyond n_t hold -inf, so any window that reaches past the end of a
//    de-dispersed series sums to -inf and can never be a maximum;
//  * wave w takes DM trials d = w, w + kWaves, ...; lane l holds the kC
//    consecutive samples t = kC*l + c (kC is odd, so lanes hit distinct LDS
//    banks at any delay);
//  * D_d[t] = sum_s z[s][t + delta[d][s]] is formed in registers (FP32);
//  * boxcars use the pairwise doubling B_2w[t] = B_w[t] + B_w[t+w]; a width
//    that is not a power of two is the sum of the power-of-two windows of its
//    binary digits placed end to end. Each output is a balanced sum, so the
//    FP32 error grows with log2(w) rather than w;
//  * a window shifted by k samples is read from register (c+k) mod kC of lane
//    l + (c+k)/kC: same lane, a DPP wave shift by one lane, or ds_bpermute.

#ifndef NSFRB_RTC_PROLOGUE
#error "compile through the search plan: the prologue defines kC, ST and nsfrb_chain"
#endif

namespace nsfrb {

constexpr int kWaves = 8;
constexpr float kNegInf = -__builtin_inff();

// Value of x held by lane l+1 (lane 63 gets -inf).
__device__ __forceinline__ float lane_next(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(kNegInf), __float_as_int(x),
                                                    0x130 /* wave_shl:1 */, 0xf, 0xf, false));
}
// Value of x held by lane l+q, q >= 2 (-inf beyond lane 63).
__device__ __forceinline__ float lane_ahead(float x, int q, int l) {
  const int v = __builtin_amdgcn_ds_bpermute((l + q) << 2, __float_as_int(x));
  return (l + q < kWave) ? __int_as_float(v) : kNegInf;
}

// out[c] = a[c] + b at sample t + K, for t = kC*l + c.
template <int K>
__device__ __forceinline__ void shift_add(float (&out)[kC], const float (&a)[kC], const float (&b)[kC]) {
  const int l = lane_id();
#pragma unroll
  for (int c = 0; c < kC; ++c) {
    const int q = (c + K) / kC;
    const int r = (c + K) % kC;
    float v;
    if (q == 0) v = b[r];
    else if (q == 1) v = lane_next(b[r]);
    else v = lane_ahead(b[r], q, l);
    out[c] = a[c] + v;
  }
}

__device__ __forceinline__ void copy_arr(float (&out)[kC], const float (&a)[kC]) {
#pragma unroll
  for (int c = 0; c < kC; ++c) out[c] = a[c];
}

__device__ __forceinline__ float wave_max_f(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}

struct Best {
  float s;
  int d, w, t;
};

__device__ __forceinline__ bool better(float s, int d, int w, const Best& b) {
  if (s > b.s) return true;
  if (s < b.s || !(s == b.s)) return false;
  return d < b.d || (d == b.d && w < b.w);
}

// Max over all samples of a boxcar array and the first sample reaching it.
__device__ __forceinline__ void max_first(const float (&b)[kC], float& M, int& T) {
  const int l = lane_id();
  float m = kNegInf;
  int idx = -1;
#pragma unroll
  for (int c = 0; c < kC; ++c) {
    const bool gt = b[c] > m;
    m = gt ? b[c] : m;
    idx = gt ? c : idx;
  }
  M = wave_max_f(m);
  const int cand = (idx >= 0 && m == M) ? kC * l + idx : 0x7fffffff;
  T = wave_min_i(cand);
  if (!(M > kNegInf)) T = -1;
}

struct Reporter {
  const float* norms;
  float* snr_max;
  int* toa;
  int n_pix, p, d, nw;
  Best best;
  __device__ __forceinline__ void emit(int iw, float M, int T) {
    const float s = (M > kNegInf) ? M / norms[iw] : kNegInf;
    if (lane_id() == 0) {
      const size_t o = ((size_t)d * nw + iw) * n_pix + p;
      snr_max[o] = s;
      toa[o] = T;
    }
    if (better(s, d, iw, best)) best = Best{s, d, iw, T};
  }
  __device__ __forceinline__ void operator()(int iw, const float (&b)[kC]) {
    float M;
    int T;
    max_first(b, M, T);
    emit(iw, M, T);
  }
  __device__ __forceinline__ void invalid(int iw) { emit(iw, kNegInf, -1); }
};

}  // namespace nsfrb

// The boxcar plan, generated per width list after this file: it forms every
// power-of-two window level from the de-dispersed series held in `cur` and
// calls rep(width_index, window_sums) once per width.
template <class R>
__device__ void nsfrb_chain(float (&cur)[kC], R& rep);

extern "C" __global__ __launch_bounds__(nsfrb::kWaves * nsfrb::kWave) void nsfrb_search_kernel(
    const ST* __restrict__ z, const int* __restrict__ delays, const int* __restrict__ dmaxv,
    const float* __restrict__ norms, int n_pix, int n_sub, int n_t, int n_dm, int rs,
    float* __restrict__ snr_max, int* __restrict__ toa, float* __restrict__ best_s,
    int* __restrict__ best_d, int* __restrict__ best_w, int* __restrict__ best_t) {
  using namespace nsfrb;
  extern __shared__ unsigned char lds_raw[];
  ST* zl = reinterpret_cast<ST*>(lds_raw);
  __shared__ Best red[kWaves];
  const int wv = threadIdx.x / kWave;
  const int l = lane_id();
  const ST neg = from_f32<ST>(kNegInf);

  for (int blk = blockIdx.x; blk < n_pix; blk += gridDim.x) {
    // pixels of one XCD are contiguous (workgroups are dealt round-robin over 8 XCDs)
    int p = blk;
    if ((n_pix & 7) == 0 && gridDim.x == n_pix) p = (blk & 7) * (n_pix >> 3) + (blk >> 3);
    // ---- stage z[p] into LDS, rows of rs samples, -inf beyond n_t
    const ST* zp = z + (size_t)p * n_sub * n_t;
    for (int s = 0; s < n_sub; ++s) {
      const ST* src = zp + (size_t)s * n_t;
      ST* dst = zl + s * rs;
      for (int u = threadIdx.x; u < rs; u += blockDim.x) dst[u] = (u < n_t) ? src[u] : neg;
    }
    __syncthreads();

    Reporter rep{norms, snr_max, toa, n_pix, p, 0, NSFRB_NW, Best{kNegInf, -1, -1, -1}};
    for (int d = wv; d < n_dm; d += kWaves) {
      rep.d = d;
      if (dmaxv[d] >= n_t) {
        for (int iw = 0; iw < NSFRB_NW; ++iw) rep.invalid(iw);
        continue;
      }
      float cur[kC];
#pragma unroll
      for (int c = 0; c < kC; ++c) cur[c] = 0.f;
      for (int s = 0; s < n_sub; ++s) {
        const int dl = delays[d * n_sub + s];
        const ST* row = zl + s * rs + dl + kC * l;
#pragma unroll
        for (int c = 0; c < kC; ++c) cur[c] += to_f32(row[c]);
      }
      nsfrb_chain(cur, rep);
    }
    if (l == 0) red[wv] = rep.best;
    __syncthreads();
    if (threadIdx.x == 0) {
      Best b = red[0];
      for (int k = 1; k < kWaves; ++k)
        if (better(red[k].s, red[k].d, red[k].w, b)) b = red[k];
      const bool ok = b.s > kNegInf;
      best_s[p] = ok ? b.s : kNegInf;
      best_d[p] = ok ? b.d : -1;
      best_w[p] = ok ? b.w : -1;
      best_t[p] = ok ? b.t : -1;
    }
    __syncthreads();
  }
}
