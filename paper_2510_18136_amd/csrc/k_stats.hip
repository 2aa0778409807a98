// Robust noise statistics and normalisation (stats + normalise stage).
//
// For every (pixel, sub-band) series of n_t samples: the FP64 median and
// median absolute deviation, sigma = 1.482602218505602 * MAD, and the
// normalised series z = (x - median) / sigma formed in FP64, rounded to FP32
// and then to the store dtype (paper section 2.2: median subtraction per pixel
// and normalisation by the noise; section 3.2: a robust estimate is needed
// because wide pulses bias a plain one).
//
// Launch: one workgroup of 8 waves per (tile of 16 pixels, sub-band). The
// raw cube [t][s][p] is read in coalesced 16-pixel rows and transposed through
// LDS so that each wave holds two pixels' series in registers (lane l, register
// j <-> sample t = 64 j + l). The z series is written time-contiguous to the
// search layout [p][s][t].
//
// Exact selection: order statistics are found by adaptive histogramming of the
// FP64 values over [lo, hi] into 256 equal bins (bin = floor((v - lo) * scale),
// a monotone map, so rank bookkeeping is exact whatever the rounding), keeping
// only the bin that holds the wanted rank, until <= 64 candidates remain; those
// are sorted across the wave. Each round shrinks the range strictly, so the
// loop ends; a degenerate range falls back to stepping through distinct values.
#include "device_common.h"
#include "nsfrb_internal.h"

namespace nsfrb {

constexpr int kStatTilePix = 16;
constexpr int kStatWaves = 8;
constexpr double kMadToSigma = 1.482602218505602;

struct SeriesCtx {
  uint32_t* hist;   // 256 bins (this wave)
  double* list;     // 64 candidates (this wave)
  int n_t;
};

// k-th smallest (0-based) of the values val(j) over valid registers j.
template <int V, class Val>
__device__ __forceinline__ double select_kth(const Val& val, int k, const SeriesCtx& cx) {
  const int l = lane_id();
  double lo = __builtin_inf(), hi = -__builtin_inf();
#pragma unroll
  for (int j = 0; j < V; ++j) {
    if (64 * j + l < cx.n_t) { double v = val(j); lo = fmin(lo, v); hi = fmax(hi, v); }
  }
  lo = wave_min(lo);
  hi = wave_max(hi);
  int krem = k;
  for (int iter = 0; iter < 80; ++iter) {
    if (!(lo < hi)) return lo;
    const double scale = 256.0 / (hi - lo);
    if (!(scale < 1e300)) break;   // range too narrow to bin: step through values
    cx.hist[4 * l + 0] = 0; cx.hist[4 * l + 1] = 0; cx.hist[4 * l + 2] = 0; cx.hist[4 * l + 3] = 0;
    wave_lds_sync();
#pragma unroll
    for (int j = 0; j < V; ++j) {
      if (64 * j + l < cx.n_t) {
        double v = val(j);
        if (v >= lo && v <= hi) {
          int b = (int)((v - lo) * scale);
          b = b > 255 ? 255 : b;
          atomicAdd(&cx.hist[b], 1u);
        }
      }
    }
    wave_lds_sync();
    uint32_t h0 = cx.hist[4 * l], h1 = cx.hist[4 * l + 1], h2 = cx.hist[4 * l + 2], h3 = cx.hist[4 * l + 3];
    uint32_t s = h0 + h1 + h2 + h3;
    uint32_t incl = wave_incl_scan(s);
    uint32_t excl = incl - s;
    bool hit = (excl <= (uint32_t)krem) && ((uint32_t)krem < incl);
    uint64_t m = ballot(hit);
    int L = __ffsll((long long)m) - 1;
    // the bin inside lane L that holds rank krem
    uint32_t e = __shfl(excl, L);
    uint32_t a0 = __shfl(h0, L), a1 = __shfl(h1, L), a2 = __shfl(h2, L), a3 = __shfl(h3, L);
    uint32_t r = (uint32_t)krem - e;
    int bsel; uint32_t before, cnt;
    if (r < a0) { bsel = 0; before = 0; cnt = a0; }
    else if (r < a0 + a1) { bsel = 1; before = a0; cnt = a1; }
    else if (r < a0 + a1 + a2) { bsel = 2; before = a0 + a1; cnt = a2; }
    else { bsel = 3; before = a0 + a1 + a2; cnt = a3; }
    const int B = 4 * L + bsel;
    krem = (int)(r - before);
    if (cnt <= 64) {
      int base = 0;
#pragma unroll
      for (int j = 0; j < V; ++j) {
        bool mem = false;
        double v = 0.0;
        if (64 * j + l < cx.n_t) {
          v = val(j);
          if (v >= lo && v <= hi) {
            int b = (int)((v - lo) * scale);
            b = b > 255 ? 255 : b;
            mem = (b == B);
          }
        }
        uint64_t mm = ballot(mem);
        if (mem) cx.list[base + lanes_below(mm)] = v;
        base += popc64(mm);
      }
      wave_lds_sync();
      double c = (l < (int)cnt) ? cx.list[l] : __builtin_inf();
      wave_lds_sync();
      c = wave_sort_asc(c);
      return __shfl(c, krem);
    }
    double nlo = __builtin_inf(), nhi = -__builtin_inf();
#pragma unroll
    for (int j = 0; j < V; ++j) {
      if (64 * j + l < cx.n_t) {
        double v = val(j);
        if (v >= lo && v <= hi) {
          int b = (int)((v - lo) * scale);
          b = b > 255 ? 255 : b;
          if (b == B) { nlo = fmin(nlo, v); nhi = fmax(nhi, v); }
        }
      }
    }
    lo = wave_min(nlo);
    hi = wave_max(nhi);
  }
  // Fallback: walk the distinct values upward from lo.
  double cur = lo;
  for (;;) {
    int ceq = 0;
    double nxt = __builtin_inf();
#pragma unroll
    for (int j = 0; j < V; ++j) {
      if (64 * j + l < cx.n_t) {
        double v = val(j);
        ceq += (v == cur);
        if (v > cur) nxt = fmin(nxt, v);
      }
    }
    ceq = wave_sum(ceq);
    if (krem < ceq) return cur;
    krem -= ceq;
    cur = wave_min(nxt);
    if (!(cur < __builtin_inf())) return cur;
  }
}

// The order statistic right after `a` (= the k-th smallest): the (k+1)-th.
template <int V, class Val>
__device__ __forceinline__ double next_order_stat(const Val& val, double a, int k, const SeriesCtx& cx) {
  const int l = lane_id();
  int cle = 0;
  double gt = __builtin_inf();
#pragma unroll
  for (int j = 0; j < V; ++j) {
    if (64 * j + l < cx.n_t) {
      double v = val(j);
      cle += (v <= a);
      if (v > a) gt = fmin(gt, v);
    }
  }
  cle = wave_sum(cle);
  gt = wave_min(gt);
  return (cle > k + 1) ? a : gt;
}

template <int V, class Val>
__device__ __forceinline__ double median_of(const Val& val, const SeriesCtx& cx) {
  const int n = cx.n_t;
  const int k1 = (n - 1) / 2;
  double a = select_kth<V>(val, k1, cx);
  if (n & 1) return a;
  double b = next_order_stat<V>(val, a, k1, cx);
  return (a + b) * 0.5;
}

// Statistics + normalisation of one series held as xv[j] <-> t = 64 j + lane.
template <int V, typename ST>
__device__ __forceinline__ void process_series(const float (&xv)[V], int p, int s, int n_t, int n_sub, int mode,
                                               const double* __restrict__ med_in, const double* __restrict__ sig_in,
                                               double* __restrict__ med_out, double* __restrict__ sig_out,
                                               ST* __restrict__ z, unsigned long long* __restrict__ flag_count,
                                               const SeriesCtx& cx) {
  const int l = lane_id();
  bool bad = false;
#pragma unroll
  for (int j = 0; j < V; ++j)
    if (64 * j + l < n_t && !__builtin_isfinite(xv[j])) bad = true;
  const bool any_bad = ballot(bad) != 0;

  long long nflag = 0;
  double med = 0.0, sig = 1.0;
  bool usable = true;
  if (mode == NORM_PIXEL_SUBBAND) {
    if (any_bad) {
      med = __builtin_nan(""); sig = __builtin_nan(""); usable = false;
    } else {
      auto vx = [&](int j) { return (double)xv[j]; };
      med = median_of<V>(vx, cx);
      const double mm = med;
      auto vd = [&](int j) { return fabs((double)xv[j] - mm); };
      const double mad = median_of<V>(vd, cx);
      sig = kMadToSigma * mad;
      usable = (sig > 0.0) && (sig < __builtin_inf());
    }
    if (l == 0) {
      med_out[(size_t)p * n_sub + s] = med;
      sig_out[(size_t)p * n_sub + s] = sig;
    }
    if (!usable) nflag = 1;
  } else if (mode == NORM_EXTERNAL) {
    med = med_in[(size_t)p * n_sub + s];
    sig = sig_in[(size_t)p * n_sub + s];
    usable = __builtin_isfinite(med) && __builtin_isfinite(sig) && sig > 0.0;
    if (!usable) nflag = 1;
  }
  ST* zrow = z + ((size_t)p * n_sub + s) * n_t;
  int nbad_samples = 0;
#pragma unroll
  for (int j = 0; j < V; ++j) {
    const int t = 64 * j + l;
    if (t < n_t) {
      float zf;
      const bool fin = __builtin_isfinite(xv[j]);
      if (mode == NORM_NONE) {
        zf = fin ? xv[j] : 0.0f;
        nbad_samples += !fin;
      } else if (!usable) {
        zf = 0.0f;
      } else if (mode == NORM_EXTERNAL && !fin) {
        zf = 0.0f;
        nbad_samples += 1;
      } else {
        zf = (float)(((double)xv[j] - med) / sig);
      }
      zrow[t] = from_f32<ST>(zf);
    }
  }
  if (mode == NORM_NONE || mode == NORM_EXTERNAL) nflag += wave_sum(nbad_samples);
  if (l == 0 && nflag) atomicAdd(flag_count, (unsigned long long)nflag);
}

template <int V, typename InT, typename ST>
__global__ __launch_bounds__(kStatWaves * kWave) void k_stats_norm(
    const InT* __restrict__ x, int n_t, int n_sub, int n_pix, int mode,
    const double* __restrict__ med_in, const double* __restrict__ sig_in,
    double* __restrict__ med_out, double* __restrict__ sig_out,
    ST* __restrict__ z, unsigned long long* __restrict__ flag_count) {
  constexpr int VC = V < 4 ? V : 4;               // registers filled per LDS chunk
  constexpr int CT = 64 * VC;                     // samples per chunk
  constexpr int RS = kStatTilePix + 1;            // padded LDS row
  __shared__ float tile[CT * RS];
  __shared__ uint32_t hist_all[kStatWaves][256];
  __shared__ double list_all[kStatWaves][64];

  const int s = blockIdx.y;
  const int p0 = blockIdx.x * kStatTilePix;
  const int w = threadIdx.x / kWave;
  const int l = lane_id();
  const size_t plane = (size_t)n_sub * n_pix;

  // this wave's two pixels: p0 + w and p0 + w + kStatWaves
  float xa[V], xb[V];
  // ---- load: coalesced rows of 16 pixels, transposed through LDS
#pragma unroll
  for (int ch = 0; ch < V / VC; ++ch) {
    const int t0 = ch * CT;
    for (int i = threadIdx.x; i < CT * kStatTilePix; i += kStatWaves * kWave) {
      const int r = i / kStatTilePix, c = i % kStatTilePix;
      const int t = t0 + r, pp = p0 + c;
      float v = __builtin_nanf("");
      if (t < n_t && pp < n_pix) v = to_f32(x[(size_t)t * plane + (size_t)s * n_pix + pp]);
      tile[r * RS + c] = v;
    }
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < VC; ++jj) {
      xa[ch * VC + jj] = tile[(64 * jj + l) * RS + w];
      xb[ch * VC + jj] = tile[(64 * jj + l) * RS + w + kStatWaves];
    }
    __syncthreads();
  }
  SeriesCtx cx{hist_all[w], list_all[w], n_t};
  if (p0 + w < n_pix)
    process_series<V, ST>(xa, p0 + w, s, n_t, n_sub, mode, med_in, sig_in, med_out, sig_out, z, flag_count, cx);
  if (p0 + w + kStatWaves < n_pix)
    process_series<V, ST>(xb, p0 + w + kStatWaves, s, n_t, n_sub, mode, med_in, sig_in, med_out, sig_out, z,
                          flag_count, cx);
}

// ------------------------------------------------------------ launcher
template <int V, typename InT, typename ST>
static hipError_t launch_stats_v(const StatsLaunch& a, hipStream_t st) {
  dim3 grid((a.n_pix + kStatTilePix - 1) / kStatTilePix, a.n_sub);
  hipLaunchKernelGGL((k_stats_norm<V, InT, ST>), grid, dim3(kStatWaves * kWave), 0, st,
                     (const InT*)a.x, a.n_t, a.n_sub, a.n_pix, a.mode, a.med_in, a.sig_in,
                     a.med_out, a.sig_out, (ST*)a.z, a.flag_count);
  return hipGetLastError();
}

template <typename InT, typename ST>
static hipError_t launch_stats_t(const StatsLaunch& a, hipStream_t st) {
  const int v = (a.n_t + 63) / 64;
  if (v <= 1) return launch_stats_v<1, InT, ST>(a, st);
  if (v <= 2) return launch_stats_v<2, InT, ST>(a, st);
  if (v <= 4) return launch_stats_v<4, InT, ST>(a, st);
  if (v <= 8) return launch_stats_v<8, InT, ST>(a, st);
  if (v <= 16) return launch_stats_v<16, InT, ST>(a, st);
  if (v <= 32) return launch_stats_v<32, InT, ST>(a, st);
  return launch_stats_v<64, InT, ST>(a, st);
}

template <typename InT>
static hipError_t launch_stats_in(const StatsLaunch& a, hipStream_t st) {
  switch (a.store_dtype) {
    case DT_F32: return launch_stats_t<InT, float>(a, st);
    case DT_F16: return launch_stats_t<InT, _Float16>(a, st);
    default: return launch_stats_t<InT, bf16_t>(a, st);
  }
}

__global__ void k_zero_u64(unsigned long long* p) {
  if (threadIdx.x == 0) p[0] = 0ull;
}

hipError_t launch_zero_u64(unsigned long long* p, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_stats(const StatsLaunch& a, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, a.flag_count);
  switch (a.in_dtype) {
    case DT_F32: return launch_stats_in<float>(a, st);
    case DT_F16: return launch_stats_in<_Float16>(a, st);
    default: return launch_stats_in<bf16_t>(a, st);
  }
}

}  // namespace nsfrb
