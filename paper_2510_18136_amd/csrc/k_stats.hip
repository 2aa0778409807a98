// Robust noise statistics and normalisation (stats + normalise stage).
//
// For every (pixel, sub-band) series of n_t samples: the FP64 median and
// median absolute deviation, sigma = 1.482602218505602 * MAD, and the
// normalised series z = (x - median) / sigma formed in FP64, rounded to FP32
// and then to the store dtype (paper section 2.2: median subtraction per pixel
// and normalisation by the noise; section 3.2: a robust estimate is needed
// because wide pulses bias a plain one).
//
// Launch: one workgroup of W waves per (tile of W pixels, sub-band), W = 16
// (8 for series longer than 1024 samples). The raw cube [t][s][p] (or a ring
// of its last n_t samples, read oldest first) is loaded in coalesced W-pixel
// rows into one padded LDS row per pixel; wave w works on pixel w's row, lane l
// and step j reading sample t = 64 j + l. The z series is written
// time-contiguous to the search layout [p][s][t].
//
// Exact selection: an order statistic of FP32 keys is found by adaptive
// histogramming over [lo, hi] into 256 equal bins (bin = (v - lo) * scale
// rounded down, a monotone map, so rank bookkeeping is exact whatever the
// rounding),
// keeping only the bin that holds the wanted rank, until <= 64 candidates
// remain; those are sorted across the wave. Each round shrinks the range
// strictly, so the loop ends; a range too narrow to bin falls back to stepping
// through distinct values.
//
// The median selects over the FP32 samples themselves. The MAD selects over
// the FP32 roundings of the FP64 distances |x - median|: rounding is monotone,
// so all samples of a lower key bin have smaller FP64 distances than those of
// the bin holding the wanted rank, and all samples of a higher bin larger ones.
// When that bin has <= 64 members, the FP64 values of its members are gathered
// and sorted across the wave, which yields both middle order statistics at
// once. The median's key range comes from the finite-check pass; the MAD's is
// [0, largest distance], the largest distance being that of the series' minimum
// or maximum. Ranges that cannot be binned that far (long runs of equal keys)
// take a general path: the k-th key, then the FP64 values among its ties.
// Usually the MAD needs no histogram of its own: the median's one-round
// histogram predicts a narrow bracket of distances around it, and one exact pass
// checks that the bracket holds the middle ranks (see mad_from_bracket).
//
// Normalisation divides in FP64 by Markstein's method: with r = RN(1/sigma)
// (a correctly rounded division, once per series), q0 = RN(a*r),
// e = fma(-q0, sigma, a) (exact) and q = fma(e, r, q0) is the correctly rounded
// quotient a/sigma (Markstein, IBM J. Res. Dev. 34(1), 1990); sigma far from
// 1 in exponent takes the plain division instead.
#include "device_common.h"
#include "nsfrb_internal.h"

namespace nsfrb {

// Waves per workgroup (= pixels per tile): 16 for short series, 8 for long
// ones (the LDS rows of 16 series of 2048 samples would not leave room for a
// second workgroup on the CU).
template <int V> struct StatShape {
  static constexpr int kWaves = V >= 32 ? 8 : 16;
  // two workgroups per CU (8 waves each) for series up to 2048 samples: at most
  // 128 VGPRs; longer series fill the CU's LDS with one workgroup
  static constexpr int kMinWavesPerEU = V <= 32 ? 4 : 1;
};
constexpr double kMadToSigma = 1.482602218505602;

typedef const __attribute__((address_space(1))) char* gptr;   // global memory
// One input sample at a global address, as FP32.
template <typename InT> __device__ __forceinline__ float load_global_f32(gptr a) {
  if constexpr (sizeof(InT) == 4) {
    return __uint_as_float(*(const __attribute__((address_space(1))) uint32_t*)a);
  } else {
    const uint16_t bits = *(const __attribute__((address_space(1))) uint16_t*)a;
    InT v;
    __builtin_memcpy(&v, &bits, 2);
    return to_f32(v);
  }
}

struct SeriesCtx {
  uint32_t* hist;   // 256 bins (this wave)
  double* list;     // 64 candidates (this wave)
  int n_t;
};

// Result of a selection over FP32 keys: the key value, and the rank of the
// wanted element among the samples whose key equals it.
struct Sel {
  float key;
  int rank_in_ties;
};

// Keys of a series seen through an accessor key(j), j = 0..V-1 (sample
// 64 j + lane): the series itself in LDS, or a value derived from it.
struct LdsSeries {
  const float* x;     // this wave's series, sample t at x[t]
  int l;
  __device__ __forceinline__ float operator()(int j) const { return x[64 * j + l]; }
};
// FP32-rounded distances |x - med| (FP64 difference), formed from the LDS
// series on each read instead of being held in registers.
struct DistKeys {
  LdsSeries x;
  double med;
  __device__ __forceinline__ float operator()(int j) const { return (float)fabs((double)x(j) - med); }
};

// Passes that write LDS (histogram atomics, candidate lists) read their keys
// kChunk registers at a time ahead of that work: the compiler does not move a
// read of the series above an LDS write that might alias it, so without the
// grouping every sample would wait a full LDS round trip.
constexpr int kChunk = 8;
template <int V, class Key, class Fn>
__device__ __forceinline__ void for_each_key(const Key& key, Fn&& fn) {
#pragma unroll
  for (int j0 = 0; j0 < V; j0 += kChunk) {
    float v[kChunk];
#pragma unroll
    for (int b = 0; b < kChunk; ++b)
      if (j0 + b < V) v[b] = key(j0 + b);
#pragma unroll
    for (int b = 0; b < kChunk; ++b)
      if (j0 + b < V) fn(j0 + b, v[b]);
  }
}

// k-th smallest (0-based) of the FP32 keys key(j). Registers past the end of
// the series hold NaN, which fails every comparison and is ignored by
// fminf/fmaxf, so they never take part.
template <int V, class Key>
__device__ __forceinline__ Sel select_kth_f32(const Key& key, int k, const SeriesCtx& cx) {
  const int l = lane_id();
  float lo = __builtin_inff(), hi = -__builtin_inff();
#pragma unroll
  for (int j = 0; j < V; ++j)
    { lo = fminf(lo, key(j)); hi = fmaxf(hi, key(j)); }
  lo = wave_min_f(lo);
  hi = wave_max_f(hi);
  int krem = k;                                    // rank among keys in [lo, hi]
  for (int iter = 0; iter < 48; ++iter) {
    if (!(lo < hi)) return Sel{lo, krem};
    const float scale = 256.0f / (hi - lo);
    if (!(scale > 0.0f && scale < 1e30f)) break;
    cx.hist[4 * l + 0] = 0; cx.hist[4 * l + 1] = 0; cx.hist[4 * l + 2] = 0; cx.hist[4 * l + 3] = 0;
    wave_lds_sync();
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const float v = key(j);
      if (v >= lo && v <= hi) {
        int b = (int)((v - lo) * scale);
        b = b > 255 ? 255 : b;
        atomicAdd(&cx.hist[b], 1u);
      }
    }
    wave_lds_sync();
    const uint32_t h0 = cx.hist[4 * l], h1 = cx.hist[4 * l + 1], h2 = cx.hist[4 * l + 2], h3 = cx.hist[4 * l + 3];
    const uint32_t s4 = h0 + h1 + h2 + h3;
    const uint32_t incl = wave_incl_scan(s4);
    const uint32_t excl = incl - s4;
    const uint64_t m = ballot((excl <= (uint32_t)krem) && ((uint32_t)krem < incl));
    const int L = __ffsll((long long)m) - 1;
    const uint32_t e = (uint32_t)__builtin_amdgcn_readlane((int)excl, L);
    const uint32_t a0 = (uint32_t)__builtin_amdgcn_readlane((int)h0, L), a1 = (uint32_t)__builtin_amdgcn_readlane((int)h1, L);
    const uint32_t a2 = (uint32_t)__builtin_amdgcn_readlane((int)h2, L), a3 = (uint32_t)__builtin_amdgcn_readlane((int)h3, L);
    const uint32_t r = (uint32_t)krem - e;
    int bsel;
    uint32_t before, cnt;
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
        const float v = key(j);
        bool mem = false;
        if (v >= lo && v <= hi) {
          int b = (int)((v - lo) * scale);
          b = b > 255 ? 255 : b;
          mem = (b == B);
        }
        const uint64_t mm = ballot(mem);
        if (mem) cx.list[base + lanes_below(mm)] = (double)v;
        base += popc64(mm);
      }
      wave_lds_sync();
      double c = (l < (int)cnt) ? cx.list[l] : __builtin_inf();
      wave_lds_sync();
      c = wave_sort_asc(c, (int)cnt);
      const float kv = (float)readlane_d(c, krem);
      // rank among equal keys: krem minus the candidates below it
      const int below = popc64(ballot(l < (int)cnt && c < (double)kv));
      return Sel{kv, krem - below};
    }
    float nlo = __builtin_inff(), nhi = -__builtin_inff();
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const float v = key(j);
      if (v >= lo && v <= hi) {
        int b = (int)((v - lo) * scale);
        b = b > 255 ? 255 : b;
        if (b == B) { nlo = fminf(nlo, v); nhi = fmaxf(nhi, v); }
      }
    }
    lo = wave_min_f(nlo);
    hi = wave_max_f(nhi);
  }
  // Fallback: walk the distinct keys upward from lo.
  float cur = lo;
  for (;;) {
    int ceq = 0;
    float nxt = __builtin_inff();
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const float v = key(j);
      ceq += (v == cur);
      if (v > cur) nxt = fminf(nxt, v);
    }
    ceq = wave_sum(ceq);
    if (krem < ceq) return Sel{cur, krem};
    krem -= ceq;
    cur = wave_min_f(nxt);
    if (!(cur < __builtin_inff())) return Sel{cur, 0};
  }
}

// Exact FP64 order statistics k and (if want_second) k + 1 of val(j), where the
// FP32 keys key(j) = RN32(val(j)) all lie in [lo, hi]. Rounding is monotone, so
// every sample of a lower key bin has a smaller value than every sample of the
// bin holding rank k, and every sample of a higher bin a larger one: once that
// bin has <= 64 members, their FP64 values sorted across the wave give the
// answer directly. Returns the number of histogram rounds used, or 0 (nothing
// decided) when the range cannot be binned down to such a bin; the caller then
// takes the general path. After a one-round answer, cx.hist still holds the
// histogram of the whole range [lo, hi].
template <int V, class Key, class Val>
__device__ __forceinline__ int select_values(const Key& key, const Val& val, int k, bool want_second, float lo,
                                              float hi, bool all_in, const SeriesCtx& cx, double& first,
                                              double& second) {
  const int l = lane_id();
  int krem = k;                                    // rank among keys in [lo, hi]
  for (int iter = 0; iter < 48; ++iter) {
    if (!(lo < hi)) return 0;
    const float scale = 256.0f / (hi - lo);
    if (!(scale > 0.0f && scale < 1e30f)) return 0;
    // bin(v) = trunc(fma(v, scale, -lo scale)) clamped to [0, 255]: monotone
    // in v (the rounding of -lo scale shifts every bin edge alike)
    const float off = -lo * scale;
    auto bin_of = [&](float v) {
      const int b = (int)__builtin_fmaf(v, scale, off);
      return min(max(b, 0), 255);
    };
    // keys known to lie in [lo, hi]: the first round when every register holds
    // a finite key and [lo, hi] spans them all
    const bool in_range = all_in && iter == 0;
    cx.hist[4 * l + 0] = 0; cx.hist[4 * l + 1] = 0; cx.hist[4 * l + 2] = 0; cx.hist[4 * l + 3] = 0;
    wave_lds_sync();
    if (in_range) {
      for_each_key<V>(key, [&](int, float v) { atomicAdd(&cx.hist[bin_of(v)], 1u); });
      asm volatile("");                             // keeps this loop from being merged with the checked one
    } else {
      // keys outside [lo, hi] (and NaN padding) are masked off; sending them
      // all to one discard bin instead would make up to 64 lanes of an atomic
      // hit the same address, which the LDS serialises
      for_each_key<V>(key, [&](int, float v) {
        if (v >= lo && v <= hi) atomicAdd(&cx.hist[bin_of(v)], 1u);
      });
    }
    wave_lds_sync();
    const uint32_t h0 = cx.hist[4 * l], h1 = cx.hist[4 * l + 1], h2 = cx.hist[4 * l + 2], h3 = cx.hist[4 * l + 3];
    const uint32_t s4 = h0 + h1 + h2 + h3;
    const uint32_t incl = wave_incl_scan(s4);
    const uint32_t excl = incl - s4;
    const uint64_t m = ballot((excl <= (uint32_t)krem) && ((uint32_t)krem < incl));
    const int L = __ffsll((long long)m) - 1;
    const uint32_t e = (uint32_t)__builtin_amdgcn_readlane((int)excl, L);
    const uint32_t a0 = (uint32_t)__builtin_amdgcn_readlane((int)h0, L), a1 = (uint32_t)__builtin_amdgcn_readlane((int)h1, L);
    const uint32_t a2 = (uint32_t)__builtin_amdgcn_readlane((int)h2, L), a3 = (uint32_t)__builtin_amdgcn_readlane((int)h3, L);
    const uint32_t r = (uint32_t)krem - e;
    int bsel;
    uint32_t before, cnt;
    if (r < a0) { bsel = 0; before = 0; cnt = a0; }
    else if (r < a0 + a1) { bsel = 1; before = a0; cnt = a1; }
    else if (r < a0 + a1 + a2) { bsel = 2; before = a0 + a1; cnt = a2; }
    else { bsel = 3; before = a0 + a1 + a2; cnt = a3; }
    const int B = 4 * L + bsel;
    krem = (int)(r - before);
    if (cnt <= 64) {
      int base = 0;
      for_each_key<V>(key, [&](int j, float v) {
        const bool mem = (in_range || (v >= lo && v <= hi)) && bin_of(v) == B;
        const uint64_t mm = ballot(mem);
        if (mem) cx.list[base + lanes_below(mm)] = val(j);
        base += popc64(mm);
      });
      wave_lds_sync();
      double c = (l < (int)cnt) ? cx.list[l] : __builtin_inf();
      wave_lds_sync();
      c = wave_sort_asc(c, (int)cnt);
      first = readlane_d(c, krem);
      if (!want_second) return iter + 1;
      if (krem + 1 < (int)cnt) {
        second = readlane_d(c, krem + 1);
        return iter + 1;
      }
      // rank k is the bin's largest value: rank k + 1 is the smallest value above it
      double nx = __builtin_inf();
#pragma unroll
      for (int j = 0; j < V; ++j) {
        const double v = val(j);
        if (v > first) nx = fmin(nx, v);
      }
      second = wave_min(nx);
      return iter + 1;
    }
    float nlo = __builtin_inff(), nhi = -__builtin_inff();
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const float v = key(j);
      if ((v >= lo && v <= hi) && bin_of(v) == B) { nlo = fminf(nlo, v); nhi = fmaxf(nhi, v); }
    }
    lo = wave_min_f(nlo);
    hi = wave_max_f(nhi);
  }
  return 0;
}

// MAD from a bracket (a shortcut; the result is exact or nothing is decided).
// cx.hist holds the one-round histogram of the samples over [lo, lo + 256/scale]
// that found the median. Reading it as a piecewise-uniform distribution, two
// parallel 64-point searches find the distance d at which the count of samples
// within d of the median reaches the middle rank, and the bracket [d_lo, d_hi]
// around it is sized to hold about 40 samples. One pass then counts, exactly in
// FP64, the distances below d_lo and gathers those inside the bracket. If the
// middle rank(s) fall inside and at most 64 were gathered, their sorted FP64
// values give the answer; otherwise the caller runs the general selection.
template <int V>
__device__ __forceinline__ bool mad_from_bracket(const LdsSeries& x, double med, int k, bool even, float lo,
                                                 float scale, float dmax, const SeriesCtx& cx, double& mad) {
  const int l = lane_id();
  // exclusive prefix counts P[b] in place of the counts (P[256] = total)
  const uint32_t h0 = cx.hist[4 * l], h1 = cx.hist[4 * l + 1], h2 = cx.hist[4 * l + 2], h3 = cx.hist[4 * l + 3];
  const uint32_t s4 = h0 + h1 + h2 + h3;
  const uint32_t incl = wave_incl_scan(s4);
  const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
  wave_lds_sync();
  const uint32_t e0 = incl - s4;
  cx.hist[4 * l] = e0;
  cx.hist[4 * l + 1] = e0 + h0;
  cx.hist[4 * l + 2] = e0 + h0 + h1;
  cx.hist[4 * l + 3] = e0 + h0 + h1 + h2;
  wave_lds_sync();
  const float mf = (float)med;
  auto cdf = [&](float p) {                         // interpolated count of samples below p
    const float u = (p - lo) * scale;
    if (!(u > 0.0f)) return 0.0f;
    if (!(u < 256.0f)) return (float)total;
    const int b = (int)u;
    const float pb = (float)cx.hist[b];
    const float pn = b < 255 ? (float)cx.hist[b + 1] : (float)total;
    return pb + (u - (float)b) * (pn - pb);
  };
  const float target = (float)k + (even ? 1.5f : 1.0f);
  // coarse: d = dmax (i + 1) / 64; fine: 64 steps inside the first coarse step reaching the target
  float d = dmax * (float)(l + 1) * (1.0f / 64.0f);
  uint64_t m = ballot(cdf(mf + d) - cdf(mf - d) >= target);
  int i = m ? __ffsll((long long)m) - 1 : 63;
  const float c1 = dmax * (float)(i + 1) * (1.0f / 64.0f), c0 = dmax * (float)i * (1.0f / 64.0f);
  d = c0 + (c1 - c0) * (float)(l + 1) * (1.0f / 64.0f);
  m = ballot(cdf(mf + d) - cdf(mf - d) >= target);
  i = m ? __ffsll((long long)m) - 1 : 63;
  const float dh = c0 + (c1 - c0) * (float)(i + 1) * (1.0f / 64.0f);
  // local density (samples per unit distance) on both sides, from the bins there
  auto dens = [&](float p) {
    const float u = (p - lo) * scale;
    if (!(u >= 0.0f && u < 256.0f)) return 0.0f;
    const int b = (int)u;
    const float pn = b < 255 ? (float)cx.hist[b + 1] : (float)total;
    return (pn - (float)cx.hist[b]) * scale;
  };
  const float rho = dens(mf + dh) + dens(mf - dh);
  const float half = rho > 0.0f ? 20.0f / rho : dmax;
  const double d_lo = fmax(0.0, (double)dh - (double)half), d_hi = (double)dh + (double)half;
  wave_lds_sync();
  // exact pass: distances below the bracket, and the ones inside it
  int below = 0, base = 0;
  for_each_key<V>(x, [&](int, float xv) {
    const double dv = fabs((double)xv - med);       // NaN padding fails both tests
    below += dv < d_lo;
    const bool in = dv >= d_lo && dv <= d_hi;
    const uint64_t mm = ballot(in);
    const int pos = base + lanes_below(mm);
    if (in && pos < 64) cx.list[pos] = dv;
    base += popc64(mm);
  });
  below = wave_sum(below);
  const int need = k + (even ? 1 : 0);               // highest rank needed
  if (!(below <= k && below + base > need && base <= 64)) return false;
  wave_lds_sync();
  double c = (l < base) ? cx.list[l] : __builtin_inf();
  wave_lds_sync();
  c = wave_sort_asc(c, base);
  const double a = readlane_d(c, k - below);
  mad = even ? (a + readlane_d(c, k - below + 1)) * 0.5 : a;
  return true;
}

// The (rank)-th and (rank+1)-th smallest FP64 values val(j) among the samples
// whose key equals kv; `second` is +inf when there is no (rank+1)-th tie.
template <int V, class Key, class Val>
__device__ __forceinline__ void resolve_ties(const Key& key, float kv, int rank, const Val& val,
                                             const SeriesCtx& cx, double& first, double& second) {
  const int l = lane_id();
  int base = 0;
#pragma unroll
  for (int j = 0; j < V; ++j) {
    const bool mem = key(j) == kv;
    const uint64_t mm = ballot(mem);
    if (mem) {
      const int pos = base + lanes_below(mm);
      if (pos < 64) cx.list[pos] = val(j);
    }
    base += popc64(mm);
  }
  if (base <= 64) {
    wave_lds_sync();
    double c = (l < base) ? cx.list[l] : __builtin_inf();
    wave_lds_sync();
    c = wave_sort_asc(c, base);
    first = readlane_d(c, rank);
    second = (rank + 1 < base) ? readlane_d(c, rank + 1) : __builtin_inf();
    return;
  }
  // more than 64 equal keys: step through their distinct FP64 values
  double cur = -__builtin_inf();
  bool have_first = false;
  for (;;) {
    double nxt = __builtin_inf();
#pragma unroll
    for (int j = 0; j < V; ++j)
      if (key(j) == kv) {
        const double v = val(j);
        if (v > cur) nxt = fmin(nxt, v);
      }
    cur = wave_min(nxt);
    if (!(cur < __builtin_inf())) { second = __builtin_inf(); return; }
    int ceq = 0;
#pragma unroll
    for (int j = 0; j < V; ++j)
      if (key(j) == kv) ceq += (val(j) == cur);
    ceq = wave_sum(ceq);
    if (have_first) { second = cur; return; }
    if (rank < ceq) {
      first = cur;
      if (rank + 1 < ceq) { second = cur; return; }
      have_first = true;
    } else {
      rank -= ceq;
    }
  }
}

// Smallest key strictly above kv (+inf if none).
template <int V, class Key>
__device__ __forceinline__ float next_key(const Key& key, float kv, int n_t) {
  const int l = lane_id();
  float m = __builtin_inff();
#pragma unroll
  for (int j = 0; j < V; ++j)
    if (key(j) > kv) m = fminf(m, key(j));
  return wave_min_f(m);
}

// FP64 median of val(j) given FP32 keys with key(j) = RN32(val(j)) (rounding
// is monotone); when kExact, the keys are the values themselves.
template <bool kExact, int V, class Key, class Val>
__device__ __forceinline__ double median_via_keys(const Key& key, const Val& val, const SeriesCtx& cx) {
  const int n = cx.n_t;
  const int k1 = (n - 1) / 2;
  const Sel s = select_kth_f32<V>(key, k1, cx);
  double a, b;
  if (kExact) {
    a = (double)s.key;
    if (n & 1) return a;
    // the next order statistic: a again if another sample shares the key, else the next key
    const int l = lane_id();
    int ceq = 0;
#pragma unroll
    for (int j = 0; j < V; ++j) ceq += key(j) == s.key;
    ceq = wave_sum(ceq);
    b = (s.rank_in_ties + 1 < ceq) ? a : (double)next_key<V>(key, s.key, n);
  } else {
    resolve_ties<V>(key, s.key, s.rank_in_ties, val, cx, a, b);
    if (n & 1) return a;
    if (!(b < __builtin_inf())) {
      const float k2 = next_key<V>(key, s.key, n);
      double dummy;
      resolve_ties<V>(key, k2, 0, val, cx, b, dummy);
    }
  }
  return (a + b) * 0.5;
}

// A z sample written with the non-temporal hint: the z cube is streamed out
// once (the search reads it back much later), so its lines should not displace
// the raw cube's, which neighbouring tiles still read.
template <typename ST> __device__ __forceinline__ void store_z(ST* p, float zf) {
  const ST v = from_f32<ST>(zf);
  if constexpr (sizeof(ST) == 4)
    __builtin_nontemporal_store(__builtin_bit_cast(uint32_t, v), (uint32_t*)p);
  else
    __builtin_nontemporal_store(__builtin_bit_cast(uint16_t, v), (uint16_t*)p);
}

__device__ __forceinline__ double div_markstein(double a, double b, double r) {
  const double q0 = a * r;
  const double e = __builtin_fma(-q0, b, a);
  return __builtin_fma(e, r, q0);
}

// Statistics + normalisation of one series held in LDS (sample t at xs[t];
// NaN from n_t up to 64 V), read as x(j) <-> t = 64 j + lane.
// xmin, xmax: this lane's partial extremes of the series (NaN padding is
// ignored by fminf/fmaxf), any_bad: whether the series holds a non-finite
// sample; both come from the load, which sees every sample once.
template <int V, typename ST>
__device__ __forceinline__ void process_series(const float* xs, int p, int s, int n_t, int n_sub, int mode,
                                               const double* __restrict__ med_in, const double* __restrict__ sig_in,
                                               double* __restrict__ med_out, double* __restrict__ sig_out,
                                               ST* __restrict__ z, unsigned long long* __restrict__ flag_count,
                                               const SeriesCtx& cx, float xmin, float xmax, bool any_bad) {
  const int l = lane_id();
  const LdsSeries x{xs, l};

  long long nflag = 0;
  double med = 0.0, sig = 1.0;
  bool usable = true;
  if (mode == NORM_PIXEL_SUBBAND) {
    if (any_bad) {
      med = __builtin_nan(""); sig = __builtin_nan(""); usable = false;
    } else {
      xmin = wave_min_f(xmin);
      xmax = wave_max_f(xmax);
      const int k1 = (n_t - 1) / 2;
      const bool even = (n_t & 1) == 0;
      double a = 0.0, b = 0.0;
      auto vx = [&](int j) { return (double)x(j); };
      const bool full = n_t == 64 * V;              // no NaN padding
      const int rounds = select_values<V>(x, vx, k1, even, xmin, xmax, full, cx, a, b);
      if (rounds)
        med = even ? (a + b) * 0.5 : a;
      else
        med = median_via_keys<true, V>(x, vx, cx);
      // separate copies of the median for each use, so the compiler recomputes the
      // FP64 differences instead of keeping all of them live
      double mk = med, mv = med;
      asm volatile("" : "+v"(mk));
      asm volatile("" : "+v"(mv));
      auto vd = [&](int j) { return fabs((double)x(j) - mv); };
      // distance keys lie in [0, RN32(largest distance)], the largest distance
      // being that of the series' minimum or maximum (the map is monotone on
      // each side of the median)
      const float dhi = fmaxf((float)fabs((double)xmax - med), (float)fabs((double)xmin - med));
      double mad;
      if (rounds == 1 && mad_from_bracket<V>(x, mv, k1, even, xmin, 256.0f / (xmax - xmin), dhi, cx, mad)) {
      } else if (select_values<V>(DistKeys{x, mk}, vd, k1, even, 0.0f, dhi, full, cx, a, b)) {
        mad = even ? (a + b) * 0.5 : a;
      } else {
        mad = median_via_keys<false, V>(DistKeys{x, mk}, vd, cx);
      }
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
  const double r = 1.0 / sig;
  const bool fast_div = sig > 0x1p-900 && sig < 0x1p900;
  asm volatile("" : "+v"(med));
  ST* zrow = z + ((size_t)p * n_sub + s) * n_t;
  int nbad_samples = 0;
  if (mode == NORM_PIXEL_SUBBAND && usable && fast_div && n_t == 64 * V) {
    // the usual case, with no per-sample branch: every register holds a
    // sample, every sample is finite (a non-finite one makes the series
    // unusable) and the quotient is Markstein's
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const double a = (double)x(j) - med;
      float zf = (float)div_markstein(a, sig, r);
      // z is rounded to FP32 first and then to the store type; without the
      // barrier the compiler merges the two roundings into one from FP64
      asm("" : "+v"(zf));
      store_z<ST>(zrow + 64 * j + l, zf);
      if ((j & 3) == 3) __builtin_amdgcn_sched_barrier(0);   // bound the live FP64 temporaries
    }
  } else if (mode == NORM_PIXEL_SUBBAND && usable && fast_div) {
    // the same with registers left over: four quotients are formed before
    // their stores, which only lanes holding a sample make
#pragma unroll
    for (int j0 = 0; j0 < V; j0 += 4) {
      float zf[4];
#pragma unroll
      for (int b = 0; b < 4 && j0 + b < V; ++b) {
        zf[b] = (float)div_markstein((double)x(j0 + b) - med, sig, r);
        asm("" : "+v"(zf[b]));
      }
#pragma unroll
      for (int b = 0; b < 4 && j0 + b < V; ++b)
        if (64 * (j0 + b) + l < n_t) store_z<ST>(zrow + 64 * (j0 + b) + l, zf[b]);
      __builtin_amdgcn_sched_barrier(0);
    }
  } else {
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const int t = 64 * j + l;
      if (t < n_t) {
        float zf;
        const float xj = x(j);
        const bool fin = __builtin_isfinite(xj);
        if (mode == NORM_NONE) {
          zf = fin ? xj : 0.0f;
          nbad_samples += !fin;
        } else if (!usable) {
          zf = 0.0f;
        } else if (mode == NORM_EXTERNAL && !fin) {
          zf = 0.0f;
          nbad_samples += 1;
        } else {
          const double a = (double)xj - med;
          zf = (float)(fast_div ? div_markstein(a, sig, r) : a / sig);
        }
        store_z<ST>(zrow + t, zf);
      }
      if ((j & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
  }
  if (mode == NORM_NONE || mode == NORM_EXTERNAL) nflag += wave_sum(nbad_samples);
  if (l == 0 && nflag) atomicAdd(flag_count, (unsigned long long)nflag);
}

template <int V, typename InT, typename ST>
__global__ __launch_bounds__(StatShape<V>::kWaves * kWave)
__attribute__((amdgpu_waves_per_eu(StatShape<V>::kMinWavesPerEU))) void k_stats_norm(
    const InT* __restrict__ x, int n_t, int n_sub, int n_pix, int mode,
    const double* __restrict__ med_in, const double* __restrict__ sig_in,
    double* __restrict__ med_out, double* __restrict__ sig_out,
    ST* __restrict__ z, unsigned long long* __restrict__ flag_count, int t_start) {
  constexpr int kStatWaves = StatShape<V>::kWaves;
  constexpr int kStatTilePix = kStatWaves;        // one pixel (series) per wave
  // each wave's series lives in LDS, sample t at row[t]; rows are padded so that
  // the load's stores (kStatTilePix pixels x 64/kStatTilePix times per wave
  // instruction) fall in distinct banks, and a wave's reads of 64 consecutive
  // samples are conflict-free anyway
  constexpr int RS = 64 * V + 64 / kStatTilePix;
  __shared__ float series[kStatWaves * RS];
  __shared__ uint32_t hist_all[kStatWaves][256];
  __shared__ double list_all[kStatWaves][64];

  // Workgroups are dealt to the 8 XCDs round-robin; remap so that each XCD
  // takes a contiguous run of (pixel tile, sub-band) items: neighbouring
  // tiles share 128-byte lines of the [t][s][p] rows, which then stay in one
  // L2 instead of being fetched once per XCD.
  const unsigned n_items = gridDim.x * gridDim.y;
  unsigned item = blockIdx.x + blockIdx.y * gridDim.x;
  if ((n_items & 7u) == 0) item = (item & 7u) * (n_items >> 3) + (item >> 3);
  const int s = (int)(item / gridDim.x);
  const int p0 = (int)(item % gridDim.x) * kStatTilePix;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const size_t plane = (size_t)n_sub * n_pix;

  // ---- load: rows of kStatTilePix pixels; every global load of the thread is
  // issued first (one memory latency), then stored into the pixels' LDS rows.
  // Thread i reads pixel p0 + i % kStatTilePix of time rows i / kStatTilePix +
  // q * kRowStep; rows beyond n_t and pixels beyond n_pix load a valid address
  // and become NaN.
  constexpr int kRowStep = kStatWaves * kWave / kStatTilePix;       // = 64
  constexpr int kPer = 64 * V / kRowStep;                           // loads per thread
  const int c_ld = threadIdx.x % kStatTilePix;
  const bool pix_ok = p0 + c_ld < n_pix;
  const int r0 = threadIdx.x / kStatTilePix;
  float stage[kPer];
  // the thread's samples all belong to series c_ld: its partial extremes and
  // non-finite flag go to that series' (not yet used) histogram slots, where
  // the series' wave combines the kRowStep partials (saves a pass over the row)
  float tmin = __builtin_inff(), tmax = -__builtin_inff();
  bool tbad = false;
  if (t_start == 0 && n_t == 64 * V && (size_t)kRowStep * plane * sizeof(InT) < 0x80000000u) {
    // Plain cube filling every register: the time rows of chunk q start at a
    // workgroup-uniform address, and each thread adds the same 32-bit offset
    // (its pixel and its row within the chunk) to every one of them. Threads
    // of pixels past n_pix read pixel p0 instead (their rows belong to no
    // processed series). fma(v, 0, acc) stays 0 unless some v is infinite or
    // NaN.
    const char* tile = (const char*)(x + (size_t)s * n_pix + p0);
    const uint32_t voff = (uint32_t)(((pix_ok ? c_ld : 0) + (size_t)r0 * plane) * sizeof(InT));
    // The row address is held in scalar registers and stepped by one add per
    // chunk, so each load adds voff to it (left to itself the compiler folds
    // the row step into a 64-bit vector multiply-add per load).
    gptr row = (gptr)tile;
    const size_t step = (size_t)kRowStep * plane * sizeof(InT);
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      stage[q] = load_global_f32<InT>(row + voff);
      row += step;
      asm("" : "+s"(row));
    }
    float nf = 0.0f;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      nf = __builtin_fmaf(stage[q], 0.0f, nf);
      tmin = fminf(tmin, stage[q]);
      tmax = fmaxf(tmax, stage[q]);
    }
    tbad = nf != 0.0f;
  } else if (t_start == 0 && (size_t)kRowStep * plane * sizeof(InT) < 0x80000000u) {
    // Plain cube of a length that leaves registers over: the same loads, and
    // a thread whose row of a chunk lies past n_t reads the chunk's first row
    // (or, for a chunk wholly past n_t, the cube's) and keeps NaN instead.
    // Every value loaded is one of the series' own samples, so the
    // non-finite check can take them all.
    const char* tile = (const char*)(x + (size_t)s * n_pix + p0);
    const uint32_t coff = (uint32_t)((pix_ok ? c_ld : 0) * sizeof(InT));
    const uint32_t voff = coff + (uint32_t)((size_t)r0 * plane * sizeof(InT));
    gptr row = (gptr)tile;
    const size_t step = (size_t)kRowStep * plane * sizeof(InT);
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      gptr rq = q * kRowStep < n_t ? row : (gptr)tile;
      asm("" : "+s"(rq));
      stage[q] = load_global_f32<InT>(rq + (q * kRowStep + r0 < n_t ? voff : coff));
      row += step;
      asm("" : "+s"(row));
    }
    float nf = 0.0f;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      nf = __builtin_fmaf(stage[q], 0.0f, nf);
      stage[q] = q * kRowStep + r0 < n_t ? stage[q] : __builtin_nanf("");
      tmin = fminf(tmin, stage[q]);
      tmax = fmaxf(tmax, stage[q]);
    }
    tbad = nf != 0.0f;
  } else {
    // Ring of the last n_t samples (read oldest first), or a plane too large
    // for 32-bit offsets. Rows beyond n_t and pixels beyond n_pix load a valid
    // address and become NaN.
    const InT* src = x + (size_t)s * n_pix + (pix_ok ? p0 + c_ld : 0);
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int t = q * kRowStep + r0;
      const bool ok = pix_ok && t < n_t;
      int tr = t + t_start;                        // ring order: oldest sample first
      tr -= tr >= n_t ? n_t : 0;
      stage[q] = to_f32(src[(size_t)(ok ? tr : 0) * plane]);
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int t = q * kRowStep + r0;
      stage[q] = pix_ok && t < n_t ? stage[q] : __builtin_nanf("");
      tbad |= (t < n_t) && !__builtin_isfinite(stage[q]);
      tmin = fminf(tmin, stage[q]);
      tmax = fmaxf(tmax, stage[q]);
    }
  }
  float* my_row = series + c_ld * RS + r0;
#pragma unroll
  for (int q = 0; q < kPer; ++q) my_row[q * kRowStep] = stage[q];
  uint32_t* part = hist_all[c_ld];
  part[r0] = __float_as_uint(tmin);
  part[kRowStep + r0] = __float_as_uint(tmax);
  part[2 * kRowStep + r0] = tbad ? 1u : 0u;
  __syncthreads();
  SeriesCtx cx{hist_all[w], list_all[w], n_t};
  const int l = lane_id();
  const float pmin = __uint_as_float(cx.hist[l]), pmax = __uint_as_float(cx.hist[kRowStep + l]);
  const bool any_bad = ballot(cx.hist[2 * kRowStep + l] != 0u) != 0;
  wave_lds_sync();                                 // the histogram slots are reused from here on
  if (p0 + w < n_pix)
    process_series<V, ST>(series + w * RS, p0 + w, s, n_t, n_sub, mode, med_in, sig_in, med_out, sig_out, z,
                          flag_count, cx, pmin, pmax, any_bad);
}

// ------------------------------------------------------------ launcher
template <int V, typename InT, typename ST>
static hipError_t launch_stats_v(const StatsLaunch& a, hipStream_t st) {
  constexpr int W = StatShape<V>::kWaves;
  dim3 grid((a.n_pix + W - 1) / W, a.n_sub);
  hipLaunchKernelGGL((k_stats_norm<V, InT, ST>), grid, dim3(W * kWave), 0, st,
                     (const InT*)a.x, a.n_t, a.n_sub, a.n_pix, a.mode, a.med_in, a.sig_in,
                     a.med_out, a.sig_out, (ST*)a.z, a.flag_count, a.t_start);
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
