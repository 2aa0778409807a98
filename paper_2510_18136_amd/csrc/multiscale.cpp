// Search at several sampling timescales (paper section 2.2): the raw cube is
// binned in time by each factor and every binned cube is searched with the
// sampling time scaled by that factor. The handle composes one search plan per
// timescale through the public entry points and owns the binned buffers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/nsfrb.h"
#include "host_util.h"
#include "nsfrb_internal.h"

using namespace nsfrb;

namespace {
constexpr int kMaxScales = 8;
}

struct nsfrb_multiscale {
  nsfrb_search_config base{};
  std::vector<int32_t> factor;
  std::vector<nsfrb_search*> search;
  std::vector<float*> binned;     // FP32 [n_time / factor][n_sub][n_pix] per scale; nullptr for factor 1
  int32_t n_pix = 0;
};

namespace {

void ms_release(nsfrb_multiscale* h) {
  if (!h) return;
  hipSetDevice(h->base.device);
  for (nsfrb_search* s : h->search) nsfrb_search_destroy(s);
  for (float* b : h->binned)
    if (b) hipFree(b);
  delete h;
}

}  // namespace

extern "C" nsfrb_status nsfrb_bin_time(const void* d_x, int32_t in_dtype, int32_t n_time, int32_t n_sub,
                                       int32_t n_pix, int32_t factor, float* d_out, void* stream) {
  host_clear_error();
  if (!d_x || !d_out) return host_fail(NSFRB_ERR_INVALID_ARG, "NULL cube pointer");
  if (in_dtype < 0 || in_dtype > 2) return host_fail(NSFRB_ERR_INVALID_ARG, "in_dtype must be F32, F16 or BF16");
  if (n_time < 1 || n_sub < 1 || n_pix < 1) return host_fail(NSFRB_ERR_INVALID_ARG, "dimensions must be >= 1");
  if (factor < 1 || n_time / factor < 1)
    return host_fail(NSFRB_ERR_INVALID_ARG, "factor must be 1..n_time (at least one whole bin)");
  NSFRB_HIP_TRY(launch_bin_time(d_x, in_dtype, n_time, n_sub, n_pix, factor, d_out, (hipStream_t)stream));
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_multiscale_create(const nsfrb_search_config* cfg, int32_t n_scales,
                                                const int32_t* factor, const double* dm_scale,
                                                nsfrb_multiscale** out) {
  host_clear_error();
  if (!cfg || !factor || !dm_scale || !out) return host_fail(NSFRB_ERR_INVALID_ARG, "NULL argument");
  *out = nullptr;
  if (n_scales < 1 || n_scales > kMaxScales)
    return host_fail(NSFRB_ERR_INVALID_ARG, "n_scales must be 1.." + std::to_string(kMaxScales));
  nsfrb_status st = nsfrb_config_validate(cfg);
  if (st != NSFRB_OK) return st;
  if (cfg->layout != NSFRB_LAYOUT_TSP)
    return host_fail(NSFRB_ERR_UNSUPPORTED, "the multi-timescale search bins a raw [time][sub-band][pixel] cube");
  for (int s = 0; s < n_scales; ++s) {
    if (factor[s] < 1 || cfg->n_time / factor[s] < 1)
      return host_fail(NSFRB_ERR_INVALID_ARG, "factor " + std::to_string(s) + " must be 1..n_time");
    if (!(dm_scale[s] >= 0.0) || !std::isfinite(dm_scale[s]))
      return host_fail(NSFRB_ERR_INVALID_ARG, "dm_scale " + std::to_string(s) + " must be finite and >= 0");
  }
  nsfrb_multiscale* h = new nsfrb_multiscale;
  h->base = *cfg;
  h->n_pix = cfg->nx * cfg->ny;
  hipError_t e = hipSetDevice(cfg->device);
  if (e != hipSuccess) {
    ms_release(h);
    return host_fail(NSFRB_ERR_DEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
  }
  for (int s = 0; s < n_scales; ++s) {
    nsfrb_search_config c = *cfg;
    const int f = factor[s];
    c.n_time = cfg->n_time / f;
    c.dt_ms = cfg->dt_ms * f;
    std::vector<double> dms;
    if (dm_scale[s] == 0.0) {
      dms.assign(1, 0.0);
    } else {
      for (int d = 0; d < cfg->n_dm; ++d) dms.push_back(cfg->dm[d] * dm_scale[s]);
    }
    c.n_dm = (int32_t)dms.size();
    c.dm = dms.data();
    if (f > 1) c.in_dtype = NSFRB_F32;
    nsfrb_search* sh = nullptr;
    st = nsfrb_search_create(&c, &sh);     // copies the host arrays
    if (st != NSFRB_OK) {
      const std::string why = nsfrb_last_error();
      ms_release(h);
      return host_fail(st, "timescale " + std::to_string(s) + " (factor " + std::to_string(f) + "): " + why);
    }
    h->factor.push_back(f);
    h->search.push_back(sh);
    float* buf = nullptr;
    if (f > 1) {
      e = hipMalloc((void**)&buf, sizeof(float) * (size_t)c.n_time * cfg->n_sub * h->n_pix);
      if (e != hipSuccess) {
        ms_release(h);
        return host_fail(e == hipErrorOutOfMemory ? NSFRB_ERR_OUT_OF_MEMORY : NSFRB_ERR_DEVICE,
                         std::string("hipMalloc (binned cube): ") + hipGetErrorString(e));
      }
    }
    h->binned.push_back(buf);
  }
  *out = h;
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_multiscale_destroy(nsfrb_multiscale* h) {
  host_clear_error();
  if (h) {
    hipSetDevice(h->base.device);
    hipDeviceSynchronize();
  }
  ms_release(h);
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_multiscale_run(nsfrb_multiscale* h, const void* d_cube, void* stream) {
  host_clear_error();
  if (!h || !d_cube) return host_fail(NSFRB_ERR_INVALID_ARG, "NULL argument");
  NSFRB_HIP_TRY(hipSetDevice(h->base.device));
  // Bin first: two timescales whose factors nest (5 and 75) are binned from one
  // read of the raw cube; any other binned timescale on its own.
  const size_t n = h->search.size();
  std::vector<bool> binned(n, false);
  for (size_t s = 0; s < n; ++s) {
    if (h->factor[s] <= 1 || binned[s]) continue;
    size_t pair = n;
    for (size_t q = s + 1; q < n && pair == n; ++q) {
      const int32_t lo = std::min(h->factor[s], h->factor[q]), hi = std::max(h->factor[s], h->factor[q]);
      if (!binned[q] && lo > 1 && hi > lo && hi % lo == 0) pair = q;
    }
    if (pair == n) {
      NSFRB_HIP_TRY(launch_bin_time(d_cube, h->base.in_dtype, h->base.n_time, h->base.n_sub, h->n_pix, h->factor[s],
                                    h->binned[s], (hipStream_t)stream));
    } else {
      const size_t a = h->factor[s] < h->factor[pair] ? s : pair, b = a == s ? pair : s;
      NSFRB_HIP_TRY(launch_bin_time_pair(d_cube, h->base.in_dtype, h->base.n_time, h->base.n_sub, h->n_pix,
                                         h->factor[a], h->binned[a], h->factor[b], h->binned[b],
                                         (hipStream_t)stream));
      binned[pair] = true;
    }
    binned[s] = true;
  }
  for (size_t s = 0; s < n; ++s) {
    nsfrb_status st = nsfrb_search_run(h->search[s], h->factor[s] > 1 ? h->binned[s] : d_cube, stream);
    if (st != NSFRB_OK) return st;
  }
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_multiscale_scale(nsfrb_multiscale* h, int32_t scale, nsfrb_search** out) {
  host_clear_error();
  if (!h || !out) return host_fail(NSFRB_ERR_INVALID_ARG, "NULL argument");
  if (scale < 0 || scale >= (int32_t)h->search.size()) return host_fail(NSFRB_ERR_INVALID_ARG, "scale out of range");
  *out = h->search[scale];
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_multiscale_candidates_get(nsfrb_multiscale* h, nsfrb_scale_candidate* host_out,
                                                        int32_t capacity, int32_t* n_written, int32_t* n_total) {
  host_clear_error();
  if (!h || (!host_out && capacity > 0) || capacity < 0)
    return host_fail(NSFRB_ERR_INVALID_ARG, "bad output buffer");
  const int K = h->base.max_candidates;
  std::vector<nsfrb_scale_candidate> all;
  int64_t total = 0;
  std::vector<nsfrb_candidate> tmp(K);
  for (size_t s = 0; s < h->search.size(); ++s) {
    int32_t w = 0, t = 0;
    nsfrb_status st = nsfrb_candidates_get(h->search[s], tmp.data(), K, &w, &t);
    if (st != NSFRB_OK) return st;
    total += t;
    for (int i = 0; i < w; ++i) all.push_back(nsfrb_scale_candidate{tmp[i], (int32_t)s});
  }
  const int nx = h->base.nx;
  std::stable_sort(all.begin(), all.end(), [nx](const nsfrb_scale_candidate& a, const nsfrb_scale_candidate& b) {
    if (a.cand.snr != b.cand.snr) return a.cand.snr > b.cand.snr;
    if (a.scale != b.scale) return a.scale < b.scale;
    return a.cand.y * nx + a.cand.x < b.cand.y * nx + b.cand.x;
  });
  const int keep = (int)std::min<size_t>(all.size(), (size_t)K);
  const int wr = std::min(keep, capacity);
  std::copy(all.begin(), all.begin() + wr, host_out);
  if (n_written) *n_written = wr;
  if (n_total) *n_total = (int32_t)std::min<int64_t>(total, INT32_MAX);
  if (wr < keep) return host_fail(NSFRB_ERR_TRUNCATED, "capacity below the merged candidate count");
  return NSFRB_OK;
}
