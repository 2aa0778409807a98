// PSF-based reduction of an image's top candidates to the most likely one
// (paper section 2.3): the simulated PSF, thresholded at a percentile, is a
// binary mask centred on each candidate in turn; the other candidates inside
// it are that candidate's possible sidelobes; the candidate whose weighted-mean
// S/N over itself and those sidelobes is largest is kept. Weights are the PSF's
// amplitude at each member's offset, the PSF normalised to its centre; the
// weighted mean of unit-noise S/N values, divided by its own noise, is
// sum(w S) / sqrt(sum(w^2)), which a point source maximises on its own pixel.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/nsfrb.h"
#include "host_util.h"

using namespace nsfrb;

extern "C" nsfrb_status nsfrb_psf_reduce(const nsfrb_candidate* cands, int32_t n, const float* psf, int32_t psf_nx,
                                         int32_t psf_ny, double percentile, int32_t* best_index,
                                         double* best_score) {
  host_clear_error();
  if (!cands || !psf || !best_index || !best_score) return host_fail(NSFRB_ERR_INVALID_ARG, "NULL argument");
  if (n < 1) return host_fail(NSFRB_ERR_INVALID_ARG, "need at least one candidate");
  if (psf_nx < 1 || psf_ny < 1 || !(psf_nx & 1) || !(psf_ny & 1))
    return host_fail(NSFRB_ERR_INVALID_ARG, "the PSF image needs odd sides (its centre is the middle pixel)");
  if (!(percentile >= 0.0 && percentile <= 100.0)) return host_fail(NSFRB_ERR_INVALID_ARG, "percentile must be 0..100");
  const int hx = psf_nx / 2, hy = psf_ny / 2;
  const size_t np = (size_t)psf_nx * psf_ny;
  std::vector<double> v(np);
  for (size_t i = 0; i < np; ++i) {
    v[i] = psf[i];
    if (!std::isfinite(v[i])) return host_fail(NSFRB_ERR_INVALID_ARG, "PSF values must be finite");
  }
  const double centre = psf[(size_t)hy * psf_nx + hx];
  if (!(centre > 0.0)) return host_fail(NSFRB_ERR_INVALID_ARG, "the PSF centre must be positive");
  // percentile with linear interpolation between order statistics; the
  // interpolation is taken from the nearer end (exact at both ends, monotone)
  std::sort(v.begin(), v.end());
  const double pos = (percentile / 100.0) * (double)(np - 1);
  const size_t lo = std::min((size_t)std::floor(pos), np - 1), hi = std::min(lo + 1, np - 1);
  const double t = pos - (double)lo, a = v[lo], b = v[hi];
  const double q = t >= 0.5 ? b - (b - a) * (1.0 - t) : a + (b - a) * t;
  int best = -1;
  double best_s = -INFINITY;
  for (int i = 0; i < n; ++i) {
    double num = cands[i].snr, w2 = 1.0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      const int dx = cands[j].x - cands[i].x, dy = cands[j].y - cands[i].y;
      if (dx < -hx || dx > hx || dy < -hy || dy > hy) continue;
      const double pv = psf[(size_t)(hy + dy) * psf_nx + (hx + dx)];
      if (pv >= q) {
        const double w = pv / centre;
        num += w * (double)cands[j].snr;
        w2 += w * w;
      }
    }
    const double s = num / std::sqrt(w2);
    if (s > best_s) {
      best = i;
      best_s = s;
    }
  }
  *best_index = best;
  *best_score = best_s;
  return NSFRB_OK;
}
