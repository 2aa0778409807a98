// Internal declarations shared by the host library and the AOT kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nsfrb {

enum { DT_F32 = 0, DT_F16 = 1, DT_BF16 = 2 };
enum { NORM_PIXEL_SUBBAND = 0, NORM_PIXEL = 1, NORM_EXTERNAL = 2, NORM_NONE = 3 };

struct StatsLaunch {
  const void* x;
  int n_t, n_sub, n_pix, mode, in_dtype, store_dtype;
  const double* med_in;
  const double* sig_in;
  double* med_out;
  double* sig_out;
  void* z;
  unsigned long long* flag_count;
};
hipError_t launch_stats(const StatsLaunch& a, hipStream_t st);

struct CandLaunch {
  const float* best_snr;
  const int* best_d;
  const int* best_w;
  const int* best_t;
  int n_pix, nx, k_max;
  float theta;
  unsigned long long* keys;   // [n_pix] scratch
  int* count;                 // [1] number of pixels >= theta
  void* out;                  // [k_max] nsfrb_candidate records
  int* n_out;                 // [2]: records written, total
};
hipError_t launch_candidates(const CandLaunch& a, hipStream_t st);

}  // namespace nsfrb
