// Internal declarations shared by the host library and the AOT kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nsfrb {

enum { DT_F32 = 0, DT_F16 = 1, DT_BF16 = 2 };
enum { NORM_PIXEL_SUBBAND = 0, NORM_EXTERNAL = 2, NORM_NONE = 3 };

struct StatsLaunch {
  const void* x;
  int n_t, n_sub, n_pix, mode, in_dtype, store_dtype;
  const double* med_in;
  const double* sig_in;
  double* med_out;
  double* sig_out;
  void* z;
  unsigned long long* flag_count;
  int t_start = 0;   // time index of the oldest sample when x is a ring of n_t samples (0: plain cube)
};
hipError_t launch_stats(const StatsLaunch& a, hipStream_t st);
hipError_t launch_zero_u64(unsigned long long* p, hipStream_t st);

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

namespace nsfrb {

// Host mirror of the device CubeDesc (same field order and types).
struct CubeDescHost {
  const void* z;
  const int* delays;
  const int* dmax;
  const float* norms;
  float* snr_max;
  int* toa;
  float* best_s;
  int* best_d;
  int* best_w;
  int* best_t;
  int n_pix, n_sub, n_t, n_dm, rs;
  int dma_w;          // batch row copy: global-to-LDS bytes per lane (16 or 4), else ordinary loads
  long long item_begin;
};
static_assert(sizeof(CubeDescHost) == 112, "CubeDesc layout");

}  // namespace nsfrb

namespace nsfrb {
hipError_t launch_philox_fill(uint32_t* out, long long n_blocks, unsigned long long seed, hipStream_t st);
hipError_t launch_noise(void* out, int dtype, long long n, unsigned long long seed, float sigma, hipStream_t st);
hipError_t launch_inject(void* cube, int dtype, int layout, int n_pix, int n_sub, int n_t, int pixel, int t0,
                         int width, float amp, const int* d_offsets, hipStream_t st);
}  // namespace nsfrb

namespace nsfrb {
// One boxcar injection (layout of nsfrb_boxcar in the C ABI).
struct BoxcarRec {
  int cube, pixel, t0, width;
  float amp;
};
// out[t'][s][p] = RN32(FP64 sum of x[t' factor + k][s][p], k = 0..factor-1 in order), t' < n_t / factor
hipError_t launch_bin_time(const void* x, int in_dtype, int n_t, int n_sub, int n_pix, int factor, float* out,
                           hipStream_t st);
// Both binnings of launch_bin_time for factors fa and fb (fa >= 2, fb a larger multiple of fa) from one read
// of x; outputs equal two launch_bin_time calls. hipErrorInvalidValue if the factors do not nest.
hipError_t launch_bin_time_pair(const void* x, int in_dtype, int n_t, int n_sub, int n_pix, int fa, float* out_a,
                                int fb, float* out_b, hipStream_t st);
hipError_t launch_inject_many(void* const* cubes, int dtype, int layout, int n_pix, int n_sub, int n_t,
                              const BoxcarRec* recs, const int* offsets, int n, hipStream_t st);
hipError_t launch_inject_rfi(void* cube, int dtype, int layout, int n_pix, int n_sub, int n_t, int kind, int t0, int len,
                             int s0, float amp, hipStream_t st);
// classifier kernels (k_cnn.hip)
hipError_t launch_conv_fwd(int cin, const uint16_t* in, const uint16_t* w, const float* bias, uint16_t* out, int N,
                           int T, int Y, hipStream_t st);
hipError_t launch_conv_bwd_data(const uint16_t* dpre, const uint16_t* wb, const uint16_t* mask_act, uint16_t* out, int N,
                                int T, int Y, hipStream_t st);
int wgrad_items(int N, int Y);   // partial-sum items of the weight-gradient kernel
hipError_t launch_conv_wgrad(int cin, const uint16_t* x, const uint16_t* dpre, float* part, float* part_db, float* dw,
                             float* db, int N, int T, int Y, hipStream_t st);
int pool_chunks(int npos);   // partial keys per sample written by launch_pool (part holds N * this * 32)
hipError_t launch_pool(const uint16_t* act, int N, int npos, int centre, uint32_t* part, float* h, int* arg,
                       hipStream_t st);
// hs: per-sample scratch of 66 floats (training only)
hipError_t launch_head(const float* h, const float* labels, int n, const float* th, float* hs, float* gh, float* dh,
                       float* logits, float* prob, float* loss, int backward, hipStream_t st);
hipError_t launch_pool_backward(const float* dh, const int* arg, const uint16_t* act, int N, int npos, int centre,
                                uint16_t* dpre, hipStream_t st);
hipError_t launch_adam(float* th, float* m, float* v, const float* g, int n, float lr, float b1, float b2, float eps,
                       float bc1, float bc2, hipStream_t st);
hipError_t launch_prep_weights(const float* wsrc, int cin, uint16_t* wf, uint16_t* wb, hipStream_t st);
hipError_t launch_cutouts(int store_dtype, const void* const* cubes, const void* desc, const int* delays, int n_cut,
                          int nx, int ny, int n_sub, int n_t, int ct, uint16_t* out, hipStream_t st);
}  // namespace nsfrb
