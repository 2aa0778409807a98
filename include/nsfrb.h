/*
 * nsfrb.h -- C ABI of the MI355X (gfx950) image-plane single-pulse search.
 *
 * The library implements the search of section 2.2 of arXiv:2510.18136 (the
 * `cerberus` pipeline of the DSA-110 NSFRB system) on one GPU:
 *   1. robust noise statistics per (pixel, sub-band): FP64 median and MAD,
 *      sigma = 1.482602218505602 * MAD                    (section 2.2; 3.2)
 *   2. normalise z = (x - median) / sigma in FP64, round to FP32 and then to
 *      the store dtype, written in the search layout    (section 2.2)
 *   3. incoherent de-dispersion with a precomputed integer shift table,
 *      delta[d][s] = rint(k_dm * DM_d * (f_s^-2 - f_ref^-2) / dt)
 *                                                       (section 2.2, t_BW law)
 *   4. boxcar sums over a list of widths, S/N = sum / sqrt(n_sub * w)
 *   5. maximum S/N over time and its time of arrival for every
 *      (DM, width, pixel)                               (sections 2.2, 2.3)
 *   6. per-pixel best trial, threshold S/N >= theta, candidates sorted by
 *      S/N (descending) then pixel index, first K kept  (sections 2.3, 3.1)
 *
 * Conventions for every entry point:
 *   - Every call returns nsfrb_status; no C++ exception crosses the ABI.
 *     nsfrb_last_error() returns a thread-local message for the last failure.
 *   - Host pointers are read (or written) during the call only; the library
 *     copies what it keeps. Device pointers stay owned by the caller.
 *   - `stream` is a hipStream_t passed as void*; NULL means the default stream.
 *   - A handle is not thread-safe; distinct handles are independent.
 *
 * Cube layout: element (t, s, p) of a raw cube is at index
 *   (t * n_sub + s) * (nx * ny) + p,  with pixel p = y * nx + x,
 * i.e. [n_time][n_sub][ny*nx], time slowest, pixel fastest.
 */
#ifndef NSFRB_H
#define NSFRB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NSFRB_OK = 0,
  NSFRB_ERR_INVALID_ARG = 1,   /* a value violates the documented domain        */
  NSFRB_ERR_UNSUPPORTED = 2,   /* valid, but beyond what the library implements */
  NSFRB_ERR_OUT_OF_MEMORY = 3, /* a device or pinned-host allocation failed     */
  NSFRB_ERR_DEVICE = 4,        /* a HIP runtime or kernel error                  */
  NSFRB_ERR_NOT_READY = 5,     /* results requested before any run              */
  NSFRB_ERR_TRUNCATED = 6      /* output capacity smaller than the result count */
} nsfrb_status;

typedef enum { NSFRB_F32 = 0, NSFRB_F16 = 1, NSFRB_BF16 = 2 } nsfrb_dtype;

typedef enum {
  NSFRB_LAYOUT_TSP = 0, /* raw cube [n_time][n_sub][ny*nx] (images as they arrive)             */
  NSFRB_LAYOUT_PST = 1  /* already normalised, in the search layout [ny*nx][n_sub][n_time];
                           requires NSFRB_NORM_NONE and in_dtype == store_dtype; searched in place */
} nsfrb_layout;

/* Normalisation (section 2.2: the median of each pixel's series is subtracted
 * and the series is scaled by its noise). The series is a (pixel, sub-band)
 * series; one set of statistics per pixel over all sub-bands is not offered
 * (value 1 is not used and is refused as unknown). */
typedef enum {
  NSFRB_NORM_PIXEL_SUBBAND = 0, /* median/MAD per (pixel, sub-band) over time        */
  NSFRB_NORM_EXTERNAL = 2,      /* caller supplies median and sigma per (p, s)       */
  NSFRB_NORM_NONE = 3           /* z = x (cast to the store dtype)                   */
} nsfrb_norm;

/* Search configuration. Host arrays are copied by nsfrb_search_create. */
typedef struct {
  uint32_t struct_size;    /* = sizeof(nsfrb_search_config), ABI check           */
  int32_t nx, ny;          /* image size in pixels, >= 1                          */
  int32_t n_sub;           /* sub-bands, 1..64                                    */
  int32_t n_time;          /* samples per series, 1..4096                          */
  const double* freq_ghz;  /* [n_sub] sub-band frequencies (GHz), finite, > 0      */
  double f_ref_ghz;        /* reference frequency, >= max(freq_ghz)               */
  double dt_ms;            /* sampling time (ms), > 0                              */
  double k_dm_ms;          /* dispersion constant (ms GHz^2 cm^3/pc); 4.15        */
  int32_t n_dm;            /* DM trials, 1..256                                   */
  const double* dm;        /* [n_dm] DM trials (pc cm^-3), finite, >= 0           */
  int32_t n_width;         /* boxcar widths, 1..32                                */
  const int32_t* width;    /* [n_width] widths in samples, 1..4096                */
  int32_t in_dtype;        /* nsfrb_dtype of the raw cube                         */
  int32_t store_dtype;     /* nsfrb_dtype of the normalised cube                  */
  int32_t norm;            /* nsfrb_norm                                          */
  float snr_threshold;     /* candidates have best S/N >= this (finite)           */
  int32_t max_candidates;  /* K of the top-K list, 1..4096                        */
  int32_t device;          /* HIP device ordinal                                  */
  int32_t layout;          /* nsfrb_layout of the input cube                      */
} nsfrb_search_config;

/* One candidate: the best (DM, width) trial of one pixel. */
typedef struct {
  int32_t x, y;            /* pixel coordinates                                   */
  int32_t dm_index;        /* index into the DM-trial list                        */
  int32_t width_index;     /* index into the width list                           */
  int32_t toa;             /* first sample of the boxcar at f_ref                 */
  float snr;               /* S/N of that trial                                   */
} nsfrb_candidate;

typedef struct nsfrb_search nsfrb_search; /* opaque handle */

/* Library version string (static storage). */
const char* nsfrb_version(void);

/* Message describing the last failure on this thread ("" if none). */
const char* nsfrb_last_error(void);

/* Host-only validation of a configuration (no GPU needed). Returns OK,
 * INVALID_ARG (e.g. f_ref below the highest frequency, which would make
 * delays negative; a width < 1; a non-positive dimension) or UNSUPPORTED. */
nsfrb_status nsfrb_config_validate(const nsfrb_search_config* cfg);

/* Host-only delay table (section 2.2): writes int32 delta[d][s] in samples,
 * computed in FP64 as ((k_dm*DM) * (1/(f*f) - 1/(f_ref*f_ref))) / dt and
 * rounded half to even, into host_out[n_dm * n_sub]. */
nsfrb_status nsfrb_plan_delays(const nsfrb_search_config* cfg, int32_t* host_out);

/* Host-only DM-trial grid from a smearing tolerance (section 2.2: the trials
 * are set by a DM tolerance; the effective width of a pulse is the quadrature
 * sum of its intrinsic width w_int, the sampling time t_s, the smearing inside
 * the lowest channel 0.0083 ms * chan_bw_MHz * DM * nu_min^-3 and the residual
 * band delay 4.15 ms * |DM - trial| * (nu_min^-2 - nu_max^-2)). Rule (the
 * paper names the tolerance but not the rule): trials start at dm_min; the next
 * trial is 2h further, h chosen so that a pulse midway between the two has an
 * effective width exactly tol times its width on a trial; the grid ends with the
 * first trial >= dm_max. Writes min(count, capacity) trials (ascending) to
 * host_out and *n_out = count; TRUNCATED when capacity < count; INVALID_ARG for
 * non-finite values, nu_min <= 0 or >= nu_max, t_s <= 0, w_int or chan_bw < 0,
 * tol <= 1, dm_min < 0 or > dm_max; UNSUPPORTED when the tolerance cannot be
 * met (channel smearing outgrowing the residual delay) or past 2^20 trials. */
nsfrb_status nsfrb_plan_dm_grid(double nu_min_ghz, double nu_max_ghz, double chan_bw_mhz, double t_s_ms,
                                double w_int_ms, double tol, double dm_min, double dm_max, double* host_out,
                                int32_t capacity, int32_t* n_out);

/* Create a search plan on cfg->device: validates, plans the delay table,
 * compiles the search kernel for this plan, allocates the device workspace
 * (normalised cube, statistics, maps, candidates) and uploads the tables. On
 * failure *out is NULL. UNSUPPORTED also when a pixel's rows do not fit in LDS,
 * or when every kernel shape would keep too little of the boxcar chain in
 * registers (more than 64 bytes of spill per lane: n_time too long for the
 * width list, e.g. 4096 samples with 32 widths); such a kernel is never
 * launched. */
nsfrb_status nsfrb_search_create(const nsfrb_search_config* cfg, nsfrb_search** out);

/* Release everything the handle owns. NULL is accepted. */
nsfrb_status nsfrb_search_destroy(nsfrb_search* h);

/* Enqueue one search of the raw device cube d_cube (layout above, in_dtype)
 * on `stream`; returns without waiting. d_cube must stay valid until the
 * stream has passed this run (e.g. until nsfrb_candidates_get returns). */
nsfrb_status nsfrb_search_run(nsfrb_search* h, const void* d_cube, void* stream);

/* Wait for the last run and copy its candidates (sorted by S/N descending,
 * then pixel index) into host_out[capacity]. *n_written = records copied,
 * *n_total = all pixels at or above the threshold. Returns TRUNCATED when
 * capacity < min(n_total, max_candidates), NOT_READY before any run. */
nsfrb_status nsfrb_candidates_get(nsfrb_search* h, nsfrb_candidate* host_out, int32_t capacity,
                                  int32_t* n_written, int32_t* n_total);

/* Introspection (each waits for the last run, then copies to host memory). */
nsfrb_status nsfrb_delay_table_get(const nsfrb_search* h, int32_t* host_out /* [n_dm*n_sub] */);
/* snr_max / toa: [n_dm][n_width][ny*nx]; -inf / -1 where no window fits. Either may be NULL. */
nsfrb_status nsfrb_maps_get(nsfrb_search* h, float* snr_max, int32_t* toa);
/* Per-pixel best trial: S/N, DM index, width index, TOA ([ny*nx] each); any may be NULL. */
nsfrb_status nsfrb_best_get(nsfrb_search* h, float* snr, int32_t* dm_index, int32_t* width_index,
                            int32_t* toa);
/* Noise statistics [ny*nx][n_sub] (FP64). NaN marks a flagged series. */
nsfrb_status nsfrb_noise_stats_get(nsfrb_search* h, double* med, double* sigma);
/* EXTERNAL normalisation: statistics used by subsequent runs, [ny*nx][n_sub]. */
nsfrb_status nsfrb_noise_stats_set(nsfrb_search* h, const double* med, const double* sigma);
/* Normalised cube in the search layout [ny*nx][n_sub][n_time], store dtype
 * (2 or 4 bytes per element). */
nsfrb_status nsfrb_zcube_get(nsfrb_search* h, void* host_out);
/* Device pointer of the normalised cube of the last run (the handle's buffer,
 * or the input itself for LAYOUT_PST), valid until the next run or destroy.
 * Does not wait. NOT_READY before any run. */
nsfrb_status nsfrb_zcube_device(nsfrb_search* h, const void** d_z);
/* Series (or, for NONE/EXTERNAL, samples) flagged as unusable by the last run. */
nsfrb_status nsfrb_flag_count_get(nsfrb_search* h, int64_t* count);

/* Device pointers of the result buffers owned by the handle (valid until
 * destroy): snr_max, toa as above. Any out-pointer may be NULL. */
nsfrb_status nsfrb_maps_device(nsfrb_search* h, float** snr_max, int32_t** toa);

/* Per-stage device time of the last run in milliseconds, measured with HIP
 * events on the run's stream: [0] statistics + normalisation,
 * [1] de-dispersion/boxcar/S/N/max, [2] candidates. Requires
 * nsfrb_profiling_enable(h, 1) before the run. */
nsfrb_status nsfrb_profiling_enable(nsfrb_search* h, int32_t on);
nsfrb_status nsfrb_stage_times_get(nsfrb_search* h, float* ms3);

/* Plan of the search kernel the autotuner chose: info[0] samples per lane,
 * info[1] pixels per workgroup, info[2] LDS row length, info[3] LDS bytes per
 * workgroup, info[4] threads per workgroup, info[5] 1 if the persistent kernel
 * (one pixel per workgroup at a time, next pixel's rows loaded during the
 * search of the current one) was chosen, else 0; for it, info[6] LDS pixel
 * buffers and info[7] workgroups (0 otherwise); info[8] is 0. `info` holds 9
 * values. */
nsfrb_status nsfrb_search_plan_info(const nsfrb_search* h, int32_t* info);

/* ---------------------------------------------------------- multi-timescale
 * The search at several sampling timescales (section 2.2: besides the native
 * sampling, the images are binned by 5 and by 75 samples and searched again;
 * the 5x-binned data are searched at 5x the DM trials, which keeps the shift
 * table of the native search because a delay in samples scales as DM / dt; the
 * 75x-binned data bypass de-dispersion, their DM delays fitting in one sample).
 *
 * Time binning (runs on the current HIP device): out[t'][s][p] =
 * RN32(x[t' f][s][p] + x[t' f + 1][s][p] + ... + x[t' f + f - 1][s][p]), the
 * sum taken in FP64 in that order, for t' < n_time / f (a trailing partial bin
 * is dropped). d_x is a raw [n_time][n_sub][n_pix] cube of in_dtype; d_out is
 * FP32 [n_time / f][n_sub][n_pix]. Asynchronous on `stream`. INVALID_ARG for
 * NULL pointers, dimensions < 1, a dtype outside nsfrb_dtype, or f outside
 * 1..n_time. */
nsfrb_status nsfrb_bin_time(const void* d_x, int32_t in_dtype, int32_t n_time, int32_t n_sub, int32_t n_pix,
                            int32_t factor, float* d_out, void* stream);

typedef struct nsfrb_multiscale nsfrb_multiscale; /* opaque handle */

/* One candidate of a multi-timescale search: the candidate of timescale
 * `scale` (its DM and width indices refer to that timescale's trial lists;
 * its TOA is in that timescale's samples). */
typedef struct {
  nsfrb_candidate cand;
  int32_t scale;
} nsfrb_scale_candidate;

/* Plan n_scales (1..8) searches of one raw TSP cube. Timescale s bins the
 * cube by factor[s] (>= 1; 1 searches the cube itself) and searches
 * n_time / factor[s] samples with dt_ms * factor[s], the DM trials of cfg
 * multiplied by dm_scale[s] (finite, >= 0; 0 means the single trial DM 0,
 * i.e. no de-dispersion), and cfg's widths, statistics, store dtype,
 * threshold and K. Binned cubes are FP32 and owned by the handle. Errors as
 * for nsfrb_search_create (the message names the timescale); UNSUPPORTED
 * unless cfg->layout is NSFRB_LAYOUT_TSP. */
nsfrb_status nsfrb_multiscale_create(const nsfrb_search_config* cfg, int32_t n_scales, const int32_t* factor,
                                     const double* dm_scale, nsfrb_multiscale** out);
/* Release the handle, its searches and binned cubes. NULL is accepted. */
nsfrb_status nsfrb_multiscale_destroy(nsfrb_multiscale* h);
/* Enqueue, for every timescale in order, the binning of d_cube and the search
 * of the result on `stream`; returns without waiting. d_cube must stay valid
 * until the stream has passed the run. */
nsfrb_status nsfrb_multiscale_run(nsfrb_multiscale* h, const void* d_cube, void* stream);
/* The search handle of timescale `scale` (owned by h, valid until destroy):
 * every introspection entry point above applies to it (maps, best trial,
 * noise statistics, normalised cube, stage times). */
nsfrb_status nsfrb_multiscale_scale(nsfrb_multiscale* h, int32_t scale, nsfrb_search** out);
/* Wait for the last run and merge the candidate lists of all timescales:
 * sorted by S/N (descending), then timescale index, then pixel index; the
 * first K (cfg->max_candidates) are kept and min(K, capacity) written.
 * *n_total = sum over timescales of the pixels at or above the threshold.
 * TRUNCATED when capacity is below the kept count; NOT_READY before any run. */
nsfrb_status nsfrb_multiscale_candidates_get(nsfrb_multiscale* h, nsfrb_scale_candidate* host_out,
                                             int32_t capacity, int32_t* n_written, int32_t* n_total);

/* --------------------------------------------------------------- streaming
 * Real-time form (section 2.2: images arrive continuously and are searched in
 * fixed 3.35 s batches, 25 samples, under a timeout; the search reports one
 * candidate per batch). The stream keeps the last n_time samples of the raw
 * cube in a device ring (cfg: TSP layout, statistics computed by the search,
 * not EXTERNAL) and, after each batch once the ring is full, searches the
 * window it holds: robust statistics over the window, then the search of
 * nsfrb_search_run. A search that takes longer than deadline_ms (measured with
 * HIP events) makes the next iteration be dropped. A sub-band that did not
 * arrive is passed as non-finite samples: its series are flagged and
 * normalised to 0 (nsfrb_flag_count_get). */
typedef struct nsfrb_stream nsfrb_stream; /* opaque handle */

typedef struct {
  int32_t searched;        /* 1 if this batch's window was searched              */
  int32_t has_candidate;   /* 1 if a pixel reached the threshold                  */
  nsfrb_candidate cand;    /* the window's best candidate (valid if has_candidate);
                              its TOA is a sample index within the window        */
  int64_t chunk_index;     /* batches pushed before this one                      */
  int64_t window_start;    /* stream sample index of the window's first sample    */
  float search_ms;         /* device time of the search (if searched)              */
  int32_t dropped_total;   /* iterations dropped so far                             */
  int64_t flagged;         /* series flagged in this window (if searched)          */
} nsfrb_stream_result;

/* chunk: samples per batch, 1..n_time; deadline_ms > 0. Errors as for
 * nsfrb_search_create; UNSUPPORTED for a PST layout or EXTERNAL statistics. */
nsfrb_status nsfrb_stream_create(const nsfrb_search_config* cfg, int32_t chunk, double deadline_ms,
                                 nsfrb_stream** out);
nsfrb_status nsfrb_stream_destroy(nsfrb_stream* s);
/* Append one batch (device [chunk][n_sub][ny*nx] of in_dtype, copied into the
 * ring on `stream`) and, when due, search the window; waits for the search and
 * fills *out. */
nsfrb_status nsfrb_stream_push(nsfrb_stream* s, const void* d_chunk, void* stream, nsfrb_stream_result* out);
/* The stream's search handle (maps, statistics, z cube of the last searched window). */
nsfrb_status nsfrb_stream_search(nsfrb_stream* s, nsfrb_search** out);

/* ----------------------------------------------------- PSF-based reduction
 * Host-only post-processing of one image's top candidates (section 2.3): the
 * simulated PSF host psf[psf_ny][psf_nx] (odd sides, centred on the middle
 * pixel, centre > 0) is thresholded at `percentile` (0..100; the paper uses 90;
 * linear interpolation between order statistics, as NumPy's default) into a
 * binary mask (pixels >= the threshold). The mask is centred on each candidate
 * in turn: the other candidates at offsets inside it are that candidate's
 * possible sidelobes, and its score is the S/N of the weighted mean of the
 * S/N values of itself (weight 1) and them (weight w = PSF at the offset / PSF
 * at the centre): sum(w S) / sqrt(sum(w^2)), each S/N having unit noise.
 * Writes the index of the highest score (ties: the earlier candidate) and that
 * score.
 * INVALID_ARG for NULL pointers, n < 1, even sides, a non-finite PSF value, a
 * centre <= 0 or a percentile outside 0..100. */
nsfrb_status nsfrb_psf_reduce(const nsfrb_candidate* cands, int32_t n, const float* psf, int32_t psf_nx,
                              int32_t psf_ny, double percentile, int32_t* best_index, double* best_score);

/* ------------------------------------------------------------------ batch
 * Many cubes of uneven shape searched together (the process server of
 * section 2.2 batches search tasks per timescale). All configurations must
 * share the DM trials, widths, store dtype, normalisation, layout, input
 * dtype and device; nx, ny, n_sub, n_time and frequencies may differ.
 * nsfrb_batch_run enqueues the statistics of every cube, then one persistent
 * search launch per kernel class (the cubes with the same samples per lane;
 * each launch's workgroups walk the pixels of its cubes, with a grid sized to
 * that kernel's occupancy), then the candidates of every cube. The sequence is
 * captured once as a hipGraph and replayed while the cube pointers stay the
 * same. Results are bitwise equal to nsfrb_batch_run_separate, which launches
 * each cube's own tuned search kernel (compiled and tuned on its first call).
 * Cube pointers must be aligned to the sample size (INVALID_ARG otherwise). */
typedef struct nsfrb_batch nsfrb_batch;

nsfrb_status nsfrb_batch_create(const nsfrb_search_config* cfgs, int32_t n_cubes, nsfrb_batch** out);
nsfrb_status nsfrb_batch_destroy(nsfrb_batch* b);
/* d_cubes: host array of n_cubes device pointers (caller-owned, valid until the run completes). */
nsfrb_status nsfrb_batch_run(nsfrb_batch* b, const void* const* d_cubes, void* stream);
nsfrb_status nsfrb_batch_run_separate(nsfrb_batch* b, const void* const* d_cubes, void* stream);
/* Graph capture on (default 1) or off. */
nsfrb_status nsfrb_batch_use_graph(nsfrb_batch* b, int32_t on);
/* Same contract as nsfrb_candidates_get / nsfrb_maps_get, for cube `cube`. */
nsfrb_status nsfrb_batch_candidates_get(nsfrb_batch* b, int32_t cube, nsfrb_candidate* host_out,
                                        int32_t capacity, int32_t* n_written, int32_t* n_total);
nsfrb_status nsfrb_batch_maps_get(nsfrb_batch* b, int32_t cube, float* snr_max, int32_t* toa);
/* Per-pixel best trial and normalised-cube pointer of one cube, as
 * nsfrb_best_get and nsfrb_zcube_device of a single search. */
nsfrb_status nsfrb_batch_best_get(nsfrb_batch* b, int32_t cube, float* snr, int32_t* dm_index, int32_t* width_index,
                                  int32_t* toa);
nsfrb_status nsfrb_batch_zcube_device(nsfrb_batch* b, int32_t cube, const void** d_z);
/* info[0] work items, [1] workgroups over all class launches, [2] largest LDS bytes, [3] kernel
 * classes, [4] 1 if the last run replayed a captured graph. */
nsfrb_status nsfrb_batch_info_get(nsfrb_batch* b, int64_t* info);

/* ------------------------------------------------------------ generator
 * Synthetic input on the device (for workloads too large to build on the
 * host). Gaussian noise N(0, sigma^2): element e of the cube (in its layout
 * order) takes value 4*(e/4) ... from one Philox4x32-10 block (Salmon et al.
 * 2011) with counter (e/4, 0, 0, 0) and key (seed low, seed high), turned into
 * two Box-Muller pairs. dtype: nsfrb_dtype; layout: nsfrb_layout. */
nsfrb_status nsfrb_generate_noise(void* d_out, int32_t dtype, int32_t layout, int32_t n_pix, int32_t n_sub,
                                  int32_t n_time, uint64_t seed, float sigma, void* stream);
/* Add `amp` to samples t0 + offsets[s] ... + width - 1 of every sub-band s of
 * pixel `pixel` (samples outside the cube are skipped); host_offsets[n_sub]. */
nsfrb_status nsfrb_inject_boxcar(void* d_cube, int32_t dtype, int32_t layout, int32_t n_pix, int32_t n_sub,
                                 int32_t n_time, int32_t pixel, int32_t t0, int32_t width, float amp,
                                 const int32_t* host_offsets, void* stream);
/* Many boxcars in one launch: record i adds amp to samples
 * t0 + host_offsets[i*n_sub + s] ... + width - 1 of every sub-band s of pixel
 * `pixel` of cube d_cubes[cube] (a HOST array of n_cubes DEVICE pointers, all
 * cubes of one shape, dtype and layout). Samples outside are skipped. Records
 * must name distinct (cube, pixel) pairs (INVALID_ARG otherwise); 1 <= n <=
 * 65535. Synchronous, like nsfrb_inject_boxcar. */
typedef struct {
  int32_t cube, pixel, t0, width;
  float amp;
} nsfrb_boxcar;
nsfrb_status nsfrb_inject_boxcars(void* const* d_cubes, int32_t n_cubes, int32_t dtype, int32_t layout, int32_t n_pix,
                                  int32_t n_sub, int32_t n_time, const nsfrb_boxcar* host_boxcars,
                                  const int32_t* host_offsets, int32_t n, void* stream);
/* nsfrb_inject_boxcars for callers that cannot allocate device memory (a
 * serving loop injecting test pulses into live data, code that forbids
 * hipMalloc): same arguments, same kernel, same result, but the host tables
 * are staged in a static device array of NSFRB_INJECT_STATIC_BYTES per GPU
 * (held until the process ends) instead of a per-call allocation; the call
 * makes no hipMalloc/hipFree. Limits: n <= 4096, and
 * align256(8 * n_cubes) + align256(20 * n) + 4 * n * n_sub <= 1 MiB
 * (align256 rounds up to a multiple of 256); beyond them INVALID_ARG, nothing
 * copied or launched. Every call on a GPU shares that GPU's array: calls that
 * overlap on one GPU (other host threads, other streams) race and must be
 * serialised by the caller. Synchronous on `stream`. */
#define NSFRB_INJECT_STATIC_BYTES (1u << 20)
nsfrb_status nsfrb_inject_boxcars_static(void* const* d_cubes, int32_t n_cubes, int32_t dtype, int32_t layout,
                                         int32_t n_pix, int32_t n_sub, int32_t n_time,
                                         const nsfrb_boxcar* host_boxcars, const int32_t* host_offsets, int32_t n,
                                         void* stream);
/* Interference over all pixels (synthetic RFI): kind 0 adds `amp` to sample
 * t0 of every sub-band (a zero-DM spike); kind 1 adds `amp` to samples
 * t0 .. t0+len-1 of sub-band `sub_band` (a stripe). Samples outside are skipped. */
nsfrb_status nsfrb_inject_rfi(void* d_cube, int32_t dtype, int32_t layout, int32_t n_pix, int32_t n_sub,
                              int32_t n_time, int32_t kind, int32_t t0, int32_t len, int32_t sub_band, float amp,
                              void* stream);
/* Raw Philox4x32-10 words: block i (4 words) of counter (i, 0, 0, 0), key
 * (seed low, seed high); d_out[4 * n_blocks] uint32. */
nsfrb_status nsfrb_philox_fill(uint32_t* d_out, int64_t n_blocks, uint64_t seed, void* stream);

/* ------------------------------------------------------------- classifier
 * Candidate classifier (paper section 2.3: a CNN over the image cube centred
 * on the TOA -- position, time, frequency -- with convolution blocks and
 * nonlinearities, a small fully connected head and one logit whose sigmoid is
 * the RFI probability, trained with Adam on binary cross-entropy; sections
 * 3.2-3.3: a probability threshold gates the S/N candidates).
 * Network: input x[n][t][y][x][16] BF16 (sub-bands as channels, x = 32),
 * four 3x3x3 'same' convolutions to 32 channels with ReLU, then 64 head
 * features: the global maximum of every channel (the first position in
 * (t, y, x) order on ties) and the channel values at the candidate's own
 * position (t = n_time/2, y = ny/2, x = 16), then 64->32 ReLU, 32->1 logit.
 * Convolutions run on BF16 MFMA with FP32 accumulation; master weights, Adam
 * moments and the head are FP32.
 * Parameters form one FP32 vector (nsfrb_classifier_param_count() values):
 *   W_l[32][27][cin_l], b_l[32] for l = 1..4 (cin = 16, 32, 32, 32; tap index
 *   kt*9 + ky*3 + kx), then W1[32][64], c1[32], w2[32], c2[1]. */
typedef struct {
  uint32_t struct_size;    /* = sizeof(nsfrb_classifier_config)                    */
  int32_t max_batch;       /* cutouts per call, 1..1024                            */
  int32_t n_time;          /* cutout samples (64 for the workload), 1..256         */
  int32_t ny;              /* cutout rows (32; x is fixed at 32), 1..256           */
  float lr, beta1, beta2, eps;   /* Adam                                            */
  uint64_t seed;           /* weight initialisation (He-uniform convolutions)      */
  int32_t device;
} nsfrb_classifier_config;

/* A dedispersion-aligned cutout request: index of its cube in the table of
 * cube pointers; centre pixel (px, py); DM trial index; toa (a candidate's
 * first boxcar sample at f_ref, placed at cutout sample n_time/2). */
typedef struct {
  int64_t cube;
  int32_t px, py, dm_index, toa;
} nsfrb_cutout;

typedef struct nsfrb_classifier nsfrb_classifier;

int32_t nsfrb_classifier_param_count(void);
nsfrb_status nsfrb_classifier_create(const nsfrb_classifier_config* cfg, nsfrb_classifier** out);
nsfrb_status nsfrb_classifier_destroy(nsfrb_classifier* c);
nsfrb_status nsfrb_classifier_params_get(nsfrb_classifier* c, float* host_out);
nsfrb_status nsfrb_classifier_params_set(nsfrb_classifier* c, const float* host_in);
/* Learning rate of later Adam steps (a schedule); the moments are kept. */
nsfrb_status nsfrb_classifier_set_lr(nsfrb_classifier* c, float lr);
/* Gradient of the mean loss from the last train step (same layout as the parameters). */
nsfrb_status nsfrb_classifier_grads_get(nsfrb_classifier* c, float* host_out);
/* Checkpoints of training (section 2.3 trains with Adam; a run that stops
 * resumes with the same result): a host byte image of
 * nsfrb_classifier_state_bytes() bytes holding a 56-byte header (magic
 * "NSFRBCK1", version 1, parameter count, Adam step count, the caller's
 * `user_counter` word, lr, beta1, beta2, eps, n_time, ny) followed by the FP32
 * parameters and Adam's first and second moments (param_count values each).
 * Train steps after nsfrb_classifier_load continue exactly as they would have
 * after the save (same weights, moments, step count and bias corrections).
 * save: waits for the device; capacity < state_bytes -> TRUNCATED (n_written
 * still set). load: INVALID_ARG if the size, magic, version, parameter count or
 * cutout shape (n_time, ny) differ from this classifier's, or the optimiser
 * settings are not finite; nothing is changed then. *user_counter (may be
 * NULL) receives the saved word. */
int64_t nsfrb_classifier_state_bytes(void);
nsfrb_status nsfrb_classifier_save(nsfrb_classifier* c, uint64_t user_counter, void* host_out, int64_t capacity,
                                   int64_t* n_written);
nsfrb_status nsfrb_classifier_load(nsfrb_classifier* c, const void* host_in, int64_t n_bytes, uint64_t* user_counter);
/* One step on n cutouts (device BF16 [n][n_time][ny][32][16]) with device FP32
 * labels (1 = RFI/noise, 0 = astrophysical): forward, BCE loss, backward and,
 * if `update`, one Adam step. *host_loss (may be NULL) receives the mean loss
 * (the call then waits for the stream). */
nsfrb_status nsfrb_classifier_train_step(nsfrb_classifier* c, const void* d_cutouts, const float* d_labels, int32_t n,
                                         int32_t update, float* host_loss, void* stream);
/* p_rfi = sigmoid(logit) for n cutouts into device d_prob[n]. */
nsfrb_status nsfrb_classifier_infer(nsfrb_classifier* c, const void* d_cutouts, int32_t n, float* d_prob,
                                    void* stream);
/* Test/introspection: after a train step or inference on n' >= n cutouts, the
 * BF16 output a_layer (layer 1..4) of that forward pass for its first n
 * cutouts, host_out uint16 [n][n_time][ny][32][32] (BF16 bits); after a train
 * step, the BF16 gradient of the loss with respect to conv layer `layer`'s
 * pre-activation (ReLU derivative applied), same layout; and the FP32 logits
 * z (p_rfi = sigmoid(z)), host_out[n]. Wait for the device. INVALID_ARG for
 * NULL pointers, layer outside 1..4 or n outside 1..max_batch. */
nsfrb_status nsfrb_classifier_activations_get(nsfrb_classifier* c, int32_t layer, int32_t n, void* host_out);
nsfrb_status nsfrb_classifier_grad_pre_get(nsfrb_classifier* c, int32_t layer, int32_t n, void* host_out);
nsfrb_status nsfrb_classifier_logits_get(nsfrb_classifier* c, int32_t n, float* host_out);
/* Cut n_cut dedispersion-aligned cutouts (section 2.3: the classifier sees
 * the image cube centred on the candidate's TOA) out of normalised cubes in
 * the search layout [ny*nx][n_sub][n_time] (store dtype; n_sub must be 16).
 * d_z_cubes is a HOST array of n_cubes DEVICE pointers (e.g. from
 * nsfrb_zcube_device); all cubes share the shape and the delay table
 * host_delays[n_dm * n_sub] (delta[d][s] in samples). Sample tt of sub-band s
 * of cutout k is z[pixel][s][toa - n_time_c/2 + tt + delta[dm][s]], pixels
 * centred on (px, py), zero outside the image or the series; d_out BF16
 * [n_cut][n_time_c][32][32][16], n_time_c = the classifier's n_time (its ny
 * must be 32). Waits for `stream` (the descriptor buffers are reused), then
 * enqueues the copy on it. INVALID_ARG for NULL pointers, n_cut outside
 * 1..max_batch or a descriptor whose cube or DM index is out of range. */
nsfrb_status nsfrb_cutouts_extract(nsfrb_classifier* c, const void* const* d_z_cubes, int32_t n_cubes,
                                   int32_t store_dtype, int32_t nx, int32_t ny, int32_t n_sub, int32_t n_time,
                                   const int32_t* host_delays, int32_t n_dm, const nsfrb_cutout* host_desc,
                                   int32_t n_cut, void* d_out, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* NSFRB_H */
