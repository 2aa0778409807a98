// Host side of the search library: configuration checks, the delay table,
// plan-time specialisation of the search kernel, device workspace, launches.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/nsfrb.h"
#include "nsfrb_internal.h"
#include "rtc_sources.inc"   // kRtcDeviceCommon, kRtcSearchBody (generated at build time)

using namespace nsfrb;

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;

static nsfrb_status fail(nsfrb_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(e_ == hipErrorOutOfMemory ? NSFRB_ERR_OUT_OF_MEMORY : NSFRB_ERR_DEVICE,  \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                      \
  } while (0)

extern "C" const char* nsfrb_version(void) { return "nsfrb-mi355x 0.1 (gfx950)"; }
extern "C" const char* nsfrb_last_error(void) { return g_last_error.c_str(); }

// ------------------------------------------------------------------ limits
static constexpr int kMaxSub = 64;
static constexpr int kMaxTime = 4096;
static constexpr int kMaxDm = 256;
static constexpr int kMaxWidth = 32;
static constexpr int kMaxCand = 4096;
static constexpr int kMaxAccumulators = 3;     // non-power-of-two widths open at once
static constexpr size_t kLdsBudget = 160 * 1024 - 1024;
static constexpr int kSearchThreads = 512;

static size_t dtype_size(int dt) { return dt == DT_F32 ? 4 : 2; }

// ------------------------------------------------------------ delay table
// delta[d][s] = rint(((k*DM) * (1/(f*f) - 1/(fr*fr))) / dt), FP64, no contraction.
#pragma clang fp contract(off)
static void compute_delays(const nsfrb_search_config& c, std::vector<int32_t>& out) {
  out.assign((size_t)c.n_dm * c.n_sub, 0);
  const double fr = c.f_ref_ghz;
  for (int d = 0; d < c.n_dm; ++d) {
    const double kd = c.k_dm_ms * c.dm[d];
    for (int s = 0; s < c.n_sub; ++s) {
      const double f = c.freq_ghz[s];
      const double inv = 1.0 / (f * f) - 1.0 / (fr * fr);
      const double v = (kd * inv) / c.dt_ms;
      out[(size_t)d * c.n_sub + s] = (int32_t)std::nearbyint(v);   // ties to even
    }
  }
}

static nsfrb_status validate(const nsfrb_search_config* c) {
  if (!c) return fail(NSFRB_ERR_INVALID_ARG, "config is NULL");
  if (c->struct_size != sizeof(nsfrb_search_config))
    return fail(NSFRB_ERR_INVALID_ARG, "struct_size does not match this library's nsfrb_search_config");
  if (c->nx < 1 || c->ny < 1 || c->n_sub < 1 || c->n_time < 1 || c->n_dm < 1 || c->n_width < 1)
    return fail(NSFRB_ERR_INVALID_ARG, "dimensions nx, ny, n_sub, n_time, n_dm, n_width must be >= 1");
  if (!c->freq_ghz || !c->dm || !c->width) return fail(NSFRB_ERR_INVALID_ARG, "freq_ghz, dm and width must be set");
  if ((long long)c->nx * c->ny > (1LL << 28)) return fail(NSFRB_ERR_UNSUPPORTED, "more than 2^28 pixels");
  if (c->n_sub > kMaxSub) return fail(NSFRB_ERR_UNSUPPORTED, "n_sub above 64");
  if (c->n_time > kMaxTime) return fail(NSFRB_ERR_UNSUPPORTED, "n_time above 4096");
  if (c->n_dm > kMaxDm) return fail(NSFRB_ERR_UNSUPPORTED, "n_dm above 256");
  if (c->n_width > kMaxWidth) return fail(NSFRB_ERR_UNSUPPORTED, "n_width above 32");
  double fmax = 0.0;
  for (int s = 0; s < c->n_sub; ++s) {
    const double f = c->freq_ghz[s];
    if (!std::isfinite(f) || f <= 0.0) return fail(NSFRB_ERR_INVALID_ARG, "frequencies must be finite and > 0");
    fmax = f > fmax ? f : fmax;
  }
  if (!std::isfinite(c->f_ref_ghz) || c->f_ref_ghz < fmax)
    return fail(NSFRB_ERR_INVALID_ARG, "f_ref_ghz must be >= the highest sub-band frequency (delays would be negative)");
  if (!std::isfinite(c->dt_ms) || c->dt_ms <= 0.0) return fail(NSFRB_ERR_INVALID_ARG, "dt_ms must be finite and > 0");
  if (!std::isfinite(c->k_dm_ms) || c->k_dm_ms <= 0.0) return fail(NSFRB_ERR_INVALID_ARG, "k_dm_ms must be finite and > 0");
  for (int d = 0; d < c->n_dm; ++d)
    if (!std::isfinite(c->dm[d]) || c->dm[d] < 0.0) return fail(NSFRB_ERR_INVALID_ARG, "DM trials must be finite and >= 0");
  for (int i = 0; i < c->n_width; ++i)
    if (c->width[i] < 1) return fail(NSFRB_ERR_INVALID_ARG, "widths must be >= 1");
    else if (c->width[i] > kMaxTime) return fail(NSFRB_ERR_UNSUPPORTED, "widths above 4096");
  if (c->in_dtype < 0 || c->in_dtype > 2 || c->store_dtype < 0 || c->store_dtype > 2)
    return fail(NSFRB_ERR_INVALID_ARG, "unknown dtype");
  if (c->norm < 0 || c->norm > 3) return fail(NSFRB_ERR_INVALID_ARG, "unknown normalisation mode");
  if (c->norm == NSFRB_NORM_PIXEL) return fail(NSFRB_ERR_UNSUPPORTED, "NSFRB_NORM_PIXEL is not implemented");
  if (!std::isfinite(c->snr_threshold)) return fail(NSFRB_ERR_INVALID_ARG, "snr_threshold must be finite");
  if (c->max_candidates < 1 || c->max_candidates > kMaxCand)
    return fail(NSFRB_ERR_INVALID_ARG, "max_candidates must be in 1..4096");
  if (c->device < 0) return fail(NSFRB_ERR_INVALID_ARG, "device must be >= 0");
  // delay-dependent limits: the pixel's rows (+ the largest searchable delay) must fit in LDS
  std::vector<int32_t> dl;
  compute_delays(*c, dl);
  for (int32_t v : dl)
    if (v < 0) return fail(NSFRB_ERR_INVALID_ARG, "negative delay");
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_config_validate(const nsfrb_search_config* cfg) {
  g_last_error.clear();
  return validate(cfg);
}

extern "C" nsfrb_status nsfrb_plan_delays(const nsfrb_search_config* cfg, int32_t* host_out) {
  g_last_error.clear();
  nsfrb_status st = validate(cfg);
  if (st != NSFRB_OK) return st;
  if (!host_out) return fail(NSFRB_ERR_INVALID_ARG, "host_out is NULL");
  std::vector<int32_t> dl;
  compute_delays(*cfg, dl);
  std::memcpy(host_out, dl.data(), dl.size() * sizeof(int32_t));
  return NSFRB_OK;
}

// ------------------------------------------------- search plan (codegen)
struct SearchPlan {
  int C = 0;               // samples per lane (odd), 64*C >= n_time
  int rs = 0;              // LDS row length in samples
  size_t lds_bytes = 0;
  std::string source;      // generated translation unit
};

static int lanes_per_sample_count(int n_time) {
  int c = (n_time + 63) / 64;
  if ((c & 1) == 0) c += 1;
  return c;
}

// Emit the boxcar plan: power-of-two levels by pairwise doubling, other
// widths as sums of the level windows of their binary digits.
static nsfrb_status gen_chain(const std::vector<int>& widths, int n_time, std::string& out) {
  const int nw = (int)widths.size();
  int maxb = -1;
  for (int w : widths)
    if (w <= n_time) {
      int b = 0;
      while ((2 << b) <= w) ++b;
      maxb = b > maxb ? b : maxb;
    }
  std::ostringstream o;
  o << "template <class R>\n__device__ void nsfrb_chain(float (&a0)[kC], R& rep) {\n";
  o << "  using namespace nsfrb;\n  float a1[kC];\n";
  // accumulators for non-power-of-two widths: [lowest bit, highest bit]
  struct Acc { int iw, w, lo, hi, slot, off; };
  std::vector<Acc> accs;
  for (int iw = 0; iw < nw; ++iw) {
    const int w = widths[iw];
    if (w > n_time || (w & (w - 1)) == 0) continue;
    int lo = __builtin_ctz((unsigned)w), hi = 31 - __builtin_clz((unsigned)w);
    accs.push_back({iw, w, lo, hi, -1, 0});
  }
  // slot allocation by interval scheduling
  int nslots = 0;
  std::vector<int> slot_free_after;   // level after which the slot is free
  for (auto& a : accs) {
    for (int s = 0; s < (int)slot_free_after.size(); ++s)
      if (slot_free_after[s] < a.lo) { a.slot = s; slot_free_after[s] = a.hi; break; }
    if (a.slot < 0) { a.slot = (int)slot_free_after.size(); slot_free_after.push_back(a.hi); }
  }
  nslots = (int)slot_free_after.size();
  if (nslots > kMaxAccumulators)
    return fail(NSFRB_ERR_UNSUPPORTED, "too many non-power-of-two widths open at once (max 3)");
  for (int s = 0; s < nslots; ++s) o << "  float acc" << s << "[kC];\n";
  for (int iw = 0; iw < nw; ++iw)
    if (widths[iw] > n_time) o << "  rep.invalid(" << iw << ");\n";
  for (int b = 0; b <= maxb; ++b) {
    const char* cur = (b & 1) ? "a1" : "a0";
    const char* nxt = (b & 1) ? "a0" : "a1";
    o << "  // level " << b << ": windows of " << (1 << b) << " samples in " << cur << "\n";
    for (int iw = 0; iw < nw; ++iw)
      if (widths[iw] == (1 << b)) o << "  rep(" << iw << ", " << cur << ");\n";
    for (auto& a : accs) {
      if (!((a.w >> b) & 1)) continue;
      if (b == a.lo) {
        o << "  copy_arr(acc" << a.slot << ", " << cur << ");\n";
      } else {
        o << "  shift_add<" << a.off << ">(acc" << a.slot << ", acc" << a.slot << ", " << cur << ");\n";
      }
      a.off += 1 << b;
      if (b == a.hi) o << "  rep(" << a.iw << ", acc" << a.slot << ");\n";
    }
    if (b < maxb) o << "  shift_add<" << (1 << b) << ">(" << nxt << ", " << cur << ", " << cur << ");\n";
  }
  o << "}\n";
  out = o.str();
  return NSFRB_OK;
}

static nsfrb_status build_plan(const nsfrb_search_config& c, int dmax_search, SearchPlan& plan) {
  plan.C = lanes_per_sample_count(c.n_time);
  plan.rs = 64 * plan.C + dmax_search + 1;
  plan.lds_bytes = (size_t)c.n_sub * plan.rs * dtype_size(c.store_dtype);
  if (plan.lds_bytes > kLdsBudget)
    return fail(NSFRB_ERR_UNSUPPORTED, "n_sub x (padded n_time + max delay) does not fit in LDS for this store dtype");
  std::vector<int> widths(c.width, c.width + c.n_width);
  std::string chain;
  nsfrb_status st = gen_chain(widths, c.n_time, chain);
  if (st != NSFRB_OK) return st;
  const char* st_name = c.store_dtype == DT_F32 ? "float" : (c.store_dtype == DT_F16 ? "_Float16" : "nsfrb::bf16_t");
  std::ostringstream o;
  o << "#define NSFRB_RTC_PROLOGUE 1\n#include \"device_common.h\"\n";
  o << "typedef " << st_name << " ST;\n";
  o << "constexpr int kC = " << plan.C << ";\n";
  o << "#define NSFRB_NW " << c.n_width << "\n";
  o << "#include \"k_search_body.h\"\n";
  o << chain;
  plan.source = o.str();
  return NSFRB_OK;
}

// Compiled kernels, shared by every handle on a device.
struct CompiledKernel {
  hipModule_t mod = nullptr;
  hipFunction_t fn = nullptr;
};
static std::mutex g_rtc_mu;
static std::map<std::pair<int, std::string>, CompiledKernel> g_rtc_cache;

static nsfrb_status compile_search(int device, const std::string& src, hipFunction_t* fn) {
  std::lock_guard<std::mutex> lk(g_rtc_mu);
  auto key = std::make_pair(device, src);
  auto it = g_rtc_cache.find(key);
  if (it != g_rtc_cache.end()) { *fn = it->second.fn; return NSFRB_OK; }
  hiprtcProgram prog;
  const char* hdr_names[] = {"device_common.h", "k_search_body.h"};
  const char* hdr_src[] = {kRtcDeviceCommon, kRtcSearchBody};
  if (hiprtcCreateProgram(&prog, src.c_str(), "nsfrb_search.hip", 2, hdr_src, hdr_names) != HIPRTC_SUCCESS)
    return fail(NSFRB_ERR_DEVICE, "hiprtcCreateProgram failed");
  const char* opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17",
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
  hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof(opts) / sizeof(opts[0])), opts);
  if (r != HIPRTC_SUCCESS) {
    size_t n = 0;
    hiprtcGetProgramLogSize(prog, &n);
    std::string log(n + 1, '\0');
    hiprtcGetProgramLog(prog, &log[0]);
    hiprtcDestroyProgram(&prog);
    return fail(NSFRB_ERR_DEVICE, "search kernel compilation failed: " + log);
  }
  size_t sz = 0;
  hiprtcGetCodeSize(prog, &sz);
  std::vector<char> code(sz);
  hiprtcGetCode(prog, code.data());
  hiprtcDestroyProgram(&prog);
  const char* dump = std::getenv("NSFRB_DUMP_CODE");
  if (dump && *dump) {
    FILE* f = std::fopen(dump, "wb");
    if (f) { std::fwrite(code.data(), 1, code.size(), f); std::fclose(f); }
  }
  CompiledKernel ck;
  HIP_TRY(hipModuleLoadData(&ck.mod, code.data()));
  HIP_TRY(hipModuleGetFunction(&ck.fn, ck.mod, "nsfrb_search_kernel"));
  g_rtc_cache[key] = ck;
  *fn = ck.fn;
  return NSFRB_OK;
}

// Host-only entry: generate (and optionally compile) the specialised search
// source, for build checks and inspection. Not part of the public header.
extern "C" int nsfrb_debug_plan_source(const nsfrb_search_config* cfg, char* out, int cap, int compile) {
  if (validate(cfg) != NSFRB_OK) return -1;
  std::vector<int32_t> dl;
  compute_delays(*cfg, dl);
  int dmax_search = 0;
  for (int d = 0; d < cfg->n_dm; ++d) {
    int m = 0;
    for (int s = 0; s < cfg->n_sub; ++s) m = dl[(size_t)d * cfg->n_sub + s] > m ? dl[(size_t)d * cfg->n_sub + s] : m;
    if (m < cfg->n_time && m > dmax_search) dmax_search = m;
  }
  SearchPlan plan;
  if (build_plan(*cfg, dmax_search, plan) != NSFRB_OK) return -1;
  if (out && cap > 0) {
    std::snprintf(out, (size_t)cap, "%s", plan.source.c_str());
  }
  if (compile) {
    hiprtcProgram prog;
    const char* hdr_names[] = {"device_common.h", "k_search_body.h"};
    const char* hdr_src[] = {kRtcDeviceCommon, kRtcSearchBody};
    hiprtcCreateProgram(&prog, plan.source.c_str(), "nsfrb_search.hip", 2, hdr_src, hdr_names);
    const char* opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17",
                          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
    hiprtcResult r = hiprtcCompileProgram(prog, 7, opts);
    if (r != HIPRTC_SUCCESS) {
      size_t n = 0;
      hiprtcGetProgramLogSize(prog, &n);
      std::string log(n + 1, '\0');
      hiprtcGetProgramLog(prog, &log[0]);
      g_last_error = log;
      hiprtcDestroyProgram(&prog);
      return -2;
    }
    size_t sz = 0;
    hiprtcGetCodeSize(prog, &sz);
    const char* dump = std::getenv("NSFRB_DUMP_CODE");
    if (dump && *dump) {
      std::vector<char> code(sz);
      hiprtcGetCode(prog, code.data());
      FILE* f = std::fopen(dump, "wb");
      if (f) { std::fwrite(code.data(), 1, code.size(), f); std::fclose(f); }
    }
    hiprtcDestroyProgram(&prog);
  }
  return (int)plan.source.size();
}

// ------------------------------------------------------------------ handle
struct nsfrb_search {
  nsfrb_search_config cfg{};
  std::vector<double> freqs, dms;
  std::vector<int32_t> widths, delays, dmaxv;
  int n_pix = 0, device = 0;
  SearchPlan plan;
  hipFunction_t search_fn = nullptr;
  // device buffers
  int32_t *d_delays = nullptr, *d_dmax = nullptr;
  float* d_norms = nullptr;
  void* d_z = nullptr;
  double *d_med = nullptr, *d_sig = nullptr, *d_ext_med = nullptr, *d_ext_sig = nullptr;
  float* d_snr = nullptr;
  int32_t* d_toa = nullptr;
  float* d_best_s = nullptr;
  int32_t *d_best_d = nullptr, *d_best_w = nullptr, *d_best_t = nullptr;
  unsigned long long* d_keys = nullptr;
  int32_t* d_count = nullptr;
  nsfrb_candidate* d_cands = nullptr;
  int32_t* d_nout = nullptr;
  unsigned long long* d_flags = nullptr;
  // pinned host mirrors
  nsfrb_candidate* h_cands = nullptr;
  int32_t* h_nout = nullptr;
  hipEvent_t done = nullptr;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  bool profiling = false, ran = false, ext_set = false;
};

template <typename T>
static hipError_t dalloc(T** p, size_t n) {
  return hipMalloc((void**)p, n * sizeof(T) > 0 ? n * sizeof(T) : 16);
}

static void release(nsfrb_search* h) {
  if (!h) return;
  hipSetDevice(h->device);
  void* bufs[] = {h->d_delays, h->d_dmax, h->d_norms, h->d_z, h->d_med, h->d_sig, h->d_ext_med, h->d_ext_sig,
                  h->d_snr, h->d_toa, h->d_best_s, h->d_best_d, h->d_best_w, h->d_best_t, h->d_keys,
                  h->d_count, h->d_cands, h->d_nout, h->d_flags};
  for (void* b : bufs)
    if (b) hipFree(b);
  if (h->h_cands) hipHostFree(h->h_cands);
  if (h->h_nout) hipHostFree(h->h_nout);
  if (h->done) hipEventDestroy(h->done);
  for (auto& e : h->ev)
    if (e) hipEventDestroy(e);
  delete h;
}

extern "C" nsfrb_status nsfrb_search_create(const nsfrb_search_config* cfg, nsfrb_search** out) {
  g_last_error.clear();
  if (!out) return fail(NSFRB_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  nsfrb_status st = validate(cfg);
  if (st != NSFRB_OK) return st;
  std::unique_ptr<nsfrb_search, void (*)(nsfrb_search*)> h(new nsfrb_search, release);
  h->cfg = *cfg;
  h->freqs.assign(cfg->freq_ghz, cfg->freq_ghz + cfg->n_sub);
  h->dms.assign(cfg->dm, cfg->dm + cfg->n_dm);
  h->widths.assign(cfg->width, cfg->width + cfg->n_width);
  h->cfg.freq_ghz = h->freqs.data();
  h->cfg.dm = h->dms.data();
  h->cfg.width = h->widths.data();
  h->n_pix = cfg->nx * cfg->ny;
  h->device = cfg->device;
  compute_delays(h->cfg, h->delays);
  h->dmaxv.assign(cfg->n_dm, 0);
  int dmax_search = 0;
  for (int d = 0; d < cfg->n_dm; ++d) {
    int m = 0;
    for (int s = 0; s < cfg->n_sub; ++s) m = std::max(m, (int)h->delays[(size_t)d * cfg->n_sub + s]);
    h->dmaxv[d] = m;
    if (m < cfg->n_time) dmax_search = std::max(dmax_search, m);
  }
  st = build_plan(h->cfg, dmax_search, h->plan);
  if (st != NSFRB_OK) return st;
  const char* force = std::getenv("NSFRB_FORCE_ALLOC_FAIL");
  if (force && std::atoi(force) != 0) return fail(NSFRB_ERR_OUT_OF_MEMORY, "allocation failure forced by NSFRB_FORCE_ALLOC_FAIL");

  HIP_TRY(hipSetDevice(h->device));
  st = compile_search(h->device, h->plan.source, &h->search_fn);
  if (st != NSFRB_OK) return st;
  const size_t n_pix = (size_t)h->n_pix, ns = (size_t)cfg->n_sub, nt = (size_t)cfg->n_time;
  const size_t nmaps = (size_t)cfg->n_dm * cfg->n_width * n_pix;
  HIP_TRY(dalloc(&h->d_delays, h->delays.size()));
  HIP_TRY(dalloc(&h->d_dmax, h->dmaxv.size()));
  HIP_TRY(dalloc(&h->d_norms, (size_t)cfg->n_width));
  HIP_TRY(hipMalloc(&h->d_z, n_pix * ns * nt * dtype_size(cfg->store_dtype)));
  HIP_TRY(dalloc(&h->d_med, n_pix * ns));
  HIP_TRY(dalloc(&h->d_sig, n_pix * ns));
  if (cfg->norm == NSFRB_NORM_EXTERNAL) {
    HIP_TRY(dalloc(&h->d_ext_med, n_pix * ns));
    HIP_TRY(dalloc(&h->d_ext_sig, n_pix * ns));
  }
  HIP_TRY(dalloc(&h->d_snr, nmaps));
  HIP_TRY(dalloc(&h->d_toa, nmaps));
  HIP_TRY(dalloc(&h->d_best_s, n_pix));
  HIP_TRY(dalloc(&h->d_best_d, n_pix));
  HIP_TRY(dalloc(&h->d_best_w, n_pix));
  HIP_TRY(dalloc(&h->d_best_t, n_pix));
  HIP_TRY(dalloc(&h->d_keys, n_pix));
  HIP_TRY(dalloc(&h->d_count, 4));
  HIP_TRY(dalloc(&h->d_cands, (size_t)cfg->max_candidates));
  HIP_TRY(dalloc(&h->d_nout, 4));
  HIP_TRY(dalloc(&h->d_flags, 1));
  HIP_TRY(hipHostMalloc((void**)&h->h_cands, sizeof(nsfrb_candidate) * cfg->max_candidates, hipHostMallocDefault));
  HIP_TRY(hipHostMalloc((void**)&h->h_nout, sizeof(int32_t) * 4, hipHostMallocDefault));
  HIP_TRY(hipEventCreateWithFlags(&h->done, hipEventDisableTiming));
  for (auto& e : h->ev) HIP_TRY(hipEventCreate(&e));
  std::vector<float> norms(cfg->n_width);
  for (int i = 0; i < cfg->n_width; ++i) norms[i] = (float)std::sqrt((double)cfg->n_sub * (double)h->widths[i]);
  HIP_TRY(hipMemcpy(h->d_delays, h->delays.data(), h->delays.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(h->d_dmax, h->dmaxv.data(), h->dmaxv.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(h->d_norms, norms.data(), norms.size() * sizeof(float), hipMemcpyHostToDevice));
  HIP_TRY(hipMemset(h->d_flags, 0, sizeof(unsigned long long)));
  *out = h.release();
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_search_destroy(nsfrb_search* h) {
  g_last_error.clear();
  if (h) {
    hipSetDevice(h->device);
    if (h->ran) hipEventSynchronize(h->done);
  }
  release(h);
  return NSFRB_OK;
}

static nsfrb_status launch_search(nsfrb_search* h, hipStream_t st) {
  const nsfrb_search_config& c = h->cfg;
  const void* z = h->d_z;
  int n_pix = h->n_pix, n_sub = c.n_sub, n_t = c.n_time, n_dm = c.n_dm, rs = h->plan.rs;
  void* args[] = {(void*)&z, (void*)&h->d_delays, (void*)&h->d_dmax, (void*)&h->d_norms,
                  (void*)&n_pix, (void*)&n_sub, (void*)&n_t, (void*)&n_dm, (void*)&rs,
                  (void*)&h->d_snr, (void*)&h->d_toa, (void*)&h->d_best_s, (void*)&h->d_best_d,
                  (void*)&h->d_best_w, (void*)&h->d_best_t};
  HIP_TRY(hipModuleLaunchKernel(h->search_fn, (unsigned)n_pix, 1, 1, kSearchThreads, 1, 1,
                                (unsigned)h->plan.lds_bytes, st, args, nullptr));
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_search_run(nsfrb_search* h, const void* d_cube, void* stream) {
  g_last_error.clear();
  if (!h || !d_cube) return fail(NSFRB_ERR_INVALID_ARG, "handle and d_cube must be non-NULL");
  if (h->cfg.norm == NSFRB_NORM_EXTERNAL && !h->ext_set)
    return fail(NSFRB_ERR_INVALID_ARG, "EXTERNAL normalisation needs nsfrb_noise_stats_set before run");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(h->device));
  const nsfrb_search_config& c = h->cfg;
  if (h->profiling) HIP_TRY(hipEventRecord(h->ev[0], st));
  StatsLaunch sa{d_cube, c.n_time, c.n_sub, h->n_pix, c.norm, c.in_dtype, c.store_dtype,
                 h->d_ext_med, h->d_ext_sig, h->d_med, h->d_sig, h->d_z, h->d_flags};
  HIP_TRY(launch_stats(sa, st));
  if (h->profiling) HIP_TRY(hipEventRecord(h->ev[1], st));
  nsfrb_status s2 = launch_search(h, st);
  if (s2 != NSFRB_OK) return s2;
  if (h->profiling) HIP_TRY(hipEventRecord(h->ev[2], st));
  CandLaunch ca{h->d_best_s, h->d_best_d, h->d_best_w, h->d_best_t, h->n_pix, c.nx, c.max_candidates,
                c.snr_threshold, h->d_keys, h->d_count, h->d_cands, h->d_nout};
  HIP_TRY(launch_candidates(ca, st));
  if (h->profiling) HIP_TRY(hipEventRecord(h->ev[3], st));
  HIP_TRY(hipMemcpyAsync(h->h_nout, h->d_nout, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(h->h_cands, h->d_cands, sizeof(nsfrb_candidate) * c.max_candidates,
                         hipMemcpyDeviceToHost, st));
  HIP_TRY(hipEventRecord(h->done, st));
  h->ran = true;
  return NSFRB_OK;
}

static nsfrb_status wait_run(const nsfrb_search* h) {
  if (!h) return fail(NSFRB_ERR_INVALID_ARG, "handle is NULL");
  if (!h->ran) return fail(NSFRB_ERR_NOT_READY, "no run has been enqueued on this handle");
  HIP_TRY(hipSetDevice(h->device));
  HIP_TRY(hipEventSynchronize(h->done));
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_candidates_get(nsfrb_search* h, nsfrb_candidate* host_out, int32_t capacity,
                                             int32_t* n_written, int32_t* n_total) {
  g_last_error.clear();
  nsfrb_status st = wait_run(h);
  if (st != NSFRB_OK) return st;
  if (capacity < 0 || (capacity > 0 && !host_out)) return fail(NSFRB_ERR_INVALID_ARG, "bad output buffer");
  const int k = h->h_nout[0], total = h->h_nout[1];
  const int nw = k < capacity ? k : capacity;
  if (nw > 0) std::memcpy(host_out, h->h_cands, sizeof(nsfrb_candidate) * nw);
  if (n_written) *n_written = nw;
  if (n_total) *n_total = total;
  if (nw < k) return fail(NSFRB_ERR_TRUNCATED, "capacity below the number of candidates");
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_delay_table_get(const nsfrb_search* h, int32_t* host_out) {
  g_last_error.clear();
  if (!h || !host_out) return fail(NSFRB_ERR_INVALID_ARG, "NULL argument");
  std::memcpy(host_out, h->delays.data(), h->delays.size() * sizeof(int32_t));
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_maps_get(nsfrb_search* h, float* snr_max, int32_t* toa) {
  g_last_error.clear();
  nsfrb_status st = wait_run(h);
  if (st != NSFRB_OK) return st;
  const size_t n = (size_t)h->cfg.n_dm * h->cfg.n_width * h->n_pix;
  if (snr_max) HIP_TRY(hipMemcpy(snr_max, h->d_snr, n * sizeof(float), hipMemcpyDeviceToHost));
  if (toa) HIP_TRY(hipMemcpy(toa, h->d_toa, n * sizeof(int32_t), hipMemcpyDeviceToHost));
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_maps_device(nsfrb_search* h, float** snr_max, int32_t** toa) {
  g_last_error.clear();
  if (!h) return fail(NSFRB_ERR_INVALID_ARG, "handle is NULL");
  if (snr_max) *snr_max = h->d_snr;
  if (toa) *toa = h->d_toa;
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_best_get(nsfrb_search* h, float* snr, int32_t* dm_index, int32_t* width_index,
                                       int32_t* toa) {
  g_last_error.clear();
  nsfrb_status st = wait_run(h);
  if (st != NSFRB_OK) return st;
  const size_t n = (size_t)h->n_pix;
  if (snr) HIP_TRY(hipMemcpy(snr, h->d_best_s, n * sizeof(float), hipMemcpyDeviceToHost));
  if (dm_index) HIP_TRY(hipMemcpy(dm_index, h->d_best_d, n * sizeof(int32_t), hipMemcpyDeviceToHost));
  if (width_index) HIP_TRY(hipMemcpy(width_index, h->d_best_w, n * sizeof(int32_t), hipMemcpyDeviceToHost));
  if (toa) HIP_TRY(hipMemcpy(toa, h->d_best_t, n * sizeof(int32_t), hipMemcpyDeviceToHost));
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_noise_stats_get(nsfrb_search* h, double* med, double* sigma) {
  g_last_error.clear();
  nsfrb_status st = wait_run(h);
  if (st != NSFRB_OK) return st;
  const size_t n = (size_t)h->n_pix * h->cfg.n_sub;
  const double* sm = h->cfg.norm == NSFRB_NORM_EXTERNAL ? h->d_ext_med : h->d_med;
  const double* ss = h->cfg.norm == NSFRB_NORM_EXTERNAL ? h->d_ext_sig : h->d_sig;
  if (med) HIP_TRY(hipMemcpy(med, sm, n * sizeof(double), hipMemcpyDeviceToHost));
  if (sigma) HIP_TRY(hipMemcpy(sigma, ss, n * sizeof(double), hipMemcpyDeviceToHost));
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_noise_stats_set(nsfrb_search* h, const double* med, const double* sigma) {
  g_last_error.clear();
  if (!h || !med || !sigma) return fail(NSFRB_ERR_INVALID_ARG, "NULL argument");
  if (h->cfg.norm != NSFRB_NORM_EXTERNAL) return fail(NSFRB_ERR_INVALID_ARG, "handle is not in EXTERNAL mode");
  HIP_TRY(hipSetDevice(h->device));
  if (h->ran) HIP_TRY(hipEventSynchronize(h->done));
  const size_t n = (size_t)h->n_pix * h->cfg.n_sub;
  HIP_TRY(hipMemcpy(h->d_ext_med, med, n * sizeof(double), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(h->d_ext_sig, sigma, n * sizeof(double), hipMemcpyHostToDevice));
  h->ext_set = true;
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_zcube_get(nsfrb_search* h, void* host_out) {
  g_last_error.clear();
  nsfrb_status st = wait_run(h);
  if (st != NSFRB_OK) return st;
  if (!host_out) return fail(NSFRB_ERR_INVALID_ARG, "host_out is NULL");
  const size_t n = (size_t)h->n_pix * h->cfg.n_sub * h->cfg.n_time * dtype_size(h->cfg.store_dtype);
  HIP_TRY(hipMemcpy(host_out, h->d_z, n, hipMemcpyDeviceToHost));
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_flag_count_get(nsfrb_search* h, int64_t* count) {
  g_last_error.clear();
  nsfrb_status st = wait_run(h);
  if (st != NSFRB_OK) return st;
  unsigned long long v = 0;
  HIP_TRY(hipMemcpy(&v, h->d_flags, sizeof(v), hipMemcpyDeviceToHost));
  if (count) *count = (int64_t)v;
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_profiling_enable(nsfrb_search* h, int32_t on) {
  g_last_error.clear();
  if (!h) return fail(NSFRB_ERR_INVALID_ARG, "handle is NULL");
  h->profiling = on != 0;
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_stage_times_get(nsfrb_search* h, float* ms3) {
  g_last_error.clear();
  nsfrb_status st = wait_run(h);
  if (st != NSFRB_OK) return st;
  if (!h->profiling) return fail(NSFRB_ERR_NOT_READY, "profiling was not enabled for the last run");
  for (int i = 0; i < 3; ++i) HIP_TRY(hipEventElapsedTime(&ms3[i], h->ev[i], h->ev[i + 1]));
  return NSFRB_OK;
}
