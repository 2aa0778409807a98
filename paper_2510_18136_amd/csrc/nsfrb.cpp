// Host side of the search library: configuration checks, the delay table,
// plan-time specialisation of the search kernel, device workspace, launches.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <tuple>
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
#include "host_util.h"
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

namespace nsfrb {
nsfrb_status host_fail(nsfrb_status st, const std::string& msg) { return fail(st, msg); }
void host_clear_error() { g_last_error.clear(); }
}  // namespace nsfrb

extern "C" const char* nsfrb_version(void) { return "nsfrb-mi355x 0.1 (gfx950)"; }
extern "C" const char* nsfrb_last_error(void) { return g_last_error.c_str(); }

// ------------------------------------------------------------------ limits
static constexpr int kMaxSub = 64;
static constexpr int kMaxTime = 4096;
static constexpr int kMaxDm = 256;
static constexpr int kMaxWidth = 32;
static constexpr int kMaxCand = 4096;
static constexpr int kMaxAccumulators = 3;     // non-power-of-two widths open at once
static constexpr int kMaxScratchPerLane = 64;  // bytes of register spill a launched search kernel may use

// Largest per-lane scratch (register spill) a search kernel may have to be
// launched: a few dozen bytes of spill run correctly and fast; kernels whose
// private segment approaches the runtime's per-thread stack limit are never
// launched (such a kernel, 1.9 KB per lane, was rejected at dispatch).
static int scratch_allowance() {
  size_t stack = 0;
  if (hipDeviceGetLimit(&stack, hipLimitStackSize) != hipSuccess) return 0;
  return (int)std::min<size_t>(stack, (size_t)kMaxScratchPerLane);
}
static constexpr size_t kLdsBudget = 160 * 1024 - 1024;

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
  if (c->norm != NSFRB_NORM_PIXEL_SUBBAND && c->norm != NSFRB_NORM_EXTERNAL && c->norm != NSFRB_NORM_NONE)
    return fail(NSFRB_ERR_INVALID_ARG, "unknown normalisation mode");
  if (c->layout != NSFRB_LAYOUT_TSP && c->layout != NSFRB_LAYOUT_PST) return fail(NSFRB_ERR_INVALID_ARG, "unknown layout");
  if (c->layout == NSFRB_LAYOUT_PST && (c->norm != NSFRB_NORM_NONE || c->in_dtype != c->store_dtype))
    return fail(NSFRB_ERR_INVALID_ARG, "NSFRB_LAYOUT_PST needs NSFRB_NORM_NONE and in_dtype == store_dtype");
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
struct KernelClass {
  int C;     // samples per lane
  int PIX;   // pixels per workgroup
  int NW;    // waves per workgroup (8 or 16)
};
std::string single_kernel_name(const KernelClass& k);
// Samples per lane: odd, so 64 lanes reading rows at a common delay hit
// distinct LDS banks; 64*C > n_time, so every series ends in padding.
// Samples per lane C: 64 C > n_time, so every series has a -inf padding sample.
// FP32 rows are read one sample per register and C is odd: lanes C samples
// apart hit distinct LDS banks. FP16 rows are read two samples per dword and C
// is even with C/2 odd: every lane then starts on the same half of a dword (the
// parity of the delay) and lanes C/2 dwords apart hit distinct banks.
// DM-trial grid from a smearing tolerance (see nsfrb.h): with A = 4.15 ms *
// (nu_min^-2 - nu_max^-2), B = 0.0083 ms * dnu * nu_min^-3, C^2 = W_int^2 + t_s^2
// and q = tol^2 - 1, the half spacing h after trial D solves
// A^2 h^2 = q (C^2 + B^2 (D + h)^2), a quadratic with one positive root.
extern "C" nsfrb_status nsfrb_plan_dm_grid(double nu_min_ghz, double nu_max_ghz, double chan_bw_mhz, double t_s_ms,
                                           double w_int_ms, double tol, double dm_min, double dm_max,
                                           double* host_out, int32_t capacity, int32_t* n_out) {
  g_last_error.clear();
  const double v[] = {nu_min_ghz, nu_max_ghz, chan_bw_mhz, t_s_ms, w_int_ms, tol, dm_min, dm_max};
  for (double x : v)
    if (!std::isfinite(x)) return fail(NSFRB_ERR_INVALID_ARG, "every parameter must be finite");
  if (!(nu_min_ghz > 0.0 && nu_max_ghz > nu_min_ghz))
    return fail(NSFRB_ERR_INVALID_ARG, "need 0 < nu_min < nu_max");
  if (!(chan_bw_mhz >= 0.0 && t_s_ms > 0.0 && w_int_ms >= 0.0 && tol > 1.0))
    return fail(NSFRB_ERR_INVALID_ARG, "need chan_bw >= 0, t_s > 0, w_int >= 0 and tol > 1");
  if (!(dm_min >= 0.0 && dm_max >= dm_min)) return fail(NSFRB_ERR_INVALID_ARG, "need 0 <= dm_min <= dm_max");
  if (capacity < 0 || (capacity > 0 && !host_out) || !n_out) return fail(NSFRB_ERR_INVALID_ARG, "bad output buffer");
  const double A = 4.15 * (1.0 / (nu_min_ghz * nu_min_ghz) - 1.0 / (nu_max_ghz * nu_max_ghz));
  const double B = 0.0083 * chan_bw_mhz / (nu_min_ghz * nu_min_ghz * nu_min_ghz);
  const double C2 = w_int_ms * w_int_ms + t_s_ms * t_s_ms;
  const double q = tol * tol - 1.0;
  const double a2 = A * A - q * B * B;
  if (!(a2 > 0.0))
    return fail(NSFRB_ERR_UNSUPPORTED, "tolerance unattainable: channel smearing grows as fast as the residual delay");
  constexpr int kMaxTrials = 1 << 20;
  int n = 0;
  double d = dm_min;
  for (;;) {
    if (n < capacity) host_out[n] = d;
    ++n;
    if (d >= dm_max) break;
    if (n >= kMaxTrials) return fail(NSFRB_ERR_UNSUPPORTED, "more than 2^20 trials");
    const double bd = q * B * B * d;
    const double h = (bd + std::sqrt(bd * bd + a2 * q * (C2 + B * B * d * d))) / a2;
    d += 2.0 * h;
  }
  *n_out = n;
  if (n > capacity) return fail(NSFRB_ERR_TRUNCATED, "capacity below the number of trials");
  return NSFRB_OK;
}

static int samples_per_lane(int n_time, int store) {
  int c = (n_time + 64) / 64;
  if (store == NSFRB_F16) {
    if (c & 1) c += 1;
    if (((c / 2) & 1) == 0) c += 2;
  } else if ((c & 1) == 0) {
    c += 1;
  }
  return c;
}
// Row length in samples: 64 C + the largest searched delay + 1 (whole dwords for FP16).
static int row_len(int C, int dmax_search, int store) {
  const int rs = 64 * C + dmax_search + 1;
  return store == NSFRB_F32 ? rs : (rs + 1) & ~1;      // 16-bit rows start on a dword
}
static size_t lds_bytes_for(int pix, int n_sub, int rs, int store) {
  return (size_t)pix * n_sub * rs * dtype_size(store);
}

// Emit the boxcar plan: power-of-two levels by pairwise doubling, other
// widths as sums of the level windows of their binary digits. A width that
// is not a power of two needs an accumulator from its lowest to its highest
// binary digit; widths are split into passes so that at most max_acc
// (<= kMaxAccumulators) accumulators are open at any level of a pass (each
// extra pass re-forms the de-dispersed series). Power-of-two widths go in pass 0.
static nsfrb_status gen_chain(const std::vector<int>& widths, std::string& out, int* npass_out = nullptr,
                              int max_acc = kMaxAccumulators) {
  const int nw = (int)widths.size();
  struct Acc { int iw, w, lo, hi, pass, slot, off; };
  std::vector<Acc> accs;
  for (int iw = 0; iw < nw; ++iw) {
    const int w = widths[iw];
    if ((w & (w - 1)) == 0) continue;
    const int lo = __builtin_ctz((unsigned)w), hi = 31 - __builtin_clz((unsigned)w);
    accs.push_back({iw, w, lo, hi, -1, -1, 0});
  }
  std::sort(accs.begin(), accs.end(), [](const Acc& x, const Acc& y) { return x.lo < y.lo || (x.lo == y.lo && x.hi < y.hi); });
  // passes[p][slot] = last level the slot is busy through
  std::vector<std::vector<int>> passes(1);
  for (auto& a : accs) {
    for (int p = 0; p < (int)passes.size() && a.pass < 0; ++p) {
      for (int s = 0; s < (int)passes[p].size(); ++s)
        if (passes[p][s] < a.lo) { a.pass = p; a.slot = s; passes[p][s] = a.hi; break; }
      if (a.pass < 0 && (int)passes[p].size() < max_acc) {
        a.pass = p; a.slot = (int)passes[p].size(); passes[p].push_back(a.hi);
      }
    }
    if (a.pass < 0) { passes.push_back({a.hi}); a.pass = (int)passes.size() - 1; a.slot = 0; }
  }
  const int npass = (int)passes.size();
  std::ostringstream o;
  o << "template <int C, class R>\n__device__ __forceinline__ void nsfrb_chain(int pass, float (&a0)[C], R& rep) {\n";
  o << "  using namespace nsfrb;\n  float a1[C];\n";
  for (int s = 0; s < max_acc; ++s) o << "  float acc" << s << "[C];\n";
  o << "  switch (pass) {\n";
  for (int p = 0; p < npass; ++p) {
    int maxb = 0;
    for (int iw = 0; iw < nw; ++iw) {
      if (p == 0 && (widths[iw] & (widths[iw] - 1)) == 0) maxb = std::max(maxb, __builtin_ctz((unsigned)widths[iw]));
    }
    for (auto& a : accs)
      if (a.pass == p) maxb = std::max(maxb, a.hi);
    o << "  case " << p << ": {\n";
    for (int b = 0; b <= maxb; ++b) {
      const char* cur = (b & 1) ? "a1" : "a0";
      const char* nxt = (b & 1) ? "a0" : "a1";
      o << "    // level " << b << ": windows of " << (1 << b) << " samples in " << cur << "\n";
      if (p == 0)
        for (int iw = 0; iw < nw; ++iw)
          if (widths[iw] == (1 << b)) o << "    rep(" << iw << ", " << cur << ");\n";
      for (auto& a : accs) {
        if (a.pass != p || !((a.w >> b) & 1)) continue;
        if (b == a.lo) o << "    copy_arr(acc" << a.slot << ", " << cur << ");\n";
        else o << "    shift_add<" << a.off << ">(acc" << a.slot << ", acc" << a.slot << ", " << cur << ");\n";
        a.off += 1 << b;
        if (b == a.hi) o << "    rep(" << a.iw << ", acc" << a.slot << ");\n";
      }
      if (b < maxb) o << "    shift_add<" << (1 << b) << ">(" << nxt << ", " << cur << ", " << cur << ");\n";
    }
    o << "  } break;\n";
  }
  o << "  default: break;\n  }\n}\n";
  out = o.str();
  if (npass_out) *npass_out = npass;
  return NSFRB_OK;
}

static const char* store_type_name(int store) {
  return store == DT_F32 ? "float" : (store == DT_F16 ? "_Float16" : "nsfrb::bf16_t");
}

// A persistent kernel to instantiate: samples per lane, waves, LDS buffers.
struct PersistentKernel {
  int C, NW, n_buf;
};
// A persistent batch kernel: samples per lane, waves, LDS buffers, pixels per item.
struct BatchKernel {
  int C, NW, n_buf, pix;
};
// Translation unit with the per-DM kernels of `single` (C, PIX, NW), the
// persistent single-cube kernels, and one persistent batch kernel per entry of
// `batch`.
static std::string gen_source(int store, int nw, int npass, const std::string& chain,
                              const std::vector<KernelClass>& single, const std::vector<BatchKernel>& batch,
                              const std::vector<PersistentKernel>& persistent = {}) {
  std::ostringstream o;
  o << "#define NSFRB_RTC_PROLOGUE 1\n#include \"device_common.h\"\n";
  o << "#define NSFRB_NPASS " << npass << "\n";
  o << "typedef " << store_type_name(store) << " ST;\n";
  o << "#define NSFRB_NW " << nw << "\n";
  o << "#include \"k_search_body.h\"\n";
  o << chain;
  for (const auto& k : single)
    o << "extern \"C\" __global__ __launch_bounds__(" << 64 * k.NW << ") void " << single_kernel_name(k)
      << "(nsfrb::CubeDesc cd) { search_cube<" << k.C << ", " << k.PIX << ", " << k.NW << ">(cd); }\n";
  for (const auto& k : persistent)
    o << "extern \"C\" __global__ __launch_bounds__(" << 64 * k.NW << ") void nsfrb_persistent_c" << k.C << "_w"
      << k.NW << "_b" << k.n_buf
      << "(nsfrb::CubeDesc cd, const int* __restrict__ delays, const int* __restrict__ dmax) { "
         "nsfrb::search_persistent<" << k.C << ", " << k.NW << ", " << k.n_buf << ">(cd, delays, dmax); }\n";
  // one persistent kernel per class of the batch
  for (size_t i = 0; i < batch.size(); ++i)
    o << "extern \"C\" __global__ __launch_bounds__(" << 64 * batch[i].NW << ") void nsfrb_batch_kernel_" << i
      << "(const nsfrb::CubeDesc* __restrict__ descs, int n_cubes, long long n_items, int buf_stride) {\n"
         "  nsfrb::search_batch_persistent<" << batch[i].C << ", " << batch[i].NW << ", " << batch[i].n_buf << ", "
      << batch[i].pix << ">(descs, n_cubes, n_items, buf_stride);\n}\n";
  return o.str();
}

std::string single_kernel_name(const KernelClass& k) {
  return "nsfrb_search_c" + std::to_string(k.C) + "_p" + std::to_string(k.PIX) + "_w" + std::to_string(k.NW);
}

// Compiled modules, shared by every handle on a device.
struct CompiledModule {
  hipModule_t mod = nullptr;
};
static std::mutex g_rtc_mu;
static std::map<std::pair<int, std::string>, CompiledModule> g_rtc_cache;

static const char* kRtcOpts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-fno-honor-nans", "-mno-amdgpu-ieee",
                                 "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};

static nsfrb_status rtc_compile(const std::string& src, std::vector<char>& code) {
  hiprtcProgram prog;
  const char* hdr_names[] = {"device_common.h", "k_search_body.h"};
  const char* hdr_src[] = {kRtcDeviceCommon, kRtcSearchBody};
  if (hiprtcCreateProgram(&prog, src.c_str(), "nsfrb_search.hip", 2, hdr_src, hdr_names) != HIPRTC_SUCCESS)
    return fail(NSFRB_ERR_DEVICE, "hiprtcCreateProgram failed");
  hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof(kRtcOpts) / sizeof(kRtcOpts[0])), kRtcOpts);
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
  code.resize(sz);
  hiprtcGetCode(prog, code.data());
  hiprtcDestroyProgram(&prog);
  const char* dump = std::getenv("NSFRB_DUMP_CODE");
  if (dump && *dump) {
    FILE* f = std::fopen(dump, "wb");
    if (f) { std::fwrite(code.data(), 1, code.size(), f); std::fclose(f); }
  }
  return NSFRB_OK;
}

nsfrb_status load_module(int device, const std::string& src, hipModule_t* mod) {
  std::lock_guard<std::mutex> lk(g_rtc_mu);
  auto key = std::make_pair(device, src);
  auto it = g_rtc_cache.find(key);
  if (it != g_rtc_cache.end()) { *mod = it->second.mod; return NSFRB_OK; }
  std::vector<char> code;
  nsfrb_status st = rtc_compile(src, code);
  if (st != NSFRB_OK) return st;
  CompiledModule cm;
  HIP_TRY(hipModuleLoadData(&cm.mod, code.data()));
  g_rtc_cache[key] = cm;
  *mod = cm.mod;
  return NSFRB_OK;
}

static int max_delay_searchable(const std::vector<int32_t>& delays, int n_dm, int n_sub, int n_time,
                                std::vector<int32_t>* dmaxv) {
  int dmax_search = 0;
  if (dmaxv) dmaxv->assign(n_dm, 0);
  for (int d = 0; d < n_dm; ++d) {
    int m = 0;
    for (int s = 0; s < n_sub; ++s) m = std::max(m, (int)delays[(size_t)d * n_sub + s]);
    if (dmaxv) (*dmaxv)[d] = m;
    if (m < n_time) dmax_search = std::max(dmax_search, m);
  }
  return dmax_search;
}

// Kernel shapes that fit in LDS, best first by the default heuristic (enough
// waves per pixel to cover the DM trials): PIX pixels per workgroup of 8
// waves, and one or two pixels per workgroup of 16 waves. A single large
// workgroup may take most of a CU's LDS, so 16 waves of one workgroup reach an
// occupancy that two 8-wave workgroups with that much LDS do not.
static std::vector<KernelClass> plan_candidates(int C, int n_dm, int n_sub, int rs, int store) {
  std::vector<KernelClass> out;
  for (int pix : {1, 2, 4, 8})
    if (lds_bytes_for(pix, n_sub, rs, store) <= kLdsBudget) out.push_back({C, pix, 8});
  std::sort(out.begin(), out.end(), [&](const KernelClass& a, const KernelClass& b) {
    const int wa = 8 / a.PIX, wb = 8 / b.PIX;     // waves per pixel
    const bool fa = wa <= n_dm, fb = wb <= n_dm;  // no idle waves
    if (fa != fb) return fa;
    return fa ? a.PIX < b.PIX : a.PIX > b.PIX;
  });
  for (int pix : {1, 2})
    if (lds_bytes_for(pix, n_sub, rs, store) <= kLdsBudget && 16 / pix <= n_dm) out.push_back({C, pix, 16});
  return out;
}

// ------------------------------------------------ persistent kernel plans
// The persistent kernel keeps one pixel per workgroup of NW waves (DM trials
// round-robin, as the per-DM kernel) and walks its pixels (ItemWalk);
// the next pixel's rows are requested with global-to-LDS loads while the
// current one is searched. Rows are whole 16-byte vectors (n_t * store bytes a
// multiple of 16, pitch padded to 16 bytes), in one or two LDS buffers.
struct PersistentPlan {
  int NW = 16, rs = 0, n_buf = 1;
  size_t lds = 0;
};

// LDS buffers for a persistent kernel of nw waves with a tile of `tile` bytes:
// two (the next pixel's rows load during the whole current pixel) unless that
// leaves fewer workgroups on a CU than one buffer does, counting at most the 16
// waves per CU that a search kernel's register use allows; 0 if no tile fits.
static int persistent_buffers(size_t tile, int nw) {
  if (tile > kLdsBudget) return 0;
  if (2 * tile > kLdsBudget) return 1;
  auto wgs = [&](size_t nb) { return (int)((160 * 1024) / (nb * tile + 1024)); };
  return wgs(2) >= std::min(wgs(1), std::max(1, 16 / nw)) ? 2 : 1;
}

static bool plan_persistent(int n_sub, int n_t, int C, int dmax_search, int store, int NW, PersistentPlan& out) {
  out = PersistentPlan{};
  out.NW = NW;
  if (((size_t)n_t * dtype_size(store)) % 16 != 0) return false;
  const int align = store == DT_F32 ? 4 : 8;
  out.rs = (64 * C + dmax_search + 1 + align - 1) / align * align;
  const size_t tile = (size_t)n_sub * out.rs * dtype_size(store);
  out.n_buf = persistent_buffers(tile, NW);
  out.lds = out.n_buf * tile;
  return out.n_buf > 0;
}

// 16 waves when there are at least 16 DM trials, and 8.
static std::vector<PersistentPlan> persistent_candidates(int n_dm, int n_sub, int n_t, int C, int dmax_search,
                                                         int store) {
  std::vector<PersistentPlan> out;
  for (int NW : {16, 8}) {
    PersistentPlan pp;
    if ((NW == 8 || n_dm >= NW) && plan_persistent(n_sub, n_t, C, dmax_search, store, NW, pp)) out.push_back(pp);
  }
  return out;
}

static std::string persistent_kernel_name(int C, const PersistentPlan& pp) {
  return "nsfrb_persistent_c" + std::to_string(C) + "_w" + std::to_string(pp.NW) + "_b" + std::to_string(pp.n_buf);
}

// Host-only entry: generate (and optionally compile) the specialised search
// source, for build checks and inspection. Not part of the public header.
extern "C" int nsfrb_debug_plan_source(const nsfrb_search_config* cfg, char* out, int cap, int compile) {
  if (validate(cfg) != NSFRB_OK) return -1;
  std::vector<int32_t> dl;
  compute_delays(*cfg, dl);
  const int dmax_search = max_delay_searchable(dl, cfg->n_dm, cfg->n_sub, cfg->n_time, nullptr);
  const int C = samples_per_lane(cfg->n_time, cfg->store_dtype);
  const int rs = row_len(C, dmax_search, cfg->store_dtype);
  std::vector<KernelClass> ks = plan_candidates(C, cfg->n_dm, cfg->n_sub, rs, cfg->store_dtype);
  if (ks.empty()) {
    fail(NSFRB_ERR_UNSUPPORTED, "a pixel's rows do not fit in LDS");
    return -1;
  }
  std::string chain;
  int npass = 1;
  // NSFRB_DEBUG_MAX_ACC=n emits the plan with at most n accumulators per pass (inspection of register use)
  int max_acc = kMaxAccumulators;
  if (const char* e = std::getenv("NSFRB_DEBUG_MAX_ACC")) max_acc = std::max(1, std::min(kMaxAccumulators, std::atoi(e)));
  if (gen_chain(std::vector<int>(cfg->width, cfg->width + cfg->n_width), chain, &npass, max_acc) != NSFRB_OK)
    return -1;
  std::vector<PersistentKernel> pks;
  std::vector<BatchKernel> bks;          // batch kernels of the same shapes, one and two pixels per item
  for (const PersistentPlan& pp : persistent_candidates(cfg->n_dm, cfg->n_sub, cfg->n_time, C, dmax_search,
                                                        cfg->store_dtype)) {
    pks.push_back({C, pp.NW, pp.n_buf});
    bks.push_back({C, pp.NW, pp.n_buf, 1});
    bks.push_back({C, pp.NW, 1, 2});
  }
  const std::string src = gen_source(cfg->store_dtype, cfg->n_width, npass, chain, ks, bks, pks);
  if (out && cap > 0) std::snprintf(out, (size_t)cap, "%s", src.c_str());
  if (compile) {
    std::vector<char> code;
    if (rtc_compile(src, code) != NSFRB_OK) return -2;
  }
  return (int)src.size();
}

// ------------------------------------------------------------------ handle
struct nsfrb_search {
  nsfrb_search_config cfg{};
  std::vector<double> freqs, dms;
  std::vector<int32_t> widths, delays, dmaxv;
  int n_pix = 0, device = 0;
  int C = 0, rs = 0, pix = 1, nw = 8;  // chosen kernel class and LDS row length
  int dmax_search = 0;                 // largest delay of a searchable trial
  int max_acc = kMaxAccumulators;      // accumulators per pass of the boxcar plan (no register spills)
  std::vector<KernelClass> cands;      // per-DM shapes that fit LDS
  bool planned = false;                // kernels compiled and tuned (a batch's cubes plan on first separate run)
  size_t lds_bytes = 0;
  std::string source;                  // generated search translation unit
  hipModule_t mod = nullptr;
  hipFunction_t search_fn = nullptr;
  std::vector<KernelClass> tuned;      // candidates timed by the autotuner
  std::vector<float> tuned_ms;
  // persistent kernels that compiled without spills, their persistent grids and
  // tuned times; `pers` is the one in use (-1: the per-DM kernel above)
  std::vector<PersistentPlan> pers_plans;
  std::vector<hipFunction_t> pers_fns;
  std::vector<unsigned> pers_grids;
  std::vector<float> pers_ms;
  int pers = -1;
  int32_t* d_delays_zeroed = nullptr;  // delays with zero rows for trials that have no valid sample
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
  const void* last_z = nullptr;        // normalised cube searched by the last run
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
  if (h->d_delays_zeroed) hipFree(h->d_delays_zeroed);
  if (h->h_cands) hipHostFree(h->h_cands);
  if (h->h_nout) hipHostFree(h->h_nout);
  if (h->done) hipEventDestroy(h->done);
  for (auto& e : h->ev)
    if (e) hipEventDestroy(e);
  delete h;
}

static nsfrb_status autotune(nsfrb_search* h, const std::vector<KernelClass>& ks);

// Compiles the handle's kernels (dropping shapes that would spill), sizes the
// persistent grids and runs the autotuner.
static nsfrb_status plan_kernels(nsfrb_search* h) {
  const nsfrb_search_config* cfg = &h->cfg;
  nsfrb_status st = NSFRB_OK;
  HIP_TRY(hipSetDevice(h->device));
  // Only kernels that keep the boxcar chain in registers (up to a few dozen
  // bytes of spill) are ever launched: each compiled candidate's scratch use is
  // queried and a heavily spilling one is dropped. If every shape spills, the
  // plan is regenerated with fewer accumulators per pass (more passes, each
  // re-forming the de-dispersed series) before the configuration is refused.
  const int allowance = scratch_allowance();
  std::vector<KernelClass> usable;
  // NSFRB_PERSISTENT: "0" per-DM kernel only; "NW" only the persistent kernel of NW waves (studies)
  const char* pers_env = std::getenv("NSFRB_PERSISTENT");
  const int pers_only = pers_env ? std::atoi(pers_env) : -1;
  for (int max_acc = kMaxAccumulators; max_acc >= 1 && usable.empty(); --max_acc) {
    std::string chain;
    int npass = 1;
    st = gen_chain(h->widths, chain, &npass, max_acc);
    if (st != NSFRB_OK) return st;
    std::vector<PersistentPlan> pps;
    if (pers_only != 0)
      for (const PersistentPlan& pp : persistent_candidates(cfg->n_dm, cfg->n_sub, cfg->n_time, h->C, h->dmax_search,
                                                            cfg->store_dtype))
        if (pers_only < 0 || pp.NW == pers_only) pps.push_back(pp);
    std::vector<PersistentKernel> pks;
    for (const PersistentPlan& pp : pps) pks.push_back({h->C, pp.NW, pp.n_buf});
    h->source = gen_source(cfg->store_dtype, cfg->n_width, npass, chain, h->cands, {}, pks);
    st = load_module(h->device, h->source, &h->mod);
    if (st != NSFRB_OK) return st;
    for (const KernelClass& k : h->cands) {
      hipFunction_t fn = nullptr;
      HIP_TRY(hipModuleGetFunction(&fn, h->mod, single_kernel_name(k).c_str()));
      int scratch = 0;
      HIP_TRY(hipFuncGetAttribute(&scratch, HIP_FUNC_ATTRIBUTE_LOCAL_SIZE_BYTES, fn));
      if (scratch <= allowance) usable.push_back(k);
    }
    h->pers_plans.clear();
    h->pers_fns.clear();
    for (const PersistentPlan& pp : pps) {
      hipFunction_t fn = nullptr;
      HIP_TRY(hipModuleGetFunction(&fn, h->mod, persistent_kernel_name(h->C, pp).c_str()));
      int scratch = 0;
      HIP_TRY(hipFuncGetAttribute(&scratch, HIP_FUNC_ATTRIBUTE_LOCAL_SIZE_BYTES, fn));
      if (scratch > 0) continue;   // a spill reload would wait for the row requests in flight
      h->pers_plans.push_back(pp);
      h->pers_fns.push_back(fn);
    }
    h->max_acc = max_acc;
  }
  if (usable.empty())
    return fail(NSFRB_ERR_UNSUPPORTED, "every kernel shape for " + std::to_string(h->C) +
                                           " samples per lane and these widths would spill more than " +
                                           std::to_string(allowance) +
                                           " bytes of registers per lane (n_time too long for the width list)");
  int n_cu = 0;
  HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, h->device));
  h->pers_grids.clear();
  for (size_t i = 0; i < h->pers_plans.size(); ++i) {
    int per_cu = 0;
    HIP_TRY(hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, h->pers_fns[i], 64 * h->pers_plans[i].NW,
                                                               h->pers_plans[i].lds));
    h->pers_grids.push_back((unsigned)(std::max(1, n_cu) * std::max(1, per_cu)));
  }
  st = autotune(h, usable);
  if (st != NSFRB_OK) return st;
  h->lds_bytes = lds_bytes_for(h->pix, cfg->n_sub, h->rs, cfg->store_dtype);
  h->planned = true;
  return NSFRB_OK;
}

// A handle with its buffers; its kernels are planned now or (plan_now false,
// for a batch's cubes) before its first separate launch.
static nsfrb_status search_create(const nsfrb_search_config* cfg, bool plan_now, nsfrb_search** out) {
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
  h->dmax_search = max_delay_searchable(h->delays, cfg->n_dm, cfg->n_sub, cfg->n_time, &h->dmaxv);
  h->C = samples_per_lane(cfg->n_time, cfg->store_dtype);
  h->rs = row_len(h->C, h->dmax_search, cfg->store_dtype);
  h->cands = plan_candidates(h->C, cfg->n_dm, cfg->n_sub, h->rs, cfg->store_dtype);
  if (h->cands.empty())
    return fail(NSFRB_ERR_UNSUPPORTED, "n_sub x (padded n_time + max delay) does not fit in LDS for this store dtype");
  const char* force = std::getenv("NSFRB_FORCE_ALLOC_FAIL");
  if (force && std::atoi(force) != 0) return fail(NSFRB_ERR_OUT_OF_MEMORY, "allocation failure forced by NSFRB_FORCE_ALLOC_FAIL");

  HIP_TRY(hipSetDevice(h->device));
  const size_t n_pix = (size_t)h->n_pix, ns = (size_t)cfg->n_sub, nt = (size_t)cfg->n_time;
  const size_t nmaps = (size_t)cfg->n_dm * cfg->n_width * n_pix;
  HIP_TRY(dalloc(&h->d_delays, h->delays.size()));
  HIP_TRY(dalloc(&h->d_dmax, h->dmaxv.size()));
  HIP_TRY(dalloc(&h->d_norms, (size_t)cfg->n_width));
  if (cfg->layout == NSFRB_LAYOUT_TSP) HIP_TRY(hipMalloc(&h->d_z, n_pix * ns * nt * dtype_size(cfg->store_dtype)));
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
  {
    std::vector<int32_t> dz(h->delays);
    for (int d = 0; d < cfg->n_dm; ++d)
      if (h->dmaxv[(size_t)d] >= cfg->n_time)
        std::fill(dz.begin() + (long)d * cfg->n_sub, dz.begin() + (long)(d + 1) * cfg->n_sub, 0);
    HIP_TRY(dalloc(&h->d_delays_zeroed, dz.size()));
    HIP_TRY(hipMemcpy(h->d_delays_zeroed, dz.data(), dz.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  }
  if (plan_now) {
    st = plan_kernels(h.get());
    if (st != NSFRB_OK) return st;
  }
  *out = h.release();
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_search_create(const nsfrb_search_config* cfg, nsfrb_search** out) {
  g_last_error.clear();
  return search_create(cfg, true, out);
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

static CubeDescHost cube_desc(const nsfrb_search* h, const void* z, int n_pix) {
  const nsfrb_search_config& c = h->cfg;
  CubeDescHost d{};
  d.z = z;
  d.delays = h->d_delays;
  d.dmax = h->d_dmax;
  d.norms = h->d_norms;
  d.snr_max = h->d_snr;
  d.toa = h->d_toa;
  d.best_s = h->d_best_s;
  d.best_d = h->d_best_d;
  d.best_w = h->d_best_w;
  d.best_t = h->d_best_t;
  d.n_pix = n_pix;
  d.n_sub = c.n_sub;
  d.n_t = c.n_time;
  d.n_dm = c.n_dm;
  d.rs = h->rs;
  d.dma_w = 0;
  d.item_begin = 0;
  return d;
}

static nsfrb_status launch_search_fn(const nsfrb_search* h, hipFunction_t fn, const KernelClass& k, const void* z,
                                     int n_pix, hipStream_t st) {
  CubeDescHost d = cube_desc(h, z, n_pix);
  void* args[] = {(void*)&d};
  const unsigned n_items = (unsigned)((n_pix + k.PIX - 1) / k.PIX);
  const size_t lds = lds_bytes_for(k.PIX, h->cfg.n_sub, h->rs, h->cfg.store_dtype);
  HIP_TRY(hipModuleLaunchKernel(fn, n_items, 1, 1, 64 * k.NW, 1, 1, (unsigned)lds, st, args, nullptr));
  return NSFRB_OK;
}

static nsfrb_status launch_persistent(const nsfrb_search* h, size_t i, const void* z, int n_pix, hipStream_t st) {
  const PersistentPlan& pp = h->pers_plans[i];
  CubeDescHost d = cube_desc(h, z, n_pix);
  d.rs = pp.rs;
  const int32_t* delays = h->d_delays_zeroed;
  const int32_t* dmax = h->d_dmax;
  void* args[] = {(void*)&d, (void*)&delays, (void*)&dmax};
  const unsigned grid = (unsigned)std::min<long long>(h->pers_grids[i], std::max(1, n_pix));
  HIP_TRY(hipModuleLaunchKernel(h->pers_fns[i], grid, 1, 1, 64 * pp.NW, 1, 1, (unsigned)pp.lds, st, args, nullptr));
  return NSFRB_OK;
}

// The per-DM kernel the autotuner chose (the batch's separate launches use it too).
static nsfrb_status launch_search_per_dm(const nsfrb_search* h, const void* z, hipStream_t st) {
  return launch_search_fn(h, h->search_fn, {h->C, h->pix, h->nw}, z, h->n_pix, st);
}

static nsfrb_status launch_search(const nsfrb_search* h, const void* z, hipStream_t st) {
  // the persistent kernel stages with global-to-LDS loads, which need a 16-byte aligned cube
  if (h->pers >= 0 && (reinterpret_cast<uintptr_t>(z) & 15u) == 0)
    return launch_persistent(h, (size_t)h->pers, z, h->n_pix, st);
  return launch_search_per_dm(h, z, st);
}

// Autotuner: time every per-DM candidate (pixels and waves per workgroup) and
// every persistent candidate (waves per workgroup) on this plan's shape (the
// normalised-cube buffer, zeroed) and keep the fastest; all give bitwise equal
// results. Choices are cached per shape for the process. NSFRB_AUTOTUNE=0
// keeps the heuristic first per-DM candidate.
struct TuneKey {
  int C, n_sub, n_t, n_dm, n_pix_bucket, store;
  std::vector<int32_t> widths;
  std::vector<int32_t> pers;    // the persistent candidates' waves
  bool operator<(const TuneKey& o) const {
    return std::tie(C, n_sub, n_t, n_dm, n_pix_bucket, store, widths, pers) <
           std::tie(o.C, o.n_sub, o.n_t, o.n_dm, o.n_pix_bucket, o.store, o.widths, o.pers);
  }
};
struct TuneChoice {
  int pix, nw, pers;      // pers: index of the persistent candidate used, -1 for the per-DM kernel
};
static std::mutex g_tune_mu;
static std::map<TuneKey, TuneChoice> g_tune_cache;

static nsfrb_status autotune(nsfrb_search* h, const std::vector<KernelClass>& ks) {
  const nsfrb_search_config& c = h->cfg;
  std::vector<hipFunction_t> fns(ks.size());
  for (size_t i = 0; i < ks.size(); ++i)
    HIP_TRY(hipModuleGetFunction(&fns[i], h->mod, single_kernel_name(ks[i]).c_str()));
  auto choose = [&](size_t i) { h->pix = ks[i].PIX; h->nw = ks[i].NW; h->search_fn = fns[i]; };
  auto choose_pers = [&](int i) { h->pers = (i >= 0 && i < (int)h->pers_plans.size()) ? i : -1; };
  choose(0);
  h->pers = -1;
  // NSFRB_PLAN="pixels,waves" picks that per-DM shape when it is a candidate (for tuning studies)
  if (const char* plan = std::getenv("NSFRB_PLAN")) {
    int pp = 0, ww = 0;
    if (std::sscanf(plan, "%d,%d", &pp, &ww) == 2)
      for (size_t i = 0; i < ks.size(); ++i)
        if (ks[i].PIX == pp && ks[i].NW == ww) { choose(i); return NSFRB_OK; }
  }
  // NSFRB_PERSISTENT=NW (NW > 0) keeps that persistent kernel (for studies)
  if (const char* pe = std::getenv("NSFRB_PERSISTENT"))
    if (std::atoi(pe) > 0 && !h->pers_plans.empty()) { h->pers = 0; return NSFRB_OK; }
  const char* env = std::getenv("NSFRB_AUTOTUNE");
  if ((ks.size() == 1 && h->pers_plans.empty()) || (env && std::atoi(env) == 0)) return NSFRB_OK;
  int bucket = 0;
  while ((1 << bucket) < h->n_pix) ++bucket;
  TuneKey key{h->C, c.n_sub, c.n_time, c.n_dm, bucket > 13 ? 13 : bucket, c.store_dtype, h->widths, {}};
  for (const PersistentPlan& pp : h->pers_plans) key.pers.push_back(pp.NW);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      for (size_t i = 0; i < ks.size(); ++i)
        if (ks[i].PIX == it->second.pix && ks[i].NW == it->second.nw) choose(i);
      choose_pers(it->second.pers);
      return NSFRB_OK;
    }
  }
  // time on up to 8192 pixels of a zeroed scratch cube (the cost per pixel does not depend on the data)
  const int n_tune = h->n_pix < 8192 ? h->n_pix : 8192;
  const size_t zbytes = (size_t)n_tune * c.n_sub * c.n_time * dtype_size(c.store_dtype);
  void* zt = nullptr;
  HIP_TRY(hipMalloc(&zt, zbytes));
  std::unique_ptr<void, hipError_t (*)(void*)> zt_guard(zt, hipFree);
  HIP_TRY(hipMemset(zt, 0, zbytes));
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  // candidates are timed in interleaved rounds and each keeps its best round, so
  // clock ramp-up after an idle spell (e.g. the plan compile) favours none of them
  const size_t n_all = ks.size() + h->pers_plans.size();
  auto launch = [&](size_t i) {
    return i < ks.size() ? launch_search_fn(h, fns[i], ks[i], zt, n_tune, nullptr)
                         : launch_persistent(h, i - ks.size(), zt, n_tune, nullptr);
  };
  std::vector<float> ms_best(n_all, 1e30f);
  for (int round = 0; round < 3; ++round) {
    for (size_t i = 0; i < n_all; ++i) {
      nsfrb_status st = launch(i);   // warm-up
      if (st != NSFRB_OK) return st;
      HIP_TRY(hipEventRecord(e0, nullptr));
      for (int r = 0; r < 2; ++r) {
        st = launch(i);
        if (st != NSFRB_OK) return st;
      }
      HIP_TRY(hipEventRecord(e1, nullptr));
      HIP_TRY(hipEventSynchronize(e1));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      ms_best[i] = std::min(ms_best[i], ms / 2.f);
    }
  }
  float best_ms = 1e30f;
  for (size_t i = 0; i < ks.size(); ++i) {
    h->tuned.push_back(ks[i]);
    h->tuned_ms.push_back(ms_best[i]);
    if (ms_best[i] < best_ms) { best_ms = ms_best[i]; choose(i); }
  }
  h->pers_ms.assign(ms_best.begin() + (long)ks.size(), ms_best.end());
  for (size_t i = 0; i < h->pers_plans.size(); ++i)
    if (h->pers_ms[i] < best_ms) { best_ms = h->pers_ms[i]; h->pers = (int)i; }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache[key] = {h->pix, h->nw, h->pers};
  return NSFRB_OK;
}

static nsfrb_status run_impl(nsfrb_search* h, const void* d_cube, int t_start, void* stream);

extern "C" nsfrb_status nsfrb_search_run(nsfrb_search* h, const void* d_cube, void* stream) {
  g_last_error.clear();
  return run_impl(h, d_cube, 0, stream);
}

// One search; d_cube is a raw TSP cube or, with t_start > 0, a ring of n_time
// samples whose oldest sample is at time index t_start.
static nsfrb_status run_impl(nsfrb_search* h, const void* d_cube, int t_start, void* stream) {
  if (!h || !d_cube) return fail(NSFRB_ERR_INVALID_ARG, "handle and d_cube must be non-NULL");
  if (h->cfg.norm == NSFRB_NORM_EXTERNAL && !h->ext_set)
    return fail(NSFRB_ERR_INVALID_ARG, "EXTERNAL normalisation needs nsfrb_noise_stats_set before run");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(h->device));
  const nsfrb_search_config& c = h->cfg;
  if (h->profiling) HIP_TRY(hipEventRecord(h->ev[0], st));
  const void* z = d_cube;
  if (c.layout == NSFRB_LAYOUT_TSP) {
    StatsLaunch sa{d_cube, c.n_time, c.n_sub, h->n_pix, c.norm, c.in_dtype, c.store_dtype,
                   h->d_ext_med, h->d_ext_sig, h->d_med, h->d_sig, h->d_z, h->d_flags, t_start};
    HIP_TRY(launch_stats(sa, st));
    z = h->d_z;
  } else {
    HIP_TRY(launch_zero_u64(h->d_flags, st));
  }
  h->last_z = z;
  if (h->profiling) HIP_TRY(hipEventRecord(h->ev[1], st));
  nsfrb_status s2 = launch_search(h, z, st);
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
  HIP_TRY(hipMemcpy(host_out, h->last_z, n, hipMemcpyDeviceToHost));
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_zcube_device(nsfrb_search* h, const void** d_z) {
  g_last_error.clear();
  if (!h || !d_z) return fail(NSFRB_ERR_INVALID_ARG, "NULL argument");
  if (!h->last_z) return fail(NSFRB_ERR_NOT_READY, "no run has been enqueued on this handle");
  *d_z = h->last_z;
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

extern "C" nsfrb_status nsfrb_search_plan_info(const nsfrb_search* h, int32_t* info) {
  g_last_error.clear();
  if (!h || !info) return fail(NSFRB_ERR_INVALID_ARG, "NULL argument");
  const bool pe = h->pers >= 0;
  const PersistentPlan* pp = pe ? &h->pers_plans[(size_t)h->pers] : nullptr;
  info[0] = h->C;
  info[1] = pe ? 1 : h->pix;
  info[2] = pe ? pp->rs : h->rs;
  info[3] = (int32_t)(pe ? pp->lds : h->lds_bytes);
  info[4] = 64 * (pe ? pp->NW : h->nw);
  info[5] = pe ? 1 : 0;
  info[6] = pe ? pp->n_buf : 0;
  info[7] = pe ? (int32_t)h->pers_grids[(size_t)h->pers] : 0;
  info[8] = 0;
  return NSFRB_OK;
}

// ------------------------------------------------------------------- batch
// One kernel class of a batch: the cubes whose tuned plan has this (C, PIX).
// One kernel class of a batch: the cubes with the same samples per lane (C) and
// waves per workgroup; one persistent kernel walks all their pixels.
struct BatchClass {
  KernelClass k;                         // C, PIX (pixels per work item), NW
  int n_buf = 1;                         // LDS buffers (PIX tiles each)
  int buf_stride = 0;                    // elements between the buffers (PIX times the class's largest tile)
  hipFunction_t fn = nullptr;
  int first_desc = 0, n_cubes = 0;       // descriptors [first_desc, first_desc + n_cubes)
  long long n_items = 0;
  size_t lds = 0;
  unsigned grid = 0;
};

struct nsfrb_batch {
  std::vector<nsfrb_search*> cubes;
  int device = 0, store = 0, nw = 0;
  std::vector<BatchClass> classes;
  std::vector<CubeDescHost> descs;        // grouped by class; item_begin relative to the class
  std::vector<int> desc_of_cube;          // cube index -> descriptor index
  CubeDescHost* d_descs = nullptr;
  long long n_items = 0;
  hipModule_t mod = nullptr;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<const void*> desc_ptrs;     // cube pointers the device descriptors were written for
  std::vector<const void*> graph_ptrs;    // cube pointers baked into the captured graph (if any)
  bool use_graph = true, last_graph = false, ran = false;
  hipEvent_t done = nullptr;
};

static void batch_release(nsfrb_batch* b) {
  if (!b) return;
  hipSetDevice(b->device);
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  if (b->cap_stream) hipStreamDestroy(b->cap_stream);
  if (b->d_descs) hipFree(b->d_descs);
  if (b->done) hipEventDestroy(b->done);
  for (auto* h : b->cubes) release(h);
  delete b;
}

// Pixels per batch work item (tile: one pixel's LDS rows in bytes): two for
// short series (C <= 18 samples per lane), whose items are short enough that
// the per-item wait for rows and the barriers show; one otherwise, where a
// second pixel's tile would cost a workgroup per CU. Measured per class on the
// 64-cube benchmark batch: two pixels saved 4-10% on C = 6..18 and cost
// 28-50% on C = 22..30. NSFRB_BATCH_PIX = 1, 2 or 4 sets the count (studies);
// never more than fit in LDS.
static int batch_pixels_per_item(int C, int nw, int env, size_t tile) {
  int pix = (env == 1 || env == 2 || env == 4) ? env : (C <= 18 ? 2 : 1);
  pix = std::min(pix, nw);
  while (pix > 1 && (size_t)pix * tile > kLdsBudget) pix >>= 1;
  return pix;
}

extern "C" nsfrb_status nsfrb_batch_create(const nsfrb_search_config* cfgs, int32_t n_cubes, nsfrb_batch** out) {
  g_last_error.clear();
  if (!out || !cfgs || n_cubes < 1) return fail(NSFRB_ERR_INVALID_ARG, "need cfgs, n_cubes >= 1 and out");
  *out = nullptr;
  const nsfrb_search_config& c0 = cfgs[0];
  for (int i = 0; i < n_cubes; ++i) {
    const nsfrb_search_config& c = cfgs[i];
    nsfrb_status st = validate(&c);
    if (st != NSFRB_OK) return fail(st, "cube " + std::to_string(i) + ": " + g_last_error);
    bool same = c.n_dm == c0.n_dm && c.n_width == c0.n_width && c.store_dtype == c0.store_dtype &&
                c.in_dtype == c0.in_dtype && c.norm == c0.norm && c.layout == c0.layout && c.device == c0.device;
    for (int d = 0; same && d < c.n_dm; ++d) same = c.dm[d] == c0.dm[d];
    for (int w = 0; same && w < c.n_width; ++w) same = c.width[w] == c0.width[w];
    if (!same) return fail(NSFRB_ERR_INVALID_ARG, "cube " + std::to_string(i) + " differs in DMs, widths, dtypes, "
                                                  "normalisation, layout or device");
  }
  std::unique_ptr<nsfrb_batch, void (*)(nsfrb_batch*)> b(new nsfrb_batch, batch_release);
  b->device = c0.device;
  b->store = c0.store_dtype;
  b->nw = c0.n_width;
  for (int i = 0; i < n_cubes; ++i) {
    nsfrb_search* h = nullptr;
    nsfrb_status st = search_create(&cfgs[i], false, &h);
    if (st != NSFRB_OK) return fail(st, "cube " + std::to_string(i) + ": " + g_last_error);
    b->cubes.push_back(h);
  }
  // kernel classes: cubes with the same samples per lane; 16 waves when there
  // are at least 16 DM trials (the trials are shared by all cubes), else 8
  const int nw_b = c0.n_dm >= 16 ? 16 : 8;
  int pix_env = 0;
  if (const char* e = std::getenv("NSFRB_BATCH_PIX")) pix_env = std::atoi(e);
  const size_t sz = dtype_size(c0.store_dtype);
  const int align = c0.store_dtype == DT_F32 ? 4 : 8;          // row pitch: whole 16-byte vectors
  std::vector<int> cls_of(b->cubes.size());
  for (size_t i = 0; i < b->cubes.size(); ++i) {
    nsfrb_search* h = b->cubes[i];
    int cls = -1;
    for (size_t k = 0; k < b->classes.size(); ++k)
      if (b->classes[k].k.C == h->C) cls = (int)k;
    if (cls < 0) {
      cls = (int)b->classes.size();
      b->classes.emplace_back();
      b->classes.back().k = {h->C, 1, nw_b};
    }
    cls_of[i] = cls;
  }
  b->desc_of_cube.assign(b->cubes.size(), -1);
  for (size_t c = 0; c < b->classes.size(); ++c) {
    BatchClass& bc = b->classes[c];
    int tile1 = 0;                       // the class's largest one-pixel tile (elements)
    for (size_t i = 0; i < b->cubes.size(); ++i)
      if (cls_of[i] == (int)c)
        tile1 = std::max(tile1, b->cubes[i]->cfg.n_sub * ((b->cubes[i]->rs + align - 1) / align * align));
    bc.k.PIX = batch_pixels_per_item(bc.k.C, nw_b, pix_env, (size_t)tile1 * sz);
    bc.first_desc = (int)b->descs.size();
    for (size_t i = 0; i < b->cubes.size(); ++i) {
      if (cls_of[i] != (int)c) continue;
      nsfrb_search* h = b->cubes[i];
      CubeDescHost d = cube_desc(h, nullptr, h->n_pix);
      d.rs = (h->rs + align - 1) / align * align;
      d.delays = h->d_delays_zeroed;
      d.item_begin = bc.n_items;
      bc.n_items += (h->n_pix + bc.k.PIX - 1) / bc.k.PIX;
      b->desc_of_cube[i] = (int)b->descs.size();
      b->descs.push_back(d);
      bc.buf_stride = std::max(bc.buf_stride, bc.k.PIX * h->cfg.n_sub * d.rs);
    }
    bc.n_cubes = (int)b->descs.size() - bc.first_desc;
    const size_t tile = (size_t)bc.buf_stride * sz;
    bc.n_buf = persistent_buffers(tile, nw_b);
    if (bc.n_buf == 0)
      return fail(NSFRB_ERR_UNSUPPORTED, "a batch cube's rows do not fit in LDS with 16-byte row pitches");
    bc.lds = bc.n_buf * tile;
    b->n_items += bc.n_items;
  }
  // one module with a persistent kernel per class; like a single cube's plan it
  // is regenerated with fewer accumulators per pass while a class kernel would
  // spill more than a search kernel may, and refused only after that
  HIP_TRY(hipSetDevice(b->device));
  int n_cu = 0;
  HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, b->device));
  std::vector<BatchKernel> ks;
  for (const auto& bc : b->classes) ks.push_back({bc.k.C, bc.k.NW, bc.n_buf, bc.k.PIX});
  bool fits = false;
  for (int max_acc = kMaxAccumulators; max_acc >= 1 && !fits; --max_acc) {
    std::string chain;
    int npass = 1;
    nsfrb_status st = gen_chain(b->cubes[0]->widths, chain, &npass, max_acc);
    if (st != NSFRB_OK) return st;
    st = load_module(b->device, gen_source(b->store, b->nw, npass, chain, {}, ks), &b->mod);
    if (st != NSFRB_OK) return st;
    fits = true;
    for (size_t c = 0; c < b->classes.size(); ++c) {
      BatchClass& bc = b->classes[c];
      HIP_TRY(hipModuleGetFunction(&bc.fn, b->mod, ("nsfrb_batch_kernel_" + std::to_string(c)).c_str()));
      int scratch = 0;
      HIP_TRY(hipFuncGetAttribute(&scratch, HIP_FUNC_ATTRIBUTE_LOCAL_SIZE_BYTES, bc.fn));
      fits = fits && scratch <= scratch_allowance();
    }
  }
  if (!fits)
    return fail(NSFRB_ERR_UNSUPPORTED, "a class's persistent kernel would spill more registers than a search kernel "
                                       "may at every accumulator count");
  for (size_t c = 0; c < b->classes.size(); ++c) {
    BatchClass& bc = b->classes[c];
    // a persistent grid of as many workgroups as this class's kernel keeps resident
    int per_cu = 0;
    HIP_TRY(hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, bc.fn, 64 * bc.k.NW, bc.lds));
    const long long g = (long long)n_cu * std::max(1, per_cu);
    bc.grid = (unsigned)std::max(1LL, std::min(g, bc.n_items));
  }
  HIP_TRY(dalloc(&b->d_descs, b->descs.size()));
  HIP_TRY(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
  HIP_TRY(hipEventCreateWithFlags(&b->done, hipEventDisableTiming));
  *out = b.release();
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_batch_destroy(nsfrb_batch* b) {
  g_last_error.clear();
  if (b && b->ran) {
    hipSetDevice(b->device);
    hipEventSynchronize(b->done);
  }
  batch_release(b);
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_batch_use_graph(nsfrb_batch* b, int32_t on) {
  g_last_error.clear();
  if (!b) return fail(NSFRB_ERR_INVALID_ARG, "batch is NULL");
  b->use_graph = on != 0;
  return NSFRB_OK;
}

// Statistics of every cube (or flag reset for search-layout input); sets last_z.
static nsfrb_status batch_stats(nsfrb_batch* b, const void* const* d_cubes, hipStream_t st) {
  for (size_t i = 0; i < b->cubes.size(); ++i) {
    nsfrb_search* h = b->cubes[i];
    const nsfrb_search_config& c = h->cfg;
    if (c.layout == NSFRB_LAYOUT_TSP) {
      StatsLaunch sa{d_cubes[i], c.n_time, c.n_sub, h->n_pix, c.norm, c.in_dtype, c.store_dtype,
                     h->d_ext_med, h->d_ext_sig, h->d_med, h->d_sig, h->d_z, h->d_flags};
      HIP_TRY(launch_stats(sa, st));
      h->last_z = h->d_z;
    } else {
      HIP_TRY(launch_zero_u64(h->d_flags, st));
      h->last_z = d_cubes[i];
    }
  }
  return NSFRB_OK;
}

static nsfrb_status batch_candidates(nsfrb_batch* b, hipStream_t st) {
  for (auto* h : b->cubes) {
    const nsfrb_search_config& c = h->cfg;
    CandLaunch ca{h->d_best_s, h->d_best_d, h->d_best_w, h->d_best_t, h->n_pix, c.nx, c.max_candidates,
                  c.snr_threshold, h->d_keys, h->d_count, h->d_cands, h->d_nout};
    HIP_TRY(launch_candidates(ca, st));
    HIP_TRY(hipMemcpyAsync(h->h_nout, h->d_nout, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(h->h_cands, h->d_cands, sizeof(nsfrb_candidate) * c.max_candidates,
                           hipMemcpyDeviceToHost, st));
  }
  return NSFRB_OK;
}

static nsfrb_status batch_enqueue(nsfrb_batch* b, const void* const* d_cubes, hipStream_t st) {
  nsfrb_status s = batch_stats(b, d_cubes, st);
  if (s != NSFRB_OK) return s;
  for (size_t c = 0; c < b->classes.size(); ++c) {
    const BatchClass& bc = b->classes[c];
    const CubeDescHost* descs = b->d_descs + bc.first_desc;
    int n = bc.n_cubes;
    long long items = bc.n_items;
    int stride = bc.buf_stride;
    void* args[] = {(void*)&descs, &n, &items, &stride};
    HIP_TRY(hipModuleLaunchKernel(bc.fn, bc.grid, 1, 1, 64 * bc.k.NW, 1, 1, (unsigned)bc.lds, st, args, nullptr));
  }
  return batch_candidates(b, st);
}

extern "C" nsfrb_status nsfrb_batch_run(nsfrb_batch* b, const void* const* d_cubes, void* stream) {
  g_last_error.clear();
  if (!b || !d_cubes) return fail(NSFRB_ERR_INVALID_ARG, "batch and d_cubes must be non-NULL");
  for (size_t i = 0; i < b->cubes.size(); ++i)
    if (!d_cubes[i]) return fail(NSFRB_ERR_INVALID_ARG, "a cube pointer is NULL");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(b->device));
  std::vector<const void*> ptrs(d_cubes, d_cubes + b->cubes.size());
  // descriptors carry the normalised-cube pointers; refresh them when the inputs change
  if (ptrs != b->desc_ptrs || !b->ran) {
    if (b->ran) HIP_TRY(hipEventSynchronize(b->done));
    for (size_t i = 0; i < b->cubes.size(); ++i) {
      nsfrb_search* h = b->cubes[i];
      CubeDescHost& d = b->descs[b->desc_of_cube[i]];
      d.z = h->cfg.layout == NSFRB_LAYOUT_TSP ? h->d_z : d_cubes[i];
      // row copy the cube allows: global-to-LDS loads of 16 (4) bytes per lane
      // for rows of whole 16-byte (4-byte) vectors from a 16-byte (4-byte)
      // aligned cube, else (2) 16-bit rows placed at their dword parity
      const size_t es = dtype_size(h->cfg.store_dtype), row_bytes = (size_t)h->cfg.n_time * es;
      const uintptr_t zp = reinterpret_cast<uintptr_t>(d.z);
      if (zp % es != 0) return fail(NSFRB_ERR_INVALID_ARG, "cube " + std::to_string(i) + " is not aligned to its sample size");
      d.dma_w = (row_bytes % 16 == 0 && zp % 16 == 0) ? 16 : (row_bytes % 4 == 0 && zp % 4 == 0) ? 4 : 2;
    }
    HIP_TRY(hipMemcpy(b->d_descs, b->descs.data(), b->descs.size() * sizeof(CubeDescHost), hipMemcpyHostToDevice));
    b->desc_ptrs = ptrs;
  }
  if (!b->use_graph) {
    nsfrb_status s = batch_enqueue(b, d_cubes, st);
    if (s != NSFRB_OK) return s;
    b->last_graph = false;
  } else {
    // the graph bakes in the raw cube pointers of its statistics launches:
    // re-capture whenever they differ from this run's, whichever path ran last
    if (ptrs != b->graph_ptrs || !b->exec) {
      if (b->exec) { hipGraphExecDestroy(b->exec); b->exec = nullptr; }
      if (b->graph) { hipGraphDestroy(b->graph); b->graph = nullptr; }
      HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
      nsfrb_status s = batch_enqueue(b, d_cubes, b->cap_stream);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
      if (s != NSFRB_OK) { if (g) hipGraphDestroy(g); return s; }
      HIP_TRY(e);
      b->graph = g;
      HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
      b->graph_ptrs = ptrs;
    }
    HIP_TRY(hipGraphLaunch(b->exec, st));
    b->last_graph = true;
  }
  HIP_TRY(hipEventRecord(b->done, st));
  for (auto* h : b->cubes) h->ran = true;
  b->ran = true;
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_batch_run_separate(nsfrb_batch* b, const void* const* d_cubes, void* stream) {
  g_last_error.clear();
  if (!b || !d_cubes) return fail(NSFRB_ERR_INVALID_ARG, "batch and d_cubes must be non-NULL");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(b->device));
  // first separate run: compile and tune each cube's own kernels (synchronous;
  // the tuner's launches finish before this run's work is enqueued)
  for (auto* h : b->cubes)
    if (!h->planned) {
      nsfrb_status s = plan_kernels(h);
      if (s != NSFRB_OK) return s;
    }
  nsfrb_status s = batch_stats(b, d_cubes, st);
  if (s != NSFRB_OK) return s;
  for (auto* h : b->cubes) {
    s = launch_search_per_dm(h, h->last_z, st);
    if (s != NSFRB_OK) return s;
  }
  s = batch_candidates(b, st);
  if (s != NSFRB_OK) return s;
  HIP_TRY(hipEventRecord(b->done, st));
  for (auto* h : b->cubes) h->ran = true;
  b->ran = true;
  b->last_graph = false;
  return NSFRB_OK;
}

static nsfrb_status batch_cube(nsfrb_batch* b, int32_t cube, nsfrb_search** h) {
  if (!b) return fail(NSFRB_ERR_INVALID_ARG, "batch is NULL");
  if (cube < 0 || cube >= (int)b->cubes.size()) return fail(NSFRB_ERR_INVALID_ARG, "cube index out of range");
  if (!b->ran) return fail(NSFRB_ERR_NOT_READY, "no run has been enqueued on this batch");
  HIP_TRY(hipSetDevice(b->device));
  HIP_TRY(hipEventSynchronize(b->done));
  *h = b->cubes[cube];
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_batch_candidates_get(nsfrb_batch* b, int32_t cube, nsfrb_candidate* host_out,
                                                   int32_t capacity, int32_t* n_written, int32_t* n_total) {
  g_last_error.clear();
  nsfrb_search* h = nullptr;
  nsfrb_status st = batch_cube(b, cube, &h);
  if (st != NSFRB_OK) return st;
  return nsfrb_candidates_get(h, host_out, capacity, n_written, n_total);
}

extern "C" nsfrb_status nsfrb_batch_maps_get(nsfrb_batch* b, int32_t cube, float* snr_max, int32_t* toa) {
  g_last_error.clear();
  nsfrb_search* h = nullptr;
  nsfrb_status st = batch_cube(b, cube, &h);
  if (st != NSFRB_OK) return st;
  return nsfrb_maps_get(h, snr_max, toa);
}

extern "C" nsfrb_status nsfrb_batch_best_get(nsfrb_batch* b, int32_t cube, float* snr, int32_t* dm_index,
                                             int32_t* width_index, int32_t* toa) {
  g_last_error.clear();
  nsfrb_search* h = nullptr;
  nsfrb_status st = batch_cube(b, cube, &h);
  if (st != NSFRB_OK) return st;
  return nsfrb_best_get(h, snr, dm_index, width_index, toa);
}

extern "C" nsfrb_status nsfrb_batch_zcube_device(nsfrb_batch* b, int32_t cube, const void** d_z) {
  g_last_error.clear();
  nsfrb_search* h = nullptr;
  nsfrb_status st = batch_cube(b, cube, &h);
  if (st != NSFRB_OK) return st;
  return nsfrb_zcube_device(h, d_z);
}

extern "C" nsfrb_status nsfrb_batch_info_get(nsfrb_batch* b, int64_t* info) {
  g_last_error.clear();
  if (!b || !info) return fail(NSFRB_ERR_INVALID_ARG, "NULL argument");
  int64_t grid = 0, lds = 0;
  for (const auto& bc : b->classes) {
    grid += bc.grid;
    lds = std::max<int64_t>(lds, (int64_t)bc.lds);
  }
  info[0] = b->n_items;
  info[1] = grid;
  info[2] = lds;
  info[3] = (int64_t)b->classes.size();
  info[4] = b->last_graph ? 1 : 0;
  return NSFRB_OK;
}

// --------------------------------------------------------------- generator
static size_t elem_count(int32_t n_pix, int32_t n_sub, int32_t n_time) {
  return (size_t)n_pix * n_sub * n_time;
}

extern "C" nsfrb_status nsfrb_generate_noise(void* d_out, int32_t dtype, int32_t layout, int32_t n_pix,
                                             int32_t n_sub, int32_t n_time, uint64_t seed, float sigma,
                                             void* stream) {
  g_last_error.clear();
  if (!d_out || dtype < 0 || dtype > 2 || (layout != 0 && layout != 1) || n_pix < 1 || n_sub < 1 || n_time < 1 ||
      !std::isfinite(sigma))
    return fail(NSFRB_ERR_INVALID_ARG, "bad generator arguments");
  HIP_TRY(launch_noise(d_out, dtype, (long long)elem_count(n_pix, n_sub, n_time), seed, sigma, (hipStream_t)stream));
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_inject_boxcar(void* d_cube, int32_t dtype, int32_t layout, int32_t n_pix,
                                            int32_t n_sub, int32_t n_time, int32_t pixel, int32_t t0,
                                            int32_t width, float amp, const int32_t* host_offsets, void* stream) {
  g_last_error.clear();
  if (!d_cube || !host_offsets || dtype < 0 || dtype > 2 || (layout != 0 && layout != 1) || n_pix < 1 ||
      n_sub < 1 || n_time < 1 || pixel < 0 || pixel >= n_pix || width < 1 || !std::isfinite(amp))
    return fail(NSFRB_ERR_INVALID_ARG, "bad injection arguments");
  // a utility for building inputs: synchronous, so the host offsets can be released on return
  int* d_off = nullptr;
  HIP_TRY(hipMalloc((void**)&d_off, sizeof(int) * n_sub));
  std::unique_ptr<void, hipError_t (*)(void*)> guard(d_off, hipFree);
  HIP_TRY(hipMemcpy(d_off, host_offsets, sizeof(int) * n_sub, hipMemcpyHostToDevice));
  HIP_TRY(launch_inject(d_cube, dtype, layout, n_pix, n_sub, n_time, pixel, t0, width, amp, d_off,
                        (hipStream_t)stream));
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_inject_boxcars(void* const* d_cubes, int32_t n_cubes, int32_t dtype, int32_t layout,
                                             int32_t n_pix, int32_t n_sub, int32_t n_time,
                                             const nsfrb_boxcar* host_boxcars, const int32_t* host_offsets,
                                             int32_t n, void* stream) {
  static_assert(sizeof(nsfrb_boxcar) == sizeof(BoxcarRec), "nsfrb_boxcar layout");
  g_last_error.clear();
  if (!d_cubes || n_cubes < 1 || !host_boxcars || !host_offsets || n < 1 || dtype < 0 || dtype > 2 ||
      (layout != 0 && layout != 1) || n_pix < 1 || n_sub < 1 || n_time < 1 || n > 65535)
    return fail(NSFRB_ERR_INVALID_ARG, "bad injection arguments");
  for (int i = 0; i < n_cubes; ++i)
    if (!d_cubes[i]) return fail(NSFRB_ERR_INVALID_ARG, "cube pointer " + std::to_string(i) + " is NULL");
  std::vector<long long> keys((size_t)n);
  for (int i = 0; i < n; ++i) {
    const nsfrb_boxcar& b = host_boxcars[i];
    if (b.cube < 0 || b.cube >= n_cubes || b.pixel < 0 || b.pixel >= n_pix || b.width < 1 || !std::isfinite(b.amp))
      return fail(NSFRB_ERR_INVALID_ARG, "boxcar " + std::to_string(i) + " out of range");
    keys[(size_t)i] = (long long)b.cube * n_pix + b.pixel;
  }
  std::sort(keys.begin(), keys.end());
  if (std::adjacent_find(keys.begin(), keys.end()) != keys.end())
    return fail(NSFRB_ERR_INVALID_ARG, "two boxcars share a (cube, pixel)");
  // a utility for building inputs: synchronous, so host arrays can be released on return
  const size_t bytes_ptr = sizeof(void*) * n_cubes, bytes_rec = sizeof(BoxcarRec) * n,
               bytes_off = sizeof(int) * (size_t)n * n_sub;
  char* d_buf = nullptr;
  HIP_TRY(hipMalloc((void**)&d_buf, bytes_ptr + bytes_rec + bytes_off));
  std::unique_ptr<void, hipError_t (*)(void*)> guard(d_buf, hipFree);
  HIP_TRY(hipMemcpy(d_buf, d_cubes, bytes_ptr, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(d_buf + bytes_ptr, host_boxcars, bytes_rec, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(d_buf + bytes_ptr + bytes_rec, host_offsets, bytes_off, hipMemcpyHostToDevice));
  HIP_TRY(launch_inject_many((void* const*)d_buf, dtype, layout, n_pix, n_sub, n_time,
                             (const BoxcarRec*)(d_buf + bytes_ptr), (const int*)(d_buf + bytes_ptr + bytes_rec), n,
                             (hipStream_t)stream));
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_philox_fill(uint32_t* d_out, int64_t n_blocks, uint64_t seed, void* stream) {
  g_last_error.clear();
  if (!d_out || n_blocks < 0) return fail(NSFRB_ERR_INVALID_ARG, "bad arguments");
  HIP_TRY(launch_philox_fill(d_out, n_blocks, seed, (hipStream_t)stream));
  return NSFRB_OK;
}

// --------------------------------------------------------------- streaming
// Real-time form (section 2.2): images arrive in fixed batches of `chunk`
// samples; the last n_time samples sit in a device ring (raw layout, one row
// of n_sub x n_pix per sample) and are searched after each batch once the ring
// is full; a search that overruns the deadline makes the next iteration be
// dropped so the stream catches up.
struct nsfrb_stream {
  nsfrb_search* search = nullptr;
  void* ring = nullptr;
  size_t row_bytes = 0;
  int n_time = 0, chunk = 0, head = 0;
  int64_t received = 0, pushes = 0;
  double deadline_ms = 0.0;
  bool drop_next = false;
  int32_t dropped = 0;
  hipEvent_t t0 = nullptr, t1 = nullptr;
};

static void stream_release(nsfrb_stream* s) {
  if (!s) return;
  if (s->search) {
    hipSetDevice(s->search->device);
    nsfrb_search_destroy(s->search);
  }
  if (s->ring) hipFree(s->ring);
  if (s->t0) hipEventDestroy(s->t0);
  if (s->t1) hipEventDestroy(s->t1);
  delete s;
}

extern "C" nsfrb_status nsfrb_stream_create(const nsfrb_search_config* cfg, int32_t chunk, double deadline_ms,
                                            nsfrb_stream** out) {
  g_last_error.clear();
  if (!cfg || !out) return fail(NSFRB_ERR_INVALID_ARG, "NULL argument");
  *out = nullptr;
  nsfrb_status st = validate(cfg);
  if (st != NSFRB_OK) return st;
  if (cfg->layout != NSFRB_LAYOUT_TSP) return fail(NSFRB_ERR_UNSUPPORTED, "a stream takes raw [time][sub-band][pixel] batches");
  if (cfg->norm == NSFRB_NORM_EXTERNAL) return fail(NSFRB_ERR_UNSUPPORTED, "a stream computes its own statistics");
  if (chunk < 1 || chunk > cfg->n_time) return fail(NSFRB_ERR_INVALID_ARG, "chunk must be 1..n_time");
  if (!(deadline_ms > 0.0) || !std::isfinite(deadline_ms)) return fail(NSFRB_ERR_INVALID_ARG, "deadline_ms must be > 0");
  std::unique_ptr<nsfrb_stream, void (*)(nsfrb_stream*)> s(new nsfrb_stream, stream_release);
  st = nsfrb_search_create(cfg, &s->search);
  if (st != NSFRB_OK) return st;
  s->n_time = cfg->n_time;
  s->chunk = chunk;
  s->deadline_ms = deadline_ms;
  s->row_bytes = (size_t)cfg->n_sub * cfg->nx * cfg->ny * dtype_size(cfg->in_dtype);
  HIP_TRY(hipSetDevice(cfg->device));
  HIP_TRY(hipMalloc(&s->ring, s->row_bytes * cfg->n_time));
  HIP_TRY(hipEventCreate(&s->t0));
  HIP_TRY(hipEventCreate(&s->t1));
  *out = s.release();
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_stream_destroy(nsfrb_stream* s) {
  g_last_error.clear();
  if (s && s->search) {
    hipSetDevice(s->search->device);
    hipDeviceSynchronize();
  }
  stream_release(s);
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_stream_push(nsfrb_stream* s, const void* d_chunk, void* stream,
                                          nsfrb_stream_result* out) {
  g_last_error.clear();
  if (!s || !d_chunk || !out) return fail(NSFRB_ERR_INVALID_ARG, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(s->search->device));
  // append the batch at the ring's head (two copies when it wraps)
  const int first = std::min(s->chunk, s->n_time - s->head);
  HIP_TRY(hipMemcpyAsync((char*)s->ring + (size_t)s->head * s->row_bytes, d_chunk, (size_t)first * s->row_bytes,
                         hipMemcpyDeviceToDevice, st));
  if (first < s->chunk)
    HIP_TRY(hipMemcpyAsync(s->ring, (const char*)d_chunk + (size_t)first * s->row_bytes,
                           (size_t)(s->chunk - first) * s->row_bytes, hipMemcpyDeviceToDevice, st));
  s->head = (s->head + s->chunk) % s->n_time;
  s->received += s->chunk;
  s->pushes += 1;
  nsfrb_stream_result r{};
  r.chunk_index = s->pushes - 1;
  r.window_start = s->received - s->n_time;
  r.dropped_total = s->dropped;
  if (s->received < s->n_time) {             // the window is not full yet
    HIP_TRY(hipStreamSynchronize(st));
    *out = r;
    return NSFRB_OK;
  }
  if (s->drop_next) {                        // the previous search overran: skip this one
    s->drop_next = false;
    s->dropped += 1;
    r.dropped_total = s->dropped;
    HIP_TRY(hipStreamSynchronize(st));
    *out = r;
    return NSFRB_OK;
  }
  HIP_TRY(hipEventRecord(s->t0, st));
  nsfrb_status rs = run_impl(s->search, s->ring, s->head, stream);    // oldest sample at the head
  if (rs != NSFRB_OK) return rs;
  HIP_TRY(hipEventRecord(s->t1, st));
  rs = wait_run(s->search);
  if (rs != NSFRB_OK) return rs;
  HIP_TRY(hipEventSynchronize(s->t1));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, s->t0, s->t1));
  r.searched = 1;
  r.search_ms = ms;
  if (ms > s->deadline_ms) s->drop_next = true;
  unsigned long long flags = 0;
  HIP_TRY(hipMemcpy(&flags, s->search->d_flags, sizeof(flags), hipMemcpyDeviceToHost));
  r.flagged = (int64_t)flags;
  if (s->search->h_nout[0] > 0) {            // one candidate per batch: the window's best
    r.has_candidate = 1;
    r.cand = s->search->h_cands[0];
  }
  *out = r;
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_stream_search(nsfrb_stream* s, nsfrb_search** out) {
  g_last_error.clear();
  if (!s || !out) return fail(NSFRB_ERR_INVALID_ARG, "NULL argument");
  *out = s->search;
  return NSFRB_OK;
}
