// Host side of the candidate classifier: parameters, Adam state, activation
// buffers and the forward / backward / update sequence of one training step.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/nsfrb.h"
#include "host_util.h"
#include "nsfrb_internal.h"

using namespace nsfrb;

namespace {

constexpr int kCin = 16, kCh = 32, kTap = 27, kX = 32;
constexpr int kLayerCin[4] = {kCin, kCh, kCh, kCh};

// Offsets of the parameter blocks in the flat FP32 vector:
// W_l[32][27][cin], b_l[32] for l = 1..4, then W1[32][64], c1[32], w2[32], c2[1].
struct Layout {
  int w[4], b[4], head, total;
  Layout() {
    int o = 0;
    for (int l = 0; l < 4; ++l) {
      w[l] = o;
      o += kCh * kTap * kLayerCin[l];
      b[l] = o;
      o += kCh;
    }
    head = o;
    o += kCh * 2 * kCh + kCh + kCh + 1;
    total = o;
  }
};
const Layout kL;

// SplitMix64 (Steele, Lea & Flood 2014): a counter-based stream for weight init.
uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
double uniform01(uint64_t& s) { return (double)(splitmix64(s) >> 11) * (1.0 / 9007199254740992.0); }

}  // namespace

struct nsfrb_classifier {
  nsfrb_classifier_config cfg{};
  int device = 0;
  float* d_theta = nullptr;
  float* d_m = nullptr;
  float* d_v = nullptr;
  float* d_grad = nullptr;
  uint16_t* d_wf[4] = {};      // BF16 forward weights in convolution-operand order
  uint16_t* d_wb[4] = {};      // BF16 backward-data weights (flipped taps, transposed channels; layers 2..4)
  uint16_t* d_act[4] = {};     // conv outputs a_1..a_4 [n][t][y][x][32]
  uint16_t* d_dpre[4] = {};    // pre-activation gradients of conv layers 1..4 (kept for inspection)
  float* d_part = nullptr;
  float* d_part_db = nullptr;
  float* d_h = nullptr;         // head input [n][64]: channel maxima, candidate-position features
  float* d_dh = nullptr;
  int* d_arg = nullptr;         // position of each channel's maximum [n][32]
  uint32_t* d_pool_part = nullptr;  // per-chunk maximum keys of the pooling pass
  float* d_hs = nullptr;        // head's per-sample backward record [n][66]
  float* d_logits = nullptr;
  float* d_prob = nullptr;
  float* d_loss = nullptr;
  void* d_cut_desc = nullptr;
  int* d_delays = nullptr;
  int delays_cap = 0;
  const void** d_cube_ptrs = nullptr;
  int cube_ptrs_cap = 0;
  float* h_loss = nullptr;
  long long step = 0;
  bool weights_dirty = true;
};

namespace {

void release(nsfrb_classifier* c) {
  if (!c) return;
  hipSetDevice(c->device);
  void* bufs[] = {c->d_theta, c->d_m, c->d_v, c->d_grad, c->d_part, c->d_part_db, c->d_h, c->d_dh, (void*)c->d_arg,
                  (void*)c->d_pool_part, c->d_hs,
                  c->d_logits, c->d_prob, c->d_loss, c->d_cut_desc, c->d_delays, (void*)c->d_cube_ptrs};
  for (void* b : bufs)
    if (b) hipFree(b);
  for (int l = 0; l < 4; ++l) {
    if (c->d_wf[l]) hipFree(c->d_wf[l]);
    if (c->d_wb[l]) hipFree(c->d_wb[l]);
    if (c->d_act[l]) hipFree(c->d_act[l]);
  }
  for (auto* p : c->d_dpre)
    if (p) hipFree(p);
  if (c->h_loss) hipHostFree(c->h_loss);
  delete c;
}

template <typename T>
hipError_t dalloc(T** p, size_t n) {
  return hipMalloc((void**)p, (n ? n : 1) * sizeof(T));
}

nsfrb_status prep_weights(nsfrb_classifier* c, hipStream_t st) {
  for (int l = 0; l < 4; ++l)
    NSFRB_HIP_TRY(launch_prep_weights(c->d_theta + kL.w[l], kLayerCin[l], c->d_wf[l], l ? c->d_wb[l] : nullptr, st));
  c->weights_dirty = false;
  return NSFRB_OK;
}

// Flat (t, y, x) index of the candidate's own position: TOA at sample T/2, pixel at the centre.
int centre_pos(const nsfrb_classifier* c) { return ((c->cfg.n_time / 2) * c->cfg.ny + c->cfg.ny / 2) * kX + kX / 2; }

nsfrb_status forward(nsfrb_classifier* c, const uint16_t* x, int n, hipStream_t st) {
  const int T = c->cfg.n_time, Y = c->cfg.ny;
  if (c->weights_dirty) {
    nsfrb_status s = prep_weights(c, st);
    if (s != NSFRB_OK) return s;
  }
  const uint16_t* in = x;
  for (int l = 0; l < 4; ++l) {
    NSFRB_HIP_TRY(launch_conv_fwd(kLayerCin[l], in, c->d_wf[l], c->d_theta + kL.b[l], c->d_act[l], n, T, Y, st));
    in = c->d_act[l];
  }
  NSFRB_HIP_TRY(launch_pool(c->d_act[3], n, T * Y * kX, centre_pos(c), c->d_pool_part, c->d_h, c->d_arg, st));
  return NSFRB_OK;
}

}  // namespace

extern "C" nsfrb_status nsfrb_classifier_create(const nsfrb_classifier_config* cfg, nsfrb_classifier** out) {
  host_clear_error();
  if (!cfg || !out) return host_fail(NSFRB_ERR_INVALID_ARG, "cfg and out must be non-NULL");
  *out = nullptr;
  if (cfg->struct_size != sizeof(nsfrb_classifier_config))
    return host_fail(NSFRB_ERR_INVALID_ARG, "struct_size does not match this library's nsfrb_classifier_config");
  if (cfg->max_batch < 1 || cfg->max_batch > 1024) return host_fail(NSFRB_ERR_INVALID_ARG, "max_batch must be 1..1024");
  if (cfg->n_time < 1 || cfg->n_time > 256 || cfg->ny < 1 || cfg->ny > 256)
    return host_fail(NSFRB_ERR_INVALID_ARG, "n_time and ny must be 1..256");
  if (!(cfg->lr >= 0.f) || !(cfg->beta1 >= 0.f && cfg->beta1 < 1.f) || !(cfg->beta2 >= 0.f && cfg->beta2 < 1.f) ||
      !(cfg->eps > 0.f))
    return host_fail(NSFRB_ERR_INVALID_ARG, "bad Adam hyper-parameters");
  std::unique_ptr<nsfrb_classifier, void (*)(nsfrb_classifier*)> c(new nsfrb_classifier, release);
  c->cfg = *cfg;
  c->device = cfg->device;
  NSFRB_HIP_TRY(hipSetDevice(c->device));
  const size_t P = (size_t)kL.total;
  const size_t N = (size_t)cfg->max_batch, npos = (size_t)cfg->n_time * cfg->ny * kX;
  NSFRB_HIP_TRY(dalloc(&c->d_theta, P));
  NSFRB_HIP_TRY(dalloc(&c->d_m, P));
  NSFRB_HIP_TRY(dalloc(&c->d_v, P));
  NSFRB_HIP_TRY(dalloc(&c->d_grad, P));
  for (int l = 0; l < 4; ++l) {
    NSFRB_HIP_TRY(dalloc(&c->d_wf[l], (size_t)kCh * kTap * kLayerCin[l]));
    if (l) NSFRB_HIP_TRY(dalloc(&c->d_wb[l], (size_t)kCh * kTap * kLayerCin[l]));
    NSFRB_HIP_TRY(dalloc(&c->d_act[l], N * npos * kCh));
  }
  for (auto& p : c->d_dpre) NSFRB_HIP_TRY(dalloc(&p, N * npos * kCh));
  const size_t items = (size_t)wgrad_items((int)N, cfg->ny);
  NSFRB_HIP_TRY(dalloc(&c->d_part, items * kTap * kCh * kCh));
  NSFRB_HIP_TRY(dalloc(&c->d_part_db, items * kCh));
  NSFRB_HIP_TRY(dalloc(&c->d_h, N * 2 * kCh));
  NSFRB_HIP_TRY(dalloc(&c->d_dh, N * 2 * kCh));
  NSFRB_HIP_TRY(dalloc(&c->d_arg, N * kCh));
  NSFRB_HIP_TRY(dalloc(&c->d_pool_part, N * pool_chunks((int)npos) * kCh));
  NSFRB_HIP_TRY(dalloc(&c->d_hs, N * (2 * kCh + 2)));
  NSFRB_HIP_TRY(dalloc(&c->d_logits, N));
  NSFRB_HIP_TRY(dalloc(&c->d_prob, N));
  NSFRB_HIP_TRY(dalloc(&c->d_loss, 4));
  NSFRB_HIP_TRY(hipHostMalloc((void**)&c->h_loss, sizeof(float) * 4, hipHostMallocDefault));
  // He-uniform convolution weights, uniform(+-sqrt(6/fan_in)) head weights, zero biases
  std::vector<float> th(P, 0.f);
  uint64_t s = cfg->seed;
  for (int l = 0; l < 4; ++l) {
    const double lim = std::sqrt(6.0 / (kTap * kLayerCin[l]));
    for (int i = 0; i < kCh * kTap * kLayerCin[l]; ++i) th[kL.w[l] + i] = (float)((2 * uniform01(s) - 1) * lim);
  }
  const double lim1 = std::sqrt(6.0 / (2 * kCh)), lim2 = std::sqrt(6.0 / kCh);
  for (int i = 0; i < kCh * 2 * kCh; ++i) th[kL.head + i] = (float)((2 * uniform01(s) - 1) * lim1);
  for (int i = 0; i < kCh; ++i) th[kL.head + 2 * kCh * kCh + kCh + i] = (float)((2 * uniform01(s) - 1) * lim2);
  NSFRB_HIP_TRY(hipMemcpy(c->d_theta, th.data(), P * sizeof(float), hipMemcpyHostToDevice));
  NSFRB_HIP_TRY(hipMemset(c->d_m, 0, P * sizeof(float)));
  NSFRB_HIP_TRY(hipMemset(c->d_v, 0, P * sizeof(float)));
  NSFRB_HIP_TRY(hipMemset(c->d_grad, 0, P * sizeof(float)));
  *out = c.release();
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_classifier_destroy(nsfrb_classifier* c) {
  host_clear_error();
  if (c) {
    hipSetDevice(c->device);
    hipDeviceSynchronize();
  }
  release(c);
  return NSFRB_OK;
}

extern "C" int32_t nsfrb_classifier_param_count(void) { return kL.total; }

extern "C" nsfrb_status nsfrb_classifier_params_get(nsfrb_classifier* c, float* host) {
  host_clear_error();
  if (!c || !host) return host_fail(NSFRB_ERR_INVALID_ARG, "NULL argument");
  NSFRB_HIP_TRY(hipSetDevice(c->device));
  NSFRB_HIP_TRY(hipDeviceSynchronize());
  NSFRB_HIP_TRY(hipMemcpy(host, c->d_theta, sizeof(float) * kL.total, hipMemcpyDeviceToHost));
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_classifier_params_set(nsfrb_classifier* c, const float* host) {
  host_clear_error();
  if (!c || !host) return host_fail(NSFRB_ERR_INVALID_ARG, "NULL argument");
  NSFRB_HIP_TRY(hipSetDevice(c->device));
  NSFRB_HIP_TRY(hipDeviceSynchronize());
  NSFRB_HIP_TRY(hipMemcpy(c->d_theta, host, sizeof(float) * kL.total, hipMemcpyHostToDevice));
  c->weights_dirty = true;
  return NSFRB_OK;
}

// ------------------------------------------------------------ checkpoints
// A checkpoint is a host byte image: a fixed header, then the FP32 parameter
// vector, then Adam's first and second moments (each nsfrb_classifier_param_count
// values, little-endian as the host stores them).
namespace {
struct CkptHeader {
  char magic[8];            // "NSFRBCK1"
  uint32_t version;         // 1
  uint32_t n_params;
  int64_t step;             // Adam steps taken (bias corrections continue from it)
  uint64_t user_counter;    // caller's word, e.g. the position of its data generator
  float lr, beta1, beta2, eps;
  int32_t n_time, ny;       // cutout shape the classifier was created for
};
static_assert(sizeof(CkptHeader) == 56, "checkpoint header layout");
constexpr char kCkptMagic[8] = {'N', 'S', 'F', 'R', 'B', 'C', 'K', '1'};
}  // namespace

extern "C" int64_t nsfrb_classifier_state_bytes(void) {
  return (int64_t)sizeof(CkptHeader) + 3 * (int64_t)sizeof(float) * kL.total;
}

extern "C" nsfrb_status nsfrb_classifier_save(nsfrb_classifier* c, uint64_t user_counter, void* host_out,
                                              int64_t capacity, int64_t* n_written) {
  host_clear_error();
  if (!c || !host_out || !n_written) return host_fail(NSFRB_ERR_INVALID_ARG, "NULL argument");
  const int64_t need = nsfrb_classifier_state_bytes();
  *n_written = need;
  if (capacity < need) return host_fail(NSFRB_ERR_TRUNCATED, "capacity below nsfrb_classifier_state_bytes()");
  NSFRB_HIP_TRY(hipSetDevice(c->device));
  NSFRB_HIP_TRY(hipDeviceSynchronize());
  CkptHeader h{};
  std::memcpy(h.magic, kCkptMagic, 8);
  h.version = 1;
  h.n_params = (uint32_t)kL.total;
  h.step = c->step;
  h.user_counter = user_counter;
  h.lr = c->cfg.lr;
  h.beta1 = c->cfg.beta1;
  h.beta2 = c->cfg.beta2;
  h.eps = c->cfg.eps;
  h.n_time = c->cfg.n_time;
  h.ny = c->cfg.ny;
  unsigned char* out = static_cast<unsigned char*>(host_out);
  std::memcpy(out, &h, sizeof h);
  float* body = reinterpret_cast<float*>(out + sizeof h);
  const size_t nb = sizeof(float) * kL.total;
  NSFRB_HIP_TRY(hipMemcpy(body, c->d_theta, nb, hipMemcpyDeviceToHost));
  NSFRB_HIP_TRY(hipMemcpy(body + kL.total, c->d_m, nb, hipMemcpyDeviceToHost));
  NSFRB_HIP_TRY(hipMemcpy(body + 2 * kL.total, c->d_v, nb, hipMemcpyDeviceToHost));
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_classifier_load(nsfrb_classifier* c, const void* host_in, int64_t n_bytes,
                                              uint64_t* user_counter) {
  host_clear_error();
  if (!c || !host_in) return host_fail(NSFRB_ERR_INVALID_ARG, "NULL argument");
  if (n_bytes != nsfrb_classifier_state_bytes())
    return host_fail(NSFRB_ERR_INVALID_ARG, "checkpoint size differs from nsfrb_classifier_state_bytes()");
  CkptHeader h;
  std::memcpy(&h, host_in, sizeof h);
  if (std::memcmp(h.magic, kCkptMagic, 8) != 0 || h.version != 1)
    return host_fail(NSFRB_ERR_INVALID_ARG, "not a classifier checkpoint (magic or version)");
  if (h.n_params != (uint32_t)kL.total || h.n_time != c->cfg.n_time || h.ny != c->cfg.ny)
    return host_fail(NSFRB_ERR_INVALID_ARG, "checkpoint of another network or cutout shape");
  if (h.step < 0 || !std::isfinite(h.lr) || !(h.lr >= 0.f) || !std::isfinite(h.beta1) || !std::isfinite(h.beta2) ||
      !std::isfinite(h.eps))
    return host_fail(NSFRB_ERR_INVALID_ARG, "checkpoint header holds invalid optimiser settings");
  NSFRB_HIP_TRY(hipSetDevice(c->device));
  NSFRB_HIP_TRY(hipDeviceSynchronize());
  const float* body = reinterpret_cast<const float*>(static_cast<const unsigned char*>(host_in) + sizeof h);
  const size_t nb = sizeof(float) * kL.total;
  NSFRB_HIP_TRY(hipMemcpy(c->d_theta, body, nb, hipMemcpyHostToDevice));
  NSFRB_HIP_TRY(hipMemcpy(c->d_m, body + kL.total, nb, hipMemcpyHostToDevice));
  NSFRB_HIP_TRY(hipMemcpy(c->d_v, body + 2 * kL.total, nb, hipMemcpyHostToDevice));
  c->step = h.step;
  c->cfg.lr = h.lr;
  c->cfg.beta1 = h.beta1;
  c->cfg.beta2 = h.beta2;
  c->cfg.eps = h.eps;
  c->weights_dirty = true;
  if (user_counter) *user_counter = h.user_counter;
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_classifier_set_lr(nsfrb_classifier* c, float lr) {
  host_clear_error();
  if (!c) return host_fail(NSFRB_ERR_INVALID_ARG, "classifier is NULL");
  if (!(lr >= 0.f) || !std::isfinite(lr)) return host_fail(NSFRB_ERR_INVALID_ARG, "lr must be finite and >= 0");
  c->cfg.lr = lr;
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_classifier_grads_get(nsfrb_classifier* c, float* host) {
  host_clear_error();
  if (!c || !host) return host_fail(NSFRB_ERR_INVALID_ARG, "NULL argument");
  NSFRB_HIP_TRY(hipSetDevice(c->device));
  NSFRB_HIP_TRY(hipDeviceSynchronize());
  NSFRB_HIP_TRY(hipMemcpy(host, c->d_grad, sizeof(float) * kL.total, hipMemcpyDeviceToHost));
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_classifier_train_step(nsfrb_classifier* c, const void* d_cutouts, const float* d_labels,
                                                    int32_t n, int32_t update, float* host_loss, void* stream) {
  host_clear_error();
  if (!c || !d_cutouts || !d_labels) return host_fail(NSFRB_ERR_INVALID_ARG, "NULL argument");
  if (n < 1 || n > c->cfg.max_batch) return host_fail(NSFRB_ERR_INVALID_ARG, "n must be 1..max_batch");
  hipStream_t st = (hipStream_t)stream;
  NSFRB_HIP_TRY(hipSetDevice(c->device));
  const int T = c->cfg.n_time, Y = c->cfg.ny, npos = T * Y * kX;
  const uint16_t* x = (const uint16_t*)d_cutouts;
  nsfrb_status s = forward(c, x, n, st);
  if (s != NSFRB_OK) return s;
  NSFRB_HIP_TRY(launch_head(c->d_h, d_labels, n, c->d_theta + kL.head, c->d_hs, c->d_grad + kL.head, c->d_dh, c->d_logits,
                            c->d_prob, c->d_loss, 1, st));
  NSFRB_HIP_TRY(launch_pool_backward(c->d_dh, c->d_arg, c->d_act[3], n, npos, centre_pos(c), c->d_dpre[3], st));
  for (int l = 3; l >= 0; --l) {
    const uint16_t* in = l ? c->d_act[l - 1] : x;
    NSFRB_HIP_TRY(launch_conv_wgrad(kLayerCin[l], in, c->d_dpre[l], c->d_part, c->d_part_db, c->d_grad + kL.w[l],
                                    c->d_grad + kL.b[l], n, T, Y, st));
    if (l) NSFRB_HIP_TRY(launch_conv_bwd_data(c->d_dpre[l], c->d_wb[l], c->d_act[l - 1], c->d_dpre[l - 1], n, T, Y, st));
  }
  if (update) {
    c->step += 1;
    const float b1 = c->cfg.beta1, b2 = c->cfg.beta2;
    const float bc1 = (float)(1.0 - std::pow((double)b1, (double)c->step));
    const float bc2 = (float)(1.0 - std::pow((double)b2, (double)c->step));
    NSFRB_HIP_TRY(launch_adam(c->d_theta, c->d_m, c->d_v, c->d_grad, kL.total, c->cfg.lr, b1, b2, c->cfg.eps, bc1, bc2,
                              st));
    c->weights_dirty = true;
  }
  if (host_loss) {
    NSFRB_HIP_TRY(hipMemcpyAsync(c->h_loss, c->d_loss, sizeof(float), hipMemcpyDeviceToHost, st));
    NSFRB_HIP_TRY(hipStreamSynchronize(st));
    *host_loss = c->h_loss[0];
  }
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_classifier_activations_get(nsfrb_classifier* c, int32_t layer, int32_t n,
                                                          void* host_out) {
  host_clear_error();
  if (!c || !host_out) return host_fail(NSFRB_ERR_INVALID_ARG, "NULL argument");
  if (layer < 1 || layer > 4) return host_fail(NSFRB_ERR_INVALID_ARG, "layer must be 1..4");
  if (n < 1 || n > c->cfg.max_batch) return host_fail(NSFRB_ERR_INVALID_ARG, "n must be 1..max_batch");
  NSFRB_HIP_TRY(hipSetDevice(c->device));
  NSFRB_HIP_TRY(hipDeviceSynchronize());
  const size_t per = (size_t)c->cfg.n_time * c->cfg.ny * kX * kCh;
  NSFRB_HIP_TRY(hipMemcpy(host_out, c->d_act[layer - 1], per * n * sizeof(uint16_t), hipMemcpyDeviceToHost));
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_classifier_grad_pre_get(nsfrb_classifier* c, int32_t layer, int32_t n,
                                                       void* host_out) {
  host_clear_error();
  if (!c || !host_out) return host_fail(NSFRB_ERR_INVALID_ARG, "NULL argument");
  if (layer < 1 || layer > 4) return host_fail(NSFRB_ERR_INVALID_ARG, "layer must be 1..4");
  if (n < 1 || n > c->cfg.max_batch) return host_fail(NSFRB_ERR_INVALID_ARG, "n must be 1..max_batch");
  NSFRB_HIP_TRY(hipSetDevice(c->device));
  NSFRB_HIP_TRY(hipDeviceSynchronize());
  const size_t per = (size_t)c->cfg.n_time * c->cfg.ny * kX * kCh;
  NSFRB_HIP_TRY(hipMemcpy(host_out, c->d_dpre[layer - 1], per * n * sizeof(uint16_t), hipMemcpyDeviceToHost));
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_classifier_logits_get(nsfrb_classifier* c, int32_t n, float* host_out) {
  host_clear_error();
  if (!c || !host_out) return host_fail(NSFRB_ERR_INVALID_ARG, "NULL argument");
  if (n < 1 || n > c->cfg.max_batch) return host_fail(NSFRB_ERR_INVALID_ARG, "n must be 1..max_batch");
  NSFRB_HIP_TRY(hipSetDevice(c->device));
  NSFRB_HIP_TRY(hipDeviceSynchronize());
  NSFRB_HIP_TRY(hipMemcpy(host_out, c->d_logits, sizeof(float) * n, hipMemcpyDeviceToHost));
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_classifier_infer(nsfrb_classifier* c, const void* d_cutouts, int32_t n, float* d_prob,
                                               void* stream) {
  host_clear_error();
  if (!c || !d_cutouts || !d_prob) return host_fail(NSFRB_ERR_INVALID_ARG, "NULL argument");
  if (n < 1 || n > c->cfg.max_batch) return host_fail(NSFRB_ERR_INVALID_ARG, "n must be 1..max_batch");
  hipStream_t st = (hipStream_t)stream;
  NSFRB_HIP_TRY(hipSetDevice(c->device));
  nsfrb_status s = forward(c, (const uint16_t*)d_cutouts, n, st);
  if (s != NSFRB_OK) return s;
  NSFRB_HIP_TRY(launch_head(c->d_h, nullptr, n, c->d_theta + kL.head, nullptr, nullptr, nullptr, c->d_logits, d_prob, nullptr,
                            0, st));
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_cutouts_extract(nsfrb_classifier* c, const void* const* d_z_cubes, int32_t n_cubes,
                                              int32_t store_dtype, int32_t nx, int32_t ny, int32_t n_sub,
                                              int32_t n_time, const int32_t* host_delays, int32_t n_dm,
                                              const nsfrb_cutout* host_desc, int32_t n_cut, void* d_out,
                                              void* stream) {
  host_clear_error();
  if (!c || !d_z_cubes || !host_delays || !host_desc || !d_out) return host_fail(NSFRB_ERR_INVALID_ARG, "NULL argument");
  if (n_cubes < 1) return host_fail(NSFRB_ERR_INVALID_ARG, "n_cubes must be >= 1");
  for (int i = 0; i < n_cubes; ++i)
    if (!d_z_cubes[i]) return host_fail(NSFRB_ERR_INVALID_ARG, "cube pointer " + std::to_string(i) + " is NULL");
  if (n_cut < 1 || n_cut > c->cfg.max_batch) return host_fail(NSFRB_ERR_INVALID_ARG, "n_cut must be 1..max_batch");
  if (n_sub != kCin) return host_fail(NSFRB_ERR_UNSUPPORTED, "cutouts need 16 sub-bands (the network's input channels)");
  if (store_dtype < 0 || store_dtype > 2 || nx < 1 || ny < 1 || n_time < 1 || n_dm < 1)
    return host_fail(NSFRB_ERR_INVALID_ARG, "bad cube description");
  if (c->cfg.ny != kX) return host_fail(NSFRB_ERR_UNSUPPORTED, "cutouts are 32 x 32 pixels (classifier ny must be 32)");
  for (int i = 0; i < n_cut; ++i)
    if (host_desc[i].dm_index < 0 || host_desc[i].dm_index >= n_dm || host_desc[i].cube < 0 ||
        host_desc[i].cube >= n_cubes)
      return host_fail(NSFRB_ERR_INVALID_ARG, "cutout descriptor " + std::to_string(i) + " out of range");
  hipStream_t st = (hipStream_t)stream;
  NSFRB_HIP_TRY(hipSetDevice(c->device));
  NSFRB_HIP_TRY(hipStreamSynchronize(st));   // descriptor buffers are reused across calls
  if (!c->d_cut_desc) NSFRB_HIP_TRY(hipMalloc(&c->d_cut_desc, sizeof(nsfrb_cutout) * c->cfg.max_batch));
  if (c->delays_cap < n_dm * n_sub) {
    if (c->d_delays) NSFRB_HIP_TRY(hipFree(c->d_delays));
    c->d_delays = nullptr;
    NSFRB_HIP_TRY(hipMalloc((void**)&c->d_delays, sizeof(int) * n_dm * n_sub));
    c->delays_cap = n_dm * n_sub;
  }
  if (c->cube_ptrs_cap < n_cubes) {
    if (c->d_cube_ptrs) NSFRB_HIP_TRY(hipFree((void*)c->d_cube_ptrs));
    c->d_cube_ptrs = nullptr;
    NSFRB_HIP_TRY(hipMalloc((void**)&c->d_cube_ptrs, sizeof(void*) * n_cubes));
    c->cube_ptrs_cap = n_cubes;
  }
  NSFRB_HIP_TRY(hipMemcpy(c->d_cut_desc, host_desc, sizeof(nsfrb_cutout) * n_cut, hipMemcpyHostToDevice));
  NSFRB_HIP_TRY(hipMemcpy(c->d_delays, host_delays, sizeof(int) * n_dm * n_sub, hipMemcpyHostToDevice));
  NSFRB_HIP_TRY(hipMemcpy((void*)c->d_cube_ptrs, d_z_cubes, sizeof(void*) * n_cubes, hipMemcpyHostToDevice));
  NSFRB_HIP_TRY(launch_cutouts(store_dtype, c->d_cube_ptrs, c->d_cut_desc, c->d_delays, n_cut, nx, ny, n_sub, n_time,
                               c->cfg.n_time, (uint16_t*)d_out, st));
  return NSFRB_OK;
}

extern "C" nsfrb_status nsfrb_inject_rfi(void* d_cube, int32_t dtype, int32_t layout, int32_t n_pix, int32_t n_sub,
                                         int32_t n_time, int32_t kind, int32_t t0, int32_t len, int32_t sub_band,
                                         float amp, void* stream) {
  host_clear_error();
  if (!d_cube || dtype < 0 || dtype > 2 || (layout != 0 && layout != 1) || n_pix < 1 || n_sub < 1 || n_time < 1 ||
      (kind != 0 && kind != 1) || (kind == 1 && (len < 1 || sub_band < 0 || sub_band >= n_sub)) || !std::isfinite(amp))
    return host_fail(NSFRB_ERR_INVALID_ARG, "bad interference arguments");
  NSFRB_HIP_TRY(launch_inject_rfi(d_cube, dtype, layout, n_pix, n_sub, n_time, kind, t0, len, sub_band, amp,
                                  (hipStream_t)stream));
  return NSFRB_OK;
}
