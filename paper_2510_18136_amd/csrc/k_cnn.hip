// Candidate classifier on the GPU: a 3-D CNN over dedispersed candidate
// cutouts, trained with hand-written BF16 MFMA kernels (paper section 2.3: a
// CNN over the image cube centred on the TOA, convolution blocks with
// nonlinearities, a small fully connected head, a logit whose sigmoid is the
// RFI probability, Adam on a binary cross-entropy loss).
//
// Network (fixed shape): input x[n][t][y][x][16] (sub-bands as channels,
// x = 32 wide), four 3x3x3 'same' convolutions with 32 output channels and
// ReLU; head input = every channel's global maximum and its value at the
// candidate's position (64 features); 64->32 ReLU, 32->1 logit.
//
// Tensors are channels-last BF16; accumulation is FP32 on the matrix cores
// (v_mfma_f32_32x32x8_bf16: D[32x32] += A[32x8] * B[8x32]; lane l holds
// A[l%32][4(l/32)..+3], B[4(l/32)..+3][l%32], D[8(r/4)+4(l/32)+r%4][l%32]).
//  * convolution (forward, and backward-data with transposed, flipped
//    weights): one wave per output row (n, t, y): M = 32 output channels,
//    N = the 32 x positions, K = 27 taps x input channels; weights in LDS;
//  * weight gradient: M = 32 output channels, N = input channels, K =
//    positions; each output row's pre-activation gradient (transposed) and
//    the nine input rows of its taps are staged in LDS; each workgroup writes
//    its partial sums, which a second kernel adds in a fixed order.
#include <algorithm>

#include "device_common.h"
#include "nsfrb_internal.h"

namespace nsfrb {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int kCH = 32;       // hidden channels (conv outputs)
constexpr int kXW = 32;       // cutout width (x)
constexpr int kTaps = 27;

__device__ __forceinline__ uint16_t f2bf(float v) { return from_f32<bf16_t>(v).bits; }
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// ------------------------------------------------------------ convolution
// MODE 0: out = bf16(relu(conv + bias)).   MODE 1: out = bf16(conv * (mask > 0)).
template <int CIN, int MODE>
__global__ __launch_bounds__(256) void k_conv3(const uint16_t* __restrict__ in, const uint16_t* __restrict__ w,
                                               const float* __restrict__ bias, const uint16_t* __restrict__ mask,
                                               uint16_t* __restrict__ out, int N, int T, int Y) {
  __shared__ __attribute__((aligned(16))) uint16_t wl[kCH * kTaps * CIN];
  for (int i = threadIdx.x; i < kCH * kTaps * CIN / 4; i += blockDim.x)
    reinterpret_cast<uint2*>(wl)[i] = reinterpret_cast<const uint2*>(w)[i];
  __syncthreads();
  const long long rows = (long long)N * T * Y;
  const long long row = (long long)blockIdx.x * 4 + threadIdx.x / 64;
  if (row >= rows) return;                                   // no barrier below
  const int l = lane_id();
  const int n = (int)(row / ((long long)T * Y));
  const int t = (int)((row / Y) % T);
  const int y = (int)(row % Y);
  const int x = l & 31, kq = l >> 5, co = l & 31;
  v16f acc = {};
#pragma unroll 1
  for (int tap = 0; tap < kTaps; ++tap) {
    const int kt = tap / 9, ky = (tap / 3) % 3, kx = tap % 3;
    const int tt = t + kt - 1, yy = y + ky - 1, xx = x + kx - 1;
    const bool ok = tt >= 0 && tt < T && yy >= 0 && yy < Y && xx >= 0 && xx < kXW;
    const uint16_t* src = in + ((((size_t)n * T + (ok ? tt : 0)) * Y + (ok ? yy : 0)) * kXW + (ok ? xx : 0)) * CIN;
#pragma unroll
    for (int k8 = 0; k8 < CIN / 8; ++k8) {
      const int ci = k8 * 8 + kq * 4;
      const v4s a = *reinterpret_cast<const v4s*>(&wl[(co * kTaps + tap) * CIN + ci]);
      v4s b = {0, 0, 0, 0};
      if (ok) b = *reinterpret_cast<const v4s*>(src + ci);
      acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
    }
  }
  const size_t pos = (((size_t)n * T + t) * Y + y) * kXW + x;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int c0 = 8 * g + 4 * kq;
    uint16_t o[4];
    if (MODE == 1) {
      const uint2 mk = *reinterpret_cast<const uint2*>(mask + pos * kCH + c0);
      const uint16_t mv[4] = {(uint16_t)(mk.x & 0xffff), (uint16_t)(mk.x >> 16), (uint16_t)(mk.y & 0xffff),
                              (uint16_t)(mk.y >> 16)};
#pragma unroll
      for (int j = 0; j < 4; ++j) o[j] = f2bf(bf2f(mv[j]) > 0.0f ? acc[4 * g + j] : 0.0f);
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) o[j] = f2bf(fmaxf(acc[4 * g + j] + bias[c0 + j], 0.0f));
    }
    uint2 pk;
    pk.x = (uint32_t)o[0] | ((uint32_t)o[1] << 16);
    pk.y = (uint32_t)o[2] | ((uint32_t)o[3] << 16);
    *reinterpret_cast<uint2*>(out + pos * kCH + c0) = pk;
  }
}

// --------------------------------------------------------- weight gradient
// Work item = (n, chunk of kTch time planes). Per output row (t, y) the
// pre-activation gradient row is staged transposed (dT[co][x], so an A operand
// is one aligned 8-byte read) and the nine input rows of the taps are staged
// channels-last with a zero halo in x (xr[r][x + 1][ci]); a B operand (four
// positions of one channel) is four 2-byte reads. Wave w accumulates taps
// w, w + 4, ... (at most 7) for all (co, ci).
constexpr int kTch = 8;
constexpr int kXP = 36;       // transposed row pitch (x = 0..31, multiple of 4)

template <int CIN>
__global__ __launch_bounds__(256) void k_conv3_wgrad(const uint16_t* __restrict__ x, const uint16_t* __restrict__ dpre,
                                                     float* __restrict__ part, float* __restrict__ part_db, int N,
                                                     int T, int Y) {
  __shared__ __attribute__((aligned(16))) uint16_t dT[kCH * kXP];
  __shared__ __attribute__((aligned(16))) uint16_t xr[9 * (kXW + 2) * CIN];
  const int l = lane_id(), wv = threadIdx.x / 64;
  const int chunks = (T + kTch - 1) / kTch;
  const int n = blockIdx.x / chunks, t0 = (blockIdx.x % chunks) * kTch;
  const int col = l & 31, kq = l >> 5;
  v16f acc[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) acc[k] = v16f{};
  float dbsum = 0.f;
  constexpr int V8 = CIN / 8;              // 16-byte vectors per position
  for (int t = t0; t < t0 + kTch && t < T; ++t) {
    for (int y = 0; y < Y; ++y) {
      __syncthreads();
      for (int i = threadIdx.x; i < kXW * kCH; i += blockDim.x) {
        const int xx = i / kCH, c = i % kCH;
        dT[c * kXP + xx] = dpre[((((size_t)n * T + t) * Y + y) * kXW + xx) * kCH + c];
      }
      for (int i = threadIdx.x; i < 9 * (kXW + 2) * V8; i += blockDim.x) {
        const int r = i / ((kXW + 2) * V8), rem = i % ((kXW + 2) * V8);
        const int xh = rem / V8, v8 = rem % V8;          // xh = x + 1
        const int tt = t + r / 3 - 1, yy = y + r % 3 - 1, xs = xh - 1;
        uint4 v = {0u, 0u, 0u, 0u};
        if (tt >= 0 && tt < T && yy >= 0 && yy < Y && xs >= 0 && xs < kXW)
          v = *reinterpret_cast<const uint4*>(x + ((((size_t)n * T + tt) * Y + yy) * kXW + xs) * CIN + v8 * 8);
        *reinterpret_cast<uint4*>(&xr[(r * (kXW + 2) + xh) * CIN + v8 * 8]) = v;
      }
      __syncthreads();
      if (threadIdx.x < kCH) {
        float sacc = 0.f;
        for (int xx = 0; xx < kXW; ++xx) sacc += bf2f(dT[threadIdx.x * kXP + xx]);
        dbsum += sacc;
      }
#pragma unroll
      for (int k = 0; k < 7; ++k) {
        const int tap = wv + 4 * k;
        if (tap < kTaps) {
          const int r = (tap / 9) * 3 + (tap / 3) % 3, kx = tap % 3;
#pragma unroll
          for (int s8 = 0; s8 < kXW / 8; ++s8) {
            const int xb = s8 * 8 + kq * 4;
            const v4s a = *reinterpret_cast<const v4s*>(&dT[col * kXP + xb]);   // A[co][pos]
            v4s b = {0, 0, 0, 0};                                                // B[pos][ci]
            if (col < CIN) {
              const uint16_t* pb = &xr[(r * (kXW + 2) + xb + kx) * CIN + col];   // input x = xb + kx - 1
              b[0] = (short)pb[0];
              b[1] = (short)pb[CIN];
              b[2] = (short)pb[2 * CIN];
              b[3] = (short)pb[3 * CIN];
            }
            acc[k] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc[k], 0, 0, 0);
          }
        }
      }
    }
  }
  // partial sums of this item, in the parameter layout: part[item][co][tap][ci]
  float* pb = part + (size_t)blockIdx.x * kTaps * kCH * CIN;
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    const int tap = wv + 4 * k;
    if (tap < kTaps && col < CIN) {
#pragma unroll
      for (int rg = 0; rg < 16; ++rg) {
        const int co = 8 * (rg / 4) + 4 * kq + (rg % 4);
        pb[((size_t)co * kTaps + tap) * CIN + col] = acc[k][rg];
      }
    }
  }
  if (threadIdx.x < kCH) part_db[(size_t)blockIdx.x * kCH + threadIdx.x] = dbsum;
}

// out[i] = sum over items of part[item][i] (fixed order, deterministic).
__global__ void k_reduce_items(const float* __restrict__ part, int n_items, int len, float* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  float s = 0.f;
  for (int it = 0; it < n_items; ++it) s += part[(size_t)it * len + i];
  out[i] = s;
}

// ------------------------------------------------------------------- head
// h[n] = [m, q]: m[c] = max over positions of act[n][pos][c] (first position on
// ties; its index goes to arg[n][c]), q[c] = act at the candidate's position.
__global__ __launch_bounds__(256) void k_pool(const uint16_t* __restrict__ act, int npos, int centre,
                                              float* __restrict__ h, int* __restrict__ arg) {
  __shared__ float rv[8 * kCH];
  __shared__ int ri[8 * kCH];
  const int n = blockIdx.x;
  const int c = threadIdx.x % kCH, part = threadIdx.x / kCH;          // 8 interleaved parts of the positions
  const uint16_t* a = act + (size_t)n * npos * kCH + c;
  float best = -1.f;                                                  // activations are >= 0
  int bi = 0;
  for (int p = part; p < npos; p += 8) {
    const float v = bf2f(a[(size_t)p * kCH]);
    if (v > best) { best = v; bi = p; }                               // increasing p: first maximum kept
  }
  rv[part * kCH + c] = best;
  ri[part * kCH + c] = bi;
  __syncthreads();
  if (threadIdx.x < kCH) {
    float m = rv[c];
    int mi = ri[c];
    for (int k = 1; k < 8; ++k) {
      const float v = rv[k * kCH + c];
      const int i = ri[k * kCH + c];
      if (v > m || (v == m && i < mi)) { m = v; mi = i; }
    }
    h[(size_t)n * 2 * kCH + c] = m;
    h[(size_t)n * 2 * kCH + kCH + c] = bf2f(a[(size_t)centre * kCH]);
    arg[(size_t)n * kCH + c] = mi;
  }
}

// MLP head (64 -> 32 ReLU -> 1), BCE-with-logits loss and its backward pass for
// a batch of n <= 1024. theta_head = [W1[32][64], c1[32], w2[32], c2[1]];
// gradients are written in the same order.
constexpr int kH = 2 * kCH;
__global__ __launch_bounds__(256) void k_head(const float* __restrict__ h, const float* __restrict__ labels, int n,
                                              const float* __restrict__ th, float* __restrict__ gh,
                                              float* __restrict__ dh, float* __restrict__ logits,
                                              float* __restrict__ prob, float* __restrict__ loss_out, int backward) {
  __shared__ float W1[kCH * kH], c1[kCH], w2[kCH];
  __shared__ float gW1[kCH * kH], gc1[kCH], gw2[kCH], gc2, lsum;
  for (int i = threadIdx.x; i < kCH * kH; i += blockDim.x) { W1[i] = th[i]; gW1[i] = 0.f; }
  if (threadIdx.x < kCH) {
    c1[threadIdx.x] = th[kCH * kH + threadIdx.x];
    w2[threadIdx.x] = th[kCH * kH + kCH + threadIdx.x];
    gc1[threadIdx.x] = 0.f;
    gw2[threadIdx.x] = 0.f;
  }
  if (threadIdx.x == 0) { gc2 = 0.f; lsum = 0.f; }
  __syncthreads();
  const float c2 = th[kCH * kH + 2 * kCH];
  // one thread per sample: forward, loss, backward into per-sample dh; weight
  // gradients summed with atomics in LDS (float adds of one batch)
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const float* hv = h + (size_t)i * kH;
    float u[kCH];
    float z = c2;
    for (int j = 0; j < kCH; ++j) {
      float s = c1[j];
      for (int c = 0; c < kH; ++c) s += W1[j * kH + c] * hv[c];
      u[j] = s;
      z += w2[j] * fmaxf(s, 0.f);
    }
    logits[i] = z;
    prob[i] = 1.0f / (1.0f + expf(-z));
    if (backward) {
      const float yv = labels[i];
      const float li = fmaxf(z, 0.f) - z * yv + log1pf(expf(-fabsf(z)));
      atomicAdd(&lsum, li / (float)n);
      const float dz = (1.0f / (1.0f + expf(-z)) - yv) / (float)n;
      atomicAdd(&gc2, dz);
      for (int j = 0; j < kCH; ++j) {
        atomicAdd(&gw2[j], dz * fmaxf(u[j], 0.f));
        u[j] = u[j] > 0.f ? dz * w2[j] : 0.f;                         // u now holds d(loss)/du
        if (u[j] != 0.f) {
          atomicAdd(&gc1[j], u[j]);
          for (int c = 0; c < kH; ++c) atomicAdd(&gW1[j * kH + c], u[j] * hv[c]);
        }
      }
      for (int c = 0; c < kH; ++c) {
        float d = 0.f;
        for (int j = 0; j < kCH; ++j) d += u[j] * W1[j * kH + c];
        dh[(size_t)i * kH + c] = d;
      }
    }
  }
  __syncthreads();
  if (backward) {
    for (int i = threadIdx.x; i < kCH * kH; i += blockDim.x) gh[i] = gW1[i];
    if (threadIdx.x < kCH) {
      gh[kCH * kH + threadIdx.x] = gc1[threadIdx.x];
      gh[kCH * kH + kCH + threadIdx.x] = gw2[threadIdx.x];
    }
    if (threadIdx.x == 0) {
      gh[kCH * kH + 2 * kCH] = gc2;
      loss_out[0] = lsum;
    }
  }
}

// dpre4[n][pos][c] = bf16(g * (act4[n][pos][c] > 0)) with g = dm[n][c] at the
// channel's maximum, + dq[n][c] at the candidate position, 0 elsewhere.
__global__ void k_pool_backward(const float* __restrict__ dh, const int* __restrict__ arg,
                                const uint16_t* __restrict__ act, int npos, int centre, long long total,
                                uint16_t* __restrict__ dpre) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const int c = (int)(i % kCH);
    const long long r = i / kCH;
    const int pos = (int)(r % npos);
    const long long n = r / npos;
    float g = 0.f;
    if (pos == arg[n * kCH + c]) g = dh[n * kH + c];
    if (pos == centre) g += dh[n * kH + kCH + c];
    dpre[i] = f2bf(bf2f(act[i]) > 0.f ? g : 0.f);
  }
}

// ------------------------------------------------------------ optimiser
__global__ void k_adam(float* __restrict__ th, float* __restrict__ m, float* __restrict__ v, const float* __restrict__ g,
                       int n, float lr, float b1, float b2, float eps, float bc1, float bc2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// BF16 copies of a conv layer's weights: forward layout [co][tap][ci] and the
// backward-data layout [ci][26 - tap][co] (transposed channels, flipped taps).
__global__ void k_prep_weights(const float* __restrict__ wsrc, int cin, uint16_t* __restrict__ wf,
                               uint16_t* __restrict__ wb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int total = kCH * kTaps * cin;
  if (i >= total) return;
  const int co = i / (kTaps * cin), tap = (i / cin) % kTaps, ci = i % cin;
  const uint16_t b = f2bf(wsrc[i]);
  wf[i] = b;
  if (wb) wb[((size_t)ci * kTaps + (kTaps - 1 - tap)) * kCH + co] = b;
}

// ------------------------------------------------------------- cutouts
// Dedispersion-aligned cutout around a candidate: out[k][tt][y][x][s] =
// z[pixel (px + x - 16, py + y - 16)][s][toa - ct/2 + tt + delta[dm][s]], zero
// outside the image or the series. Each z cube is [n_pix][n_sub][n_t] in the
// store dtype; descriptor k names its cube by an index into a pointer table.
struct CutoutDesc {
  long long cube;
  int px, py, dm, toa;
};

template <typename ST>
__global__ void k_cutouts(const ST* const* __restrict__ cubes, const CutoutDesc* __restrict__ desc,
                          const int* __restrict__ delays, int nx, int ny, int n_sub, int n_t, int ct,
                          uint16_t* __restrict__ out, long long total) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const int s = (int)(i % n_sub);
    long long r = i / n_sub;
    const int x = (int)(r % kXW); r /= kXW;
    const int y = (int)(r % kXW); r /= kXW;
    const int tt = (int)(r % ct);
    const int k = (int)(r / ct);
    const CutoutDesc d = desc[k];
    const int xi = d.px + x - kXW / 2, yi = d.py + y - kXW / 2;
    const int t = d.toa - ct / 2 + tt + delays[d.dm * n_sub + s];
    float v = 0.f;
    if (xi >= 0 && xi < nx && yi >= 0 && yi < ny && t >= 0 && t < n_t)
      v = to_f32(cubes[d.cube][((size_t)(yi * nx + xi) * n_sub + s) * n_t + t]);
    out[i] = f2bf(v);
  }
}

// --------------------------------------------------------------- launchers
hipError_t launch_conv_fwd(int cin, const uint16_t* in, const uint16_t* w, const float* bias, uint16_t* out, int N,
                           int T, int Y, hipStream_t st) {
  const long long rows = (long long)N * T * Y;
  const unsigned grid = (unsigned)((rows + 3) / 4);
  if (cin == 16) hipLaunchKernelGGL((k_conv3<16, 0>), dim3(grid), dim3(256), 0, st, in, w, bias, nullptr, out, N, T, Y);
  else hipLaunchKernelGGL((k_conv3<32, 0>), dim3(grid), dim3(256), 0, st, in, w, bias, nullptr, out, N, T, Y);
  return hipGetLastError();
}

hipError_t launch_conv_bwd_data(const uint16_t* dpre, const uint16_t* wb, const uint16_t* mask_act, uint16_t* out, int N,
                                int T, int Y, hipStream_t st) {
  const long long rows = (long long)N * T * Y;
  hipLaunchKernelGGL((k_conv3<32, 1>), dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st, dpre, wb, nullptr, mask_act,
                     out, N, T, Y);
  return hipGetLastError();
}

int wgrad_items(int N, int T) { return N * ((T + kTch - 1) / kTch); }

hipError_t launch_conv_wgrad(int cin, const uint16_t* x, const uint16_t* dpre, float* part, float* part_db, float* dw,
                             float* db, int N, int T, int Y, hipStream_t st) {
  const int items = wgrad_items(N, T);
  if (cin == 16) hipLaunchKernelGGL((k_conv3_wgrad<16>), dim3(items), dim3(256), 0, st, x, dpre, part, part_db, N, T, Y);
  else hipLaunchKernelGGL((k_conv3_wgrad<32>), dim3(items), dim3(256), 0, st, x, dpre, part, part_db, N, T, Y);
  const int len = kTaps * kCH * cin;
  hipLaunchKernelGGL(k_reduce_items, dim3((len + 255) / 256), dim3(256), 0, st, part, items, len, dw);
  hipLaunchKernelGGL(k_reduce_items, dim3(1), dim3(kCH), 0, st, part_db, items, kCH, db);
  return hipGetLastError();
}

hipError_t launch_pool(const uint16_t* act, int N, int npos, int centre, float* h, int* arg, hipStream_t st) {
  hipLaunchKernelGGL(k_pool, dim3(N), dim3(256), 0, st, act, npos, centre, h, arg);
  return hipGetLastError();
}

hipError_t launch_head(const float* h, const float* labels, int n, const float* th, float* gh, float* dh, float* logits,
                       float* prob, float* loss, int backward, hipStream_t st) {
  hipLaunchKernelGGL(k_head, dim3(1), dim3(256), 0, st, h, labels, n, th, gh, dh, logits, prob, loss, backward);
  return hipGetLastError();
}

hipError_t launch_pool_backward(const float* dh, const int* arg, const uint16_t* act, int N, int npos, int centre,
                                uint16_t* dpre, hipStream_t st) {
  const long long total = (long long)N * npos * kCH;
  const unsigned grid = (unsigned)std::min<long long>((total + 255) / 256, 65536LL * 4);
  hipLaunchKernelGGL(k_pool_backward, dim3(grid), dim3(256), 0, st, dh, arg, act, npos, centre, total, dpre);
  return hipGetLastError();
}

hipError_t launch_adam(float* th, float* m, float* v, const float* g, int n, float lr, float b1, float b2, float eps,
                       float bc1, float bc2, hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, st, th, m, v, g, n, lr, b1, b2, eps, bc1, bc2);
  return hipGetLastError();
}

hipError_t launch_prep_weights(const float* wsrc, int cin, uint16_t* wf, uint16_t* wb, hipStream_t st) {
  const int total = kCH * kTaps * cin;
  hipLaunchKernelGGL(k_prep_weights, dim3((total + 255) / 256), dim3(256), 0, st, wsrc, cin, wf, wb);
  return hipGetLastError();
}

hipError_t launch_cutouts(int store_dtype, const void* const* cubes, const void* desc, const int* delays, int n_cut,
                          int nx, int ny, int n_sub, int n_t, int ct, uint16_t* out, hipStream_t st) {
  const long long total = (long long)n_cut * ct * kXW * kXW * n_sub;
  const unsigned grid = (unsigned)std::min<long long>((total + 255) / 256, 65536LL * 4);
  const CutoutDesc* d = (const CutoutDesc*)desc;
  if (store_dtype == DT_F32)
    hipLaunchKernelGGL(k_cutouts<float>, dim3(grid), dim3(256), 0, st, (const float* const*)cubes, d, delays, nx, ny,
                       n_sub, n_t, ct, out, total);
  else if (store_dtype == DT_F16)
    hipLaunchKernelGGL(k_cutouts<_Float16>, dim3(grid), dim3(256), 0, st, (const _Float16* const*)cubes, d, delays, nx,
                       ny, n_sub, n_t, ct, out, total);
  else
    hipLaunchKernelGGL(k_cutouts<bf16_t>, dim3(grid), dim3(256), 0, st, (const bf16_t* const*)cubes, d, delays, nx, ny,
                       n_sub, n_t, ct, out, total);
  return hipGetLastError();
}

}  // namespace nsfrb
