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
// Tensors are channels-last BF16; accumulation is FP32 on the matrix cores.
//  * convolution (forward, and backward-data with transposed, flipped
//    weights): implicit GEMM on v_mfma_f32_32x32x16_bf16 with the weights and a
//    ring of input planes in LDS (see k_conv3);
//  * weight gradient (v_mfma_f32_32x32x8_bf16: lane l holds A[l%32][4(l/32)..+3],
//    B[4(l/32)..+3][l%32], D[8(r/4)+4(l/32)+r%4][l%32]): M = 32 output
//    channels, N = input channels, K = positions; each output row's
//    pre-activation gradient (transposed) and the nine input rows of its taps
//    are staged in LDS; each workgroup writes its partial sums, which a second
//    kernel adds in a fixed order.
#include <algorithm>

#include "device_common.h"
#include "nsfrb_internal.h"

namespace nsfrb {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int kCH = 32;       // hidden channels (conv outputs)
constexpr int kXW = 32;       // cutout width (x)
constexpr int kTaps = 27;

__device__ __forceinline__ uint16_t f2bf(float v) { return from_f32<bf16_t>(v).bits; }
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// ------------------------------------------------------------ convolution
// MODE 0: out = bf16(relu(conv + bias)).   MODE 1: out = bf16(conv * (mask > 0)).
//
// Implicit GEMM on v_mfma_f32_32x32x16_bf16 (D[32x32] += A[32x16] * B[16x32];
// lane l holds A[l%32][8(l/32)..+7] and B[8(l/32)..+7][l%32] as eight BF16, and
// D as for the 32x32x8 form). Per output row (n, t, y): M = 32 output channels,
// N = the 32 x positions, K = 27 taps x CIN input channels in steps of 16.
// A workgroup of 8 waves takes (n, 8 consecutive y, up to kConvTT consecutive
// t); wave w computes row y0 + w of each plane in turn. The weights sit in LDS
// in operand order (step s, lane l: 16 bytes), so each A operand is one
// conflict-free 16-byte read. Input planes t-1, t, t+1 (rows y0-1 .. y0+8, a
// zero halo in x) live in a 4-slot ring; the loads of plane t+2 are issued
// before the matrix work of plane t and stored into the free slot after it. In
// a staged row the 16-byte channel chunk c of position xs sits at chunk
// c ^ swz(xs), so the 32 lanes of a B read hit distinct banks.
constexpr int kConvWaves = 8;
constexpr int kConvYT = kConvWaves;       // output rows (y) per plane per workgroup
constexpr int kConvRY = kConvYT + 2;      // staged rows per plane (y halo)
constexpr int kConvXS = kXW + 2;          // staged positions per row (x halo)
constexpr int kConvTT = 16;               // planes per workgroup

template <int CIN>
__device__ __forceinline__ int conv_swz(int xs) {
  constexpr int G8 = CIN / 8;             // 16-byte chunks per position
  return (xs / (8 / G8)) & (G8 - 1);
}

template <int CIN, int MODE>
__global__ __launch_bounds__(kConvWaves * kWave) void k_conv3(const uint16_t* __restrict__ in,
                                                              const uint16_t* __restrict__ wm,
                                                              const float* __restrict__ bias,
                                                              const uint16_t* __restrict__ mask,
                                                              uint16_t* __restrict__ out, int N, int T, int Y) {
  constexpr int G8 = CIN / 8;
  constexpr int S = kTaps * CIN / 16;                    // K steps
  constexpr int ROW = kConvXS * G8;                      // 16-byte chunks per staged row
  constexpr int SLOT = kConvRY * ROW;
  constexpr int PLANE = kConvRY * kXW * G8;              // chunks loaded per plane
  constexpr int NT = kConvWaves * kWave;
  constexpr int PER = (PLANE + NT - 1) / NT;
  __shared__ uint4 wl[S * kWave];
  __shared__ uint4 xl[4 * SLOT];

  const int n_yb = (Y + kConvYT - 1) / kConvYT, n_tb = (T + kConvTT - 1) / kConvTT;
  const int blk = blockIdx.x;
  const int tb = blk % n_tb, yb = (blk / n_tb) % n_yb, n = blk / (n_tb * n_yb);
  const int y0 = yb * kConvYT, t0 = tb * kConvTT, t1 = min(t0 + kConvTT, T);
  const int tid = threadIdx.x, l = lane_id();
  const int w = __builtin_amdgcn_readfirstlane(tid / kWave);

  for (int i = tid; i < S * kWave; i += NT) wl[i] = reinterpret_cast<const uint4*>(wm)[i];
  for (int i = tid; i < 4 * kConvRY * 2 * G8; i += NT) {           // x halo of every slot and row
    const int c = i % G8, side = (i / G8) % 2, r = i / (2 * G8);
    xl[r * ROW + (side ? kConvXS - 1 : 0) * G8 + c] = make_uint4(0u, 0u, 0u, 0u);
  }
  // plane tp -> registers (zero outside the cube)
  auto fetch = [&](int tp, uint4 (&v)[PER]) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int i = tid + q * NT;
      const int c = i % G8, x = (i / G8) % kXW, ry = i / (G8 * kXW);
      const int y = y0 - 1 + ry;
      const bool ok = i < PLANE && tp >= 0 && tp < T && y >= 0 && y < Y;
      v[q] = ok ? reinterpret_cast<const uint4*>(in + ((((size_t)n * T + tp) * Y + y) * kXW + x) * CIN)[c]
                : make_uint4(0u, 0u, 0u, 0u);
    }
  };
  auto stage = [&](int tp, const uint4 (&v)[PER]) {
    uint4* sl = xl + (tp & 3) * SLOT;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int i = tid + q * NT;
      if (i < PLANE) {
        const int c = i % G8, x = (i / G8) % kXW, ry = i / (G8 * kXW);
        const int xs = x + 1;
        sl[ry * ROW + xs * G8 + (c ^ conv_swz<CIN>(xs))] = v[q];
      }
    }
  };
  {
    uint4 v[PER];
    fetch(t0 - 1, v);
    stage(t0 - 1 + 4, v);            // slot index uses tp & 3; keep it non-negative
    fetch(t0, v);
    stage(t0, v);
    fetch(t0 + 1, v);
    stage(t0 + 1, v);
  }
  __syncthreads();

  const int x = l & 31, half = l >> 5;
  int hs[3];
#pragma unroll
  for (int dx = 0; dx < 3; ++dx) hs[dx] = half ^ conv_swz<CIN>(x + dx);
  const int y = y0 + w;
  const bool row_ok = y < Y;
  const v8bf* wa = reinterpret_cast<const v8bf*>(wl) + l;
  for (int t = t0; t < t1; ++t) {
    uint4 v[PER];
    fetch(t + 2, v);
    if (row_ok) {
      v16f acc = {};
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int tap = s / (CIN / 16), kb = s % (CIN / 16);
        const int dt = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
        const uint4* rowp = xl + ((t - 1 + dt + 4) & 3) * SLOT + (w + dy) * ROW + (x + dx) * G8;
        const uint4 bv = rowp[(2 * kb) ^ hs[dx]];
        v8bf b;
        __builtin_memcpy(&b, &bv, 16);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa[s * kWave], b, acc, 0, 0, 0);
      }
      const size_t pos = (((size_t)n * T + t) * Y + y) * kXW + x;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int c0 = 8 * g + 4 * half;
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
    stage(t + 2, v);                 // slot of plane t - 2, which step t does not read
    __syncthreads();
  }
}

// --------------------------------------------------------- weight gradient
// dW[co][tap][ci] = sum over positions of dpre[p][co] * in[p + offset(tap)][ci]
// and db[co] = sum of dpre[p][co]: per tap a GEMM with M = 32 output channels,
// N = input channels, K = positions, on v_mfma_f32_32x32x16_bf16.
//
// Work item = (sample n, 4 consecutive output rows y0 .. y0+3), streamed over
// every plane t. K at plane t runs over k = 32 r + x (row y0 + r, input
// position x). Both operands want eight consecutive k per lane, so the data
// are staged transposed: input rows y0-1 .. y0+4 of planes t-1, t, t+1 as
// inT[ci][x] in a 4-slot ring, and the plane's output-gradient rows as three
// copies dT_dx[co][32 r + x] = dpre[y0 + r][x + 1 - dx][co] (one per x-offset
// of the taps, zero where x + 1 - dx leaves the row), double-buffered. Wave w
// takes the three taps (dt, dy) = (w / 3, w % 3), dx = 0..2: per K step one B
// read and three A reads, all 16 bytes and conflict-free (row pitches padded).
// The next plane's loads are issued before the matrix work and stored after
// it. Each item writes its partial sums, which a second kernel adds in a fixed
// order (deterministic).
constexpr int kWgR = 4;                    // output rows per item
constexpr int kWgWaves = 9;                // one per (dt, dy)
constexpr int kWgRows = kWgR + 2;          // staged input rows per plane
constexpr int kWgXP = kXW + 8;             // inT row pitch (bf16): 80 bytes
constexpr int kWgKP = kWgR * kXW + 8;      // dT row pitch (bf16): 272 bytes

int wgrad_items(int N, int Y) { return N * ((Y + kWgR - 1) / kWgR); }

template <int CIN>
__global__ __launch_bounds__(kWgWaves * kWave) void k_conv3_wgrad(const uint16_t* __restrict__ x,
                                                                  const uint16_t* __restrict__ dpre,
                                                                  float* __restrict__ part,
                                                                  float* __restrict__ part_db, int N, int T,
                                                                  int Y) {
  constexpr int NT = kWgWaves * kWave;
  constexpr int G8 = CIN / 8;
  constexpr int SLOT = kWgRows * CIN * kWgXP;                 // bf16 per ring slot
  constexpr int DCOPY = kCH * kWgKP;                          // bf16 per dT copy
  constexpr int IN_CH = kWgRows * kXW * G8;                   // 16-byte chunks per input plane slice
  constexpr int D_CH = kWgR * kXW * (kCH / 8);                // 16-byte chunks per dpre plane slice
  constexpr int IN_PER = (IN_CH + NT - 1) / NT;
  static_assert(D_CH <= NT, "one dpre chunk per thread");
  __shared__ __attribute__((aligned(16))) uint16_t inT[4 * SLOT];
  __shared__ __attribute__((aligned(16))) uint16_t dT[2 * 3 * DCOPY];
  __shared__ float dbs[kCH * (D_CH / (kCH / 8))];              // per-thread bias partials, reduced at the end

  const int n_yb = (Y + kWgR - 1) / kWgR;
  const int n = blockIdx.x / n_yb, y0 = (blockIdx.x % n_yb) * kWgR;
  const int tid = threadIdx.x, l = lane_id();
  const int w = __builtin_amdgcn_readfirstlane(tid / kWave);
  const int dt = w / 3, dy = w % 3;

  // dT entries that no store reaches (the row ends of the shifted copies) stay 0
  for (int i = tid; i < 2 * 3 * DCOPY; i += NT) dT[i] = 0;
  __syncthreads();

  auto fetch_in = [&](int tp, uint4 (&v)[IN_PER]) {
#pragma unroll
    for (int q = 0; q < IN_PER; ++q) {
      const int i = tid + q * NT;
      const int c = i % G8, xx = (i / G8) % kXW, ry = i / (G8 * kXW);
      const int y = y0 - 1 + ry;
      const bool ok = i < IN_CH && tp >= 0 && tp < T && y >= 0 && y < Y;
      v[q] = ok ? reinterpret_cast<const uint4*>(x + ((((size_t)n * T + tp) * Y + y) * kXW + xx) * CIN)[c]
                : make_uint4(0u, 0u, 0u, 0u);
    }
  };
  auto stage_in = [&](int tp, const uint4 (&v)[IN_PER]) {
    uint16_t* s = inT + ((tp + 4) & 3) * SLOT;
#pragma unroll
    for (int q = 0; q < IN_PER; ++q) {
      const int i = tid + q * NT;
      if (i < IN_CH) {
        const int c = i % G8, xx = (i / G8) % kXW, ry = i / (G8 * kXW);
        uint16_t* d = s + (ry * CIN + 8 * c) * kWgXP + xx;
        const uint32_t wv[4] = {v[q].x, v[q].y, v[q].z, v[q].w};
#pragma unroll
        for (int j = 0; j < 8; ++j) d[j * kWgXP] = (uint16_t)(wv[j / 2] >> (16 * (j & 1)));
      }
    }
  };
  // dpre plane tp (rows y0 .. y0+3) -> one chunk per thread (8 output channels of one position)
  const int dc = tid % (kCH / 8), dxp = (tid / (kCH / 8)) % kXW, dr = tid / (kCH / 8 * kXW);
  auto fetch_d = [&](int tp) {
    const bool ok = tid < D_CH && tp < T && y0 + dr < Y;
    return ok ? reinterpret_cast<const uint4*>(dpre + ((((size_t)n * T + tp) * Y + y0 + dr) * kXW + dxp) * kCH)[dc]
              : make_uint4(0u, 0u, 0u, 0u);
  };
  float dbp[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  auto stage_d = [&](int buf, const uint4& v) {
    if (tid < D_CH) {
      const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const uint16_t b = (uint16_t)(wv[j / 2] >> (16 * (j & 1)));
        dbp[j] += bf2f(b);
        uint16_t* d = dT + (size_t)buf * 3 * DCOPY + (8 * dc + j) * kWgKP + dr * kXW;
#pragma unroll
        for (int ddx = 0; ddx < 3; ++ddx) {
          const int xs = dxp - 1 + ddx;                      // input position paired with dpre position dxp
          if (xs >= 0 && xs < kXW) d[ddx * DCOPY + xs] = b;
        }
      }
    }
  };

  {
    uint4 v[IN_PER];
    fetch_in(-1, v);
    stage_in(-1, v);
    fetch_in(0, v);
    stage_in(0, v);
    fetch_in(1, v);
    stage_in(1, v);
    stage_d(0, fetch_d(0));
  }
  __syncthreads();

  v16f acc[3] = {v16f{}, v16f{}, v16f{}};
  const int col = l & 31, h = l >> 5;
  for (int t = 0; t < T; ++t) {
    uint4 vin[IN_PER];
    fetch_in(t + 2, vin);
    const uint4 vd = fetch_d(t + 1);
    const uint16_t* sb = inT + ((t - 1 + dt + 4) & 3) * SLOT + col * kWgXP;      // inT[.][ci = col][x]
    const uint16_t* sa = dT + (size_t)(t & 1) * 3 * DCOPY + col * kWgKP;         // dT_dx[co = col][k]
#pragma unroll
    for (int r = 0; r < kWgR; ++r) {
#pragma unroll
      for (int xh = 0; xh < 2; ++xh) {
        const int xo = 16 * xh + 8 * h;
        v8bf b = {};
        if (col < CIN) __builtin_memcpy(&b, sb + (r + dy) * CIN * kWgXP + xo, 16);
#pragma unroll
        for (int ddx = 0; ddx < 3; ++ddx) {
          v8bf a;
          __builtin_memcpy(&a, sa + ddx * DCOPY + r * kXW + xo, 16);
          acc[ddx] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[ddx], 0, 0, 0);
        }
      }
    }
    stage_in(t + 2, vin);            // ring slot of plane t - 2, not read at step t
    stage_d((t + 1) & 1, vd);        // the other dT buffer
    __syncthreads();
  }

  // partial sums of this item, in the parameter layout part[item][co][tap][ci]
  float* pb = part + (size_t)blockIdx.x * kTaps * kCH * CIN;
  if (col < CIN) {
#pragma unroll
    for (int ddx = 0; ddx < 3; ++ddx) {
      const int tap = dt * 9 + dy * 3 + ddx;
#pragma unroll
      for (int rg = 0; rg < 16; ++rg) {
        const int co = 8 * (rg / 4) + 4 * h + (rg % 4);
        pb[((size_t)co * kTaps + tap) * CIN + col] = acc[ddx][rg];
      }
    }
  }
  // bias: thread tid holds channels 8 dc .. 8 dc + 7 of its positions
  if (tid < D_CH) {
#pragma unroll
    for (int j = 0; j < 8; ++j) dbs[(8 * dc + j) * (D_CH / (kCH / 8)) + tid / (kCH / 8)] = dbp[j];
  }
  __syncthreads();
  if (tid < kCH) {
    float s = 0.f;
    for (int i = 0; i < D_CH / (kCH / 8); ++i) s += dbs[tid * (D_CH / (kCH / 8)) + i];
    part_db[(size_t)blockIdx.x * kCH + tid] = s;
  }
}

// out[i] = sum over items of part[item][i] in a fixed order (deterministic):
// a workgroup takes 32 outputs; thread (o, c) adds items c, c + 8, ... of output
// o, and the eight partial sums are then added in order of c.
constexpr int kRedOut = 32, kRedPar = 8;
__global__ __launch_bounds__(kRedOut * kRedPar) void k_reduce_items(const float* __restrict__ part, int n_items,
                                                                    int len, float* __restrict__ out) {
  __shared__ float ps[kRedPar][kRedOut];
  const int o = threadIdx.x % kRedOut, c = threadIdx.x / kRedOut;
  const int i = blockIdx.x * kRedOut + o;
  float s = 0.f;
  if (i < len)
    for (int it = c; it < n_items; it += kRedPar) s += part[(size_t)it * len + i];
  ps[c][o] = s;
  __syncthreads();
  if (c == 0 && i < len) {
    float t = ps[0][o];
    for (int k = 1; k < kRedPar; ++k) t += ps[k][o];
    out[i] = t;
  }
}

// ------------------------------------------------------------------- head
// h[n] = [m, q]: m[c] = max over positions of act[n][pos][c] (first position on
// ties; its index goes to arg[n][c]), q[c] = act at the candidate's position.
//
// Pass 1: G workgroups per sample, each over one chunk of positions, reduce a
// 32-bit key per channel, (value bits << 16) | (0xFFFF - offset in the chunk):
// activations are >= 0, so their BF16 bits order like their values and the
// larger key is the larger value, then the earlier position (a maximum, so the
// result does not depend on the order of the reduction). Pass 2 takes, for each
// (sample, channel), the first chunk that holds the largest value.
constexpr int kPoolChunks = 64;
constexpr int kPoolThreads = 256;

__device__ __forceinline__ uint32_t pool_key(uint32_t bits16, int off) {
  const uint32_t v = (bits16 & 0x8000u) ? 0u : bits16;               // -0 counts as 0
  return (v << 16) | (uint32_t)(0xFFFF - off);
}

__global__ __launch_bounds__(kPoolThreads) void k_pool_partial(const uint16_t* __restrict__ act, int npos, int chunk,
                                                               uint32_t* __restrict__ part) {
  __shared__ uint32_t red[kPoolThreads / kWave][kCH];
  const int n = blockIdx.y, g = blockIdx.x;
  const int cg = threadIdx.x & 3, r = threadIdx.x >> 2;                // 8 channels (16 bytes) per thread
  const int p0 = g * chunk, p1 = min(p0 + chunk, npos);
  const uint4* a = reinterpret_cast<const uint4*>(act + (size_t)n * npos * kCH) + cg;
  uint32_t k[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) k[q] = 0u;
#pragma unroll 4
  for (int p = p0 + r; p < p1; p += kPoolThreads / 4) {
    const uint4 v = a[(size_t)p * 4];
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
    const int off = p - p0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      k[2 * q] = max(k[2 * q], pool_key(w[q] & 0xFFFFu, off));
      k[2 * q + 1] = max(k[2 * q + 1], pool_key(w[q] >> 16, off));
    }
  }
#pragma unroll
  for (int q = 0; q < 8; ++q)
#pragma unroll
    for (int s = 4; s < kWave; s <<= 1) k[q] = max(k[q], (uint32_t)__shfl_xor((int)k[q], s));
  const int wv = threadIdx.x / kWave, l = threadIdx.x % kWave;
  if (l < 4) {
#pragma unroll
    for (int q = 0; q < 8; ++q) red[wv][cg * 8 + q] = k[q];
  }
  __syncthreads();
  if (threadIdx.x < kCH) {
    uint32_t m = red[0][threadIdx.x];
    for (int w = 1; w < kPoolThreads / kWave; ++w) m = max(m, red[w][threadIdx.x]);
    part[((size_t)n * gridDim.x + g) * kCH + threadIdx.x] = m;
  }
}

__global__ void k_pool_finish(const uint32_t* __restrict__ part, int n_chunks, int chunk, const uint16_t* __restrict__ act,
                              int N, int npos, int centre, float* __restrict__ h, int* __restrict__ arg) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N * kCH) return;
  const int n = i / kCH, c = i % kCH;
  uint32_t best = part[(size_t)n * n_chunks * kCH + c];
  int g_best = 0;
  for (int g = 1; g < n_chunks; ++g) {
    const uint32_t k = part[((size_t)n * n_chunks + g) * kCH + c];
    if ((k >> 16) > (best >> 16)) { best = k; g_best = g; }            // strictly larger: earlier chunk kept on ties
  }
  h[(size_t)n * 2 * kCH + c] = bf2f((uint16_t)(best >> 16));
  h[(size_t)n * 2 * kCH + kCH + c] = bf2f(act[((size_t)n * npos + centre) * kCH + c]);
  arg[i] = g_best * chunk + (0xFFFF - (int)(best & 0xFFFFu));
}

// MLP head (64 -> 32 ReLU -> 1) and BCE-with-logits loss for a batch of n.
// theta_head = [W1[32][64], c1[32], w2[32], c2[1]]; gradients use the same order.
// k_head_sample: one wave per sample (lane l: hidden unit l % 32, half l / 32 of
// the inputs): logit, probability and, when training, the sample's loss, its
// gradient dz, d(loss)/du, relu(u) (into hs[i][66]) and d(loss)/dh.
// k_head_grad: one thread per head parameter sums the samples in index order.
constexpr int kH = 2 * kCH;
constexpr int kHS = 2 * kCH + 2;          // per-sample record: du[32], relu(u)[32], dz, loss
constexpr int kHeadParams = kCH * kH + 2 * kCH + 1;

__global__ __launch_bounds__(256) void k_head_sample(const float* __restrict__ h, const float* __restrict__ labels,
                                                     int n, const float* __restrict__ th, float* __restrict__ hs,
                                                     float* __restrict__ dh, float* __restrict__ logits,
                                                     float* __restrict__ prob, int backward) {
  const int i = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  if (i >= n) return;                                                  // whole waves leave together
  const int l = threadIdx.x % kWave, j = l % kCH, hf = l / kCH;
  const float* hv = h + (size_t)i * kH + hf * kCH;
  const float* wr = th + j * kH + hf * kCH;
  float s = 0.f;
#pragma unroll 8
  for (int c = 0; c < kCH; ++c) s += wr[c] * hv[c];
  s += __shfl_xor(s, kCH);
  const float u = s + th[kCH * kH + j];
  const float ru = fmaxf(u, 0.f);
  const float w2 = th[kCH * kH + kCH + j];
  float t = hf == 0 ? w2 * ru : 0.f;
#pragma unroll
  for (int k = 1; k < kWave; k <<= 1) t += __shfl_xor(t, k);          // same sum in every lane
  const float z = th[kCH * kH + 2 * kCH] + t;
  const float p = 1.0f / (1.0f + expf(-z));
  if (l == 0) {
    logits[i] = z;
    prob[i] = p;
  }
  if (!backward) return;
  const float yv = labels[i];
  const float dz = (p - yv) / (float)n;
  const float du = u > 0.f ? dz * w2 : 0.f;
  float* rec = hs + (size_t)i * kHS;
  rec[l] = hf == 0 ? du : ru;
  if (l == 0) {
    rec[2 * kCH] = dz;
    rec[2 * kCH + 1] = fmaxf(z, 0.f) - z * yv + log1pf(expf(-fabsf(z)));
  }
  float d = 0.f;
  for (int k = 0; k < kCH; ++k) d += __shfl(du, k) * th[k * kH + l];
  dh[(size_t)i * kH + l] = d;
}

__global__ void k_head_grad(const float* __restrict__ h, const float* __restrict__ hs, int n, float* __restrict__ gh,
                            float* __restrict__ loss_out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > kHeadParams) return;
  float s = 0.f;
  if (p < kCH * kH) {                                                  // W1[j][c]: du_j * h_c
    const int j = p / kH, c = p % kH;
    for (int i = 0; i < n; ++i) s += hs[(size_t)i * kHS + j] * h[(size_t)i * kH + c];
  } else if (p < kCH * kH + kCH) {                                     // c1[j]: du_j
    const int j = p - kCH * kH;
    for (int i = 0; i < n; ++i) s += hs[(size_t)i * kHS + j];
  } else if (p < kCH * kH + 2 * kCH) {                                 // w2[j]: dz * relu(u_j)
    const int j = p - kCH * kH - kCH;
    for (int i = 0; i < n; ++i) s += hs[(size_t)i * kHS + 2 * kCH] * hs[(size_t)i * kHS + kCH + j];
  } else if (p == kHeadParams - 1) {                                   // c2: dz
    for (int i = 0; i < n; ++i) s += hs[(size_t)i * kHS + 2 * kCH];
  } else {                                                             // mean loss
    for (int i = 0; i < n; ++i) s += hs[(size_t)i * kHS + 2 * kCH + 1];
    loss_out[0] = s / (float)n;
    return;
  }
  gh[p] = s;
}

// dpre4[n][pos][c] = bf16(g * (act4[n][pos][c] > 0)) with g = dm[n][c] at the
// channel's maximum, + dq[n][c] at the candidate position, 0 elsewhere; eight
// channels (16 bytes) per thread.
__global__ void k_pool_backward(const float* __restrict__ dh, const int* __restrict__ arg,
                                const uint16_t* __restrict__ act, int npos, int centre, long long total8,
                                uint16_t* __restrict__ dpre) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total8;
       i += (long long)gridDim.x * blockDim.x) {
    const int cg = (int)(i & 3);
    const long long r = i >> 2;
    const int pos = (int)(r % npos);
    const long long n = r / npos;
    const uint4 av = reinterpret_cast<const uint4*>(act)[i];
    const uint32_t aw[4] = {av.x, av.y, av.z, av.w};
    const int* ar = arg + n * kCH + cg * 8;
    const float* dm = dh + n * kH + cg * 8;
    uint32_t ow[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      uint32_t o = 0;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int c = 2 * q + e;
        float g = 0.f;
        if (pos == ar[c]) g = dm[c];
        if (pos == centre) g += dm[kCH + c];
        const uint16_t ab = (uint16_t)(aw[q] >> (16 * e));
        o |= (uint32_t)f2bf(bf2f(ab) > 0.f ? g : 0.f) << (16 * e);
      }
      ow[q] = o;
    }
    reinterpret_cast<uint4*>(dpre)[i] = make_uint4(ow[0], ow[1], ow[2], ow[3]);
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

// BF16 copies of a conv layer's weights in convolution-operand order: element
// (s, l, j) (K step s, lane l, element j; 16 bytes per lane and step) holds the
// weight of output channel l % 32 at K index 16 s + 8 (l / 32) + j, K running
// over (tap, input channel). Forward: W[co][tap][ci]. Backward-data (input
// gradient as a convolution of the output gradient): output channel = forward
// input channel, K over (tap', forward output channel) with tap' = 26 - tap
// (flipped taps, transposed channels).
__global__ void k_prep_weights(const float* __restrict__ wsrc, int cin, uint16_t* __restrict__ wf,
                               uint16_t* __restrict__ wb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int total = kCH * kTaps * cin;
  if (i >= total) return;
  const int s = i / 512, l = (i / 8) % 64, j = i % 8;
  const int m = l % 32, kk = 16 * s + 8 * (l / 32) + j;
  {
    const int tap = kk / cin, ci = kk % cin;
    wf[i] = f2bf(wsrc[((size_t)m * kTaps + tap) * cin + ci]);
  }
  if (wb) {                                           // cin == 32 here: K = 27 x 32 forward outputs
    const int tapb = kk / kCH, cof = kk % kCH;
    wb[i] = f2bf(wsrc[((size_t)cof * kTaps + (kTaps - 1 - tapb)) * cin + m]);
  }
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
static unsigned conv_blocks(int N, int T, int Y) {
  return (unsigned)N * ((Y + kConvYT - 1) / kConvYT) * ((T + kConvTT - 1) / kConvTT);
}

hipError_t launch_conv_fwd(int cin, const uint16_t* in, const uint16_t* w, const float* bias, uint16_t* out, int N,
                           int T, int Y, hipStream_t st) {
  const dim3 grid(conv_blocks(N, T, Y)), block(kConvWaves * kWave);
  if (cin == 16) hipLaunchKernelGGL((k_conv3<16, 0>), grid, block, 0, st, in, w, bias, nullptr, out, N, T, Y);
  else hipLaunchKernelGGL((k_conv3<32, 0>), grid, block, 0, st, in, w, bias, nullptr, out, N, T, Y);
  return hipGetLastError();
}

hipError_t launch_conv_bwd_data(const uint16_t* dpre, const uint16_t* wb, const uint16_t* mask_act, uint16_t* out, int N,
                                int T, int Y, hipStream_t st) {
  hipLaunchKernelGGL((k_conv3<32, 1>), dim3(conv_blocks(N, T, Y)), dim3(kConvWaves * kWave), 0, st, dpre, wb, nullptr,
                     mask_act, out, N, T, Y);
  return hipGetLastError();
}

hipError_t launch_conv_wgrad(int cin, const uint16_t* x, const uint16_t* dpre, float* part, float* part_db, float* dw,
                             float* db, int N, int T, int Y, hipStream_t st) {
  const int items = wgrad_items(N, Y);
  const dim3 block(kWgWaves * kWave);
  if (cin == 16) hipLaunchKernelGGL((k_conv3_wgrad<16>), dim3(items), block, 0, st, x, dpre, part, part_db, N, T, Y);
  else hipLaunchKernelGGL((k_conv3_wgrad<32>), dim3(items), block, 0, st, x, dpre, part, part_db, N, T, Y);
  const int len = kTaps * kCH * cin;
  hipLaunchKernelGGL(k_reduce_items, dim3((len + kRedOut - 1) / kRedOut), dim3(kRedOut * kRedPar), 0, st, part, items,
                     len, dw);
  hipLaunchKernelGGL(k_reduce_items, dim3(1), dim3(kRedOut * kRedPar), 0, st, part_db, items, kCH, db);
  return hipGetLastError();
}

int pool_chunks(int npos) { return std::max(1, std::min(kPoolChunks, (npos + 1023) / 1024)); }

hipError_t launch_pool(const uint16_t* act, int N, int npos, int centre, uint32_t* part, float* h, int* arg,
                       hipStream_t st) {
  const int G = pool_chunks(npos), chunk = (npos + G - 1) / G;
  if (chunk > 0x10000) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pool_partial, dim3(G, N), dim3(kPoolThreads), 0, st, act, npos, chunk, part);
  hipLaunchKernelGGL(k_pool_finish, dim3((N * kCH + 255) / 256), dim3(256), 0, st, part, G, chunk, act, N, npos,
                     centre, h, arg);
  return hipGetLastError();
}

hipError_t launch_head(const float* h, const float* labels, int n, const float* th, float* hs, float* gh, float* dh,
                       float* logits, float* prob, float* loss, int backward, hipStream_t st) {
  hipLaunchKernelGGL(k_head_sample, dim3((n + 3) / 4), dim3(256), 0, st, h, labels, n, th, hs, dh, logits, prob,
                     backward);
  if (backward)
    hipLaunchKernelGGL(k_head_grad, dim3((kHeadParams + 1 + 255) / 256), dim3(256), 0, st, h, hs, n, gh, loss);
  return hipGetLastError();
}

hipError_t launch_pool_backward(const float* dh, const int* arg, const uint16_t* act, int N, int npos, int centre,
                                uint16_t* dpre, hipStream_t st) {
  const long long total8 = (long long)N * npos * (kCH / 8);
  const unsigned grid = (unsigned)std::min<long long>((total8 + 255) / 256, 65536LL);
  hipLaunchKernelGGL(k_pool_backward, dim3(grid), dim3(256), 0, st, dh, arg, act, npos, centre, total8, dpre);
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
