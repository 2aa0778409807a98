// De-dispersion, boxcar filtering, S/N and max/argmax over time (search stage).
//
// Paper section 2.2: every pixel's time series is de-dispersed over a grid of
// DM trials with precomputed integer shifts, filtered with boxcars of several
// widths, normalised to S/N, and reduced to the maximum S/N over time and its
// TOA; section 2.3 keeps those S/N and TOA maps for all pixels, widths and DM
// trials.
//
// This file is compiled at plan time. The generated prologue fixes the store
// dtype (ST), the number of widths (NSFRB_NW) and the shape classes; the
// generated boxcar plan (nsfrb_chain) follows this file. DM trials, delays,
// n_sub and n_t stay runtime values.
//
// Layout and work split (gfx950, wave64):
//  * a workgroup of NW waves (8 or 16) takes PIX pixels at a time; their normalised
//    series z[s][0..n_t) are staged in LDS, one row per sub-band of rs
//    samples; samples at and beyond n_t hold -inf, so any window that reaches
//    past the end of a de-dispersed series sums to -inf and is never a maximum;
//  * NW/PIX waves share a pixel and split its DM trials round-robin (the
//    "DM chunk" of a wave is every (NW/PIX)-th trial);
//  * lane l holds the C consecutive samples t = C*l + c (FP32 rows: C odd, so
//    lanes hit distinct LDS banks at any delay; FP16 rows: C even with C/2
//    odd, read as dwords holding two samples);
//  * D_d[t] = sum_s z[s][t + delta[d][s]] is formed in registers (FP32); an
//    FP16 sample is added by v_fma_mix_f32 (f16 operand * 1.0 + f32), one
//    rounding, the same result as converting and then adding;
//  * boxcars use the pairwise doubling B_2w[t] = B_w[t] + B_w[t+w]; a width
//    that is not a power of two is the sum of the power-of-two windows of its
//    binary digits placed end to end. Each output is a balanced sum, so the
//    FP32 error grows with log2(w) rather than w;
//  * a window shifted by k samples is read from register (c+k) mod C of lane
//    l + (c+k)/C: the same lane, one or two DPP wave shifts by one lane (two
//    VALU moves return sooner than one ds_bpermute round trip through the LDS
//    pipeline), or ds_bpermute.

#ifndef NSFRB_RTC_PROLOGUE
#error "compile through the search plan: the prologue defines ST, NSFRB_NW and the shape classes"
#endif

namespace nsfrb {

constexpr float kNegInf = -__builtin_inff();

// Work-item and workgroup indices read inline from the hardware registers and
// the HSA dispatch packet. The generated kernels are compiled with IEEE mode
// off, and the runtime's index accessors then stay out-of-line calls whose
// results the compiler must treat as per-lane values.
__device__ __forceinline__ int tid_x() { return (int)__builtin_amdgcn_workitem_id_x(); }
__device__ __forceinline__ int wg_id() { return (int)__builtin_amdgcn_workgroup_id_x(); }
// Workgroups in the launch: grid_size_x (work-items, a 32-bit field at byte 12
// of the packet) over the workgroup size WG the kernel is launched with.
template <int WG>
__device__ __forceinline__ int n_wg() {
  const auto* pk = (const __attribute__((address_space(4))) unsigned char*)__builtin_amdgcn_dispatch_ptr();
  return (int)(*(const __attribute__((address_space(4))) unsigned int*)(pk + 12) / (unsigned)WG);
}

// Value of x held by lane l+1 (lane 63 reads 0). Only used where the sum it
// feeds is already -inf for lane 63 (see shift_add).
__device__ __forceinline__ float lane_next(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x130 /* wave_shl:1 */, 0xf, 0xf, true));
}
// Value of x held by lane (l+q) mod 64, q >= 2.
__device__ __forceinline__ float lane_ahead(float x, int q, int l) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(((l + q) & 63) << 2, __float_as_int(x)));
}

// out[c] = a[c] + b at sample t + K, for t = C*l + c.
// Samples t + K >= 64*C lie beyond the lanes and read 0 or a wrapped value; the
// sums they feed are still -inf: every series has at least one padding sample
// (64*C > n_t), so a window a[c] that ends at or beyond 64*C already covers a
// -inf sample, and wrapped values are finite or -inf, never +inf or NaN.
template <int K, int C>
__device__ __forceinline__ void shift_add(float (&out)[C], const float (&a)[C], const float (&b)[C]) {
  const int l = lane_id();
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int q = (c + K) / C;
    const int r = (c + K) % C;
    float v;
    if (q == 0) v = b[r];
    else if (q == 1) v = lane_next(b[r]);
    else if (q == 2) v = lane_next(lane_next(b[r]));
    else v = lane_ahead(b[r], q, l);
    out[c] = a[c] + v;
  }
}

template <int C>
__device__ __forceinline__ void copy_arr(float (&out)[C], const float (&a)[C]) {
#pragma unroll
  for (int c = 0; c < C; ++c) out[c] = a[c];
}

// acc + (FP16 sample in the low / high half of w), rounded once.
__device__ __forceinline__ float add_f16_lo(float acc, uint32_t w) {
  float r;
  asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(r) : "v"(w), "v"(acc));
  return r;
}
__device__ __forceinline__ float add_f16_hi(float acc, uint32_t w) {
  float r;
  asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(r) : "v"(w), "v"(acc));
  return r;
}

// cur[c] += row[e0 + c] for c < C, e0 = delay + C * lane.
template <int C, typename T>
__device__ __forceinline__ void add_row(float (&cur)[C], const T* row, int dl, int l) {
  const T* r = row + dl + C * l;
#pragma unroll
  for (int c = 0; c < C; ++c) cur[c] += to_f32(r[c]);
}
// FP16 rows (row start dword-aligned, C even): the samples of a lane start at
// element e0 = dl + C*l, whose parity is that of dl (uniform); dword k of the
// lane holds elements (2k, 2k+1) counted from e0 rounded down to even.
template <int C>
__device__ __forceinline__ void add_row(float (&cur)[C], const _Float16* row, int dl, int l) {
  static_assert((C & 1) == 0, "FP16 rows need an even number of samples per lane");
  const uint32_t* w = reinterpret_cast<const uint32_t*>(row) + ((dl + C * l) >> 1);
  if (dl & 1) {
    cur[0] = add_f16_hi(cur[0], w[0]);
#pragma unroll
    for (int k = 0; k < C / 2; ++k) {
      const uint32_t v = w[k + 1];
      cur[2 * k + 1] = add_f16_lo(cur[2 * k + 1], v);
      if (2 * k + 2 < C) cur[2 * k + 2] = add_f16_hi(cur[2 * k + 2], v);
    }
  } else {
#pragma unroll
    for (int k = 0; k < C / 2; ++k) {
      const uint32_t v = w[k];
      cur[2 * k] = add_f16_lo(cur[2 * k], v);
      cur[2 * k + 1] = add_f16_hi(cur[2 * k + 1], v);
    }
  }
}

struct Best {
  float s;
  int d, w, t;
};

// (s, d, w) beats b: higher S/N, then the smaller DM index, then the smaller
// width index (written without branches, so the reporting code stays in one
// basic block with the boxcar arithmetic around it).
__device__ __forceinline__ bool better(float s, int d, int w, const Best& b) {
  return (s > b.s) | ((s == b.s) & ((d < b.d) | ((d == b.d) & (w < b.w))));
}

// Max over all samples of a boxcar array and the first sample reaching it:
// lane maxima by a max3 tree over groups of three registers, the wave maximum
// by DPP, the first lane L holding it by a ballot, then the first register of
// lane L holding it from one ballot per register (compares write lane masks
// to scalar registers; lane L's bit is tested on the scalar unit).
template <int C>
__device__ __forceinline__ void max_first(const float (&b)[C], float& M, int& T) {
  constexpr int G = (C + 2) / 3;
  float g[G];
#pragma unroll
  for (int k = 0; k < G; ++k) {
    float v = b[3 * k];
    if (3 * k + 1 < C) v = fmaxf(v, b[3 * k + 1]);
    if (3 * k + 2 < C) v = fmaxf(v, b[3 * k + 2]);
    g[k] = v;
  }
  float m = g[0];
#pragma unroll
  for (int k = 1; k < G; k += 2) m = (k + 1 < G) ? fmaxf(m, fmaxf(g[k], g[k + 1])) : fmaxf(m, g[k]);
  M = wave_max_f(m);
  // some lane's maximum equals M, so the ballot is never empty
  const int L = __ffsll((long long)ballot(m == M)) - 1;
  int cf = C - 1;
#pragma unroll
  for (int c = C - 2; c >= 0; --c) {
    // cf = c if lane L's bit of the compare mask is set: s_bitcmp1_b64 tests
    // the bit straight into SCC (two scalar instructions per register; the
    // compiler's mask-and-compare form takes three)
    const uint64_t mk = ballot(b[c] == M);
    asm("s_bitcmp1_b64 %1, %2\n\ts_cselect_b32 %0, %3, %0" : "+s"(cf) : "s"(mk), "s"(L), "n"(c) : "scc");
  }
  T = (M > kNegInf) ? C * L + cf : -1;
}

// Where one cube's results go.
struct CubeOut {
  const float* norms;
  float* snr_max;
  int* toa;
  int n_pix;
};

// Per-DM results: the raw maximum of width iw and its TOA are kept in lane iw
// of two registers. flush() turns all of them into S/N at once (lane iw
// divides by its own normaliser), stores them ([d][iw][p], lanes
// 0..NSFRB_NW-1), and folds the DM's best width into the running best.
struct Reporter {
  CubeOut o;
  int p, d;
  Best best;
  float snr_lane;
  int toa_lane;
  float norm_lane;          // lane iw: sqrt(n_sub * width[iw])
  __device__ __forceinline__ void emit(int iw, float M, int T) {
    const bool mine = lane_id() == iw;
    snr_lane = mine ? M : snr_lane;
    toa_lane = mine ? T : toa_lane;
  }
  __device__ __forceinline__ void flush() {
    const int l = lane_id();
    const bool act = l < NSFRB_NW;
    const float s = (act && snr_lane > kNegInf) ? snr_lane / norm_lane : kNegInf;
    if (act && p < o.n_pix) {         // (a batch item's last pixels may lie past the cube)
      const size_t idx = ((size_t)d * NSFRB_NW + l) * o.n_pix + p;
      o.snr_max[idx] = s;
      o.toa[idx] = toa_lane;
    }
    // the DM's best width: the largest S/N, the smallest width index on ties
    // (with every width at -inf, width 0 at -inf never beats the running best)
    const float smax = wave_max_f(s);
    const int w = __ffsll((long long)ballot(act && s == smax)) - 1;
    const int t = __builtin_amdgcn_readlane(toa_lane, w);
    const bool up = better(smax, d, w, best);
    best.s = up ? smax : best.s;
    best.d = up ? d : best.d;
    best.w = up ? w : best.w;
    best.t = up ? t : best.t;
  }
  template <int C>
  __device__ __forceinline__ void operator()(int iw, const float (&b)[C]) {
    float M;
    int T;
    max_first<C>(b, M, T);
    emit(iw, M, T);
  }
  __device__ __forceinline__ void invalid(int iw) { emit(iw, kNegInf, -1); }
};

// Everything the search needs about one cube (also the batch descriptor).
struct CubeDesc {
  const ST* z;              // [n_pix][n_sub][n_t]
  const int* delays;        // [n_dm][n_sub]
  const int* dmax;          // [n_dm]
  const float* norms;       // [NSFRB_NW]
  float* snr_max;           // [n_dm][NSFRB_NW][n_pix]
  int* toa;
  float* best_s;            // [n_pix]
  int* best_d;
  int* best_w;
  int* best_t;
  int n_pix, n_sub, n_t, n_dm, rs;
  int dma_w;                // batch row copy: global-to-LDS bytes per lane (16 or 4), else ordinary loads
  long long item_begin;     // first work item of this cube in a batch
};

}  // namespace nsfrb

// The boxcar plan, generated per width list after this file: pass `pass`
// forms the power-of-two window levels it needs from the de-dispersed series
// held in `cur` and calls rep(width_index, window_sums) for its widths; the
// passes together report every width once (NSFRB_NPASS passes).
template <int C, class R>
__device__ __forceinline__ void nsfrb_chain(int pass, float (&cur)[C], R& rep);

namespace nsfrb {

// One work item: PIX consecutive pixels starting at p0 of one cube.
// Requires all NW waves of the workgroup (it contains barriers).
template <int C, int PIX, int NW>
__device__ __forceinline__ void search_group(const CubeDesc& cd, int p0, ST* zl, Best* red) {
  static_assert(NW % PIX == 0, "every pixel of a group gets the same number of waves");
  constexpr int WPP = NW / PIX;            // waves per pixel
  // the wave index is uniform across the wave; saying so lets every per-DM
  // value (delays, DM bounds) come through the scalar cache
  const int wv = __builtin_amdgcn_readfirstlane(tid_x() / kWave);
  const int l = lane_id();
  const int slot = wv / WPP;               // which pixel of the group
  const int wq = wv % WPP;                 // this wave's DM chunk: d = wq, wq + WPP, ...
  const int rs = cd.rs, n_sub = cd.n_sub, n_t = cd.n_t;
  const ST neg = from_f32<ST>(kNegInf);
  // ---- stage the group's rows into LDS, -inf beyond n_t. A pixel's n_sub x n_t
  // samples are contiguous in memory: when rows split into whole 16-byte
  // vectors and the cube is 16-byte aligned, every thread issues all its
  // vector loads (up to kStageBatch) before storing any, so the staging costs
  // about one memory latency instead of one per sample.
  constexpr int VW = 16 / (int)sizeof(ST);          // samples per 16-byte vector
  constexpr int kStageBatch = 8;
  const bool vec = (n_t % VW) == 0 && (reinterpret_cast<unsigned long long>(cd.z) & 15ull) == 0;
  for (int k = 0; k < PIX; ++k) {
    const int p = p0 + k;
    ST* dstp = zl + (size_t)k * n_sub * rs;
    if (p >= cd.n_pix) continue;
    const ST* zp = cd.z + (size_t)p * n_sub * n_t;
    if (vec) {
      const int nv = n_sub * n_t / VW;
      const uint4* src = reinterpret_cast<const uint4*>(zp);
      for (int v0 = tid_x(); v0 < nv; v0 += kStageBatch * 64 * NW) {
        uint4 buf[kStageBatch];
#pragma unroll
        for (int b = 0; b < kStageBatch; ++b) {
          const int v = v0 + b * 64 * NW;
          buf[b] = v < nv ? src[v] : make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (int b = 0; b < kStageBatch; ++b) {
          const int v = v0 + b * 64 * NW;
          if (v < nv) {
            const int e = v * VW, s = e / n_t, u = e - s * n_t;
            // FP32 samples are dwords; 16-bit rows have even pitches and u is a
            // multiple of VW, so every store below is dword-aligned
            uint32_t* d = reinterpret_cast<uint32_t*>(dstp + s * rs + u);
            d[0] = buf[b].x;
            d[1] = buf[b].y;
            d[2] = buf[b].z;
            d[3] = buf[b].w;
          }
        }
      }
      const int tail = rs - n_t;
      for (int i = tid_x(); i < n_sub * tail; i += 64 * NW) {
        const int s = i / tail;
        dstp[s * rs + n_t + (i - s * tail)] = neg;
      }
    } else {
      for (int s = 0; s < n_sub; ++s) {
        const ST* src = zp + (size_t)s * n_t;
        ST* dst = dstp + s * rs;
        for (int u = tid_x(); u < rs; u += 64 * NW) dst[u] = (u < n_t) ? src[u] : neg;
      }
    }
  }
  __syncthreads();
  const int p = p0 + slot;
  Reporter rep{CubeOut{cd.norms, cd.snr_max, cd.toa, cd.n_pix}, p, 0, Best{kNegInf, -1, -1, -1}, 0.f, 0,
               l < NSFRB_NW ? cd.norms[l] : 1.f};
  if (p < cd.n_pix) {
    const ST* zbase = zl + (size_t)slot * n_sub * rs;
    // a DM's delays sit in lanes 0..n_sub-1 of one register (one coalesced
    // load, issued a DM ahead); the sub-band loop reads them with v_readlane
    const int n_dm = cd.n_dm;
    int dl_next = (wq < n_dm && l < n_sub) ? cd.delays[wq * n_sub + l] : 0;
    int dmax_next = wq < n_dm ? cd.dmax[wq] : 0;
    for (int d = wq; d < n_dm; d += WPP) {
      const int dl_cur = dl_next;
      const int dmax_d = __builtin_amdgcn_readfirstlane(dmax_next);
      const int dn = d + WPP;
      dl_next = (dn < n_dm && l < n_sub) ? cd.delays[dn * n_sub + l] : 0;
      dmax_next = dn < n_dm ? cd.dmax[dn] : 0;
      rep.d = d;
      if (dmax_d >= n_t) {
        for (int iw = 0; iw < NSFRB_NW; ++iw) rep.invalid(iw);
        rep.flush();
        continue;
      }
      for (int pass = 0; pass < NSFRB_NPASS; ++pass) {
        float cur[C];
#pragma unroll
        for (int c = 0; c < C; ++c) cur[c] = 0.f;
        for (int s = 0; s < n_sub; ++s)
          add_row<C>(cur, zbase + s * rs, __builtin_amdgcn_readlane(dl_cur, s), l);
        nsfrb_chain<C>(pass, cur, rep);
      }
      rep.flush();
    }
  }
  if (l == 0) red[wv] = rep.best;
  __syncthreads();
  if (tid_x() < PIX && p0 + tid_x() < cd.n_pix) {
    const int k = tid_x();
    Best b = red[k * WPP];
    for (int j = 1; j < WPP; ++j)
      if (better(red[k * WPP + j].s, red[k * WPP + j].d, red[k * WPP + j].w, b)) b = red[k * WPP + j];
    const bool ok = b.s > kNegInf;
    const int pp = p0 + k;
    cd.best_s[pp] = ok ? b.s : kNegInf;
    cd.best_d[pp] = ok ? b.d : -1;
    cd.best_w[pp] = ok ? b.w : -1;
    cd.best_t[pp] = ok ? b.t : -1;
  }
  __syncthreads();
}


// Global-to-LDS staging: row s of pixel p is n_t * sizeof(ST) bytes, a whole
// number of 16-byte vectors; wave wv requests pieces wv, wv + NW, ... of
// 64 vectors (one instruction each), lanes beyond the row's end disabled.
// The loads land asynchronously; the caller waits (vmcnt) and synchronises.
template <int NW, int W = 16>   // W: 16 or 4 bytes per lane
__device__ __forceinline__ void stage_rows_async(const CubeDesc& cd, int p, ST* buf, int wv, int l) {
  typedef __attribute__((address_space(3))) void* lds_ptr;
  const int rs = cd.rs, n_sub = cd.n_sub, n_t = cd.n_t;
  const int row_bytes = n_t * (int)sizeof(ST);
  const int per_row = (row_bytes + 64 * W - 1) / (64 * W);    // instructions per row
  const unsigned char* zp = reinterpret_cast<const unsigned char*>(cd.z + (size_t)p * n_sub * n_t);
  for (int i = wv; i < n_sub * per_row; i += NW) {
    const int s = i / per_row, piece = i - s * per_row;
    const int off = (piece * 64 + l) * W;                         // byte offset of this lane in the row
    if (off < row_bytes) {
      const unsigned char* g = zp + ((size_t)s * row_bytes + (size_t)off);
      unsigned char* d = reinterpret_cast<unsigned char*>(buf + (size_t)s * rs) + (size_t)piece * 64 * W;
      if constexpr (W == 16) __builtin_amdgcn_global_load_lds(g, (lds_ptr)d, 16, 0, 0);
      else __builtin_amdgcn_global_load_lds(g, (lds_ptr)d, 4, 0, 0);
    }
  }
}
// 16-bit rows whose start is not dword-aligned (odd n_t, or a cube 2 bytes
// past a dword boundary). Row s of pixel p goes to LDS index off_s + t, off_s
// the parity of its first sample's position (row_offset), so that the global
// and LDS dword boundaries coincide and the row is copied as the whole dwords
// that cover it, with 4-byte global-to-LDS loads. The dword before the row
// (off_s = 1) puts the previous row's last sample at index 0, never read; the
// dword after it (n_t + off_s odd) puts the next row's first sample at index
// n_t + off_s, which must read -inf: fix_row_ends rewrites it once the copies
// have landed, and the tails start after it (row_tail). The cube's first and
// last rows are copied with ordinary loads, so no copy reads outside the cube.
__device__ __forceinline__ int row_parity(const CubeDesc& cd, int p) {       // off_s of row 0 of pixel p
  return (int)((((unsigned long long)cd.z >> 1) + (unsigned long long)p * cd.n_sub * cd.n_t) & 1ull);
}
__device__ __forceinline__ int row_offset(int par, int s, int n_t) { return (par + s * n_t) & 1; }
__device__ __forceinline__ int row_tail(int n_t, int off) { return n_t + off + ((n_t + off) & 1); }

template <int NW>
__device__ __forceinline__ void stage_rows_par(const CubeDesc& cd, int p, ST* buf, int wv, int l) {
  static_assert(sizeof(ST) == 2, "only 16-bit rows can start between dwords");
  typedef __attribute__((address_space(3))) void* lds_ptr;
  const int rs = cd.rs, n_sub = cd.n_sub, n_t = cd.n_t;
  const int par = row_parity(cd, p);
  const int per_row = ((n_t + 2) / 2 + 63) / 64;          // instructions per row (at most n_t/2 + 1 dwords)
  const unsigned char* zb = reinterpret_cast<const unsigned char*>(cd.z);
  const long long row0 = (long long)p * n_sub, last_row = (long long)cd.n_pix * n_sub - 1;
  for (int i = wv; i < n_sub * per_row; i += NW) {
    const int s = i / per_row, piece = i - s * per_row;
    const int off = row_offset(par, s, n_t);
    const long long gr = row0 + s;
    if ((gr == 0 && off) || (gr == last_row && ((n_t + off) & 1))) continue;   // an edge row, below
    const int j = piece * 64 + l;                          // dword of the row
    if (j < (n_t + off + 1) / 2) {
      const unsigned char* g = zb + (gr * n_t - off) * 2 + 4 * (long long)j;
      unsigned char* d = reinterpret_cast<unsigned char*>(buf + (size_t)s * rs) + (size_t)piece * 256;
      __builtin_amdgcn_global_load_lds(g, (lds_ptr)d, 4, 0, 0);
    }
  }
  // the cube's first row (if it starts between dwords) and last row (if a
  // dword would run past it), sample by sample
  for (int e = 0; e < 2; ++e) {
    const int s = e == 0 ? 0 : n_sub - 1;
    const long long gr = row0 + s;
    const int off = row_offset(par, s, n_t);
    if (!((e == 0 && gr == 0 && off) || (e == 1 && gr == last_row && ((n_t + off) & 1)))) continue;
    const ST* src = cd.z + gr * n_t;
    for (int t = tid_x(); t < n_t; t += 64 * NW) buf[(size_t)s * rs + off + t] = src[t];
  }
}
// -inf where a row's last dword put the next row's first sample, written by
// the wave that copied that dword once its copies have landed (after its own
// s_waitcnt, before the barrier that publishes the rows); lane s looks after
// row s (n_sub <= 64).
template <int NW>
__device__ __forceinline__ void fix_row_ends(const CubeDesc& cd, int p, ST* buf, int wv, int l) {
  const int par = row_parity(cd, p), n_t = cd.n_t;
  const int per_row = ((n_t + 2) / 2 + 63) / 64;          // the pieces of stage_rows_par
  const int s = l, off = row_offset(par, s, n_t);
  if (s < cd.n_sub && ((n_t + off) & 1) && (s * per_row + per_row - 1) % NW == wv)
    buf[(size_t)s * cd.rs + n_t + off] = from_f32<ST>(kNegInf);
}
// -inf tails of a tile of parity-placed rows.
template <int NW>
__device__ __forceinline__ void fill_tails_par(ST* buf, const CubeDesc& cd, int p) {
  const ST neg = from_f32<ST>(kNegInf);
  const int par = row_parity(cd, p), n_t = cd.n_t, rs = cd.rs;
  const int span = rs - n_t;                                // each row's tail is at most this long
  for (int k = tid_x(); k < cd.n_sub * span; k += 64 * NW) {
    const int s = k / span, u = row_tail(n_t, row_offset(par, s, n_t)) + (k - s * span);
    if (u < rs) buf[(size_t)s * rs + u] = neg;
  }
}
// The copy a cube's rows allow (the batch passes it per cube): global-to-LDS
// loads of 16 or 4 bytes per lane for rows of whole 16-byte vectors or dwords,
// else (dma_w 2: 16-bit rows starting between dwords) parity-placed rows.
template <int NW>
__device__ __forceinline__ void stage_rows_w(const CubeDesc& cd, int p, ST* buf, int wv, int l) {
  if (cd.dma_w == 16) stage_rows_async<NW, 16>(cd, p, buf, wv, l);
  else if (cd.dma_w == 4) stage_rows_async<NW, 4>(cd, p, buf, wv, l);
  else if constexpr (sizeof(ST) == 2) stage_rows_par<NW>(cd, p, buf, wv, l);
}

// Between requesting a pixel's rows and waiting for them, a wave issues no
// vector-memory load (the class table comes through the scalar cache, the S/N
// normalisers are read once per kernel, trial validity comes from the table):
// on gfx950 one counter tracks all vector-memory loads, so any load there
// would wait for the row requests too.
// ---------------------------------------------------------------------------
// Persistent form of search_group for one pixel per workgroup: the workgroup
// walks pixels b, b + G, ... (workgroup b of G); its NW waves split the
// DM trials round-robin as in search_group. When the layout allows, the rows of
// the next pixel are requested with global-to-LDS loads as soon as no wave will
// read the current rows again (after the last round's de-dispersion; with two
// LDS buffers, at the start of the pixel), so those loads run under the boxcar
// work. Delays and DM bounds come through the scalar cache and the S/N
// normalisers are read once, so no vector-memory load is issued while row
// requests are in flight (one counter tracks them all).
// ---------------------------------------------------------------------------
// A load through the scalar cache (the constant address space): for values the
// kernel never writes, at uniform addresses.
template <typename T>
__device__ __forceinline__ T ld_const(const T* p) {
  return *(const __attribute__((address_space(4))) T*)(p);
}

// -inf in samples n_t .. rs-1 of every row of a tile.
template <int NW>
__device__ __forceinline__ void fill_tails(ST* buf, int n_sub, int n_t, int rs) {
  const ST neg = from_f32<ST>(kNegInf);
  const int tail = rs - n_t;
  for (int k = tid_x(); k < n_sub * tail; k += 64 * NW) {
    const int r = k / tail;
    buf[r * rs + n_t + (k - r * tail)] = neg;
  }
}

// The DM trials of one pixel whose rows are in zl; `release` runs once every
// wave has read the rows for the last time (after the last round's
// de-dispersion; it is called by every wave, and must contain the barrier
// itself). The loop has no branches (a branch around the boxcar chain costs it
// registers): waves past the last trial repeat it (writing the same values
// twice), and a trial with no valid sample is searched with zero delays (its
// row of `delays` holds zeros) and then reported as -inf / -1.
template <int C, int NW, bool PAR = false, class Release>
__device__ __forceinline__ void search_pixel_dms(const CubeDesc& cd, const int* delays, const int* dmaxv,
                                                 const ST* zl, Reporter& rep, int wv, int l, Release&& release,
                                                 int par = 0) {
  const int n_dm = cd.n_dm, n_t = cd.n_t, n_sub = cd.n_sub, rs = cd.rs;
  const int n_rounds = (n_dm + NW - 1) / NW;
  for (int rd = 0; rd < n_rounds; ++rd) {
    const int d = min(rd * NW + wv, n_dm - 1);
    const int* dd = delays + (size_t)d * n_sub;
    for (int pass = 0; pass < NSFRB_NPASS; ++pass) {
      float cur[C];
#pragma unroll
      for (int c = 0; c < C; ++c) cur[c] = 0.f;
      for (int s = 0; s < n_sub; ++s)    // (PAR: rows placed at their parity offset, see stage_rows_par)
        add_row<C>(cur, zl + s * rs, ld_const(dd + s) + (PAR ? row_offset(par, s, n_t) : 0), l);
      if (pass == NSFRB_NPASS - 1 && rd == n_rounds - 1) release();
      // a wave in its boxcar chain issues ahead of waves reading rows (the
      // row readers mostly wait on the LDS; raising the chain measured 8%
      // faster at survey shape in FP32, the reverse order did not help)
      __builtin_amdgcn_s_setprio(1);
      nsfrb_chain<C>(pass, cur, rep);
      __builtin_amdgcn_s_setprio(0);
    }
    // (read after the chain: a scalar held across it would push the chain's
    // ballot masks out of scalar registers)
    const bool searched = ld_const(dmaxv + d) < n_t;
    rep.d = d;
    rep.snr_lane = searched ? rep.snr_lane : kNegInf;
    rep.toa_lane = searched ? rep.toa_lane : -1;
    rep.flush();
  }
}

// The per-pixel best (S/N, d, w, t) of pixels p0 .. p0+PIX-1 (pixel k searched
// by waves k*NW/PIX ..; pixels at or past n_pix are not written); starts with
// a barrier.
template <int NW, int PIX = 1>
__device__ __forceinline__ void write_best(const CubeDesc& cd, int p0, const Best& mine, Best* red, int wv, int l) {
  constexpr int WPP = NW / PIX;
  if (l == 0) red[wv] = mine;
  __syncthreads();
  const int k = tid_x();
  if (k < PIX && p0 + k < cd.n_pix) {
    Best b = red[k * WPP];
    for (int w = 1; w < WPP; ++w) {
      const Best& o = red[k * WPP + w];
      if (better(o.s, o.d, o.w, b)) b = o;
    }
    const bool ok = b.s > kNegInf;
    const int p = p0 + k;
    cd.best_s[p] = ok ? b.s : kNegInf;
    cd.best_d[p] = ok ? b.d : -1;
    cd.best_w[p] = ok ? b.w : -1;
    cd.best_t[p] = ok ? b.t : -1;
  }
}

// Lane iw's S/N normaliser of a cube, through the scalar cache (no vector load).
__device__ __forceinline__ float lane_norm(const CubeDesc& cd, int l) {
  float v = 1.f;
#pragma unroll
  for (int iw = 0; iw < NSFRB_NW; ++iw) v = (l == iw) ? ld_const(cd.norms + iw) : v;
  return v;
}

// The work items of one workgroup, in increasing order. When the grid is a
// multiple of 8 (workgroup b runs on XCD b mod 8), items are cut into chunks of
// 32 (one 128-byte line of a map row holds 32 pixels' entries), chunk j
// belongs to XCD j mod 8, and the workgroups of an XCD take that XCD's items in
// turn. Neighbouring pixels' map entries then leave one XCD's L2 as whole
// lines (with a plain stride every line would be written back once per XCD),
// and every XCD gets an equal share of each stretch of items, so cubes of
// unequal cost in a batch do not load one XCD more than another.
struct ItemWalk {
  long long n;
  int x, k0, step;           // XCD (-1: plain stride), first index, index step
  __device__ __forceinline__ long long item(long long k) const {
    return x < 0 ? k : ((((k >> 5) << 3) + x) << 5) + (k & 31);
  }
};
template <int NW>
__device__ __forceinline__ ItemWalk xcd_walk(long long n) {
  const int g = n_wg<64 * NW>(), b = wg_id();
  if ((g & 7) == 0) return ItemWalk{n, b & 7, b >> 3, g >> 3};
  return ItemWalk{n, -1, b, g};
}

// Persistent single-cube form: one pixel per workgroup at a time; the next
// pixel's rows (global-to-LDS, 16-byte lanes) are requested as soon as no
// wave reads the current ones (after the last round's de-dispersion; with two
// LDS buffers, at the start of the pixel). No vector-memory load is issued
// while row requests are in flight (one counter tracks them all): delays and
// DM bounds come through the scalar cache, the S/N normalisers are read once.
template <int C, int NW, int NBUF>
__device__ __forceinline__ void search_persistent(const CubeDesc& cd, const int* __restrict__ delays,
                                                  const int* __restrict__ dmaxv) {
  extern __shared__ unsigned char lds_raw[];
  __shared__ Best red[NW];
  const int wv = __builtin_amdgcn_readfirstlane(tid_x() / kWave);
  const int l = lane_id();
  const int tile = cd.n_sub * cd.rs;
  ST* bufs = reinterpret_cast<ST*>(lds_raw);
  for (int b = 0; b < NBUF; ++b) fill_tails<NW>(bufs + b * tile, cd.n_sub, cd.n_t, cd.rs);
  const float norm_l = lane_norm(cd, l);
  const ItemWalk r = xcd_walk<NW>(cd.n_pix);
  long long k = r.k0, i = r.item(k);
  if (i < r.n) stage_rows_async<NW>(cd, (int)i, bufs, wv, l);
  for (int it = 0; i < r.n; ++it) {
    const int p = (int)i;
    k += r.step;
    const long long i_next = r.item(k);
    ST* zl = bufs + (NBUF == 2 ? (it & 1) * tile : 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (NBUF == 2 && i_next < r.n) stage_rows_async<NW>(cd, (int)i_next, bufs + ((it + 1) & 1) * tile, wv, l);
    Reporter rep{CubeOut{cd.norms, cd.snr_max, cd.toa, cd.n_pix}, p, 0, Best{kNegInf, -1, -1, -1}, 0.f, 0, norm_l};
    search_pixel_dms<C, NW>(cd, delays, dmaxv, zl, rep, wv, l, [&]() {
      if (NBUF == 1) {
        __syncthreads();   // no wave reads the rows of p again
        if (i_next < r.n) stage_rows_async<NW>(cd, (int)i_next, bufs, wv, l);
      }
    });
    write_best<NW>(cd, p, rep.best, red, wv, l);
    i = i_next;
  }
  __builtin_amdgcn_s_waitcnt(0);
}

// Persistent batch: the work items of the cubes of one kernel class (PIX
// consecutive pixels of one cube each; a cube's last item may run past its
// pixels), concatenated in cube order (descs[c].item_begin), walked as in
// search_persistent. A workgroup's items increase, so its cube index only
// moves forward; descriptors, delays and normalisers come through the scalar
// cache. Pixel k of an item is searched by waves k*NW/PIX .. (k+1)*NW/PIX - 1,
// which split its DM trials. Cubes differ in n_sub, n_t, row pitch (rs) and
// delays: the -inf tails are written for each item, and each cube's rows are
// copied with the copy its alignment allows (dma_w). buf_stride: elements
// between the LDS buffers (PIX tiles of the class's largest size each).
template <int C, int NW, int NBUF, int PIX>
__device__ __forceinline__ void search_batch_persistent(const CubeDesc* __restrict__ descs, int n_cubes,
                                                        long long n_items, int buf_stride) {
  static_assert(NW % PIX == 0, "every pixel of an item gets the same number of waves");
  constexpr int WPP = NW / PIX;
  extern __shared__ unsigned char lds_raw[];
  __shared__ Best red[NW];
  const int wv = __builtin_amdgcn_readfirstlane(tid_x() / kWave);
  const int l = lane_id();
  const int slot = wv / WPP, wq = wv % WPP;
  const int tile_stride = buf_stride / PIX;
  ST* bufs = reinterpret_cast<ST*>(lds_raw);
  auto cube_of = [&](long long i, int c) {
    while (c + 1 < n_cubes && i >= ld_const(&descs[c + 1].item_begin)) ++c;
    return c;
  };
  auto stage = [&](int c, long long i, ST* buf) {
    const CubeDesc cd = ld_const(descs + c);
    const int p0 = (int)(i - cd.item_begin) * PIX;
#pragma unroll
    for (int k = 0; k < PIX; ++k) {
      const int pk = min(p0 + k, cd.n_pix - 1);
      if (sizeof(ST) == 2 && cd.dma_w == 2) fill_tails_par<NW>(buf + k * tile_stride, cd, pk);
      else fill_tails<NW>(buf + k * tile_stride, cd.n_sub, cd.n_t, cd.rs);
      stage_rows_w<NW>(cd, pk, buf + k * tile_stride, wv, l);
    }
  };
  const ItemWalk r = xcd_walk<NW>(n_items);
  long long k = r.k0, i = r.item(k);
  int c = i < r.n ? cube_of(i, 0) : 0;
  if (i < r.n) stage(c, i, bufs);
  for (int it = 0; i < r.n; ++it) {
    const CubeDesc cd = ld_const(descs + c);
    const int p0 = (int)(i - cd.item_begin) * PIX;
    k += r.step;
    const long long i_next = r.item(k);
    const int c_next = i_next < r.n ? cube_of(i_next, c) : c;
    ST* buf = bufs + (NBUF == 2 ? (it & 1) * buf_stride : 0);
    __builtin_amdgcn_s_waitcnt(0);
    if (sizeof(ST) == 2 && cd.dma_w == 2)      // parity-placed rows: restore the -inf after each row
#pragma unroll
      for (int k2 = 0; k2 < PIX; ++k2)
        fix_row_ends<NW>(cd, min(p0 + k2, cd.n_pix - 1), buf + k2 * tile_stride, wv, l);
    __syncthreads();
    if (NBUF == 2 && i_next < r.n) stage(c_next, i_next, bufs + ((it + 1) & 1) * buf_stride);
    Reporter rep{CubeOut{cd.norms, cd.snr_max, cd.toa, cd.n_pix}, p0 + slot, 0, Best{kNegInf, -1, -1, -1}, 0.f, 0,
                 lane_norm(cd, l)};
    const int par = (sizeof(ST) == 2 && cd.dma_w == 2) ? row_parity(cd, min(p0 + slot, cd.n_pix - 1)) : 0;
    search_pixel_dms<C, WPP, true>(cd, cd.delays, cd.dmax, buf + slot * tile_stride, rep, wq, l, [&]() {
      if (NBUF == 1) {
        __syncthreads();   // no wave reads the rows of this item again
        if (i_next < r.n) stage(c_next, i_next, bufs);
      }
    }, par);
    write_best<NW, PIX>(cd, p0, rep.best, red, wv, l);
    c = c_next;
    i = i_next;
  }
  __builtin_amdgcn_s_waitcnt(0);
}

}  // namespace nsfrb

// Single cube: work item i covers pixels [i*PIX, i*PIX + PIX); items are dealt
// so that the items running on one XCD at a time are neighbours.
template <int C, int PIX, int NW>
__device__ __forceinline__ void search_cube(const nsfrb::CubeDesc& cd) {
  using namespace nsfrb;
  extern __shared__ unsigned char lds_raw[];
  __shared__ Best red[NW];
  ST* zl = reinterpret_cast<ST*>(lds_raw);
  const int n_items = (cd.n_pix + PIX - 1) / PIX;
  const int g = n_wg<64 * NW>();
  for (int blk = wg_id(); blk < n_items; blk += g) {
    int item = blk;
    if ((n_items & 7) == 0 && g == n_items) item = (blk & 7) * (n_items >> 3) + (blk >> 3);
    search_group<C, PIX, NW>(cd, item * PIX, zl, red);
  }
}
