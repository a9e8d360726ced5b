// gfx950 kernels of the SIFT extraction path.
//
// Every kernel serves a whole batch: work items are decoded from prefix
// tables over the images of the batch, so one image goes through exactly
// the same per-pixel and per-keypoint arithmetic whether it is extracted
// alone or with others.  No kernel uses floating-point atomics; every sum
// has an order fixed in this source, which makes the output bit-identical
// from run to run.  The file is built with -ffp-contract=off: every fused
// multiply-add below is written out explicitly.
#include <hip/hip_runtime.h>
#include <math.h>

#include "sift_internal.h"
#include "sift_launch.h"

namespace sift {

constexpr float kTwoPi = 6.28318530717958647692f;

// ---------------------------------------------------------------------------
// Common device helpers

// Reflect-101 border: ... c b | a b c ... (index -1 -> 1), repeated with
// period 2(n-1) for indices far outside; n == 1 maps everything to 0.
__device__ __forceinline__ int mirror(int i, int n) {
  if (i >= 0 && i < n) return i;
  if (n == 1) return 0;
  const int period = 2 * (n - 1);
  i = i < 0 ? -i : i;
  i %= period;
  return i >= n ? period - i : i;
}

// Largest idx in [0, n) with prefix[idx] <= item (prefix has n + 1 entries).
__device__ __forceinline__ int find_owner(const int* prefix, int n, int item) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid] <= item) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int* counters_of(char* ws, const ImgEntry& e) {
  return reinterpret_cast<int*>(ws + e.region);
}

__device__ __forceinline__ const float* level_ptr(char* ws, const ImgEntry& e, const OctView& ov,
                                                  int level) {
  return reinterpret_cast<const float*>(ws + e.region + ov.level0 + (int64_t)level * ov.plane);
}

// Inclusive sum of an int over the 64 lanes of a wave (exact, any order).
__device__ __forceinline__ int wave_incl_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  return v;
}

// Butterfly sum over the 64 lanes.  Each step adds the partner's value; the
// two partners add the same two operands, so every lane ends with the same
// bits and the association order is fixed by the code.
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = v + __shfl_xor(v, d, 64);
  return v;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = fmaxf(v, __shfl_xor(v, d, 64));
  return v;
}

// Make this wave's LDS writes visible to its other lanes before they read.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Block-wide exclusive scan of ints (blockDim.x == 256).  Returns the
// exclusive prefix of v; *total receives the block sum.
__device__ __forceinline__ int block_excl_scan256(int v, int* s_wave, int* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int incl = wave_incl_scan(v);
  if (lane == 63) s_wave[wave] = incl;
  __syncthreads();
  int base = 0, sum = 0;
#pragma unroll
  for (int wv = 0; wv < 4; ++wv) {
    const int t = s_wave[wv];
    if (wv < wave) base += t;
    sum += t;
  }
  __syncthreads();
  *total = sum;
  return base + incl - v;
}

// ---------------------------------------------------------------------------
// Setup: copy image-table entries from kernel arguments into the workspace,
// then derive the per-octave tile and per-image band prefix sums.

__global__ void k_setup(HdrPtrs hp, SetupChunk c) {
  const int t = threadIdx.x;
  if (t < c.count) const_cast<ImgEntry*>(hp.table)[c.first + t] = c.e[t];
}

__global__ void k_finalize(HdrPtrs hp, int n, DevParams p) {
  const ImgEntry* tab = hp.table;
  int* tp = hp.tile_prefix;
  int* bp = hp.band_prefix;
  const int t = threadIdx.x;
  if (t < kNumTileH * p.n_oct) {
    // tile prefix for tile-height class t / n_oct, octave t % n_oct
    const int cls = t / p.n_oct, k = t - cls * p.n_oct;
    const int th = tile_h_of(cls);
    int* out = tp + (cls * kMaxOct + k) * (n + 1);
    int acc = 0;
    out[0] = 0;
    for (int i = 0; i < n; ++i) {
      int hk, wk;
      octave_dims(tab[i].h, tab[i].w, p.upsample, k, &hk, &wk);
      acc += cdiv(wk, kTileW) * cdiv(hk, th);
      out[i + 1] = acc;
    }
  } else if (t == kNumTileH * p.n_oct) {
    const LayoutCfg lc = layout_cfg(p);
    int acc = 0;
    bp[0] = 0;
    for (int i = 0; i < n; ++i) {
      acc += region_tail(tab[i].h, tab[i].w, lc).total_bands;
      bp[i + 1] = acc;
    }
  }
}

// ---------------------------------------------------------------------------
// Gaussian level: one separable blur of a 64 x TH tile.  The source tile plus
// an R-pixel mirrored halo is staged in LDS; the horizontal pass writes an LDS
// buffer, the vertical pass writes the level.  Each output is
//   acc = 0; for t = 0..2R: acc = fma(g[t], in[x - R + t], acc)
// for the horizontal pass and the same along columns for the vertical pass,
// whatever the tile shape.  Levels are held relative to mid-grey (L - 0.5):
// the blur is linear with unit-sum taps, so this changes no difference of
// levels and keeps fp32 rounding error proportional to |L - 0.5|.
//
// Work-groups are dealt round-robin to the 8 XCDs, each with its own L2; the
// grid is a multiple of 8 and group b takes tile (b % 8) * (grid / 8) + b / 8,
// so every XCD sweeps one contiguous run of tiles and neighbouring tiles find
// their shared halo rows in the same L2.
template <int R, int TH>
__global__ __launch_bounds__(256) void k_blur(BlurArgs a) {
  constexpr int IW = kTileW + 2 * R;
  constexpr int S = IW | 1;        // odd stride: a wave reading one column per row is conflict-free
  constexpr int IH = TH + 2 * R;
  constexpr int HS = kTileW + 1;
  constexpr int HB = 4;            // horizontal outputs per thread
  constexpr int VB = 8;            // vertical outputs per thread
  static_assert(TH % VB == 0, "tile height must be a multiple of 8");
  __shared__ float s_in[IH * S];
  __shared__ float s_h[IH * HS];

  const int* tp = a.tile_prefix;
  const int per_xcd = gridDim.x / kXcds;
  const int item = (blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds;
  if (item >= tp[a.n]) return;
  const int img = find_owner(tp, a.n, item);
  const int local = item - tp[img];
  const ImgEntry e = a.table[img];
  const LayoutCfg lc = layout_cfg(a.p);
  const int k = a.k;
  const OctView ov = octave_view(e.h, e.w, lc, k);
  const int hk = ov.h, wk = ov.w, pk = ov.pitch;
  const int tiles_x = cdiv(wk, kTileW);
  const int ty = local / tiles_x;
  const int tx = local - ty * tiles_x;
  const int x0 = tx * kTileW, y0 = ty * TH;
  float* dst = const_cast<float*>(level_ptr(a.ws, e, ov, a.dst_level));

  // ---- stage the source tile with its halo
  const int mode = a.mode;
  if (mode == kSrcImage) {
    for (int idx = threadIdx.x; idx < IH * IW; idx += 256) {
      const int rr = idx / IW, cc = idx - rr * IW;
      const int y = mirror(y0 - R + rr, hk), x = mirror(x0 - R + cc, wk);
      s_in[rr * S + cc] = e.src[(int64_t)y * e.src_pitch + x] - kCentre;
    }
  } else if (mode == kSrcUpsample) {
    // bilinear 2x: U[y][x] = I(y/2, x/2), the sample past the last row or
    // column clamped to it; computed on centred values
    for (int idx = threadIdx.x; idx < IH * IW; idx += 256) {
      const int rr = idx / IW, cc = idx - rr * IW;
      const int y = mirror(y0 - R + rr, hk), x = mirror(x0 - R + cc, wk);
      const int ya = y >> 1, xa = x >> 1;
      const int yb = min(ya + 1, e.h - 1), xb = min(xa + 1, e.w - 1);
      const float* r0 = e.src + (int64_t)ya * e.src_pitch;
      float top = r0[xa] - kCentre;
      if (x & 1) top = (top + (r0[xb] - kCentre)) * 0.5f;
      float v = top;
      if (y & 1) {
        const float* r1 = e.src + (int64_t)yb * e.src_pitch;
        float bot = r1[xa] - kCentre;
        if (x & 1) bot = (bot + (r1[xb] - kCentre)) * 0.5f;
        v = (top + bot) * 0.5f;
      }
      s_in[rr * S + cc] = v;
    }
  } else if (mode == kSrcLevel) {
    const float* src = level_ptr(a.ws, e, ov, a.dst_level - 1);
    for (int idx = threadIdx.x; idx < IH * IW; idx += 256) {
      const int rr = idx / IW, cc = idx - rr * IW;
      const int y = mirror(y0 - R + rr, hk), x = mirror(x0 - R + cc, wk);
      s_in[rr * S + cc] = src[(int64_t)y * pk + x];
    }
  } else {
    // level s of the previous octave at every second pixel
    const OctView pv = octave_view(e.h, e.w, lc, k - 1);
    const float* src = level_ptr(a.ws, e, pv, a.p.s);
    const int pp = pv.pitch;
    for (int idx = threadIdx.x; idx < IH * IW; idx += 256) {
      const int rr = idx / IW, cc = idx - rr * IW;
      const int y = mirror(y0 - R + rr, hk), x = mirror(x0 - R + cc, wk);
      s_in[rr * S + cc] = src[(int64_t)(2 * y) * pp + 2 * x];
    }
  }
  __syncthreads();

  if (mode == kSrcDown) {
    // the subsampled base is this octave's level 0
    float* l0 = const_cast<float*>(level_ptr(a.ws, e, ov, 0));
    for (int idx = threadIdx.x; idx < TH * kTileW; idx += 256) {
      const int yy = idx / kTileW, xx = idx - yy * kTileW;
      if (y0 + yy < hk && x0 + xx < wk)
        l0[(int64_t)(y0 + yy) * pk + x0 + xx] = s_in[(R + yy) * S + R + xx];
    }
  }

  // ---- horizontal pass: rows of the staged tile, HB consecutive outputs per thread
  for (int u = threadIdx.x; u < IH * (kTileW / HB); u += 256) {
    const int row = u % IH, q = u / IH;
    const float* in = &s_in[row * S + q * HB];
    float acc[HB];
#pragma unroll
    for (int m = 0; m < HB; ++m) acc[m] = 0.0f;
#pragma unroll
    for (int j = 0; j < 2 * R + HB; ++j) {
      const float v = in[j];
#pragma unroll
      for (int m = 0; m < HB; ++m) {
        const int t = j - m;
        if (t >= 0 && t <= 2 * R) acc[m] = __fmaf_rn(a.taps[t], v, acc[m]);
      }
    }
#pragma unroll
    for (int m = 0; m < HB; ++m) s_h[row * HS + q * HB + m] = acc[m];
  }
  __syncthreads();

  // ---- vertical pass: VB consecutive outputs of one column per thread
  for (int u = threadIdx.x; u < (TH / VB) * kTileW; u += 256) {
    const int x = u % kTileW, yb = u / kTileW;
    float acc[VB];
#pragma unroll
    for (int m = 0; m < VB; ++m) acc[m] = 0.0f;
#pragma unroll
    for (int j = 0; j < 2 * R + VB; ++j) {
      const float v = s_h[(yb * VB + j) * HS + x];
#pragma unroll
      for (int m = 0; m < VB; ++m) {
        const int t = j - m;
        if (t >= 0 && t <= 2 * R) acc[m] = __fmaf_rn(a.taps[t], v, acc[m]);
      }
    }
    if (x0 + x < wk) {
#pragma unroll
      for (int m = 0; m < VB; ++m) {
        const int y = y0 + yb * VB + m;
        if (y < hk) dst[(int64_t)y * pk + x0 + x] = acc[m];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Detection.  One work-group per (image, octave, band of kBand rows); each
// wave walks 64-lane column segments (lanes 1..62 are outputs, lanes 0 and 63
// their halo) down the band with a 3-row register window of the DoG layers
// D_j = L_{j+1} - L_j.  A pixel of layer i is a candidate when |D| exceeds the
// pre-gate and D is strictly above (below) the maximum (minimum) of its 26
// neighbours.  The per-row result is a 64-bit ballot word stored per
// (layer, row, segment); per-band counts feed the ordered compaction.

template <int S>
struct DetRow {
  float own[S + 2], mx3[S + 2], mn3[S + 2], lrmx[S + 2], lrmn[S + 2];
};

template <int S>
__device__ __forceinline__ void det_load_row(DetRow<S>& d, const float* const* L, int64_t off) {
  float lv[S + 3];
#pragma unroll
  for (int j = 0; j < S + 3; ++j) lv[j] = L[j][off];
#pragma unroll
  for (int j = 0; j < S + 2; ++j) {
    const float v = lv[j + 1] - lv[j];
    const float l = __shfl_up(v, 1, 64);
    const float r = __shfl_down(v, 1, 64);
    d.own[j] = v;
    d.lrmx[j] = fmaxf(l, r);
    d.lrmn[j] = fminf(l, r);
    d.mx3[j] = fmaxf(d.lrmx[j], v);
    d.mn3[j] = fminf(d.lrmn[j], v);
  }
}

template <int S>
__global__ __launch_bounds__(256) void k_detect(char* ws, HdrPtrs hp, int n, DevParams p) {
  __shared__ int s_cnt[4][S];
  const int* bp = hp.band_prefix;
  const int item = blockIdx.x;
  const int img = find_owner(bp, n, item);
  const int lb = item - bp[img];
  const ImgEntry e = hp.table[img];
  const LayoutCfg lc = layout_cfg(p);
  int k, band;
  band_owner(e.h, e.w, lc, lb, &k, &band);
  const OctView ov = octave_view(e.h, e.w, lc, k);
  const int hk = ov.h, wk = ov.w, pk = ov.pitch, nseg = ov.nseg;
  const int b = p.border;
  const int r_begin = b + band * kBand;
  const int r_end = min(r_begin + kBand, hk - b);
  const float* L[S + 3];
#pragma unroll
  for (int j = 0; j < S + 3; ++j) L[j] = level_ptr(ws, e, ov, j);
  unsigned long long* masks = reinterpret_cast<unsigned long long*>(ws + e.region + ov.masks);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const float thr = p.pre_thr;

  int cnt[S];
#pragma unroll
  for (int i = 0; i < S; ++i) cnt[i] = 0;

  for (int sg = wave; sg < nseg; sg += 4) {
    const int c = b + sg * kSeg + lane - 1;
    const int cl = min(c, wk - 1);
    const bool out_col = lane >= 1 && lane <= kSeg && c < wk - b;
    DetRow<S> w0, w1, w2;
    det_load_row<S>(w0, L, (int64_t)(r_begin - 1) * pk + cl);
    det_load_row<S>(w1, L, (int64_t)r_begin * pk + cl);
    for (int r = r_begin; r < r_end; ++r) {
      det_load_row<S>(w2, L, (int64_t)(r + 1) * pk + cl);
      float max9[S + 2], min9[S + 2];
#pragma unroll
      for (int j = 0; j < S + 2; ++j) {
        max9[j] = fmaxf(fmaxf(w0.mx3[j], w1.mx3[j]), w2.mx3[j]);
        min9[j] = fminf(fminf(w0.mn3[j], w1.mn3[j]), w2.mn3[j]);
      }
#pragma unroll
      for (int i = 1; i <= S; ++i) {
        const float v = w1.own[i];
        const float max8 = fmaxf(fmaxf(w0.mx3[i], w1.lrmx[i]), w2.mx3[i]);
        const float min8 = fminf(fminf(w0.mn3[i], w1.lrmn[i]), w2.mn3[i]);
        const float nb_max = fmaxf(fmaxf(max9[i - 1], max8), max9[i + 1]);
        const float nb_min = fminf(fminf(min9[i - 1], min8), min9[i + 1]);
        const bool flag = out_col && fabsf(v) > thr && (v > nb_max || v < nb_min);
        const unsigned long long m = __ballot(flag);
        if (lane == 0) masks[((int64_t)(i - 1) * hk + r) * nseg + sg] = m;
        cnt[i - 1] += __popcll(m);
      }
      w0 = w1;
      w1 = w2;
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < S; ++i) s_cnt[wave][i] = cnt[i];
  }
  __syncthreads();
  if (threadIdx.x < S) {
    const int i = threadIdx.x;
    const int tot = s_cnt[0][i] + s_cnt[1][i] + s_cnt[2][i] + s_cnt[3][i];
    int* bc = reinterpret_cast<int*>(ws + e.region + region_tail(e.h, e.w, lc).band_cnt);
    bc[ov.band_base * S + i * ov.nband + band] = tot;
  }
}

// Exclusive scan of the band counts of one image in canonical order
// (octave, layer, band); one work-group per image.
__global__ __launch_bounds__(256) void k_band_scan(char* ws, HdrPtrs hp, int n, DevParams p) {
  __shared__ int s_wave[4];
  const ImgEntry e = hp.table[blockIdx.x];
  const RegionTail rt = region_tail(e.h, e.w, layout_cfg(p));
  const int total_bands = rt.total_bands * p.s;
  const int* bc = reinterpret_cast<const int*>(ws + e.region + rt.band_cnt);
  int* bo = reinterpret_cast<int*>(ws + e.region + rt.band_off);
  int base = 0;
  for (int c0 = 0; c0 < total_bands; c0 += 256) {
    const int idx = c0 + threadIdx.x;
    const int v = idx < total_bands ? bc[idx] : 0;
    int tot;
    const int ex = block_excl_scan256(v, s_wave, &tot);
    if (idx < total_bands) bo[idx] = base + ex;
    base += tot;
  }
  if (threadIdx.x == 0) {
    counters_of(ws, e)[kCntCand] = base;
    if (e.n_cand) *e.n_cand = base;
  }
}

// Candidate emission: one wave per (image, octave, band) writes the set bits
// of its mask words, layer by layer, row by row, segment by segment, at the
// offsets of the band scan -- the canonical (octave, layer, row, column) order.
__global__ __launch_bounds__(64) void k_emit(char* ws, HdrPtrs hp, int n, DevParams p) {
  const int* bp = hp.band_prefix;
  const int item = blockIdx.x;
  const int img = find_owner(bp, n, item);
  const int lb = item - bp[img];
  const ImgEntry e = hp.table[img];
  const LayoutCfg lc = layout_cfg(p);
  int k, band;
  band_owner(e.h, e.w, lc, lb, &k, &band);
  const OctView ov = octave_view(e.h, e.w, lc, k);
  const RegionTail rt = region_tail(e.h, e.w, lc);
  const int hk = ov.h, nseg = ov.nseg;
  const int b = p.border;
  const int r_begin = b + band * kBand;
  const int r_end = min(r_begin + kBand, hk - b);
  const int nwords = (r_end - r_begin) * nseg;
  const unsigned long long* masks =
      reinterpret_cast<const unsigned long long*>(ws + e.region + ov.masks);
  const int* bo = reinterpret_cast<const int*>(ws + e.region + rt.band_off);
  int4* cands = reinterpret_cast<int4*>(ws + e.region + rt.cands);
  const int lane = threadIdx.x;
  for (int i = 1; i <= p.s; ++i) {
    int base = bo[ov.band_base * p.s + (i - 1) * ov.nband + band];
    for (int w0 = 0; w0 < nwords; w0 += 64) {
      const int wi = w0 + lane;
      unsigned long long m = 0ull;
      int r = 0, sg = 0;
      if (wi < nwords) {
        r = r_begin + wi / nseg;
        sg = wi - (wi / nseg) * nseg;
        m = masks[((int64_t)(i - 1) * hk + r) * nseg + sg];
      }
      const int pc = __popcll(m);
      const int incl = wave_incl_scan(pc);
      int idx = base + incl - pc;
      while (m) {
        const int bit = __ffsll((long long)m) - 1;
        m &= m - 1ull;
        if (idx < p.max_cand) cands[idx] = make_int4(k, i, r, b + sg * kSeg + bit - 1);
        ++idx;
      }
      base += __shfl(incl, 63, 64);
    }
  }
}

// Per-image prefix of min(counter, limit) over the batch (one work-group).
__global__ __launch_bounds__(256) void k_img_prefix(char* ws, HdrPtrs hp, int n, DevParams p,
                                                    int which) {
  __shared__ int s_wave[4];
  int* out = which == 0 ? hp.cand_prefix : hp.kp_prefix;
  const ImgEntry* tab = hp.table;
  int base = 0;
  for (int c0 = 0; c0 < n; c0 += 256) {
    const int i = c0 + threadIdx.x;
    int v = 0;
    if (i < n) {
      const int* cnt = counters_of(ws, tab[i]);
      if (which == 0) {
        v = min(cnt[kCntCand], p.max_cand);
      } else {
        v = min(min(cnt[kCntKp], p.max_kp), tab[i].cap);
      }
    }
    int tot;
    const int ex = block_excl_scan256(v, s_wave, &tot);
    if (i < n) out[i] = base + ex;
    base += tot;
  }
  if (threadIdx.x == 0) out[n] = base;
}

// ---------------------------------------------------------------------------
// Refinement: one thread per candidate, in double precision on the fp32 DoG
// samples.  Up to refine_iters Newton steps of the 3-D quadratic fit (the
// 3x3 system solved by Cramer's rule); a step is final when all |x^| <= 0.5,
// otherwise each coordinate with |x^| > 0.5 moves by x^ rounded half away
// from zero.  Then the contrast test on |D(x^)| and the edge test on the 2x2
// spatial Hessian.

__device__ __forceinline__ double det3d(double a00, double a01, double a02, double a10, double a11,
                                        double a12, double a20, double a21, double a22) {
  return a00 * (a11 * a22 - a12 * a21) - a01 * (a10 * a22 - a12 * a20) +
         a02 * (a10 * a21 - a11 * a20);
}

__device__ __forceinline__ double round_half_away(double x) {
  return x >= 0.0 ? floor(x + 0.5) : -floor(-x + 0.5);
}

__global__ __launch_bounds__(256) void k_refine(char* ws, HdrPtrs hp, int n, DevParams p) {
  const int* cp = hp.cand_prefix;
  const int total = cp[n];
  const ImgEntry* tab = hp.table;
  const LayoutCfg lc = layout_cfg(p);
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < total; g += gridDim.x * blockDim.x) {
    const int img = find_owner(cp, n, g);
    const int j = g - cp[img];
    const ImgEntry e = tab[img];
    const RegionTail rt = region_tail(e.h, e.w, lc);
    const int4 cd = reinterpret_cast<const int4*>(ws + e.region + rt.cands)[j];
    const int k = cd.x;
    int li = cd.y, r = cd.z, c = cd.w;
    const OctView ov = octave_view(e.h, e.w, lc, k);
    const int hk = ov.h, wk = ov.w, pk = ov.pitch;
    const int b = p.border, s = p.s;
    RefinedKp out;
    out.ok = 0;
    out.k = k;
    out.layer = li;
    out.r = r;
    out.c = c;
    out.dx = out.dy = out.sigma_oct = out.response = out.x = out.y = out.sigma = 0.0f;
    bool converged = false;
    double xs = 0.0, xy = 0.0, xx = 0.0;
    double v = 0.0, gx = 0.0, gy = 0.0, gs = 0.0, dxx = 0.0, dyy = 0.0, dxy = 0.0;
    bool bad = false;
    for (int it = 0; it < p.refine_iters; ++it) {
      // D samples of layers li-1, li, li+1 around (r, c)
      double d[3][3][3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const float* La = level_ptr(ws, e, ov, li - 1 + a);
        const float* Lb = level_ptr(ws, e, ov, li + a);
#pragma unroll
        for (int dr = 0; dr < 3; ++dr)
#pragma unroll
          for (int dc = 0; dc < 3; ++dc) {
            const int64_t off = (int64_t)(r - 1 + dr) * pk + (c - 1 + dc);
            d[a][dr][dc] = (double)(Lb[off] - La[off]);
          }
      }
      v = d[1][1][1];
      gx = (d[1][1][2] - d[1][1][0]) * 0.5;
      gy = (d[1][2][1] - d[1][0][1]) * 0.5;
      gs = (d[2][1][1] - d[0][1][1]) * 0.5;
      dxx = d[1][1][2] + d[1][1][0] - 2.0 * v;
      dyy = d[1][2][1] + d[1][0][1] - 2.0 * v;
      const double dss = d[2][1][1] + d[0][1][1] - 2.0 * v;
      dxy = (d[1][2][2] - d[1][2][0] - d[1][0][2] + d[1][0][0]) * 0.25;
      const double dxs = (d[2][1][2] - d[2][1][0] - d[0][1][2] + d[0][1][0]) * 0.25;
      const double dys = (d[2][2][1] - d[2][0][1] - d[0][2][1] + d[0][0][1]) * 0.25;
      const double det = det3d(dxx, dxy, dxs, dxy, dyy, dys, dxs, dys, dss);
      if (det == 0.0) { bad = true; break; }
      const double bx = -gx, by = -gy, bs = -gs;
      xx = det3d(bx, dxy, dxs, by, dyy, dys, bs, dys, dss) / det;
      xy = det3d(dxx, bx, dxs, dxy, by, dys, dxs, bs, dss) / det;
      xs = det3d(dxx, dxy, bx, dxy, dyy, by, dxs, dys, bs) / det;
      if (!isfinite(xx) || !isfinite(xy) || !isfinite(xs)) { bad = true; break; }
      if (fabs(xx) <= 0.5 && fabs(xy) <= 0.5 && fabs(xs) <= 0.5) { converged = true; break; }
      // any move of more than the octave size leaves the frame
      if (fabs(xx) > 1e6 || fabs(xy) > 1e6 || fabs(xs) > 1e6) { bad = true; break; }
      if (fabs(xx) > 0.5) c += (int)round_half_away(xx);
      if (fabs(xy) > 0.5) r += (int)round_half_away(xy);
      if (fabs(xs) > 0.5) li += (int)round_half_away(xs);
      if (li < 1 || li > s || r < b || r >= hk - b || c < b || c >= wk - b) { bad = true; break; }
    }
    if (!bad && converged) {
      const double contrast = v + 0.5 * (gx * xx + gy * xy + gs * xs);
      const double tr = dxx + dyy;
      const double det2 = dxx * dyy - dxy * dxy;
      const double re = (double)p.edge_ratio;
      if (fabs(contrast) >= (double)p.contrast_thr && det2 > 0.0 &&
          tr * tr * re < (re + 1.0) * (re + 1.0) * det2) {
        const int o = p.o0 + k;
        const double sig = (double)p.sigma0 * exp2((li + xs) / s);
        const double sc = ldexp(1.0, o);
        out.ok = 1;
        out.dx = (float)xx;
        out.dy = (float)xy;
        out.sigma_oct = (float)sig;
        out.response = (float)fabs(contrast);
        out.x = (float)((c + xx) * sc);
        out.y = (float)((r + xy) * sc);
        out.sigma = (float)(sig * sc);
      }
    }
    out.layer = li;
    out.r = r;
    out.c = c;
    reinterpret_cast<RefinedKp*>(ws + e.region + rt.refined)[j] = out;
  }
}

// ---------------------------------------------------------------------------
// Orientation: one wave per refined candidate.  Samples of the square window
// are dealt to lanes in a fixed order; each lane accumulates into its own
// LDS column of the 36-bin histogram (layout [bin][lane]: no two lanes share
// an address, so no atomics), a sample's weight split linearly between the
// two nearest bins.  Bins are then summed over lanes in a fixed order, smoothed
// once with [1/4, 1/2, 1/4], and every strict local maximum >= peak_ratio *
// max gives an orientation refined by a parabola through the bin and its two
// neighbours.

__global__ __launch_bounds__(256) void k_orient(char* ws, HdrPtrs hp, int n, DevParams p) {
  __shared__ float s_hist[4][kOriBins * 64];
  __shared__ float s_bins[4][kOriBins];
  const int* cp = hp.cand_prefix;
  const int total = cp[n];
  const ImgEntry* tab = hp.table;
  const LayoutCfg lc = layout_cfg(p);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float* hist = s_hist[wave];
  float* bins = s_bins[wave];
  const int nwaves = gridDim.x * 4;
  for (int g = blockIdx.x * 4 + wave; g < total; g += nwaves) {
    const int img = find_owner(cp, n, g);
    const int j = g - cp[img];
    const ImgEntry e = tab[img];
    const RegionTail rt = region_tail(e.h, e.w, lc);
    const RefinedKp kp = reinterpret_cast<const RefinedKp*>(ws + e.region + rt.refined)[j];
    int* n_ori = reinterpret_cast<int*>(ws + e.region + rt.n_ori);
    float* angles = reinterpret_cast<float*>(ws + e.region + rt.angles) + (int64_t)j * kMaxPeaks;
    if (!kp.ok) {
      if (lane == 0) n_ori[j] = 0;
      continue;
    }
    if (p.upright) {
      if (lane == 0) {
        n_ori[j] = 1;
        angles[0] = 0.0f;
      }
      continue;
    }
    const OctView ov = octave_view(e.h, e.w, lc, kp.k);
    const int hk = ov.h, wk = ov.w, pk = ov.pitch;
    const float* L = level_ptr(ws, e, ov, kp.layer);
    const float sw = p.ori_sigma_factor * kp.sigma_oct;
    const int R = (int)floorf(p.ori_radius_factor * sw + 0.5f);
    const float inv2 = 1.0f / (2.0f * sw * sw);
    const int side = 2 * R + 1;
    const int nsamp = side * side;
#pragma unroll
    for (int bn = 0; bn < kOriBins; ++bn) hist[bn * 64 + lane] = 0.0f;
    for (int q = lane; q < nsamp; q += 64) {
      const int qy = q / side;
      const int dy = qy - R, dx = q - qy * side - R;
      const int rr = kp.r + dy, cc = kp.c + dx;
      if (rr < 1 || rr > hk - 2 || cc < 1 || cc > wk - 2) continue;
      const float* row = L + (int64_t)rr * pk;
      const float gx = row[cc + 1] - row[cc - 1];
      const float gy = row[pk + cc] - row[cc - pk];
      const float mag = sqrtf(gx * gx + gy * gy);
      float th = atan2f(gy, gx);
      if (th < 0.0f) th += kTwoPi;
      const float wgt = expf(-(float)(dx * dx + dy * dy) * inv2) * mag;
      const float pos = th * ((float)kOriBins / kTwoPi);
      const float fl = floorf(pos);
      const float f = pos - fl;
      int b0 = (int)fl;
      if (b0 >= kOriBins) b0 -= kOriBins;
      int b1 = b0 + 1;
      if (b1 >= kOriBins) b1 -= kOriBins;
      hist[b0 * 64 + lane] += wgt * (1.0f - f);
      hist[b1 * 64 + lane] += wgt * f;
    }
    wave_lds_sync();
    if (lane < kOriBins) {
      float acc = 0.0f;
      for (int t = 0; t < 64; ++t) acc += hist[lane * 64 + ((lane + t) & 63)];
      bins[lane] = acc;
    }
    wave_lds_sync();
    float hs = -1.0f;
    if (lane < kOriBins) {
      const float l = bins[lane == 0 ? kOriBins - 1 : lane - 1];
      const float m = bins[lane];
      const float rt = bins[lane == kOriBins - 1 ? 0 : lane + 1];
      hs = (0.25f * l + 0.5f * m) + 0.25f * rt;
    }
    wave_lds_sync();
    if (lane < kOriBins) bins[lane] = hs;
    wave_lds_sync();
    const float hmax = wave_max(hs);
    bool peak = false;
    float ang = 0.0f;
    if (lane < kOriBins && hmax > 0.0f) {
      const float l = bins[lane == 0 ? kOriBins - 1 : lane - 1];
      const float rt = bins[lane == kOriBins - 1 ? 0 : lane + 1];
      peak = hs > l && hs > rt && hs >= p.ori_peak_ratio * hmax;
      if (peak) {
        const float delta = 0.5f * (l - rt) / ((l - 2.0f * hs) + rt);
        ang = ((float)lane + delta) * (360.0f / (float)kOriBins);
        if (ang < 0.0f) ang += 360.0f;
        if (ang >= 360.0f) ang -= 360.0f;
      }
    }
    const unsigned long long pm = __ballot(peak);
    if (peak) {
      const int rank = __popcll(pm & ((1ull << lane) - 1ull));
      angles[rank] = ang;
    }
    if (lane == 0) n_ori[j] = __popcll(pm);
    wave_lds_sync();
  }
}

// Exclusive scan of orientation counts in candidate order; one work-group per
// image.  Publishes n_found and count.
__global__ __launch_bounds__(256) void k_ori_scan(char* ws, HdrPtrs hp, int n, DevParams p) {
  __shared__ int s_wave[4];
  const ImgEntry e = hp.table[blockIdx.x];
  const RegionTail rt = region_tail(e.h, e.w, layout_cfg(p));
  int* cnt = counters_of(ws, e);
  const int nc = min(cnt[kCntCand], p.max_cand);
  const int* n_ori = reinterpret_cast<const int*>(ws + e.region + rt.n_ori);
  int* kp_off = reinterpret_cast<int*>(ws + e.region + rt.kp_off);
  int base = 0;
  for (int c0 = 0; c0 < nc; c0 += 256) {
    const int idx = c0 + threadIdx.x;
    const int v = idx < nc ? n_ori[idx] : 0;
    int tot;
    const int ex = block_excl_scan256(v, s_wave, &tot);
    if (idx < nc) kp_off[idx] = base + ex;
    base += tot;
  }
  if (threadIdx.x == 0) {
    cnt[kCntKp] = base;
    if (e.n_found) *e.n_found = base;
    *e.count = min(min(base, p.max_kp), e.cap);
  }
}

// ---------------------------------------------------------------------------
// Descriptor: one wave per output keypoint.  For each pooled domain size the
// window of the rotated 4x4 grid is swept with samples dealt to lanes in a
// fixed order; each lane accumulates trilinear contributions into its own LDS
// column of the 128-bin histogram.  The lane columns are summed in a fixed
// order, averaged over domain sizes, then L2-normalised, clamped, L2-normalised
// and optionally turned into RootSIFT (L1 normalise, square root).

__global__ __launch_bounds__(64) void k_describe(char* ws, HdrPtrs hp, int n, DevParams p) {
  __shared__ float hist[kDescDim * 64];
  const int* kpp = hp.kp_prefix;
  const int total = kpp[n];
  const ImgEntry* tab = hp.table;
  const LayoutCfg lc = layout_cfg(p);
  const int lane = threadIdx.x;
  for (int g = blockIdx.x; g < total; g += gridDim.x) {
    const int img = find_owner(kpp, n, g);
    const int q = g - kpp[img];
    const ImgEntry e = tab[img];
    const RegionTail rt = region_tail(e.h, e.w, lc);
    const int* cnt = counters_of(ws, e);
    const int nc = min(cnt[kCntCand], p.max_cand);
    const int* kp_off = reinterpret_cast<const int*>(ws + e.region + rt.kp_off);
    // candidate j with kp_off[j] <= q < kp_off[j] + n_ori[j]
    int lo = 0, hi = nc;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (kp_off[mid] <= q) lo = mid; else hi = mid;
    }
    const int j = lo;
    const int pk_idx = q - kp_off[j];
    const RefinedKp kp = reinterpret_cast<const RefinedKp*>(ws + e.region + rt.refined)[j];
    const int4 cd = reinterpret_cast<const int4*>(ws + e.region + rt.cands)[j];
    const float angle =
        reinterpret_cast<const float*>(ws + e.region + rt.angles)[(int64_t)j * kMaxPeaks + pk_idx];
    const int k = kp.k;
    const OctView ov = octave_view(e.h, e.w, lc, k);
    const int hk = ov.h, wk = ov.w, pk = ov.pitch;
    const float* L = level_ptr(ws, e, ov, kp.layer);
    const float th = angle * (kTwoPi / 360.0f);
    const float st = sinf(th), ct = cosf(th);

#pragma unroll
    for (int bn = 0; bn < kDescDim; ++bn) hist[bn * 64 + lane] = 0.0f;

    for (int ds = 0; ds < p.n_dsp; ++ds) {
      const float wc = p.desc_magnif * kp.sigma_oct * p.dsp[ds];
      const float inv_wc = 1.0f / wc;
      // the rotated 5x5-cell square around the sub-pixel centre lies within
      // radius sqrt(2) * 2.5 * wc; one extra ring covers fp32 rounding
      const int R = (int)ceilf(1.41421356f * 2.5f * wc) + 1;
      const int side = 2 * R + 1;
      const int nsamp = side * side;
      for (int qq = lane; qq < nsamp; qq += 64) {
        const int qy = qq / side;
        const int dy = qy - R, dx = qq - qy * side - R;
        const int rr = kp.r + dy, cc = kp.c + dx;
        if (rr < 1 || rr > hk - 2 || cc < 1 || cc > wk - 2) continue;
        const float u = (float)dx - kp.dx;
        const float v = (float)dy - kp.dy;
        const float xr = (ct * u + st * v) * inv_wc;
        const float yr = (ct * v - st * u) * inv_wc;
        const float rb = yr + 1.5f, cb = xr + 1.5f;
        if (!(rb > -1.0f && rb < 4.0f && cb > -1.0f && cb < 4.0f)) continue;
        const float* row = L + (int64_t)rr * pk;
        const float gx = row[cc + 1] - row[cc - 1];
        const float gy = row[pk + cc] - row[cc - pk];
        const float mag = sqrtf(gx * gx + gy * gy);
        float ta = atan2f(gy, gx);
        if (ta < 0.0f) ta += kTwoPi;
        float ob = ta - th;
        if (ob < 0.0f) ob += kTwoPi;
        if (ob >= kTwoPi) ob -= kTwoPi;
        ob = ob * (8.0f / kTwoPi);
        const float wgt = mag * expf(-(xr * xr + yr * yr) * 0.125f);
        const float r0 = floorf(rb), c0 = floorf(cb), o0 = floorf(ob);
        const float fr = rb - r0, fc = cb - c0, fo = ob - o0;
        const int ir = (int)r0, ic = (int)c0;
        int io = (int)o0;
        if (io >= 8) io -= 8;
        const int io1 = (io + 1) & 7;
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const int row_b = ir + a;
          if (row_b < 0 || row_b > 3) continue;
          const float wr = a ? fr : 1.0f - fr;
#pragma unroll
          for (int bb = 0; bb < 2; ++bb) {
            const int col_b = ic + bb;
            if (col_b < 0 || col_b > 3) continue;
            const float wcl = bb ? fc : 1.0f - fc;
            const float w2 = wgt * wr * wcl;
            const int cell = (row_b * 4 + col_b) * 8;
            hist[(cell + io) * 64 + lane] += w2 * (1.0f - fo);
            hist[(cell + io1) * 64 + lane] += w2 * fo;
          }
        }
      }
    }
    wave_lds_sync();
    float h0 = 0.0f, h1 = 0.0f;
    for (int t = 0; t < 64; ++t) {
      const int col = (lane + t) & 63;
      h0 += hist[lane * 64 + col];
      h1 += hist[(lane + 64) * 64 + col];
    }
    const float kf = (float)p.n_dsp;
    h0 = h0 / kf;
    h1 = h1 / kf;
    float nrm = sqrtf(wave_sum(h0 * h0 + h1 * h1));
    if (nrm > 0.0f) { h0 = h0 / nrm; h1 = h1 / nrm; } else { h0 = 0.0f; h1 = 0.0f; }
    h0 = fminf(h0, p.desc_clamp);
    h1 = fminf(h1, p.desc_clamp);
    nrm = sqrtf(wave_sum(h0 * h0 + h1 * h1));
    if (nrm > 0.0f) { h0 = h0 / nrm; h1 = h1 / nrm; } else { h0 = 0.0f; h1 = 0.0f; }
    if (p.rootsift) {
      const float l1 = wave_sum(fabsf(h0) + fabsf(h1));
      if (l1 > 0.0f) { h0 = h0 / l1; h1 = h1 / l1; }
      h0 = sqrtf(h0);
      h1 = sqrtf(h1);
    }
    const int slot = q;
    float* dout = e.desc + (int64_t)slot * kDescDim;
    dout[lane] = h0;
    dout[lane + 64] = h1;
    if (lane == 0) {
      sift_keypoint o;
      o.x = kp.x;
      o.y = kp.y;
      o.sigma = kp.sigma;
      o.angle = angle;
      o.response = kp.response;
      o.octave = p.o0 + k;
      o.layer = kp.layer;
      o.ix = kp.c;
      o.iy = kp.r;
      o.src_layer = cd.y;
      o.src_iy = cd.z;
      o.src_ix = cd.w;
      e.kp[slot] = o;
    }
    wave_lds_sync();
  }
}

// ---------------------------------------------------------------------------
// Launch helpers: hipLaunchKernel returns the launch status directly (the
// thread's last-error slot may hold another library's stale error).

template <typename... Args>
static hipError_t launch(void (*kernel)(Args...), dim3 grid, dim3 block, hipStream_t stream,
                         Args... args) {
  void* ptrs[] = {static_cast<void*>(&args)...};
  return hipLaunchKernel(reinterpret_cast<const void*>(kernel), grid, block, ptrs, 0, stream);
}

hipError_t launch_setup(const HdrPtrs& hp, const SetupChunk& c, hipStream_t stream) {
  return launch(k_setup, dim3(1), dim3(64), stream, hp, c);
}

hipError_t launch_finalize(const HdrPtrs& hp, int n, const DevParams& p, hipStream_t stream) {
  return launch(k_finalize, dim3(1), dim3(64), stream, hp, n, p);
}

typedef void (*BlurKernel)(BlurArgs);

#define SIFT_BLUR_CASES_16(TH)                                                           \
  SIFT_BLUR_CASE(1, TH) SIFT_BLUR_CASE(2, TH) SIFT_BLUR_CASE(3, TH) SIFT_BLUR_CASE(4, TH)     \
  SIFT_BLUR_CASE(5, TH) SIFT_BLUR_CASE(6, TH) SIFT_BLUR_CASE(7, TH) SIFT_BLUR_CASE(8, TH)     \
  SIFT_BLUR_CASE(9, TH) SIFT_BLUR_CASE(10, TH) SIFT_BLUR_CASE(11, TH) SIFT_BLUR_CASE(12, TH)  \
  SIFT_BLUR_CASE(13, TH) SIFT_BLUR_CASE(14, TH) SIFT_BLUR_CASE(15, TH) SIFT_BLUR_CASE(16, TH)
#define SIFT_BLUR_CASES_24(TH)                                                           \
  SIFT_BLUR_CASES_16(TH)                                                                   \
  SIFT_BLUR_CASE(17, TH) SIFT_BLUR_CASE(18, TH) SIFT_BLUR_CASE(19, TH) SIFT_BLUR_CASE(20, TH) \
  SIFT_BLUR_CASE(21, TH) SIFT_BLUR_CASE(22, TH) SIFT_BLUR_CASE(23, TH) SIFT_BLUR_CASE(24, TH)
#define SIFT_BLUR_CASE(RR, TH) \
  case RR: return k_blur<RR, TH>;

static BlurKernel blur_kernel(int radius, int th) {
  if (th == 16) {
    switch (radius) { SIFT_BLUR_CASES_24(16) default: return nullptr; }
  } else if (th == 32) {
    switch (radius) { SIFT_BLUR_CASES_24(32) default: return nullptr; }
  } else if (th == 64) {
    // 64-row tiles stay within 64 KiB of LDS up to radius 16
    switch (radius) { SIFT_BLUR_CASES_16(64) default: return nullptr; }
  }
  return nullptr;
}
#undef SIFT_BLUR_CASE

hipError_t launch_blur(const BlurArgs& a, int radius, int grid, hipStream_t stream) {
  BlurKernel fn = blur_kernel(radius, a.th);
  if (!fn) return hipErrorInvalidValue;
  return launch(fn, dim3(grid), dim3(256), stream, a);
}

hipError_t launch_detect(char* ws, const HdrPtrs& hp, int n, const DevParams& p, int grid,
                         hipStream_t stream) {
  switch (p.s) {
    case 1: return launch(k_detect<1>, dim3(grid), dim3(256), stream, ws, hp, n, p);
    case 2: return launch(k_detect<2>, dim3(grid), dim3(256), stream, ws, hp, n, p);
    case 3: return launch(k_detect<3>, dim3(grid), dim3(256), stream, ws, hp, n, p);
    case 4: return launch(k_detect<4>, dim3(grid), dim3(256), stream, ws, hp, n, p);
    case 5: return launch(k_detect<5>, dim3(grid), dim3(256), stream, ws, hp, n, p);
    case 6: return launch(k_detect<6>, dim3(grid), dim3(256), stream, ws, hp, n, p);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_band_scan(char* ws, const HdrPtrs& hp, int n, const DevParams& p,
                         hipStream_t stream) {
  return launch(k_band_scan, dim3(n), dim3(256), stream, ws, hp, n, p);
}

hipError_t launch_emit(char* ws, const HdrPtrs& hp, int n, const DevParams& p, int grid,
                         hipStream_t stream) {
  return launch(k_emit, dim3(grid), dim3(64), stream, ws, hp, n, p);
}

hipError_t launch_img_prefix(char* ws, const HdrPtrs& hp, int n, const DevParams& p, int which,
                             hipStream_t stream) {
  return launch(k_img_prefix, dim3(1), dim3(256), stream, ws, hp, n, p, which);
}

hipError_t launch_refine(char* ws, const HdrPtrs& hp, int n, const DevParams& p, int grid,
                         hipStream_t stream) {
  return launch(k_refine, dim3(grid), dim3(256), stream, ws, hp, n, p);
}

hipError_t launch_orient(char* ws, const HdrPtrs& hp, int n, const DevParams& p, int grid,
                         hipStream_t stream) {
  return launch(k_orient, dim3(grid), dim3(256), stream, ws, hp, n, p);
}

hipError_t launch_ori_scan(char* ws, const HdrPtrs& hp, int n, const DevParams& p,
                         hipStream_t stream) {
  return launch(k_ori_scan, dim3(n), dim3(256), stream, ws, hp, n, p);
}

hipError_t launch_describe(char* ws, const HdrPtrs& hp, int n, const DevParams& p, int grid,
                         hipStream_t stream) {
  return launch(k_describe, dim3(grid), dim3(64), stream, ws, hp, n, p);
}

}  // namespace sift
