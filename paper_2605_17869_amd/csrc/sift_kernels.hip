// gfx950 kernels of the SIFT extraction path.
//
// Every kernel serves a whole batch: work items are decoded from prefix
// tables over the images of the batch, so one image goes through exactly
// the same per-pixel and per-keypoint arithmetic whether it is extracted
// alone or with others.  No two lanes ever add floats into the same memory
// location in one instruction (histograms keep columns that lanes own); every
// sum has an order fixed in this source, which makes the output bit-identical
// from run to run.  The file is built with -ffp-contract=off: every fused
// multiply-add below is written out explicitly.
#include <hip/hip_runtime.h>
#include <math.h>

#include "sift_device.h"
#include "sift_launch.h"

namespace sift {

// ---------------------------------------------------------------------------
// Setup: copy image-table entries from kernel arguments into the workspace,
// then derive the per-octave tile and per-image band prefix sums.

__global__ void k_setup(HdrPtrs hp, SetupChunk c) {
  const int t = threadIdx.x;
  if (t < c.count) const_cast<ImgEntry*>(hp.table)[c.first + t] = c.e[t];
}

// Prefix sums over the batch of the blur work items of every (chunk class,
// octave) and of the detection bands, one wave, 64 images at a time: lane i
// takes image i0 + i, each table is one wave scan, and lane t keeps the
// running total of table t between chunks.
static_assert(kNumTileH * kMaxOct + 1 <= 64, "one lane per table");

__global__ void k_finalize(HdrPtrs hp, int n, DevParams p) {
  const ImgEntry* tab = hp.table;
  const LayoutCfg lc = layout_cfg(p);
  const int lane = threadIdx.x;
  const int ntile = kNumTileH * p.n_oct;   // tables 0 .. ntile - 1; the band table last
  int run = 0;
  for (int i0 = 0; i0 < n; i0 += 64) {
    const int i = i0 + lane;
    const bool has = i < n;
    const int h = has ? tab[i].h : 0, w = has ? tab[i].w : 0;
    for (int t = 0; t <= ntile; ++t) {
      int v = 0;
      int* out;
      if (t < ntile) {
        // tile prefix for class t / n_oct, octave t % n_oct
        const int cls = t / p.n_oct, k = t - cls * p.n_oct;
        if (has) {
          int hk, wk;
          octave_dims(h, w, p.upsample, k, &hk, &wk);
          v = cdiv(wk, kTileW) * cdiv(hk, tile_h_of(cls));
        }
        out = hp.tile_prefix + (cls * kMaxOct + k) * (n + 1);
      } else {
        if (has) v = region_tail(h, w, lc).total_bands;
        out = hp.band_prefix;
      }
      const int incl = wave_incl_scan(v);
      const int base = __shfl(run, t, 64);
      if (i0 == 0 && lane == 0) out[0] = 0;
      if (has) out[i + 1] = base + incl;
      const int chunk = __shfl(incl, 63, 64);
      if (lane == t) run += chunk;
    }
  }
  if (lane < kQueues) hp.queue[lane] = 0;   // the work counters of this launch sequence
}

// ---------------------------------------------------------------------------
// Detection.  One work-group per (image, octave, band of kBand = 8 rows): short
// bands keep each wave's dependent row loop short, which matters more here
// than the 2 halo rows a band re-reads.  Each wave walks 64-lane column
// segments (lanes 1..62 are outputs, lanes 0 and 63 their halo) down the band
// with a 3-row register window of the DoG layers
// D_j = L_{j+1} - L_j.  A pixel of layer i is a candidate when |D| exceeds the
// pre-gate and D is strictly above (below) the maximum (minimum) of its 26
// neighbours.  The per-row result is a 64-bit ballot word stored per
// (layer, row, segment); per-band counts feed the ordered compaction.

template <int S>
struct DetRow {
  float own[S + 2], mx3[S + 2], mn3[S + 2], lrmx[S + 2], lrmn[S + 2];
};

template <int S, bool H16>
__device__ __forceinline__ void det_load_row(DetRow<S>& d, const char* const* L, int64_t off,
                                             const Span& rs) {
  float lv[S + 3];
#pragma unroll
  for (int j = 0; j < S + 3; ++j) {
    SIFT_CHECK_IN(rs, L[j] + off * (H16 ? 2 : 4), H16 ? 2 : 4);
    lv[j] = lv_at<H16>(L[j], off);
  }
#pragma unroll
  for (int j = 0; j < S + 2; ++j) {
    const float v = lv[j + 1] - lv[j];
    const float l = lane_prev(v);
    const float r = lane_next(v);
    d.own[j] = v;
    d.lrmx[j] = fmaxf(l, r);
    d.lrmn[j] = fminf(l, r);
    d.mx3[j] = fmaxf(d.lrmx[j], v);
    d.mn3[j] = fminf(d.lrmn[j], v);
  }
}

// The rows of one band: per-layer candidate counts into cnt.  H16: the
// octave's levels are stored as fp16; W: waves of the work-group.
template <int S, bool H16, int W>
__device__ __forceinline__ void detect_band(const char* const* L, unsigned long long* masks,
                                            int hk, int wk, int pk, int nseg, int b, int r_begin,
                                            int r_end, float thr, int* cnt, const Span& rs) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int sg = wave; sg < nseg; sg += W) {
    const int c = b + sg * kSeg + lane - 1;
    const int cl = min(c, wk - 1);
    const bool out_col = lane >= 1 && lane <= kSeg && c < wk - b;
    DetRow<S> w0, w1, w2;
    det_load_row<S, H16>(w0, L, (int64_t)(r_begin - 1) * pk + cl, rs);
    det_load_row<S, H16>(w1, L, (int64_t)r_begin * pk + cl, rs);
    for (int r = r_begin; r < r_end; ++r) {
      det_load_row<S, H16>(w2, L, (int64_t)(r + 1) * pk + cl, rs);
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
        if (lane == 0) {
          SIFT_CHECK_IN(rs, &masks[((int64_t)(i - 1) * hk + r) * nseg + sg], 8);
          masks[((int64_t)(i - 1) * hk + r) * nseg + sg] = m;
        }
        cnt[i - 1] += __popcll(m);
      }
      w0 = w1;
      w1 = w2;
    }
  }
}

// H16MODE: fp16 level storage is on (the first octave stays fp32, so each
// work-group picks its octave's path).  W: waves per work-group, which share
// the band's column segments; the counts do not depend on it.
template <int S, bool H16MODE, int W>
__global__ __launch_bounds__(W * 64) void k_detect(char* ws, HdrPtrs hp, int n, DevParams p) {
  __shared__ int s_cnt[W][S];
  const int* bp = hp.band_prefix;
  // bands dealt to the XCDs in contiguous runs (the grid is a multiple of 8):
  // a band's halo rows are its neighbours' rows, read through the same L2
  const int per_xcd = gridDim.x / kXcds;
  const int item = (blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds;
  if (item >= bp[n]) return;   // a grid sized for larger images than the table's
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
  const char* L[S + 3];
#pragma unroll
  for (int j = 0; j < S + 3; ++j) L[j] = reinterpret_cast<const char*>(level_ptr(ws, e, ov, j));
  unsigned long long* masks = reinterpret_cast<unsigned long long*>(ws + e.region + ov.masks);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const float thr = p.pre_thr;

  int cnt[S];
#pragma unroll
  for (int i = 0; i < S; ++i) cnt[i] = 0;
  if (H16MODE && ov.es == 2)
    detect_band<S, true, W>(L, masks, hk, wk, pk, nseg, b, r_begin, r_end, thr, cnt,
                            SIFT_SPAN_VALUE(region_span(ws, e, lc)));
  else
    detect_band<S, false, W>(L, masks, hk, wk, pk, nseg, b, r_begin, r_end, thr, cnt,
                             SIFT_SPAN_VALUE(region_span(ws, e, lc)));
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < S; ++i) s_cnt[wave][i] = cnt[i];
  }
  __syncthreads();
  if (threadIdx.x < S) {
    const int i = threadIdx.x;
    int tot = 0;
#pragma unroll
    for (int wv = 0; wv < W; ++wv) tot += s_cnt[wv][i];
    int* bc = reinterpret_cast<int*>(ws + e.region + region_tail(e.h, e.w, lc).band_cnt);
    SIFT_CHECK_IN(region_span(ws, e, lc), &bc[ov.band_base * S + i * ov.nband + band], 4);
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
  if (item >= bp[n]) return;
  const int img = find_owner(bp, n, item);
  const int lb = item - bp[img];
  const ImgEntry e = hp.table[img];
  const LayoutCfg lc = layout_cfg(p);
  int k, band;
  band_owner(e.h, e.w, lc, lb, &k, &band);
  const OctView ov = octave_view(e.h, e.w, lc, k);
  const RegionTail rt = region_tail(e.h, e.w, lc);
  SIFT_SPAN(rspan, region_span(ws, e, lc));
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
        if (idx < p.max_cand) {
          SIFT_CHECK_IN(rspan, &cands[idx], 16);
          cands[idx] = make_int4(k, i, r, b + sg * kSeg + bit - 1);
        }
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
    SIFT_SPAN(rspan, region_span(ws, e, lc));
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
        const bool h16 = ov.es == 2;
#pragma unroll
        for (int dr = 0; dr < 3; ++dr)
#pragma unroll
          for (int dc = 0; dc < 3; ++dc) {
            const int64_t off = (int64_t)(r - 1 + dr) * pk + (c - 1 + dc);
            SIFT_CHECK_IN(rspan, reinterpret_cast<const char*>(La) + off * (h16 ? 2 : 4), h16 ? 2 : 4);
            SIFT_CHECK_IN(rspan, reinterpret_cast<const char*>(Lb) + off * (h16 ? 2 : 4), h16 ? 2 : 4);
            d[a][dr][dc] = (double)(lv_at(Lb, off, h16) - lv_at(La, off, h16));
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
// an address, so each column is a sequential sum), a sample's weight split
// linearly between the two nearest bins.  Gradient orientations come from
// a polynomial arctangent (error 1.4e-7 rad), weights from the hardware
// exponential.  Bins are then summed over lanes in a fixed order, smoothed
// once with [1/4, 1/2, 1/4], and every strict local maximum >= peak_ratio *
// max gives an orientation refined by a parabola through the bin and its two
// neighbours.

// H16MODE: fp16 level storage is on; each keypoint's octave picks the path.
// Batches of at most this many images keep their candidate (orientation) and
// keypoint (descriptor) prefix tables in LDS.
constexpr int kOriLdsPrefix = 1024;
constexpr int kDescLdsPrefix = 319;

// The next work item of a wave from a counter in the workspace header: one
// integer atomic per item, taken by whichever wave asks first.  Each item's
// results go to slots fixed by its index, so they do not depend on which
// wave computed them; waves whose items cost less take more of them.  Used
// where items are long and uneven (descriptors: the window grows with the
// keypoint's scale); for short items (orientation, with many rejected
// candidates) the atomics on one address cost more than the balance gains.
__device__ __forceinline__ int next_item(int* counter) {
  int v = 0;
  if ((threadIdx.x & 63) == 0) v = atomicAdd(counter, 1);
  return __shfl(v, 0, 64);
}

template <bool H16MODE>
__global__ __launch_bounds__(256) void k_orient(char* ws, HdrPtrs hp, int n, DevParams p) {
  // OC histogram columns per wave: lanes l, l + OC, ... share column l % OC
  // and add in turn (each group with instructions of its own)
  constexpr int OC = 16, OG = 64 / OC;
  __shared__ float s_hist[4][kOriBins * OC];
  __shared__ float s_bins[4][kOriBins];
  // the candidate prefix over the images, in LDS when it fits: each
  // candidate's image is then found without global-memory round trips
  __shared__ int s_cp[kOriLdsPrefix + 1];
  const int* cp = hp.cand_prefix;
  const bool cp_lds = n <= kOriLdsPrefix;
  if (cp_lds) {
    for (int i = threadIdx.x; i <= n; i += blockDim.x) s_cp[i] = cp[i];
    __syncthreads();
  }
  const int total = cp[n];
  const ImgEntry* tab = hp.table;
  const LayoutCfg lc = layout_cfg(p);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float* hist = s_hist[wave];
  float* bins = s_bins[wave];
  const int nwaves = gridDim.x * 4;
  for (int g = blockIdx.x * 4 + wave; g < total; g += nwaves) {
    const int img = cp_lds ? find_owner(s_cp, n, g) : find_owner(cp, n, g);
    const int j = g - (cp_lds ? s_cp[img] : cp[img]);
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
    SIFT_SPAN(rspan, region_span(ws, e, lc));
    const float sw = p.ori_sigma_factor * kp.sigma_oct;
    const int R = (int)floorf(p.ori_radius_factor * sw + 0.5f);
    const float inv2 = 1.0f / (2.0f * sw * sw);
    const int side = 2 * R + 1;
    const int nsamp = side * side;
    for (int bn = lane; bn < kOriBins * OC; bn += 64) hist[bn] = 0.0f;
    wave_lds_sync();
    // U samples per lane per pass: their loads are all issued before any is
    // used; the pass count is the same for every lane of the wave
    constexpr int U = 4;
    for (int q0 = 0; q0 < nsamp; q0 += 64 * U) {
      float ga[U], gb[U], gc[U], gd[U];
      int ddx[U], ddy[U];
      bool ok[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int q = q0 + 64 * u + lane;
        const int qy = q / side;
        const int dy = qy - R, dx = q - qy * side - R;
        const int rr = kp.r + dy, cc = kp.c + dx;
        ok[u] = q < nsamp && rr >= 1 && rr <= hk - 2 && cc >= 1 && cc <= wk - 2;
        ddx[u] = dx;
        ddy[u] = dy;
        // samples that do not contribute read the (interior) centre instead
        const int64_t at = (int64_t)(ok[u] ? rr : kp.r) * pk + (ok[u] ? cc : kp.c);
        SIFT_CHECK_IN(rspan, reinterpret_cast<const char*>(L) + (at - pk) * ov.es, ov.es);
        SIFT_CHECK_IN(rspan, reinterpret_cast<const char*>(L) + (at + pk) * ov.es, ov.es);
        if (H16MODE && ov.es == 2) {
          ga[u] = lv_at<true>(L, at + 1);
          gb[u] = lv_at<true>(L, at - 1);
          gc[u] = lv_at<true>(L, at + pk);
          gd[u] = lv_at<true>(L, at - pk);
        } else {
          const float* row = L + at;
          ga[u] = row[1];
          gb[u] = row[-1];
          gc[u] = row[pk];
          gd[u] = row[-pk];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const float gx = ga[u] - gb[u];
        const float gy = gc[u] - gd[u];
        const float mag = __builtin_amdgcn_sqrtf(gx * gx + gy * gy);
        float th = atan2_poly(gy, gx);
        if (th < 0.0f) th += kTwoPi;
        const float wgt = exp_fast(-(float)(ddx[u] * ddx[u] + ddy[u] * ddy[u]) * inv2) * mag;
        const float pos = th * ((float)kOriBins / kTwoPi);
        const float fl = floorf(pos);
        const float f = pos - fl;
        int b0 = (int)fl;
        if (b0 >= kOriBins) b0 -= kOriBins;
        int b1 = b0 + 1;
        if (b1 >= kOriBins) b1 -= kOriBins;
        const float w0 = wgt * (1.0f - f), w1 = wgt * f;
        // the two bins differ: read both, then write both
        float* c0 = &hist[b0 * OC + (lane & (OC - 1))];
        float* c1 = &hist[b1 * OC + (lane & (OC - 1))];
        SIFT_CHECK_INDEX(b0 * OC + (lane & (OC - 1)), kOriBins * OC);
        SIFT_CHECK_INDEX(b1 * OC + (lane & (OC - 1)), kOriBins * OC);
#pragma unroll
        for (int grp = 0; grp < OG; ++grp) {
          if (ok[u] && lane / OC == grp) {
            const float h0 = *c0, h1 = *c1;
            *c0 = h0 + w0;
            *c1 = h1 + w1;
          }
          // keeps the groups' updates in separate instructions, in order
          __builtin_amdgcn_wave_barrier();
        }
      }
    }
    wave_lds_sync();
    if (lane < kOriBins) {
      float acc = 0.0f;
      for (int t = 0; t < OC; ++t) acc += hist[lane * OC + ((lane + t) & (OC - 1))];
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
  int* kp_src = reinterpret_cast<int*>(ws + e.region + rt.kp_src);
  static_assert(kMaxPeaks <= 32, "peak index in five bits");
  int base = 0;
  for (int c0 = 0; c0 < nc; c0 += 256) {
    const int idx = c0 + threadIdx.x;
    const int v = idx < nc ? n_ori[idx] : 0;
    int tot;
    const int ex = block_excl_scan256(v, s_wave, &tot);
    if (idx < nc) kp_off[idx] = base + ex;
    // the inverse: which candidate and peak each keypoint slot describes
    for (int r = 0; r < v && base + ex + r < p.max_kp; ++r) {
      SIFT_CHECK_INDEX(base + ex + r, p.max_kp);
      kp_src[base + ex + r] = idx * 32 + r;
    }
    base += tot;
  }
  if (threadIdx.x == 0) {
    cnt[kCntKp] = base;
    if (e.n_found) *e.n_found = base;
    *e.count = min(min(base, p.max_kp), e.cap);
  }
}

// ---------------------------------------------------------------------------
// Descriptor: one wave per output keypoint.  The bounding square of the
// rotated 4x4 grid of the largest pooled domain size is scanned 64 samples at
// a time; the samples whose rotated cell coordinates fall in (-1, 4) (about
// 60% of the square) are packed, with their pixel gradients, into full
// 64-lane batches by a lane permutation in registers, so the trilinear
// binning runs with every lane busy; each packed pixel is binned for every
// domain size whose window holds it.  Each lane accumulates into its own LDS column of the
// 128-bin histogram.  Scan, packing and column order are fixed, so the sums
// are too.  The lane columns are summed in a fixed order, averaged over domain
// sizes, then L2-normalised, clamped, L2-normalised and optionally turned into
// RootSIFT (L1 normalise, square root).

// ND: the number of domain sizes the code is unrolled for (1, or the most).
// The launch bound asks for 16 resident groups per CU (128 registers per
// lane): the one-size build fits; the pooled-size build takes about 180
// registers and 8 groups are resident per CU.
// H16MODE: fp16 level storage is on; each keypoint's octave picks the path.
template <int ND, bool H16MODE>
__global__ __launch_bounds__(64, 16) void k_describe(char* ws, HdrPtrs hp, int n, DevParams p) {
  // DC histogram columns: lanes l, l + DC, ... share column l % DC and add
  // in turn.  Four lanes per column with one domain size; with several, two
  // (their unrolled size loop needs the registers a third resident wave would)
  constexpr int DC = ND == 1 ? 16 : 32, NG = 64 / DC;
  __shared__ float hist[kDescDim * DC];
  // the keypoint prefix over the images, in LDS when it fits (kept small:
  // the LDS of 16 resident waves per CU is nearly all histograms)
  __shared__ int s_kpp[kDescLdsPrefix + 1];
  const int* kpp = hp.kp_prefix;
  const bool kpp_lds = n <= kDescLdsPrefix;
  if (kpp_lds) {
    for (int i = threadIdx.x; i <= n; i += 64) s_kpp[i] = kpp[i];
    wave_lds_sync();
  }
  const int total = kpp[n];
  const ImgEntry* tab = hp.table;
  const LayoutCfg lc = layout_cfg(p);
  const int lane = threadIdx.x;
  int* const queue = hp.queue;
  int g_next = next_item(queue);
  for (int g = g_next; g < total; g = g_next) {
    g_next = next_item(queue);   // the wave's next keypoint, fetched while this one runs
    const int img = kpp_lds ? find_owner(s_kpp, n, g) : find_owner(kpp, n, g);
    const int q = g - (kpp_lds ? s_kpp[img] : kpp[img]);
    const ImgEntry e = tab[img];
    const RegionTail rt = region_tail(e.h, e.w, lc);
    const int* cnt = counters_of(ws, e);
    // the candidate and peak this keypoint slot describes (written by the
    // orientation scan)
    SIFT_CHECK_INDEX(q, p.max_kp);
    const int src = reinterpret_cast<const int*>(ws + e.region + rt.kp_src)[q];
    const int j = src >> 5;
    const int pk_idx = src & 31;
    const RefinedKp kp = reinterpret_cast<const RefinedKp*>(ws + e.region + rt.refined)[j];
    const int4 cd = reinterpret_cast<const int4*>(ws + e.region + rt.cands)[j];
    const float angle =
        reinterpret_cast<const float*>(ws + e.region + rt.angles)[(int64_t)j * kMaxPeaks + pk_idx];
    const int k = kp.k;
    const OctView ov = octave_view(e.h, e.w, lc, k);
    const int hk = ov.h, wk = ov.w, pk = ov.pitch;
    const float* L = level_ptr(ws, e, ov, kp.layer);
    SIFT_SPAN(rspan, region_span(ws, e, lc));
    const gchar* gL = uniform_ptr(reinterpret_cast<const gchar*>(as_global(L)));
    const uint32_t pkb = (uint32_t)pk * 4u;
    const float th = angle * (kTwoPi / 360.0f);
    const float st = sinf(th), ct = cosf(th);

#pragma unroll
    for (int bn = lane; bn < kDescDim * DC; bn += 64) hist[bn] = 0.0f;
    wave_lds_sync();

    // Domain sizes: a pixel inside the window of one size is inside the
    // window of every larger one (the cell test is monotone in 1 / cell, in
    // fp32 too), so one scan of the largest window finds every contributing
    // pixel; its gradient, magnitude and orientation bin are computed once
    // and its contribution is then added for each size whose window holds it.
    // the sizes come sorted, largest first
    const float smax = p.dsp[0];
    const float wc_max = p.desc_magnif * kp.sigma_oct * smax;
    const float inv_max = 1.0f / wc_max;
    // A sample contributes only if its rotated cell coordinates fall in
    // (-1, 4), i.e. |u|, |v| < 2.5 wc (|cos| + |sin|) around the sub-pixel
    // centre; one extra ring covers the sub-pixel offset and fp32 rounding.
    const int R = (int)ceilf(2.5f * wc_max * (fabsf(ct) + fabsf(st))) + 1;
    const int side = 2 * R + 1;
    const int nsamp = side * side;
    const float inv_side = 1.0f / (float)side;
    // 1 / cell size of every domain size, and the factor that turns a
    // squared pixel distance into the base-2 exponent of the grid's Gaussian
    // weight exp(-(xr^2 + yr^2) / 8) for that size (unused entries 0)
    float inv_ws[ND], gk_ws[ND];
#pragma unroll
    for (int ds = 0; ds < ND; ++ds) {
      inv_ws[ds] = ds < p.n_dsp ? 1.0f / (p.desc_magnif * kp.sigma_oct * p.dsp[ds]) : 0.0f;
      gk_ws[ds] = inv_ws[ds] * inv_ws[ds] * (-0.125f * 1.44269504088896341f);
    }

    // rotated offset (dx, dy) from the sub-pixel centre, in pixels
    auto rotate = [&](int dx, int dy, float& xr0, float& yr0) {
      const float fu = (float)dx - kp.dx;
      const float fv = (float)dy - kp.dy;
      xr0 = ct * fu + st * fv;
      yr0 = ct * fv - st * fu;
    };
    // rotated cell coordinates (xr, yr) relative to the grid centre: inside
    // (-1, 4) after the shift by 1.5, i.e. both below 2.5 in magnitude
    auto in_window = [](float xr, float yr) { return fmaxf(fabsf(xr), fabsf(yr)) < 2.5f; };
    // trilinear binning of one contributing pixel into this lane's column,
    // once per domain size whose window holds it; every lane of the wave
    // takes part (lanes with valid == false add nothing)
    auto accumulate = [&](int pxy, float gx, float gy, bool valid) {
      const int dx = (int)(short)(pxy & 0xffff), dy = pxy >> 16;
      float xr0, yr0;
      rotate(dx, dy, xr0, yr0);
      const float r2 = xr0 * xr0 + yr0 * yr0;
      const float mag = __builtin_amdgcn_sqrtf(gx * gx + gy * gy);
      float ta = atan2_poly(gy, gx);
      if (ta < 0.0f) ta += kTwoPi;
      float ob = ta - th;
      if (ob < 0.0f) ob += kTwoPi;
      if (ob >= kTwoPi) ob -= kTwoPi;
      ob = ob * (8.0f / kTwoPi);
      const float o0 = floorf(ob);
      const float fo = ob - o0;
      int io = (int)o0;
      if (io >= 8) io -= 8;
      const int io1 = (io + 1) & 7;
      const int col = lane & (DC - 1);
#pragma unroll
      for (int ds = 0; ds < ND; ++ds) {
        if (ds >= p.n_dsp) break;
        const float xr = xr0 * inv_ws[ds], yr = yr0 * inv_ws[ds];
        // with one size the scan's window test was this very test
        const bool add = valid && (ND == 1 || in_window(xr, yr));
        // sizes run largest first, and a pixel outside one size's window is
        // outside every smaller one's: once no lane adds, none will again
        if (ND > 1 && __ballot(add) == 0ull) break;
        const float wgt = mag * __builtin_amdgcn_exp2f(r2 * gk_ws[ds]);
        // The sample updates the 2 x 2 grid cells from (floor(rb), floor(cb))
        // clamped to 0..2, so the eight targets are always on the grid and
        // distinct.  A cell at distance d (in cells) from the sample along an
        // axis gets weight max(0, 1 - |d|): the bilinear weight for the two
        // cells the sample reaches, +0 for a block row or column it does not
        // reach (adding +0 to a non-negative sum leaves it unchanged).
        const float rb = yr + 1.5f, cb = xr + 1.5f;
        const float r0 = __builtin_amdgcn_fmed3f(floorf(rb), 0.0f, 2.0f);
        const float c0 = __builtin_amdgcn_fmed3f(floorf(cb), 0.0f, 2.0f);
        const float dr = rb - r0, dc = cb - c0;
        const float wr[2] = {fmaxf(1.0f - fabsf(dr), 0.0f), fmaxf(1.0f - fabsf(dr - 1.0f), 0.0f)};
        const float wc[2] = {fmaxf(1.0f - fabsf(dc), 0.0f), fmaxf(1.0f - fabsf(dc - 1.0f), 0.0f)};
        const float wo[2] = {wgt * (1.0f - fo), wgt * fo};
        // a lane that adds nothing keeps its (unused) addresses on the grid
        const int cell = add ? (int)(r0 * 4.0f + c0) : 0;
        float* h0 = &hist[(cell * 8 + io) * DC + col];
        float* h1 = &hist[(cell * 8 + io1) * DC + col];
        // the eight targets: cells cell .. cell + 5 (rows +0/+1, columns +0/+1)
        SIFT_CHECK_INDEX((cell * 8 + io) * DC + col, kDescDim * DC);
        SIFT_CHECK_INDEX(((cell + 5) * 8 + io1) * DC + col, kDescDim * DC);
        float wv[8];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const float ra0 = wr[a] * wo[0], ra1 = wr[a] * wo[1];
#pragma unroll
          for (int bb = 0; bb < 2; ++bb) {
            wv[4 * a + 2 * bb] = ra0 * wc[bb];
            wv[4 * a + 2 * bb + 1] = ra1 * wc[bb];
          }
        }
        // the lane groups sharing a column update it in turn, each with its
        // own instructions: read the eight targets, then write them
#pragma unroll
        for (int grp = 0; grp < NG; ++grp) {
          if (add && lane / DC == grp) {
            float hv[8];
#pragma unroll
            for (int a = 0; a < 2; ++a) {
#pragma unroll
              for (int bb = 0; bb < 2; ++bb) {
                const int off = (a * 4 + bb) * 8 * DC;   // cell step: 8 bins of DC columns
                hv[4 * a + 2 * bb] = h0[off];
                hv[4 * a + 2 * bb + 1] = h1[off];
              }
            }
#pragma unroll
            for (int a = 0; a < 2; ++a) {
#pragma unroll
              for (int bb = 0; bb < 2; ++bb) {
                const int off = (a * 4 + bb) * 8 * DC;
                h0[off] = hv[4 * a + 2 * bb] + wv[4 * a + 2 * bb];
                h1[off] = hv[4 * a + 2 * bb + 1] + wv[4 * a + 2 * bb + 1];
              }
            }
          }
          // keeps the groups' updates in separate instructions, in order
          __builtin_amdgcn_wave_barrier();
        }
      }
    };

    // Pending contributing pixels sit in lanes [0, fill): packed offset
    // (dy << 16 | dx & 0xffff) and gradient.
    int fill = 0;
    int p_xy = 0;
    float p_gx = 0.0f, p_gy = 0.0f;
    constexpr int U = 4;   // scan batches whose loads are issued together
    for (int q0 = 0; q0 < nsamp; q0 += 64 * U) {
      float ga[U], gb[U], gc[U], gd[U];
      int sxy[U];
      bool ok[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int qq = q0 + 64 * u + lane;
        // qq / side: an fp32 estimate within one of the quotient, then one
        // correction step on the remainder makes it exact
        int qy = (int)(((float)qq + 0.5f) * inv_side);
        int qx = qq - qy * side;
        if (qx < 0) {
          --qy;
          qx += side;
        } else if (qx >= side) {
          ++qy;
          qx -= side;
        }
        const int dy = qy - R, dx = qx - R;
        const int rr = kp.r + dy, cc = kp.c + dx;
        float xr0, yr0;
        rotate(dx, dy, xr0, yr0);
        ok[u] = qq < nsamp && rr >= 1 && rr <= hk - 2 && cc >= 1 && cc <= wk - 2 &&
                in_window(xr0 * inv_max, yr0 * inv_max);
        sxy[u] = (dy << 16) | (dx & 0xffff);
        // samples that do not contribute read the (interior) centre instead
        const uint32_t idx = (uint32_t)((ok[u] ? rr : kp.r) * pk + (ok[u] ? cc : kp.c));
        SIFT_CHECK_IN(rspan, gL + (uint64_t)idx * ov.es - (uint64_t)pk * ov.es, ov.es);
        SIFT_CHECK_IN(rspan, gL + (uint64_t)idx * ov.es + (uint64_t)pk * ov.es, ov.es);
        if (H16MODE && ov.es == 2) {
          const uint32_t at = idx * 2u, pkh = (uint32_t)pk * 2u;
          ga[u] = load_lv<true>(gL, at + 2u);
          gb[u] = load_lv<true>(gL, at - 2u);
          gc[u] = load_lv<true>(gL, at + pkh);
          gd[u] = load_lv<true>(gL, at - pkh);
        } else {
          const uint32_t at = idx * 4u;
          ga[u] = load_at(gL, at + 4u);
          gb[u] = load_at(gL, at - 4u);
          gc[u] = load_at(gL, at + pkb);
          gd[u] = load_at(gL, at - pkb);
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint64_t m = __ballot(ok[u]);
        const int cnt = __popcll(m);
        const int rank = __popcll(m & lanemask_lt());
        // contributing lanes go to [fill, fill + cnt), the others after them
        const int dest = (ok[u] ? fill + rank : fill + cnt + (lane - rank)) & 63;
        const int r_xy = lane_send(dest, sxy[u]);
        const float r_gx = lane_send(dest, ga[u] - gb[u]);
        const float r_gy = lane_send(dest, gc[u] - gd[u]);
        const int nf = fill + cnt;
        if (nf >= 64) {
          // lanes [fill, 64) complete the batch; lanes [0, nf - 64) overflow
          const bool fresh = lane >= fill;
          accumulate(fresh ? r_xy : p_xy, fresh ? r_gx : p_gx, fresh ? r_gy : p_gy, true);
          p_xy = r_xy;
          p_gx = r_gx;
          p_gy = r_gy;
          fill = nf - 64;
        } else {
          const bool take = lane >= fill && lane < nf;
          p_xy = take ? r_xy : p_xy;
          p_gx = take ? r_gx : p_gx;
          p_gy = take ? r_gy : p_gy;
          fill = nf;
        }
      }
    }
    accumulate(p_xy, p_gx, p_gy, lane < fill);
    wave_lds_sync();
    float h0 = 0.0f, h1 = 0.0f;
    for (int t = 0; t < DC; ++t) {
      const int col = (lane + t) & (DC - 1);
      h0 += hist[lane * DC + col];
      h1 += hist[(lane + 64) * DC + col];
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
    SIFT_CHECK_INDEX(slot, e.cap);
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
// Launch helpers

hipError_t launch_setup(const HdrPtrs& hp, const SetupChunk& c, hipStream_t stream) {
  return launch(k_setup, dim3(1), dim3(64), stream, hp, c);
}

hipError_t launch_finalize(const HdrPtrs& hp, int n, const DevParams& p, hipStream_t stream) {
  return launch(k_finalize, dim3(1), dim3(64), stream, hp, n, p);
}

hipError_t launch_detect(char* ws, const HdrPtrs& hp, int n, const DevParams& p, int waves,
                         int grid, hipStream_t stream) {
  grid = (grid + kXcds - 1) / kXcds * kXcds;
#define SIFT_DETECT_CASE(SS, WW)                                                          \
  if (p.s == SS && waves == WW)                                                           \
    return p.h16 ? launch(k_detect<SS, true, WW>, dim3(grid), dim3(WW * 64), stream, ws, hp, \
                          n, p)                                                           \
                 : launch(k_detect<SS, false, WW>, dim3(grid), dim3(WW * 64), stream, ws, hp, \
                          n, p);
#define SIFT_DETECT_WAVES(SS) SIFT_DETECT_CASE(SS, 4) SIFT_DETECT_CASE(SS, 8)
  SIFT_DETECT_WAVES(1) SIFT_DETECT_WAVES(2) SIFT_DETECT_WAVES(3)
  SIFT_DETECT_WAVES(4) SIFT_DETECT_WAVES(5) SIFT_DETECT_WAVES(6)
#undef SIFT_DETECT_WAVES
#undef SIFT_DETECT_CASE
  return hipErrorInvalidValue;
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
  return p.h16 ? launch(k_orient<true>, dim3(grid), dim3(256), stream, ws, hp, n, p)
               : launch(k_orient<false>, dim3(grid), dim3(256), stream, ws, hp, n, p);
}

hipError_t launch_ori_scan(char* ws, const HdrPtrs& hp, int n, const DevParams& p,
                         hipStream_t stream) {
  return launch(k_ori_scan, dim3(n), dim3(256), stream, ws, hp, n, p);
}

hipError_t launch_describe(char* ws, const HdrPtrs& hp, int n, const DevParams& p, int grid,
                         hipStream_t stream) {
  // the smallest unrolled size count that covers n_dsp (5: the paper's
  // pooling set, 10: the linearly spaced set of its benchmark)
#define SIFT_DESCRIBE(NDD)                                                         \
  return p.h16 ? launch(k_describe<NDD, true>, dim3(grid), dim3(64), stream, ws, hp, n, p) \
               : launch(k_describe<NDD, false>, dim3(grid), dim3(64), stream, ws, hp, n, p)
  if (p.n_dsp == 1) SIFT_DESCRIBE(1);
  if (p.n_dsp <= 5) SIFT_DESCRIBE(5);
  if (p.n_dsp <= 10) SIFT_DESCRIBE(10);
  SIFT_DESCRIBE(kMaxDsp);
#undef SIFT_DESCRIBE
}

// The bounds-check counter of this file's kernels (see check_in).
hipError_t bounds_count_kernels(unsigned long long* count, bool reset) {
#ifdef SIFT_DEBUG_BOUNDS
  hipError_t e = hipMemcpyFromSymbol(count, HIP_SYMBOL(g_bounds_violations), sizeof *count, 0,
                                     hipMemcpyDeviceToHost);
  if (e == hipSuccess && reset) {
    const unsigned long long zero = 0;
    e = hipMemcpyToSymbol(HIP_SYMBOL(g_bounds_violations), &zero, sizeof zero, 0,
                          hipMemcpyHostToDevice);
  }
  return e;
#else
  (void)reset;
  *count = 0;
  return hipErrorNotSupported;
#endif
}

}  // namespace sift
