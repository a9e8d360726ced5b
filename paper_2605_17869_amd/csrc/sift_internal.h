// Internal definitions shared by the host runtime and the gfx950 kernels:
// octave geometry, workspace layout, the on-device image table and the
// kernel argument blocks.  Host and device compute geometry with the same
// inline functions, so launch sizes on the host and work-item decoding on the
// device always agree.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "../../include/sift.h"

#if defined(__HIPCC__)
#define SIFT_HD __host__ __device__ __forceinline__
#else
#define SIFT_HD inline
#endif

namespace sift {

constexpr int kMaxOct = 12;        // octaves including octave -1
constexpr int kMaxScales = 6;      // n_scales supported by the detector
constexpr int kMaxRadius = 24;     // largest Gaussian radius ceil(4 sigma)
constexpr int kMaxDsp = SIFT_MAX_DSP;  // pooled domain sizes
constexpr int kTileW = 192;        // blur strip width (output columns of one work-group)
constexpr int kBlurThreads = 256;  // blur work-group size (one source column per thread)
constexpr int kBlurRows = 16;      // rows a blur work-group advances per step
constexpr int kNumTileH = 5;       // blur chunk heights 32, 64, 128, 256, 512
constexpr int kXcds = 8;           // work-groups are dealt round-robin to the XCDs
constexpr int kMaxParts = 8;       // sub-batches (each with its own header) of one batched call
constexpr int kBand = 8;           // rows per detection band
constexpr int kDetectWaves = 4;    // waves of a detection work-group
constexpr int kQueues = 1;         // work counters: descriptor
constexpr int kSeg = 62;           // output columns per 64-lane detection segment
constexpr int kOriBins = 36;
constexpr int kMaxPeaks = kOriBins / 2;   // strict circular maxima of 36 bins
constexpr int kDescDim = 128;
constexpr int kSetupChunk = 24;    // image-table entries per setup launch
constexpr float kCentre = 0.5f;    // pyramid levels are stored as L - kCentre

SIFT_HD int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }
SIFT_HD int cdiv(int a, int b) { return (a + b - 1) / b; }

// Size of octave k (k = 0 is the first octave: -1 when upsampling, else 0).
SIFT_HD void octave_dims(int h, int w, int upsample, int k, int* oh, int* ow) {
  int hh = upsample ? 2 * h : h;
  int ww = upsample ? 2 * w : w;
  for (int j = 0; j < k; ++j) {
    hh = (hh + 1) / 2;
    ww = (ww + 1) / 2;
  }
  *oh = hh;
  *ow = ww;
}

SIFT_HD int level_pitch(int w) { return (int)align_up(w, 64); }

// Geometry settings that fix an image's workspace region.
struct LayoutCfg {
  int n_oct;      // total octaves
  int upsample;
  int s;          // n_scales
  int border;
  int max_cand;
  int max_kp;
  int h16;        // 1: octaves after the first hold fp16 levels
};

// Bytes per stored level element of octave k.
SIFT_HD int level_es(const LayoutCfg& c, int k) { return (c.h16 && k >= 1) ? 2 : 4; }

SIFT_HD int bands_of(int hk, int border) {
  int rows = hk - 2 * border;
  return rows > 0 ? cdiv(rows, kBand) : 0;
}

SIFT_HD int segs_of(int wk, int border) {
  int cols = wk - 2 * border;
  return cols > 0 ? cdiv(cols, kSeg) : 0;
}

// One octave of an image's workspace region (byte offsets from the region
// start).  The region holds, in order: 256 bytes of counters; the s+3
// Gaussian level planes of every octave; the detection mask words of every
// octave; then the per-image tail (band counts/offsets, candidate slots,
// refined records, orientations, keypoint offsets).
struct OctView {
  int h, w, pitch;         // size and row pitch (elements) of the octave
  int es;                  // bytes per level element: 4 (fp32) or 2 (fp16)
  int nseg, nband;         // detection segments per row, bands of kBand rows
  int band_base;           // first band of this octave within the image
  int64_t level0;          // Gaussian level 0; level j at level0 + j * plane
  int64_t plane;           // bytes per level plane
  int64_t masks;           // uint64 [s][h][nseg] detection masks
};

struct RegionTail {
  int total_bands;         // bands over all octaves
  int64_t band_cnt;        // int32 [total_bands * s], canonical (octave, layer, band)
  int64_t band_off;        // int32 exclusive offsets, same indexing
  int64_t cands;           // int4 {octave slot, layer, row, col} [max_cand]
  int64_t refined;         // RefinedKp [max_cand]
  int64_t n_ori;           // int32 [max_cand]
  int64_t angles;          // float [max_cand][kMaxPeaks]
  int64_t kp_off;          // int32 [max_cand]
  int64_t kp_src;          // int32 [max_kp]: candidate * 32 + peak of each keypoint slot
  int64_t bytes;           // region size
};

// Walk the octaves with scalar accumulators (no arrays: on the GPU every
// value stays wave-uniform).  Fills *v for octave `want` (if v) and *t (if t).
SIFT_HD void region_walk(int h, int w, const LayoutCfg& c, int want, OctView* v, RegionTail* t) {
  int64_t off = 256;
  int bb = 0;
  for (int k = 0; k < c.n_oct; ++k) {
    int hk, wk;
    octave_dims(h, w, c.upsample, k, &hk, &wk);
    const int pitch = level_pitch(wk);
    const int es = level_es(c, k);
    const int64_t plane = align_up((int64_t)pitch * hk * es, 256);
    const int nb = bands_of(hk, c.border);
    if (v && k == want) {
      v->h = hk;
      v->w = wk;
      v->pitch = pitch;
      v->es = es;
      v->plane = plane;
      v->level0 = off;
      v->nseg = segs_of(wk, c.border);
      v->nband = nb;
      v->band_base = bb;
    }
    off += plane * (c.s + 3);
    bb += nb;
  }
  for (int k = 0; k < c.n_oct; ++k) {
    int hk, wk;
    octave_dims(h, w, c.upsample, k, &hk, &wk);
    if (v && k == want) v->masks = off;
    off = align_up(off + (int64_t)c.s * hk * segs_of(wk, c.border) * 8, 256);
  }
  if (!t) return;
  t->total_bands = bb;
  t->band_cnt = off;
  off = align_up(off + (int64_t)bb * c.s * 4, 256);
  t->band_off = off;
  off = align_up(off + (int64_t)bb * c.s * 4, 256);
  t->cands = off;
  off = align_up(off + (int64_t)c.max_cand * 16, 256);
  t->refined = off;
  off = align_up(off + (int64_t)c.max_cand * 48, 256);
  t->n_ori = off;
  off = align_up(off + (int64_t)c.max_cand * 4, 256);
  t->angles = off;
  off = align_up(off + (int64_t)c.max_cand * kMaxPeaks * 4, 256);
  t->kp_off = off;
  off = align_up(off + (int64_t)c.max_cand * 4, 256);
  t->kp_src = off;
  off = align_up(off + (int64_t)c.max_kp * 4, 256);
  t->bytes = off;
}

SIFT_HD OctView octave_view(int h, int w, const LayoutCfg& c, int k) {
  OctView v;
  region_walk(h, w, c, k, &v, nullptr);
  return v;
}

SIFT_HD RegionTail region_tail(int h, int w, const LayoutCfg& c) {
  RegionTail t;
  region_walk(h, w, c, -1, nullptr, &t);
  return t;
}

// Octave slot and band within it of the image's band number lb.
SIFT_HD void band_owner(int h, int w, const LayoutCfg& c, int lb, int* k_out, int* band_out) {
  int bb = 0;
  int k = 0;
  for (; k < c.n_oct; ++k) {
    int hk, wk;
    octave_dims(h, w, c.upsample, k, &hk, &wk);
    const int nb = bands_of(hk, c.border);
    if (lb < bb + nb) break;
    bb += nb;
  }
  *k_out = k;
  *band_out = lb - bb;
}

// Counter slots inside an image region.
enum Counter { kCntCand = 0, kCntKp = 1 };

// One image of a batch as the kernels see it (written by the setup kernel).
struct ImgEntry {
  const float* src;
  int64_t src_pitch;
  int32_t h, w;
  int64_t region;          // byte offset of the image's region in the workspace
  sift_keypoint* kp;
  float* desc;
  int32_t* count;
  int32_t* n_found;
  int32_t* n_cand;
  int32_t cap;
  int32_t pad;
};

// Workspace header: image table and per-octave tile prefix sums.
SIFT_HD int tile_h_of(int cls) { return 32 << cls; }

struct Header {
  int64_t table;           // ImgEntry[n]
  int64_t tile_prefix;     // int32 [kNumTileH][kMaxOct][n + 1]
  int64_t band_prefix;     // int32 [n + 1]
  int64_t cand_prefix;     // int32 [n + 1]: refined candidates per image
  int64_t kp_prefix;       // int32 [n + 1]: described keypoints per image
  int64_t queue;           // int32 [kQueues]: next work item of the per-keypoint kernels
  int64_t bytes;
};

// Device addresses of the header arrays, computed on the host and passed to
// the kernels as arguments (the kernels never derive them from `ws` with
// alignment arithmetic: the compiler may fold such arithmetic into a scalar
// load's immediate offset and leave a base register that is not dword
// aligned, which the scalar memory unit does not honour).
struct HdrPtrs {
  const ImgEntry* table;   // ImgEntry[n]
  int* tile_prefix;        // int32 [kNumTileH][kMaxOct][n + 1]
  int* band_prefix;        // int32 [n + 1]
  int* cand_prefix;        // int32 [n + 1]
  int* kp_prefix;          // int32 [n + 1]
  int* queue;              // int32 [kQueues]
};

SIFT_HD void make_header(int n, Header* hd) {
  int64_t off = 0;
  hd->table = off;
  off = align_up(off + (int64_t)n * (int64_t)sizeof(ImgEntry), 256);
  hd->tile_prefix = off;
  off = align_up(off + (int64_t)kNumTileH * kMaxOct * (n + 1) * 4, 256);
  hd->band_prefix = off;
  off = align_up(off + (int64_t)(n + 1) * 4, 256);
  hd->cand_prefix = off;
  off = align_up(off + (int64_t)(n + 1) * 4, 256);
  hd->kp_prefix = off;
  off = align_up(off + (int64_t)(n + 1) * 4, 256);
  hd->queue = off;
  off = align_up(off + (int64_t)kQueues * 4, 256);
  hd->bytes = off;
}

// Settings the kernels read (a by-value kernel argument).
struct DevParams {
  int n_oct, o0, s, upsample, border, refine_iters, upright, rootsift;
  int max_kp, max_cand, n_dsp, h16;
  float sigma0, contrast_thr, pre_thr, edge_ratio;
  float ori_sigma_factor, ori_radius_factor, ori_peak_ratio;
  float desc_magnif, desc_clamp;
  float dsp[SIFT_MAX_DSP];
};

SIFT_HD LayoutCfg layout_cfg(const DevParams& p) {
  LayoutCfg c;
  c.n_oct = p.n_oct;
  c.upsample = p.upsample;
  c.s = p.s;
  c.border = p.border;
  c.max_cand = p.max_cand;
  c.max_kp = p.max_kp;
  c.h16 = p.h16;
  return c;
}

// Refined detection (one per candidate slot).
struct RefinedKp {
  float dx, dy;            // sub-pixel offset x^ of the extremum from (c, r)
  float sigma_oct;         // scale in octave pixels
  float response;          // |D(x^)|
  float x, y, sigma;       // input-image coordinates and scale
  int32_t ok;              // 1 accepted, 0 rejected
  int32_t layer, r, c;     // integer position after refinement
  int32_t k;               // octave slot
};

// Blur kernel fetch modes.
enum BlurSrc { kSrcImage = 0, kSrcUpsample = 1, kSrcLevel = 2, kSrcDown = 3 };

struct BlurArgs {
  char* ws;
  const ImgEntry* table;
  const int* tile_prefix;   // tiles of this octave and tile height: n + 1 entries
  int n;
  int k;            // octave slot
  int dst_level;    // level written
  int mode;         // BlurSrc
  int th;           // chunk height (64, 128, 256 or 512 rows)
  int st;           // storage: 0 fp32 -> fp32, 1 fp32 -> fp16, 2 fp16 -> fp16
  DevParams p;
  float taps[2 * kMaxRadius + 1];
};

// Chained levels (k_chain): rows per step, most levels per launch, largest
// radius (2R <= kChainB: a block of outputs needs two blocks of input rows).
constexpr int kChainB = 16;
constexpr int kChainMaxLevels = 4;
constexpr int kChainMaxR = 8;

struct ChainArgs {
  char* ws;
  const ImgEntry* table;
  const int* tile_prefix;   // tiles of this octave and chunk height: n + 1 entries
  int n;
  int k;            // octave slot
  int lv0;          // first level written
  int th;           // chunk height
  DevParams p;
  float g[kChainMaxLevels][kChainMaxR + 1];   // g[i][t]: tap at distance t of level lv0 + i
};

}  // namespace sift
