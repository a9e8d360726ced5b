// Host runtime of the SIFT library: parameter validation, Gaussian taps,
// workspace layout, and the launch sequence of one extraction.  Nothing here
// allocates device memory or synchronises; every extraction is a fixed
// sequence of kernel launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sift.h"
#include "sift_internal.h"
#include "sift_launch.h"

using namespace sift;

namespace {

thread_local std::string g_error;
// Set while this thread records a launch sequence into a graph: no events then.
thread_local bool g_capturing = false;

sift_status fail(sift_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
  return st;
}

constexpr int kMaxSide = 32768;    // per input dimension
constexpr int kMaxWindowSide = 2047;   // orientation / descriptor window side, samples
constexpr int kMaxBatch = 4096;

// Chunk height class of a blur level: the tallest chunk, up to the caller's
// tile_rows when set, that still gives at least kBlurTargetGroups work-groups
// (enough to fill every CU several times over), else the shortest.  Small
// octaves so get short chunks whatever the cap: more work-groups, shorter
// row loops.
constexpr int kBlurTargetGroups = 2048;
// Levels per blur launch when blur_chain is 0.
constexpr int kDefaultChain = 2;

int blur_class(int tile_rows, const int64_t* tiles_of_class) {
  int top = kNumTileH - 1;
  for (int c = 0; c < kNumTileH; ++c)
    if (tile_h_of(c) == tile_rows) top = c;
  for (int c = top; c > 0; --c)
    if (tiles_of_class[c] >= kBlurTargetGroups) return c;
  return 0;
}

// Sampled Gaussian exp(-t^2 / (2 sigma^2)), t = -R..R, R = ceil(4 sigma),
// normalised by its double-precision sum and rounded to float.
struct Taps {
  int radius = 0;
  float g[2 * kMaxRadius + 1] = {};
};

bool make_taps(double sigma, Taps* t) {
  const int r = (int)std::ceil(4.0 * sigma);
  if (r < 1 || r > kMaxRadius) return false;
  double w[2 * kMaxRadius + 1];
  double sum = 0.0;
  for (int i = -r; i <= r; ++i) {
    w[i + r] = std::exp(-(double)(i * i) / (2.0 * sigma * sigma));
    sum += w[i + r];
  }
  t->radius = r;
  for (int i = 0; i < 2 * r + 1; ++i) t->g[i] = (float)(w[i] / sum);
  return true;
}

}  // namespace

namespace sift {
// Sets the text sift_last_error() returns on this thread (used by the server).
void set_last_error(const std::string& msg) { g_error = msg; }
// Marks this thread as recording a graph (stage profiling skips it).
void set_capturing(bool on) { g_capturing = on; }
}  // namespace sift

// Device settings and Gaussian taps of one octave structure.
struct Config {
  DevParams dev;
  Taps init;                       // first level of the first octave
  Taps inc[kMaxScales + 2];        // level i from level i-1, i = 1..s+2
};

struct sift_handle {
  sift_params params;
  // cfg[0]: the settings as given; cfg[1]: the same without the upsampled
  // octave, for images above upsample_max_pixels (the VRAM-adaptive policy)
  Config cfg[2];
  hipStream_t part_stream[kMaxParts] = {};   // created by the first split batch
  std::once_flag streams_once;
  hipError_t streams_status = hipSuccess;
};

namespace {

sift_status validate_params(const sift_params& p) {
  if (p.n_octaves < 1) return fail(SIFT_ERR_INVALID_ARG, "n_octaves must be >= 1");
  if (p.upsample != 0 && p.upsample != 1) return fail(SIFT_ERR_INVALID_ARG, "upsample must be 0 or 1");
  if (p.n_octaves + p.upsample > kMaxOct)
    return fail(SIFT_ERR_NOT_SUPPORTED, "at most %d octaves", kMaxOct);
  if (p.n_scales < 1 || p.n_scales > kMaxScales)
    return fail(SIFT_ERR_NOT_SUPPORTED, "n_scales must be in 1..%d", kMaxScales);
  if (!(p.sigma0 > 0.0f) || !(p.sigma_in >= 0.0f))
    return fail(SIFT_ERR_INVALID_ARG, "sigma0 must be > 0 and sigma_in >= 0");
  if (!(p.contrast_threshold > 0.0f) || !(p.prefilter_ratio >= 0.0f) || !(p.edge_ratio > 0.0f))
    return fail(SIFT_ERR_INVALID_ARG, "thresholds must be positive");
  if (p.border < 1) return fail(SIFT_ERR_INVALID_ARG, "border must be >= 1");
  if (p.refine_iters < 1 || p.refine_iters > 64)
    return fail(SIFT_ERR_INVALID_ARG, "refine_iters must be in 1..64");
  if (p.ori_bins != kOriBins) return fail(SIFT_ERR_NOT_SUPPORTED, "ori_bins must be 36");
  if (!(p.ori_sigma_factor > 0.0f) || !(p.ori_radius_factor > 0.0f) ||
      !(p.ori_peak_ratio > 0.0f && p.ori_peak_ratio <= 1.0f))
    return fail(SIFT_ERR_INVALID_ARG, "bad orientation settings");
  if (p.upright != 0 && p.upright != 1) return fail(SIFT_ERR_INVALID_ARG, "upright must be 0 or 1");
  if (p.desc_width != 4 || p.desc_ori_bins != 8)
    return fail(SIFT_ERR_NOT_SUPPORTED, "descriptor must be 4x4x8");
  if (!(p.desc_magnif > 0.0f) || !(p.desc_clamp > 0.0f))
    return fail(SIFT_ERR_INVALID_ARG, "bad descriptor settings");
  if (p.n_dsp < 1 || p.n_dsp > SIFT_MAX_DSP)
    return fail(SIFT_ERR_INVALID_ARG, "n_dsp must be in 1..%d", SIFT_MAX_DSP);
  for (int i = 0; i < p.n_dsp; ++i)
    if (!(p.dsp_scales[i] > 0.0f) || !(p.dsp_scales[i] < 64.0f))
      return fail(SIFT_ERR_INVALID_ARG, "dsp_scales[%d] must be in (0, 64)", i);
  if (p.rootsift != 0 && p.rootsift != 1) return fail(SIFT_ERR_INVALID_ARG, "rootsift must be 0 or 1");
  if (p.max_keypoints < 0) return fail(SIFT_ERR_INVALID_ARG, "max_keypoints must be >= 0");
  if (p.max_candidates < 1 || p.max_candidates > (1 << 24))
    return fail(SIFT_ERR_INVALID_ARG, "max_candidates must be in 1..2^24");
  if (p.tile_rows != 0 && p.tile_rows != 32 && p.tile_rows != 64 && p.tile_rows != 128 &&
      p.tile_rows != 256 && p.tile_rows != 512)
    return fail(SIFT_ERR_INVALID_ARG, "tile_rows must be 0, 32, 64, 128, 256 or 512");
  if (p.n_streams < 0 || p.n_streams > kMaxParts)
    return fail(SIFT_ERR_INVALID_ARG, "n_streams must be in 0..%d", kMaxParts);
  if (p.upsample_max_pixels < 0)
    return fail(SIFT_ERR_INVALID_ARG, "upsample_max_pixels must be >= 0");
  if (p.pyramid_fp16 != 0 && p.pyramid_fp16 != 1)
    return fail(SIFT_ERR_INVALID_ARG, "pyramid_fp16 must be 0 or 1");
  if (p.blur_chain < 0 || p.blur_chain > kChainMaxLevels)
    return fail(SIFT_ERR_INVALID_ARG, "blur_chain must be in 0..%d", kChainMaxLevels);
  if (p.detect_waves != 0 && p.detect_waves != 4 && p.detect_waves != 8)
    return fail(SIFT_ERR_INVALID_ARG, "detect_waves must be 0, 4 or 8");
  // Window sizes.  A refined keypoint has layer + offset below s + 1/2, so
  // its octave scale stays below sigma0 * 2^((s + 1/2) / s).  The descriptor
  // scans a square of half-side ceil(2.5 * cell * (|cos| + |sin|)) + 1 for
  // the largest domain size, the orientation histogram one of half-side
  // floor(radius_factor * sigma_factor * sigma + 1/2); both sides are kept
  // below 2048 samples (at most 4M samples per keypoint).
  const double sig_max = p.sigma0 * std::pow(2.0, (p.n_scales + 0.5) / p.n_scales);
  double dmax = 0.0;
  for (int i = 0; i < p.n_dsp; ++i) dmax = std::max(dmax, (double)p.dsp_scales[i]);
  const double rd = std::ceil(2.5 * std::sqrt(2.0) * p.desc_magnif * sig_max * dmax) + 1.0;
  if (2.0 * rd + 1.0 > kMaxWindowSide)
    return fail(SIFT_ERR_NOT_SUPPORTED,
                "descriptor window side %.0f exceeds %d (desc_magnif * largest dsp_scale too large)",
                2.0 * rd + 1.0, kMaxWindowSide);
  const double ro = std::floor(p.ori_radius_factor * p.ori_sigma_factor * sig_max + 0.5);
  if (2.0 * ro + 1.0 > kMaxWindowSide)
    return fail(SIFT_ERR_NOT_SUPPORTED, "orientation window side %.0f exceeds %d",
                2.0 * ro + 1.0, kMaxWindowSide);
  return SIFT_OK;
}

// Which octave structure an image gets: without the upsampled octave when
// the handle upsamples but the image has more than upsample_max_pixels pixels
// (the paper's VRAM-adaptive suppression of the 2x base above a size).
int cfg_index(const sift_handle* h, int height, int width) {
  const sift_params& p = h->params;
  return (p.upsample && p.upsample_max_pixels > 0 &&
          (int64_t)height * width > (int64_t)p.upsample_max_pixels) ? 1 : 0;
}

const Config& cfg_for(const sift_handle* h, int height, int width) {
  return h->cfg[cfg_index(h, height, width)];
}

// Octave count, size limits and the last-octave minimum.
sift_status validate_size(const sift_handle* h, int height, int width) {
  if (height < 1 || width < 1) return fail(SIFT_ERR_INVALID_ARG, "image size must be positive");
  if (height > kMaxSide || width > kMaxSide)
    return fail(SIFT_ERR_TOO_LARGE, "image side above %d", kMaxSide);
  const DevParams& d = cfg_for(h, height, width).dev;
  int hk, wk;
  // kernels address a level with 32-bit byte offsets: the first (largest)
  // level plane must stay below 2 GiB
  octave_dims(height, width, d.upsample, 0, &hk, &wk);
  if ((int64_t)hk * level_pitch(wk) * 4 >= (int64_t(1) << 31))
    return fail(SIFT_ERR_TOO_LARGE, "a %dx%d level exceeds 2 GiB", hk, wk);
  octave_dims(height, width, d.upsample, d.n_oct - 1, &hk, &wk);
  const int need = 2 * d.border + 3;
  if (hk < need || wk < need)
    return fail(SIFT_ERR_IMAGE_TOO_SMALL, "last octave %dx%d below %dx%d", hk, wk, need, need);
  return SIFT_OK;
}

int64_t region_bytes(const sift_handle* h, int height, int width) {
  return region_tail(height, width, layout_cfg(cfg_for(h, height, width).dev)).bytes;
}

sift_status check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return SIFT_OK;
  return fail(SIFT_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

// ---- stage profiling: event pairs around stages while recording is on
enum Stage { kStSetup, kStBlur, kStDetect, kStCompact, kStRefine, kStOrient, kStDescribe, kStCount };
const char* const kStageNames[kStCount] = {"setup", "blur", "detect", "compact",
                                           "refine", "orient", "describe"};

struct ProfRecord {
  int stage;
  double bytes;
  double fmas;            // fused multiply-adds the launch must issue (0: not counted)
  char label[32];         // launch detail, e.g. "o-1 l2 R7"
  hipEvent_t a, b;
};

// Recording is process-wide; the mutex lets extractions from several host
// threads (e.g. a server's worker) record safely.
struct Profiler {
  std::mutex mu;
  bool on = false;
  std::vector<ProfRecord> recs;
  std::vector<hipEvent_t> pool;
} g_prof;

hipEvent_t prof_event() {
  if (!g_prof.pool.empty()) {
    hipEvent_t e = g_prof.pool.back();
    g_prof.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Opens a stage record (no-op when recording is off); close with prof_end.
int prof_begin(int stage, double bytes, hipStream_t stream, const char* label = "",
               double fmas = 0.0) {
  if (g_capturing) return -1;
  std::lock_guard<std::mutex> lk(g_prof.mu);
  if (!g_prof.on) return -1;
  ProfRecord r;
  r.stage = stage;
  r.bytes = bytes;
  r.fmas = fmas;
  std::snprintf(r.label, sizeof r.label, "%s", label);
  r.a = prof_event();
  r.b = prof_event();
  if (!r.a || !r.b) return -1;
  hipEventRecord(r.a, stream);
  g_prof.recs.push_back(r);
  return (int)g_prof.recs.size() - 1;
}

void prof_end(int rec, hipStream_t stream) {
  if (rec < 0) return;
  std::lock_guard<std::mutex> lk(g_prof.mu);
  hipEventRecord(g_prof.recs[rec].b, stream);
}


// Sub-batches of one batched call.  An image's arithmetic never depends on
// the others, so any partition gives the same bits; each part runs as one
// launch sequence (several run concurrently on the handle's streams).
struct Part {
  int cfg;                  // octave structure of every image of the part
  std::vector<int> idx;     // image indices, ascending
};

// Number of parts a batch of n images of one octave structure is cut into.
int parts_wanted(int32_t n, int n_streams) {
  int parts = n_streams;
  if (parts < 1) parts = n >= 8 ? 4 : 1;
  return std::min(std::min(parts, kMaxParts), (int)n);
}

// Contiguous ranges of `ids` of about equal workspace footprint.
void split_even(const sift_handle* h, int cfg, const std::vector<int>& ids, int parts,
                const int32_t* heights, const int32_t* widths, std::vector<Part>* out) {
  const int n = (int)ids.size();
  int64_t total = 0;
  std::vector<int64_t> rb(n);
  for (int i = 0; i < n; ++i) total += (rb[i] = region_bytes(h, heights[ids[i]], widths[ids[i]]));
  std::vector<int> first(parts + 1, n);
  first[0] = 0;
  int64_t acc = 0;
  int p = 1;
  for (int i = 0; i < n && p < parts; ++i) {
    acc += rb[i];
    // cut after image i once the running footprint reaches p / parts of the
    // total, leaving at least one image for each remaining part
    if (acc * parts >= total * p && n - (i + 1) >= parts - p) first[p++] = i + 1;
  }
  while (p < parts) { first[p] = first[p - 1] + 1; ++p; }   // degenerate footprints
  for (int q = 0; q < parts; ++q) {
    Part pt;
    pt.cfg = cfg;
    pt.idx.assign(ids.begin() + first[q], ids.begin() + first[q + 1]);
    out->push_back(std::move(pt));
  }
}

// The parts of a batch: images of one octave structure are split into
// parts_wanted() ranges (one range when `one_sequence`); a batch that mixes
// both structures runs one part per structure.
std::vector<Part> plan_parts(const sift_handle* h, int32_t n, const int32_t* heights,
                             const int32_t* widths, bool one_sequence) {
  std::vector<int> ids[2];
  for (int i = 0; i < n; ++i) ids[cfg_index(h, heights[i], widths[i])].push_back(i);
  std::vector<Part> parts;
  if (!ids[0].empty() && !ids[1].empty()) {
    for (int c = 0; c < 2; ++c) split_even(h, c, ids[c], 1, heights, widths, &parts);
    return parts;
  }
  const int c = ids[0].empty() ? 1 : 0;
  const int np = one_sequence ? 1 : parts_wanted(n, h->params.n_streams);
  split_even(h, c, ids[c], np, heights, widths, &parts);
  return parts;
}

int64_t part_bytes(const sift_handle* h, const Part& pt, const int32_t* heights,
                   const int32_t* widths) {
  Header hd;
  make_header((int)pt.idx.size(), &hd);
  int64_t b = hd.bytes;
  for (int i : pt.idx) b += region_bytes(h, heights[i], widths[i]);
  return b;
}

}  // namespace

extern "C" {

sift_status sift_params_default(sift_params* p) {
  if (!p) return fail(SIFT_ERR_INVALID_ARG, "null params");
  std::memset(p, 0, sizeof *p);
  p->n_octaves = 4;
  p->n_scales = 3;
  p->upsample = 0;
  p->sigma0 = 1.6f;
  p->sigma_in = 0.5f;
  p->contrast_threshold = 0.04f / 3.0f;
  p->prefilter_ratio = 0.5f;
  p->edge_ratio = 10.0f;
  p->border = 5;
  p->refine_iters = 5;
  p->ori_bins = 36;
  p->ori_sigma_factor = 1.5f;
  p->ori_radius_factor = 3.0f;
  p->ori_peak_ratio = 0.8f;
  p->upright = 0;
  p->desc_width = 4;
  p->desc_ori_bins = 8;
  p->desc_magnif = 3.0f;
  p->desc_clamp = 0.2f;
  p->n_dsp = 1;
  p->dsp_scales[0] = 1.0f;
  p->rootsift = 0;
  p->max_keypoints = 65536;
  p->max_candidates = 65536;
  return SIFT_OK;
}

sift_status sift_create(const sift_params* p, sift_handle** out) {
  if (!p || !out) return fail(SIFT_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  sift_status st = validate_params(*p);
  if (st != SIFT_OK) return st;
  sift_handle* h = new sift_handle();
  h->params = *p;
  bool ok = true;
  for (int c = 0; c < 2; ++c) {
    const int up = c == 0 ? p->upsample : 0;
    DevParams& d = h->cfg[c].dev;
    std::memset(&d, 0, sizeof d);
    d.n_oct = p->n_octaves + up;
    d.o0 = up ? -1 : 0;
    d.s = p->n_scales;
    d.upsample = up;
    d.border = p->border;
    d.refine_iters = p->refine_iters;
    d.upright = p->upright;
    d.rootsift = p->rootsift;
    d.max_kp = p->max_keypoints;
    d.max_cand = p->max_candidates;
    d.n_dsp = p->n_dsp;
    d.h16 = p->pyramid_fp16;
    d.sigma0 = p->sigma0;
    d.contrast_thr = p->contrast_threshold;
    d.pre_thr = p->prefilter_ratio * p->contrast_threshold;
    d.edge_ratio = p->edge_ratio;
    d.ori_sigma_factor = p->ori_sigma_factor;
    d.ori_radius_factor = p->ori_radius_factor;
    d.ori_peak_ratio = p->ori_peak_ratio;
    d.desc_magnif = p->desc_magnif;
    d.desc_clamp = p->desc_clamp;
    // largest domain size first: the descriptor kernel stops its size loop at
    // the first size whose window holds none of a batch's pixels
    for (int i = 0; i < p->n_dsp; ++i) d.dsp[i] = p->dsp_scales[i];
    std::sort(d.dsp, d.dsp + p->n_dsp, [](float a, float b) { return a > b; });
    // level sigmas: level i of an octave carries sigma0 * k^i, k = 2^(1/s)
    const double s0 = p->sigma0;
    const double assumed = (double)p->sigma_in * (up ? 2.0 : 1.0);
    const double sig_init = std::sqrt(std::fmax(s0 * s0 - assumed * assumed, 0.01));
    const double k2 = std::pow(2.0, 2.0 / p->n_scales);
    ok = ok && make_taps(sig_init, &h->cfg[c].init);
    for (int i = 1; i <= p->n_scales + 2; ++i)
      ok = ok && make_taps(s0 * std::sqrt(std::pow(k2, i) - std::pow(k2, i - 1)),
                           &h->cfg[c].inc[i - 1]);
  }
  if (!ok) {
    delete h;
    return fail(SIFT_ERR_NOT_SUPPORTED, "a Gaussian radius ceil(4 sigma) exceeds %d", kMaxRadius);
  }
  *out = h;
  return SIFT_OK;
}

void sift_destroy(sift_handle* h) {
  if (!h) return;
  for (int i = 0; i < kMaxParts; ++i)
    if (h->part_stream[i]) hipStreamDestroy(h->part_stream[i]);
  delete h;
}

sift_status sift_get_params(const sift_handle* h, sift_params* p) {
  if (!h || !p) return fail(SIFT_ERR_INVALID_ARG, "null argument");
  *p = h->params;
  return SIFT_OK;
}

sift_status sift_batch_workspace_size(const sift_handle* h, int32_t n, const int32_t* heights,
                                      const int32_t* widths, size_t* bytes) {
  if (!h || !heights || !widths || !bytes) return fail(SIFT_ERR_INVALID_ARG, "null argument");
  if (n < 1) return fail(SIFT_ERR_INVALID_ARG, "batch size must be >= 1");
  if (n > kMaxBatch) return fail(SIFT_ERR_TOO_LARGE, "batch above %d images", kMaxBatch);
  for (int i = 0; i < n; ++i) {
    sift_status st = validate_size(h, heights[i], widths[i]);
    if (st != SIFT_OK) return st;
  }
  // the parts' layouts one after another, for the split and for the
  // one-sequence plan (stage profiling runs a batch as one sequence)
  int64_t most = 0;
  for (bool one : {false, true}) {
    int64_t total = 0;
    for (const Part& pt : plan_parts(h, n, heights, widths, one))
      total += part_bytes(h, pt, heights, widths);
    most = std::max(most, total);
  }
  *bytes = (size_t)most;
  return SIFT_OK;
}

sift_status sift_workspace_size(const sift_handle* h, int32_t height, int32_t width, size_t* bytes) {
  return sift_batch_workspace_size(h, 1, &height, &width, bytes);
}

}  // extern "C"

namespace {

// Grid sizing of one launch sequence: work items summed over the images it
// covers (their own sizes, or a bucket's largest size for every slot).
struct Plan {
  std::vector<int64_t> tiles;   // blur strips x chunks, [octave * kNumTileH + chunk class]
  std::vector<int64_t> pixels;  // pixels per octave
  int64_t input_px = 0;
  int64_t bands = 0;
};

void plan_add(Plan* pl, const DevParams& p, int height, int width, int64_t times) {
  if (pl->tiles.empty()) {
    pl->tiles.assign((size_t)kNumTileH * p.n_oct, 0);
    pl->pixels.assign(p.n_oct, 0);
  }
  for (int k = 0; k < p.n_oct; ++k) {
    int hk, wk;
    octave_dims(height, width, p.upsample, k, &hk, &wk);
    for (int c = 0; c < kNumTileH; ++c)
      pl->tiles[k * kNumTileH + c] += times * cdiv(wk, kTileW) * cdiv(hk, tile_h_of(c));
    pl->pixels[k] += times * (int64_t)hk * wk;
  }
  pl->input_px += times * (int64_t)height * width;
  pl->bands += times * region_tail(height, width, layout_cfg(p)).total_bands;
}

HdrPtrs header_ptrs(char* ws, int n) {
  Header hd;
  make_header(n, &hd);
  HdrPtrs hp;
  hp.table = reinterpret_cast<const ImgEntry*>(ws + hd.table);
  hp.tile_prefix = reinterpret_cast<int*>(ws + hd.tile_prefix);
  hp.band_prefix = reinterpret_cast<int*>(ws + hd.band_prefix);
  hp.cand_prefix = reinterpret_cast<int*>(ws + hd.cand_prefix);
  hp.kp_prefix = reinterpret_cast<int*>(ws + hd.kp_prefix);
  hp.queue = reinterpret_cast<int*>(ws + hd.queue);
  return hp;
}

// The image table: entries[i] copied into the workspace, a chunk of entries
// per setup launch (kernel arguments carry them; nothing is copied from host
// memory by the runtime).
sift_status write_table(const std::vector<ImgEntry>& entries, const HdrPtrs& hp,
                        hipStream_t stream) {
  SetupChunk chunk;
  std::memset(&chunk, 0, sizeof chunk);
  const int n = (int)entries.size();
  for (int i = 0; i < n; ++i) {
    chunk.e[chunk.count] = entries[i];
    if (++chunk.count == kSetupChunk || i == n - 1) {
      sift_status st = check_hip(launch_setup(hp, chunk, stream), "setup");
      if (st != SIFT_OK) return st;
      chunk.first = i + 1;
      chunk.count = 0;
    }
  }
  return SIFT_OK;
}

ImgEntry make_entry(const float* img, int64_t pitch, int height, int width, int64_t region,
                    const sift_output& o) {
  ImgEntry e;
  std::memset(&e, 0, sizeof e);
  e.src = img;
  e.src_pitch = pitch;
  e.h = height;
  e.w = width;
  e.region = region;
  e.kp = o.keypoints;
  e.desc = o.descriptors;
  e.count = o.count;
  e.n_found = o.n_found;
  e.n_cand = o.n_candidates;
  e.cap = o.capacity;
  return e;
}

// Every stage after the table is in place: prefix tables, pyramid, detection,
// compaction, refinement, orientation, descriptors.  Grids come from `plan`;
// each kernel reads the actual work counts from the table on the device and
// lets surplus work-groups go, so a plan may over-cover the images.
sift_status launch_stages(const sift_handle* h, const Config& cfg, int32_t n, const Plan& plan,
                          char* ws, const HdrPtrs& hp, hipStream_t stream) {
  sift_status st = SIFT_OK;
  const DevParams& p = cfg.dev;
  for (int64_t t : plan.tiles)
    if (t > INT32_MAX - kXcds) return fail(SIFT_ERR_TOO_LARGE, "batch has too many tiles");
  if (plan.bands > INT32_MAX - kXcds) return fail(SIFT_ERR_TOO_LARGE, "batch has too many bands");
  int prec = prof_begin(kStSetup, 0.0, stream);
  if ((st = check_hip(launch_finalize(hp, n, p, stream), "finalize")) != SIFT_OK) return st;
  prof_end(prec, stream);

  // scale space: per octave, runs of consecutive levels in one launch each
  // (k_chain) where a kernel for the run is built, else one launch per level
  // (k_blur); both compute every value identically
  const int max_chain = h->params.blur_chain == 0 ? kDefaultChain : h->params.blur_chain;
  const LayoutCfg lc = layout_cfg(p);
  for (int k = 0; k < p.n_oct; ++k) {
    const int cls = blur_class(h->params.tile_rows, &plan.tiles[k * kNumTileH]);
    const int th = tile_h_of(cls);
    const int grid = (int)((plan.tiles[k * kNumTileH + cls] + kXcds - 1) / kXcds * kXcds);
    const int* tile_prefix = hp.tile_prefix + (int64_t)(cls * kMaxOct + k) * (n + 1);
    const int es_d = level_es(lc, k);
    for (int lv = (k == 0 ? 0 : 1); lv <= p.s + 2;) {
      auto taps_of = [&](int level) -> const Taps& { return level == 0 ? cfg.init : cfg.inc[level - 1]; };
      int mode;
      if (lv == 0) mode = p.upsample ? kSrcUpsample : kSrcImage;
      else if (lv == 1 && k > 0) mode = kSrcDown;
      else mode = kSrcLevel;
      // storage of the levels written and of their source
      const int es_s = lv == 0 ? 4 : level_es(lc, mode == kSrcDown ? k - 1 : k);
      const int st_mode = es_d == 4 ? 0 : (es_s == 4 ? 1 : 2);
      int nl = 1;
      int radii[kChainMaxLevels] = {};
      for (int m = std::min(max_chain, p.s + 3 - lv); m >= 2; --m) {
        for (int i = 0; i < m; ++i) radii[i] = taps_of(lv + i).radius;
        if (chain_supported(mode, st_mode, m, radii)) {
          nl = m;
          break;
        }
      }
      // algorithmic bytes: the source read once (input pixels for the first
      // level), each level written once, plus level 0 written when subsampling
      double bytes = (double)es_s * plan.pixels[k] + (double)nl * es_d * plan.pixels[k];
      if (lv == 0 && p.upsample) bytes = 4.0 * plan.input_px + 4.0 * nl * plan.pixels[k];
      if (mode == kSrcDown) bytes += (double)es_d * plan.pixels[k];
      // a vertical and a horizontal pass of 2R + 1 taps per output pixel and level
      double fmas = 0.0;
      for (int i = 0; i < nl; ++i) fmas += 2.0 * (2 * taps_of(lv + i).radius + 1) * plan.pixels[k];
      char label[32];
      if (nl == 1)
        std::snprintf(label, sizeof label, "o%d l%d R%d", k + p.o0, lv, taps_of(lv).radius);
      else if (nl == 2)
        std::snprintf(label, sizeof label, "o%d l%d-%d R%d,%d", k + p.o0, lv, lv + 1, radii[0],
                      radii[1]);
      else if (nl == 3)
        std::snprintf(label, sizeof label, "o%d l%d-%d R%d,%d,%d", k + p.o0, lv, lv + 2, radii[0],
                      radii[1], radii[2]);
      else
        std::snprintf(label, sizeof label, "o%d l%d-%d R%d,%d,%d,%d", k + p.o0, lv, lv + 3,
                      radii[0], radii[1], radii[2], radii[3]);
      prec = prof_begin(kStBlur, bytes, stream, label, fmas);
      if (nl == 1) {
        BlurArgs a;
        std::memset(&a, 0, sizeof a);
        const Taps& t = taps_of(lv);
        a.ws = ws;
        a.table = hp.table;
        a.tile_prefix = tile_prefix;
        a.n = n;
        a.k = k;
        a.dst_level = lv;
        a.mode = mode;
        a.th = th;
        a.st = st_mode;
        a.p = p;
        std::memcpy(a.taps, t.g, sizeof(float) * (2 * t.radius + 1));
        if (grid > 0 && (st = check_hip(launch_blur(a, t.radius, grid, stream), "blur")) != SIFT_OK)
          return st;
      } else {
        ChainArgs a;
        std::memset(&a, 0, sizeof a);
        a.ws = ws;
        a.table = hp.table;
        a.tile_prefix = tile_prefix;
        a.n = n;
        a.k = k;
        a.lv0 = lv;
        a.th = th;
        a.p = p;
        for (int i = 0; i < nl; ++i) {
          const Taps& t = taps_of(lv + i);
          for (int q = 0; q <= t.radius; ++q) a.g[i][q] = t.g[t.radius + q];
        }
        if (grid > 0 && (st = check_hip(launch_chain(a, mode, st_mode, nl, radii, grid, stream),
                                        "blur chain")) != SIFT_OK)
          return st;
      }
      prof_end(prec, stream);
      lv += nl;
    }
  }
  // detection and ordered compaction
  int64_t all_px = 0;
  double level_px_bytes = 0.0;
  for (int k = 0; k < p.n_oct; ++k) {
    all_px += plan.pixels[k];
    level_px_bytes += (double)level_es(layout_cfg(p), k) * plan.pixels[k];
  }
  const int bands = (int)plan.bands;
  // detection reads the s+3 levels once and writes one mask bit per pixel-layer
  prec = prof_begin(kStDetect, (p.s + 3) * level_px_bytes + p.s / 8.0 * all_px, stream);
  const int waves = h->params.detect_waves == 0 ? kDetectWaves : h->params.detect_waves;
  if (bands > 0 &&
      (st = check_hip(launch_detect(ws, hp, n, p, waves, bands, stream), "detect")) != SIFT_OK)
    return st;
  prof_end(prec, stream);
  prec = prof_begin(kStCompact, (p.s / 4.0) * all_px, stream);
  if ((st = check_hip(launch_band_scan(ws, hp, n, p, stream), "band scan")) != SIFT_OK) return st;
  if (bands > 0 && (st = check_hip(launch_emit(ws, hp, n, p, bands, stream), "emit")) != SIFT_OK)
    return st;
  if ((st = check_hip(launch_img_prefix(ws, hp, n, p, 0, stream), "prefix")) != SIFT_OK) return st;
  prof_end(prec, stream);
  // per-candidate stages; grids are persistent, work counts are read on the device
  const int64_t cand_total = (int64_t)n * p.max_cand;
  const int refine_grid = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (cand_total + 255) / 256));
  const int orient_grid = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (cand_total + 3) / 4));
  prec = prof_begin(kStRefine, 0.0, stream);
  if ((st = check_hip(launch_refine(ws, hp, n, p, refine_grid, stream), "refine")) != SIFT_OK) return st;
  prof_end(prec, stream);
  prec = prof_begin(kStOrient, 0.0, stream);
  if ((st = check_hip(launch_orient(ws, hp, n, p, orient_grid, stream), "orient")) != SIFT_OK) return st;
  if ((st = check_hip(launch_ori_scan(ws, hp, n, p, stream), "orientation scan")) != SIFT_OK) return st;
  if ((st = check_hip(launch_img_prefix(ws, hp, n, p, 1, stream), "prefix")) != SIFT_OK) return st;
  prof_end(prec, stream);
  const int desc_grid = (int)std::min<int64_t>(4096, std::max<int64_t>(1, cand_total));
  prec = prof_begin(kStDescribe, 0.0, stream);
  if ((st = check_hip(launch_describe(ws, hp, n, p, desc_grid, stream), "describe")) != SIFT_OK) return st;
  prof_end(prec, stream);
  return SIFT_OK;
}

// The launch sequence of one (sub-)batch on `stream`; arguments already checked.
sift_status launch_batch(const sift_handle* h, const Config& cfg, int32_t n,
                         const float* const* d_images, const int32_t* heights,
                         const int32_t* widths, const int64_t* pitches, void* d_workspace,
                         const sift_output* outs, hipStream_t stream) {
  char* ws = static_cast<char*>(d_workspace);
  const DevParams& p = cfg.dev;
  const LayoutCfg lc = layout_cfg(p);
  Header hd;
  make_header(n, &hd);
  const HdrPtrs hp = header_ptrs(ws, n);
  std::vector<ImgEntry> entries;
  Plan plan;
  int64_t off = hd.bytes;
  for (int i = 0; i < n; ++i) {
    entries.push_back(make_entry(d_images[i], pitches[i], heights[i], widths[i], off, outs[i]));
    off += region_tail(heights[i], widths[i], lc).bytes;
    plan_add(&plan, p, heights[i], widths[i], 1);
  }
  const int prec = prof_begin(kStSetup, 0.0, stream);
  sift_status st = write_table(entries, hp, stream);
  prof_end(prec, stream);
  if (st != SIFT_OK) return st;
  return launch_stages(h, cfg, n, plan, ws, hp, stream);
}

}  // namespace

extern "C" {

sift_status sift_extract_batch(sift_handle* h, int32_t n, const float* const* d_images,
                               const int32_t* heights, const int32_t* widths,
                               const int64_t* pitches, void* d_workspace,
                               size_t workspace_bytes, const sift_output* outs, void* stream_v) {
  if (!h || !d_images || !heights || !widths || !pitches || !d_workspace || !outs)
    return fail(SIFT_ERR_INVALID_ARG, "null argument");
  if (n < 1) return fail(SIFT_ERR_INVALID_ARG, "batch size must be >= 1");
  if (n > kMaxBatch) return fail(SIFT_ERR_TOO_LARGE, "batch above %d images", kMaxBatch);
  if (reinterpret_cast<uintptr_t>(d_workspace) % 256 != 0)
    return fail(SIFT_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  for (int i = 0; i < n; ++i) {
    if (!d_images[i]) return fail(SIFT_ERR_INVALID_ARG, "image %d is null", i);
    if (pitches[i] < widths[i]) return fail(SIFT_ERR_INVALID_ARG, "image %d: pitch < width", i);
    if (!outs[i].keypoints || !outs[i].descriptors || !outs[i].count)
      return fail(SIFT_ERR_INVALID_ARG, "image %d: null output pointer", i);
    if (outs[i].capacity < 0) return fail(SIFT_ERR_INVALID_ARG, "image %d: negative capacity", i);
  }
  size_t need = 0;
  sift_status st = sift_batch_workspace_size(h, n, heights, widths, &need);
  if (st != SIFT_OK) return st;
  if (workspace_bytes < need)
    return fail(SIFT_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes, need %zu", workspace_bytes, need);

  bool one_sequence = false;
  {
    // stage profiling times one sequence of launches on the caller's stream
    std::lock_guard<std::mutex> lk(g_prof.mu);
    one_sequence = g_prof.on && !g_capturing;
  }
  const std::vector<Part> parts = plan_parts(h, n, heights, widths, one_sequence);
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_v);
  char* ws = static_cast<char*>(d_workspace);
  // the images, sizes and outputs of one part, gathered in its order
  struct Gathered {
    std::vector<const float*> img;
    std::vector<int32_t> h, w;
    std::vector<int64_t> pitch;
    std::vector<sift_output> out;
  };
  auto gather = [&](const Part& pt) {
    Gathered g;
    for (int i : pt.idx) {
      g.img.push_back(d_images[i]);
      g.h.push_back(heights[i]);
      g.w.push_back(widths[i]);
      g.pitch.push_back(pitches[i]);
      g.out.push_back(outs[i]);
    }
    return g;
  };
  auto run_part = [&](const Part& pt, char* base, hipStream_t q) {
    const Gathered g = gather(pt);
    return launch_batch(h, h->cfg[pt.cfg], (int32_t)pt.idx.size(), g.img.data(), g.h.data(),
                        g.w.data(), g.pitch.data(), base, g.out.data(), q);
  };
  if (parts.size() == 1) return run_part(parts[0], ws, stream);
  if (one_sequence) {
    // one stream: the parts one after the other
    int64_t off = 0;
    for (const Part& pt : parts) {
      if ((st = run_part(pt, ws + off, stream)) != SIFT_OK) return st;
      off += part_bytes(h, pt, heights, widths);
    }
    return SIFT_OK;
  }
  std::call_once(h->streams_once, [h] {
    for (int i = 0; i < kMaxParts && h->streams_status == hipSuccess; ++i)
      h->streams_status = hipStreamCreateWithFlags(&h->part_stream[i], hipStreamNonBlocking);
  });
  if (h->streams_status != hipSuccess) return check_hip(h->streams_status, "sub-batch streams");
  const int np = (int)parts.size();
  hipEvent_t ev[kMaxParts + 1] = {};
  hipError_t e = hipSuccess;
  for (int q = 0; q <= np && e == hipSuccess; ++q)
    e = hipEventCreateWithFlags(&ev[q], hipEventDisableTiming);
  // fork: every sub-batch stream waits for the caller's stream
  if (e == hipSuccess) e = hipEventRecord(ev[np], stream);
  for (int q = 0; q < np && e == hipSuccess; ++q)
    e = hipStreamWaitEvent(h->part_stream[q], ev[np], 0);
  int64_t off = 0;
  for (int q = 0; q < np && e == hipSuccess && st == SIFT_OK; ++q) {
    st = run_part(parts[q], ws + off, h->part_stream[q]);
    off += part_bytes(h, parts[q], heights, widths);
    if (st == SIFT_OK) e = hipEventRecord(ev[q], h->part_stream[q]);
  }
  // join: the caller's stream waits for every sub-batch
  for (int q = 0; q < np && e == hipSuccess && st == SIFT_OK; ++q)
    e = hipStreamWaitEvent(stream, ev[q], 0);
  for (int q = 0; q <= np; ++q)
    if (ev[q]) hipEventDestroy(ev[q]);
  if (st != SIFT_OK) return st;
  return check_hip(e, "sub-batch streams");
}


// ---------------------------------------------------------------------------
// Buckets: one launch sequence recorded as a graph for up to n_slots images of
// at most max_height x max_width each.  The graph's grids cover every slot at
// the largest size; the image table it reads is rewritten by setup launches
// before every replay, and each kernel reads the actual sizes from it.

}  // extern "C"

struct sift_bucket {
  sift_handle* h = nullptr;
  int cfg = 0;
  int n_slots = 0, max_h = 0, max_w = 0;
  char* ws = nullptr;
  int64_t slot_bytes = 0;   // one image region at the largest size
  int64_t sink = 0;         // scratch outputs of empty slots
  int64_t slots = 0;        // first slot region
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

constexpr int64_t kSinkBytes = 1024;

sift_status bucket_layout(const sift_handle* h, int32_t n_slots, int32_t max_h, int32_t max_w,
                          int64_t* slot_bytes, int64_t* sink, int64_t* slots, int64_t* total) {
  if (!h) return fail(SIFT_ERR_INVALID_ARG, "null handle");
  if (n_slots < 1 || n_slots > kMaxBatch)
    return fail(SIFT_ERR_INVALID_ARG, "n_slots must be in 1..%d", kMaxBatch);
  sift_status st = validate_size(h, max_h, max_w);
  if (st != SIFT_OK) return st;
  Header hd;
  make_header(n_slots, &hd);
  *sink = hd.bytes;
  *slots = hd.bytes + kSinkBytes;
  *slot_bytes = region_bytes(h, max_h, max_w);
  *total = *slots + (int64_t)n_slots * *slot_bytes;
  return SIFT_OK;
}

}  // namespace

extern "C" {

sift_status sift_bucket_workspace_size(const sift_handle* h, int32_t n_slots, int32_t max_height,
                                       int32_t max_width, size_t* bytes) {
  if (!bytes) return fail(SIFT_ERR_INVALID_ARG, "null argument");
  int64_t sb, sink, slots, total;
  sift_status st = bucket_layout(h, n_slots, max_height, max_width, &sb, &sink, &slots, &total);
  if (st != SIFT_OK) return st;
  *bytes = (size_t)total;
  return SIFT_OK;
}

sift_status sift_bucket_create(sift_handle* h, int32_t n_slots, int32_t max_height,
                               int32_t max_width, void* d_workspace, size_t workspace_bytes,
                               sift_bucket** out) {
  if (!out || !d_workspace) return fail(SIFT_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  int64_t sb, sink, slots, total;
  sift_status st = bucket_layout(h, n_slots, max_height, max_width, &sb, &sink, &slots, &total);
  if (st != SIFT_OK) return st;
  if (reinterpret_cast<uintptr_t>(d_workspace) % 256 != 0)
    return fail(SIFT_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if ((int64_t)workspace_bytes < total)
    return fail(SIFT_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes, need %lld", workspace_bytes,
                (long long)total);
  const int cfg = cfg_index(h, max_height, max_width);
  const Config& c = h->cfg[cfg];
  Plan plan;
  plan_add(&plan, c.dev, max_height, max_width, n_slots);
  char* ws = static_cast<char*>(d_workspace);
  const HdrPtrs hp = header_ptrs(ws, n_slots);
  hipStream_t cap = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
  if (e != hipSuccess) return check_hip(e, "capture stream");
  e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    hipStreamDestroy(cap);
    return check_hip(e, "begin capture");
  }
  sift::set_capturing(true);
  st = launch_stages(h, c, n_slots, plan, ws, hp, cap);
  sift::set_capturing(false);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(cap, &graph);
  hipStreamDestroy(cap);
  if (st != SIFT_OK) {
    if (graph) hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return check_hip(e, "end capture");
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    hipGraphDestroy(graph);
    return check_hip(e, "instantiate");
  }
  sift_bucket* b = new sift_bucket();
  b->h = h;
  b->cfg = cfg;
  b->n_slots = n_slots;
  b->max_h = max_height;
  b->max_w = max_width;
  b->ws = ws;
  b->slot_bytes = sb;
  b->sink = sink;
  b->slots = slots;
  b->graph = graph;
  b->exec = exec;
  *out = b;
  return SIFT_OK;
}

sift_status sift_bucket_launch(sift_bucket* b, int32_t n, const float* const* d_images,
                               const int32_t* heights, const int32_t* widths,
                               const int64_t* pitches, const sift_output* outs, void* stream_v) {
  if (!b || !d_images || !heights || !widths || !pitches || !outs)
    return fail(SIFT_ERR_INVALID_ARG, "null argument");
  if (n < 1 || n > b->n_slots)
    return fail(SIFT_ERR_INVALID_ARG, "%d images for a bucket of %d slots", n, b->n_slots);
  for (int i = 0; i < n; ++i) {
    if (!d_images[i]) return fail(SIFT_ERR_INVALID_ARG, "image %d is null", i);
    if (heights[i] > b->max_h || widths[i] > b->max_w)
      return fail(SIFT_ERR_INVALID_ARG, "image %d (%dx%d) exceeds the bucket's %dx%d", i,
                  heights[i], widths[i], b->max_h, b->max_w);
    sift_status st = validate_size(b->h, heights[i], widths[i]);
    if (st != SIFT_OK) return st;
    if (cfg_index(b->h, heights[i], widths[i]) != b->cfg)
      return fail(SIFT_ERR_INVALID_ARG,
                  "image %d takes the other octave structure (upsample_max_pixels)", i);
    if (pitches[i] < widths[i]) return fail(SIFT_ERR_INVALID_ARG, "image %d: pitch < width", i);
    if (!outs[i].keypoints || !outs[i].descriptors || !outs[i].count)
      return fail(SIFT_ERR_INVALID_ARG, "image %d: null output pointer", i);
    if (outs[i].capacity < 0) return fail(SIFT_ERR_INVALID_ARG, "image %d: negative capacity", i);
  }
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_v);
  // empty slots: a 0 x 0 image (no work items) whose outputs land in the sink
  sift_output sink;
  std::memset(&sink, 0, sizeof sink);
  sink.keypoints = reinterpret_cast<sift_keypoint*>(b->ws + b->sink);
  sink.descriptors = reinterpret_cast<float*>(b->ws + b->sink + 64);
  sink.count = reinterpret_cast<int32_t*>(b->ws + b->sink + kSinkBytes - 16);
  sink.capacity = 0;
  std::vector<ImgEntry> entries;
  for (int i = 0; i < b->n_slots; ++i) {
    const int64_t region = b->slots + (int64_t)i * b->slot_bytes;
    if (i < n)
      entries.push_back(make_entry(d_images[i], pitches[i], heights[i], widths[i], region, outs[i]));
    else
      entries.push_back(make_entry(reinterpret_cast<const float*>(b->ws + b->sink), 0, 0, 0,
                                   region, sink));
  }
  sift_status st = write_table(entries, header_ptrs(b->ws, b->n_slots), stream);
  if (st != SIFT_OK) return st;
  return check_hip(hipGraphLaunch(b->exec, stream), "bucket launch");
}

sift_status sift_bucket_destroy(sift_bucket* b) {
  if (!b) return SIFT_OK;
  hipError_t e = hipGraphExecDestroy(b->exec);
  const hipError_t e2 = hipGraphDestroy(b->graph);
  delete b;
  if (e == hipSuccess) e = e2;
  return check_hip(e, "bucket destroy");
}

sift_status sift_extract(sift_handle* h, const float* d_image, int32_t height, int32_t width,
                         int64_t pitch, void* d_workspace, size_t workspace_bytes,
                         const sift_output* out, void* stream) {
  return sift_extract_batch(h, 1, &d_image, &height, &width, &pitch, d_workspace, workspace_bytes,
                            out, stream);
}

sift_status sift_workspace_level(const sift_handle* h, int32_t height, int32_t width,
                                 const void* d_workspace, int32_t octave, int32_t level,
                                 const float** d_level, int32_t* level_height,
                                 int32_t* level_width, int32_t* level_pitch) {
  if (!h || !d_workspace || !d_level || !level_height || !level_width || !level_pitch)
    return fail(SIFT_ERR_INVALID_ARG, "null argument");
  sift_status st = validate_size(h, height, width);
  if (st != SIFT_OK) return st;
  const DevParams& d = cfg_for(h, height, width).dev;
  const int k = octave - d.o0;
  if (k < 0 || k >= d.n_oct) return fail(SIFT_ERR_INVALID_ARG, "no octave %d", octave);
  if (level < 0 || level > d.s + 2) return fail(SIFT_ERR_INVALID_ARG, "no level %d", level);
  Header hd;
  make_header(1, &hd);
  const OctView ov = octave_view(height, width, layout_cfg(d), k);
  *d_level = reinterpret_cast<const float*>(static_cast<const char*>(d_workspace) + hd.bytes +
                                            ov.level0 + (int64_t)level * ov.plane);
  *level_height = ov.h;
  *level_width = ov.w;
  *level_pitch = ov.pitch;
  return SIFT_OK;
}

sift_status sift_workspace_level_bytes(const sift_handle* h, int32_t height, int32_t width,
                                      int32_t octave, int32_t* elem_bytes) {
  if (!h || !elem_bytes) return fail(SIFT_ERR_INVALID_ARG, "null argument");
  sift_status st = validate_size(h, height, width);
  if (st != SIFT_OK) return st;
  const DevParams& d = cfg_for(h, height, width).dev;
  const int k = octave - d.o0;
  if (k < 0 || k >= d.n_oct) return fail(SIFT_ERR_INVALID_ARG, "no octave %d", octave);
  *elem_bytes = level_es(layout_cfg(d), k);
  return SIFT_OK;
}

sift_status sift_profile_start(void) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.on = true;
  return SIFT_OK;
}

sift_status sift_profile_launches(sift_launch_stat* out, int32_t max_out, int32_t* n_out) {
  if (!out || !n_out || max_out < 0) return fail(SIFT_ERR_INVALID_ARG, "null argument");
  std::lock_guard<std::mutex> lk(g_prof.mu);
  if (!g_prof.on) return fail(SIFT_ERR_INVALID_ARG, "profiling was not started");
  sift_status st = SIFT_OK;
  int k = 0;
  for (ProfRecord& r : g_prof.recs) {
    if (k >= max_out) break;
    float ms = 0.0f;
    hipError_t e = hipEventSynchronize(r.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess && st == SIFT_OK) st = check_hip(e, "profile events");
    sift_launch_stat& o = out[k++];
    std::memset(&o, 0, sizeof o);
    std::snprintf(o.stage, sizeof o.stage, "%s", kStageNames[r.stage]);
    std::snprintf(o.label, sizeof o.label, "%s", r.label);
    o.ms = ms;
    o.bytes = r.bytes;
    o.fmas = r.fmas;
  }
  *n_out = k;
  return st;
}

sift_status sift_profile_stop(sift_stage_stat* stats, int32_t max_stats, int32_t* n_stats) {
  if (!stats || !n_stats || max_stats < 0) return fail(SIFT_ERR_INVALID_ARG, "null argument");
  std::lock_guard<std::mutex> lk(g_prof.mu);
  if (!g_prof.on) return fail(SIFT_ERR_INVALID_ARG, "profiling was not started");
  g_prof.on = false;
  sift_stage_stat tot[kStCount];
  std::memset(tot, 0, sizeof tot);
  for (int s = 0; s < kStCount; ++s) std::snprintf(tot[s].name, sizeof tot[s].name, "%s", kStageNames[s]);
  sift_status st = SIFT_OK;
  for (ProfRecord& r : g_prof.recs) {
    float ms = 0.0f;
    hipError_t e = hipEventSynchronize(r.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess && st == SIFT_OK) st = check_hip(e, "profile events");
    tot[r.stage].launches += 1;
    tot[r.stage].ms += ms;
    tot[r.stage].bytes += r.bytes;
    g_prof.pool.push_back(r.a);
    g_prof.pool.push_back(r.b);
  }
  g_prof.recs.clear();
  int k = 0;
  for (int s = 0; s < kStCount && k < max_stats; ++s)
    if (tot[s].launches) stats[k++] = tot[s];
  *n_stats = k;
  return st;
}

sift_status sift_bounds_violations(int32_t reset, uint64_t* count) {
  if (!count) return fail(SIFT_ERR_INVALID_ARG, "null argument");
  *count = 0;
#ifdef SIFT_DEBUG_BOUNDS
  hipError_t e = hipDeviceSynchronize();
  unsigned long long a = 0, b = 0, c = 0, d = 0;
  if (e == hipSuccess) e = bounds_count_blur(&a, reset != 0);
  if (e == hipSuccess) e = bounds_count_kernels(&b, reset != 0);
  if (e == hipSuccess) e = bounds_count_match(&c, reset != 0);
  if (e == hipSuccess) e = bounds_count_verify(&d, reset != 0);
  if (e != hipSuccess) return check_hip(e, "bounds counters");
  *count = (uint64_t)(a + b + c + d);
  return SIFT_OK;
#else
  (void)reset;
  return fail(SIFT_ERR_NOT_SUPPORTED,
              "built without bounds checks (libsift_mi355x_bounds.so has them)");
#endif
}

const char* sift_status_string(sift_status st) {
  switch (st) {
    case SIFT_OK: return "ok";
    case SIFT_ERR_INVALID_ARG: return "invalid argument";
    case SIFT_ERR_IMAGE_TOO_SMALL: return "image too small";
    case SIFT_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case SIFT_ERR_TOO_LARGE: return "too large";
    case SIFT_ERR_HIP: return "HIP error";
    case SIFT_ERR_NOT_SUPPORTED: return "not supported";
  }
  return "unknown status";
}

const char* sift_last_error(void) { return g_error.c_str(); }

}  // extern "C"
