// Host runtime of geometric verification: argument checks, workspace layout
// and the launch sequence (setup, point preparation, hypotheses, refinement).
// It never allocates device memory, copies or synchronises.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/sift.h"
#include "sift_verify.h"

namespace sift {
void set_last_error(const std::string& msg);
}

using namespace sift;

namespace {

sift_status fail(sift_status st, const std::string& msg) {
  set_last_error(msg);
  return st;
}

int64_t align256(int64_t v) { return (v + 255) / 256 * 256; }

sift_status check(int32_t n, const sift_verify_pair* pairs, int32_t n_hyp) {
  if (n < 1 || n > SIFT_VERIFY_MAX_PAIRS)
    return fail(SIFT_ERR_INVALID_ARG, "pairs must be in 1.." + std::to_string(SIFT_VERIFY_MAX_PAIRS));
  if (!pairs) return fail(SIFT_ERR_INVALID_ARG, "null pairs");
  if (n_hyp < 1 || n_hyp > SIFT_VERIFY_MAX_HYPOTHESES)
    return fail(SIFT_ERR_INVALID_ARG,
                "n_hyp must be in 1.." + std::to_string(SIFT_VERIFY_MAX_HYPOTHESES));
  for (int i = 0; i < n; ++i) {
    const sift_verify_pair& q = pairs[i];
    const std::string at = "pair " + std::to_string(i) + ": ";
    if (q.cap < 0 || q.cap > SIFT_MATCH_MAX_ROWS)
      return fail(SIFT_ERR_INVALID_ARG, at + "cap must be in 0.." + std::to_string(SIFT_MATCH_MAX_ROWS));
    if (q.cap > 0 && (!q.kp_a || !q.kp_b || !q.matches))
      return fail(SIFT_ERR_INVALID_ARG, at + "null keypoints or matches");
    if (!q.H || !q.score || !q.n_inliers) return fail(SIFT_ERR_INVALID_ARG, at + "null output");
  }
  return SIFT_OK;
}

struct Layout {
  int64_t table = 0;
  std::vector<int64_t> pts, raw, norm, scores, models;
  int64_t bytes = 0;
};

Layout layout_of(int32_t n, const sift_verify_pair* pairs, int32_t n_hyp) {
  Layout L;
  int64_t off = align256((int64_t)n * (int64_t)sizeof(VerifyEntry));
  for (int i = 0; i < n; ++i) {
    const int64_t cap = pairs[i].cap;
    L.pts.push_back(off);
    off = align256(off + cap * 32);
    L.raw.push_back(off);
    off = align256(off + cap * 16);
    L.norm.push_back(off);
    off = align256(off + 8 * 8);
    L.scores.push_back(off);
    off = align256(off + (int64_t)n_hyp * 8);
    L.models.push_back(off);
    off = align256(off + (int64_t)n_hyp * 9 * 8);
  }
  L.bytes = off;
  return L;
}

}  // namespace

extern "C" {

sift_status sift_verify_workspace_size(int32_t n, const sift_verify_pair* pairs, int32_t n_hyp,
                                       size_t* bytes) {
  if (!bytes) return fail(SIFT_ERR_INVALID_ARG, "null bytes");
  sift_status st = check(n, pairs, n_hyp);
  if (st != SIFT_OK) return st;
  *bytes = (size_t)layout_of(n, pairs, n_hyp).bytes;
  return SIFT_OK;
}

sift_status sift_verify_batch(int32_t n, const sift_verify_pair* pairs, const float* d_samples,
                              int32_t n_hyp, float sigma_max, int32_t refine_iters,
                              void* d_workspace, size_t workspace_bytes, void* stream_v) {
  sift_status st = check(n, pairs, n_hyp);
  if (st != SIFT_OK) return st;
  if (!d_samples) return fail(SIFT_ERR_INVALID_ARG, "null sample numbers");
  if (!(sigma_max > 0.0f)) return fail(SIFT_ERR_INVALID_ARG, "sigma_max must be > 0");
  if (refine_iters < 0 || refine_iters > 100)
    return fail(SIFT_ERR_INVALID_ARG, "refine_iters must be in 0..100");
  if (!d_workspace || reinterpret_cast<uintptr_t>(d_workspace) % 256)
    return fail(SIFT_ERR_INVALID_ARG, "workspace must be non-null and 256-byte aligned");
  const Layout L = layout_of(n, pairs, n_hyp);
  if ((int64_t)workspace_bytes < L.bytes)
    return fail(SIFT_ERR_WORKSPACE_TOO_SMALL, "workspace " + std::to_string(workspace_bytes) +
                                                  " bytes, need " + std::to_string(L.bytes));
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_v);
  char* ws = static_cast<char*>(d_workspace);
  VerifyHdr hd;
  hd.ws = ws;
  hd.table = reinterpret_cast<const VerifyEntry*>(ws);
  hd.samples = d_samples;
  hd.n_hyp = n_hyp;
  hd.hyp_groups = (n_hyp + kVerifyHypPerGroup - 1) / kVerifyHypPerGroup;
  hd.sigma_max = (double)sigma_max;
  hd.refine_iters = refine_iters;
  auto hip_fail = [](hipError_t e, const char* what) {
    return fail(SIFT_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  };
  hipError_t e;
  for (int first = 0; first < n; first += kVerifySetupChunk) {
    VerifySetupChunk c;
    std::memset(&c, 0, sizeof c);
    c.first = first;
    c.count = std::min(kVerifySetupChunk, n - first);
    for (int t = 0; t < c.count; ++t) {
      const sift_verify_pair& q = pairs[first + t];
      VerifyEntry& v = c.e[t];
      v.kp_a = q.kp_a;
      v.kp_b = q.kp_b;
      v.matches = q.matches;
      v.n_matches = q.n_matches;
      v.H = q.H;
      v.score = q.score;
      v.n_inliers = q.n_inliers;
      v.best = q.best;
      v.weights = q.weights;
      v.cap = q.cap;
      v.pts = L.pts[first + t];
      v.raw = L.raw[first + t];
      v.norm = L.norm[first + t];
      v.scores = L.scores[first + t];
      v.models = L.models[first + t];
    }
    if ((e = launch_verify_setup(hd, c, stream)) != hipSuccess) return hip_fail(e, "verify setup");
  }
  if ((e = launch_verify_prep(hd, n, stream)) != hipSuccess) return hip_fail(e, "verify prep");
  if ((e = launch_verify_models(hd, n, stream)) != hipSuccess) return hip_fail(e, "verify models");
  if ((e = launch_verify_hyp(hd, n, stream)) != hipSuccess) return hip_fail(e, "verify hypotheses");
  if ((e = launch_verify_refine(hd, n, stream)) != hipSuccess) return hip_fail(e, "verify refine");
  return SIFT_OK;
}

}  // extern "C"
