// Host runtime of descriptor matching: argument checks, workspace layout and
// the launch sequence (setup, similarity tiles, column reduction, emission).
// Like extraction, it never allocates device memory, copies or synchronises.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/sift.h"
#include "sift_match.h"

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
int cdiv_i(int a, int b) { return (a + b - 1) / b; }

struct MatchLayout {
  int64_t table, row_prefix, col_prefix, header;
  std::vector<int64_t> rowbest, colbest, colpart;
  std::vector<int> rtiles, cblocks;
  int64_t bytes;
};

sift_status check_pairs(int32_t n, const sift_match_pair* pairs) {
  if (n < 1) return fail(SIFT_ERR_INVALID_ARG, "at least one pair");
  if (n > SIFT_MATCH_MAX_PAIRS)
    return fail(SIFT_ERR_TOO_LARGE, "at most " + std::to_string(SIFT_MATCH_MAX_PAIRS) + " pairs");
  if (!pairs) return fail(SIFT_ERR_INVALID_ARG, "null pairs");
  for (int i = 0; i < n; ++i) {
    const sift_match_pair& q = pairs[i];
    const std::string at = "pair " + std::to_string(i) + ": ";
    if (q.cap_a < 0 || q.cap_a > SIFT_MATCH_MAX_ROWS || q.cap_b < 0 || q.cap_b > SIFT_MATCH_MAX_ROWS)
      return fail(SIFT_ERR_INVALID_ARG, at + "caps must be in 0.." + std::to_string(SIFT_MATCH_MAX_ROWS));
    if ((q.cap_a > 0 && !q.desc_a) || (q.cap_b > 0 && !q.desc_b))
      return fail(SIFT_ERR_INVALID_ARG, at + "null descriptors");
    if (q.capacity < 0) return fail(SIFT_ERR_INVALID_ARG, at + "negative capacity");
    if ((q.capacity > 0 && !q.matches) || !q.n_matches)
      return fail(SIFT_ERR_INVALID_ARG, at + "null output");
    if ((reinterpret_cast<uintptr_t>(q.desc_a) | reinterpret_cast<uintptr_t>(q.desc_b)) % 16)
      return fail(SIFT_ERR_INVALID_ARG, at + "descriptors must be 16-byte aligned");
  }
  return SIFT_OK;
}

MatchLayout layout_of(int32_t n, const sift_match_pair* pairs) {
  MatchLayout L;
  int64_t off = 0;
  L.table = off;
  off = align256(off + (int64_t)n * (int64_t)sizeof(MatchEntry));
  L.row_prefix = off;
  off = align256(off + (int64_t)(n + 1) * 4);
  L.col_prefix = off;
  off = align256(off + (int64_t)(n + 1) * 4);
  L.header = off;
  for (int i = 0; i < n; ++i) {
    const int rt = cdiv_i(pairs[i].cap_a, kMatchTile);
    L.rtiles.push_back(rt);
    L.cblocks.push_back(cdiv_i(pairs[i].cap_b, kMatchColBlock));
    L.rowbest.push_back(off);
    off = align256(off + (int64_t)pairs[i].cap_a * (int64_t)sizeof(Top2));
    L.colbest.push_back(off);
    off = align256(off + (int64_t)pairs[i].cap_b * (int64_t)sizeof(Top2));
    L.colpart.push_back(off);
    off = align256(off + (int64_t)pairs[i].cap_b * rt * (int64_t)sizeof(Top2));
  }
  L.bytes = off;
  return L;
}

}  // namespace

extern "C" {

sift_status sift_match_workspace_size(int32_t n, const sift_match_pair* pairs, size_t* bytes) {
  if (!bytes) return fail(SIFT_ERR_INVALID_ARG, "null bytes");
  sift_status st = check_pairs(n, pairs);
  if (st != SIFT_OK) return st;
  *bytes = (size_t)layout_of(n, pairs).bytes;
  return SIFT_OK;
}

sift_status sift_match_batch(int32_t n, const sift_match_pair* pairs, float ratio,
                             void* d_workspace, size_t workspace_bytes, void* stream_v) {
  sift_status st = check_pairs(n, pairs);
  if (st != SIFT_OK) return st;
  if (!(ratio > 0.0f && ratio <= 1.0f)) return fail(SIFT_ERR_INVALID_ARG, "ratio must be in (0, 1]");
  if (!d_workspace) return fail(SIFT_ERR_INVALID_ARG, "null workspace");
  if (reinterpret_cast<uintptr_t>(d_workspace) % 256)
    return fail(SIFT_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  const MatchLayout L = layout_of(n, pairs);
  if ((int64_t)workspace_bytes < L.bytes)
    return fail(SIFT_ERR_WORKSPACE_TOO_SMALL, "workspace " + std::to_string(workspace_bytes) +
                                                  " bytes, need " + std::to_string(L.bytes));
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_v);
  char* ws = static_cast<char*>(d_workspace);
  MatchHdr h;
  h.ws = ws;
  h.table = reinterpret_cast<const MatchEntry*>(ws + L.table);
  h.row_prefix = reinterpret_cast<int*>(ws + L.row_prefix);
  h.col_prefix = reinterpret_cast<int*>(ws + L.col_prefix);

  std::vector<int> rp(n + 1, 0), cp(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    rp[i + 1] = rp[i] + L.rtiles[i];
    cp[i + 1] = cp[i] + L.cblocks[i];
  }
  auto hip_fail = [](hipError_t e, const char* what) {
    return fail(SIFT_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  };
  hipError_t e;
  for (int first = 0; first < n; first += kMatchSetupChunk) {
    MatchSetupChunk c;
    std::memset(&c, 0, sizeof c);
    c.first = first;
    c.count = std::min(kMatchSetupChunk, n - first);
    for (int t = 0; t < c.count; ++t) {
      const sift_match_pair& q = pairs[first + t];
      MatchEntry& m = c.e[t];
      m.desc_a = q.desc_a;
      m.count_a = q.count_a;
      m.desc_b = q.desc_b;
      m.count_b = q.count_b;
      m.matches = q.matches;
      m.n_matches = q.n_matches;
      m.n_found = q.n_found;
      m.cap_a = q.cap_a;
      m.cap_b = q.cap_b;
      m.capacity = q.capacity;
      m.rtiles = L.rtiles[first + t];
      m.rowbest = L.rowbest[first + t];
      m.colbest = L.colbest[first + t];
      m.colpart = L.colpart[first + t];
    }
    for (int t = 0; t <= c.count; ++t) {
      c.row_prefix[t] = rp[first + t];
      c.col_prefix[t] = cp[first + t];
    }
    if ((e = launch_match_setup(h, c, n, stream)) != hipSuccess) return hip_fail(e, "match setup");
  }
  if (rp[n] > 0 && (e = launch_match_rows(h, n, rp[n], stream)) != hipSuccess)
    return hip_fail(e, "match similarity");
  if (cp[n] > 0 && (e = launch_match_cols(h, n, cp[n], stream)) != hipSuccess)
    return hip_fail(e, "match columns");
  const float ratio_sq = (float)((double)ratio * (double)ratio);
  if ((e = launch_match_emit(h, n, ratio_sq, stream)) != hipSuccess) return hip_fail(e, "match emit");
  return SIFT_OK;
}

}  // extern "C"
