// Replayable batches (HIP graphs of the batched launch sequence) and the
// blur chunk-height autotuner.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/sift.h"

namespace sift {
void set_last_error(const std::string& msg);
void set_capturing(bool on);
}  // namespace sift

using sift::set_last_error;

struct sift_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

sift_status hip_fail(hipError_t e, const char* what) {
  set_last_error(std::string(what) + ": " + hipGetErrorString(e));
  return SIFT_ERR_HIP;
}

}  // namespace

extern "C" {

sift_status sift_graph_create(sift_handle* h, int32_t n, const float* const* d_images,
                              const int32_t* heights, const int32_t* widths,
                              const int64_t* pitches, void* d_workspace, size_t workspace_bytes,
                              const sift_output* outs, sift_graph** out) {
  if (!out) {
    set_last_error("null argument");
    return SIFT_ERR_INVALID_ARG;
  }
  *out = nullptr;
  hipStream_t cap = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "capture stream");
  e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    hipStreamDestroy(cap);
    return hip_fail(e, "begin capture");
  }
  sift::set_capturing(true);
  const sift_status st = sift_extract_batch(h, n, d_images, heights, widths, pitches, d_workspace,
                                            workspace_bytes, outs, cap);
  sift::set_capturing(false);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(cap, &graph);
  hipStreamDestroy(cap);
  if (st != SIFT_OK) {
    if (graph) hipGraphDestroy(graph);
    return st;   // argument errors: nothing was recorded
  }
  if (e != hipSuccess) return hip_fail(e, "end capture");
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    hipGraphDestroy(graph);
    return hip_fail(e, "instantiate");
  }
  sift_graph* g = new sift_graph();
  g->graph = graph;
  g->exec = exec;
  *out = g;
  return SIFT_OK;
}

sift_status sift_graph_launch(sift_graph* g, void* stream) {
  if (!g) {
    set_last_error("null graph");
    return SIFT_ERR_INVALID_ARG;
  }
  const hipError_t e = hipGraphLaunch(g->exec, reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "graph launch");
  return SIFT_OK;
}

sift_status sift_graph_destroy(sift_graph* g) {
  if (!g) return SIFT_OK;
  hipError_t e = hipGraphExecDestroy(g->exec);
  const hipError_t e2 = hipGraphDestroy(g->graph);
  delete g;
  if (e == hipSuccess) e = e2;
  if (e != hipSuccess) return hip_fail(e, "graph destroy");
  return SIFT_OK;
}

sift_status sift_autotune_batch(const sift_params* p, int32_t n, const float* const* d_images,
                                const int32_t* heights, const int32_t* widths,
                                const int64_t* pitches, void* d_workspace,
                                size_t workspace_bytes, const sift_output* outs, void* stream_v,
                                int32_t warmup, int32_t reps, int32_t* best_tile_rows,
                                float* ms) {
  if (!p || !best_tile_rows) {
    set_last_error("null argument");
    return SIFT_ERR_INVALID_ARG;
  }
  if (warmup < 0 || reps < 1) {
    set_last_error("warmup must be >= 0 and reps >= 1");
    return SIFT_ERR_INVALID_ARG;
  }
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_v);
  const int32_t candidates[4] = {64, 128, 256, 512};
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  if (e != hipSuccess) {
    if (a) hipEventDestroy(a);
    return hip_fail(e, "autotune events");
  }
  sift_status st = SIFT_OK;
  float best = -1.0f;
  for (int c = 0; c < 4 && st == SIFT_OK; ++c) {
    sift_params q = *p;
    q.tile_rows = candidates[c];
    sift_handle* h = nullptr;
    st = sift_create(&q, &h);
    if (st != SIFT_OK) break;
    for (int i = 0; i < warmup && st == SIFT_OK; ++i)
      st = sift_extract_batch(h, n, d_images, heights, widths, pitches, d_workspace,
                              workspace_bytes, outs, stream);
    if (st == SIFT_OK && (e = hipEventRecord(a, stream)) != hipSuccess)
      st = hip_fail(e, "autotune event");
    for (int i = 0; i < reps && st == SIFT_OK; ++i)
      st = sift_extract_batch(h, n, d_images, heights, widths, pitches, d_workspace,
                              workspace_bytes, outs, stream);
    float t = 0.0f;
    if (st == SIFT_OK && (e = hipEventRecord(b, stream)) != hipSuccess)
      st = hip_fail(e, "autotune event");
    if (st == SIFT_OK && (e = hipEventSynchronize(b)) != hipSuccess)
      st = hip_fail(e, "autotune wait");
    if (st == SIFT_OK && (e = hipEventElapsedTime(&t, a, b)) != hipSuccess)
      st = hip_fail(e, "autotune timing");
    sift_destroy(h);
    if (st != SIFT_OK) break;
    t /= (float)reps;
    if (ms) ms[c] = t;
    if (best < 0.0f || t < best) {
      best = t;
      *best_tile_rows = candidates[c];
    }
  }
  hipEventDestroy(a);
  hipEventDestroy(b);
  return st;
}

}  // extern "C"

namespace {

// FNV-1a over bytes: a stable digest for cache keys.
uint64_t fnv1a(const void* data, size_t n, uint64_t h = 1469598103934665603ull) {
  const unsigned char* p = static_cast<const unsigned char*>(data);
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 1099511628211ull;
  }
  return h;
}

// Cache key: the device (name, architecture, compute units), the settings
// with the two tuned fields cleared, and the batch shape (image count and
// total input pixels rounded to two significant figures, so batches of
// similar work share an entry).
std::string tune_key(const sift_params* p, int32_t n, const int32_t* heights, const int32_t* widths) {
  int dev = 0;
  hipDeviceProp_t prop;
  std::memset(&prop, 0, sizeof prop);
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    std::snprintf(prop.name, sizeof prop.name, "unknown");
  sift_params q = *p;
  q.tile_rows = 0;
  q.n_streams = 0;
  q.blur_chain = 0;
  q.detect_waves = 0;
  double px = 0.0;
  for (int i = 0; i < n; ++i) px += (double)heights[i] * widths[i];
  const double mag = px > 0 ? std::pow(10.0, std::floor(std::log10(px)) - 1.0) : 1.0;
  const long long px2 = (long long)(std::ceil(px / mag) * mag);
  std::string name(prop.name);
  for (char& c : name)
    if (c == ' ' || c == '\t') c = '_';
  std::ostringstream k;
  k << name << "/" << prop.gcnArchName << "/cu" << prop.multiProcessorCount << "/p"
    << std::hex << fnv1a(&q, sizeof q) << std::dec << "/n" << n << "/px" << px2;
  std::string out = k.str();
  for (char& c : out)
    if (c == ' ' || c == '\t') c = '_';
  return out;
}

bool cache_lookup(const char* path, const std::string& key, sift_tuning* t) {
  if (!path) return false;
  std::ifstream f(path);
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {   // the last entry for a key wins
    std::istringstream is(line);
    std::string k;
    sift_tuning v;
    std::memset(&v, 0, sizeof v);
    if (is >> k >> v.tile_rows >> v.n_streams >> v.blur_chain >> v.detect_waves >> v.ms &&
        k == key) {
      *t = v;
      found = true;
    }
  }
  return found;
}

}  // namespace

extern "C" {

sift_status sift_autotune_workspace_size(const sift_params* p, int32_t n, const int32_t* heights,
                                         const int32_t* widths, size_t* bytes) {
  if (!p || !bytes) {
    set_last_error("null argument");
    return SIFT_ERR_INVALID_ARG;
  }
  const int32_t streams[4] = {1, 2, 4, 8};
  size_t most = 0;
  for (int q = 0; q < 4; ++q) {
    sift_params pp = *p;
    pp.n_streams = streams[q];
    sift_handle* h = nullptr;
    sift_status st = sift_create(&pp, &h);
    if (st != SIFT_OK) return st;
    size_t b = 0;
    st = sift_batch_workspace_size(h, n, heights, widths, &b);
    sift_destroy(h);
    if (st != SIFT_OK) return st;
    if (b > most) most = b;
  }
  *bytes = most;
  return SIFT_OK;
}

sift_status sift_autotune(const sift_params* p, int32_t n, const float* const* d_images,
                          const int32_t* heights, const int32_t* widths, const int64_t* pitches,
                          void* d_workspace, size_t workspace_bytes, const sift_output* outs,
                          void* stream_v, int32_t warmup, int32_t reps, int32_t as_graph,
                          const char* cache_path, sift_tuning* out) {
  if (!p || !out || !heights || !widths) {
    set_last_error("null argument");
    return SIFT_ERR_INVALID_ARG;
  }
  if (warmup < 0 || reps < 1) {
    set_last_error("warmup must be >= 0 and reps >= 1");
    return SIFT_ERR_INVALID_ARG;
  }
  if (n < 1) {
    set_last_error("batch size must be >= 1");
    return SIFT_ERR_INVALID_ARG;
  }
  std::memset(out, 0, sizeof *out);
  const std::string key =
      tune_key(p, n, heights, widths) + (as_graph ? "/graph" : "/eager") + "/v3";
  if (cache_lookup(cache_path, key, out)) {
    out->from_cache = 1;
    return SIFT_OK;
  }
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_v);
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  if (e != hipSuccess) {
    if (a) hipEventDestroy(a);
    return hip_fail(e, "autotune events");
  }
  const int32_t rows[4] = {64, 128, 256, 512};
  const int32_t streams[4] = {1, 2, 4, 8};
  sift_status st = SIFT_OK;
  float best = -1.0f;
  // times one candidate; a split the workspace cannot hold is skipped
  auto try_one = [&](int32_t tile_rows, int32_t n_streams, int32_t chain, int32_t waves) {
    sift_params pp = *p;
    pp.tile_rows = tile_rows;
    pp.n_streams = n_streams;
    pp.blur_chain = chain;
    pp.detect_waves = waves;
    sift_handle* h = nullptr;
    st = sift_create(&pp, &h);
    if (st != SIFT_OK) return;
    size_t need = 0;
    st = sift_batch_workspace_size(h, n, heights, widths, &need);
    if (st == SIFT_OK && need > workspace_bytes) {
      sift_destroy(h);
      return;
    }
    // one extraction of the batch: the launch sequence, or a replay of it
    // recorded as a graph
    sift_graph* gr = nullptr;
    if (st == SIFT_OK && as_graph)
      st = sift_graph_create(h, n, d_images, heights, widths, pitches, d_workspace,
                             workspace_bytes, outs, &gr);
    auto once = [&]() {
      return gr ? sift_graph_launch(gr, stream)
                : sift_extract_batch(h, n, d_images, heights, widths, pitches, d_workspace,
                                     workspace_bytes, outs, stream);
    };
    for (int i = 0; i < warmup && st == SIFT_OK; ++i) st = once();
    if (st == SIFT_OK && (e = hipEventRecord(a, stream)) != hipSuccess)
      st = hip_fail(e, "autotune event");
    for (int i = 0; i < reps && st == SIFT_OK; ++i) st = once();
    float t = 0.0f;
    if (st == SIFT_OK && (e = hipEventRecord(b, stream)) != hipSuccess)
      st = hip_fail(e, "autotune event");
    if (st == SIFT_OK && (e = hipEventSynchronize(b)) != hipSuccess)
      st = hip_fail(e, "autotune wait");
    if (st == SIFT_OK && (e = hipEventElapsedTime(&t, a, b)) != hipSuccess)
      st = hip_fail(e, "autotune timing");
    if (gr) {
      if (st == SIFT_OK) st = sift_graph_destroy(gr);
      else sift_graph_destroy(gr);
    }
    sift_destroy(h);
    if (st != SIFT_OK) return;
    t /= (float)reps;
    out->n_tried += 1;
    if (best < 0.0f || t < best) {
      best = t;
      out->tile_rows = tile_rows;
      out->n_streams = n_streams;
      out->blur_chain = chain;
      out->detect_waves = waves;
      out->ms = t;
    }
  };
  // chunk height x sub-batch count at the caller's chain and detection
  // settings, then the other chain lengths at the best of those (the
  // pyramid's levels per launch barely interact with the split), then the
  // other waves per detection work-group at the best so far
  const int32_t chain0 = p->blur_chain == 0 ? 2 : p->blur_chain;
  const int32_t waves0 = p->detect_waves == 0 ? 4 : p->detect_waves;
  for (int c = 0; c < 4 && st == SIFT_OK; ++c)
    for (int q = 0; q < 4 && st == SIFT_OK; ++q)
      if (streams[q] <= n) try_one(rows[c], streams[q], chain0, waves0);
  if (st == SIFT_OK && best >= 0.0f) {
    const int32_t r0 = out->tile_rows, s0 = out->n_streams;
    for (int32_t chain = 1; chain <= 3 && st == SIFT_OK; ++chain)
      if (chain != chain0) try_one(r0, s0, chain, waves0);
  }
  if (st == SIFT_OK && best >= 0.0f) {
    const int32_t r0 = out->tile_rows, s0 = out->n_streams, c0 = out->blur_chain;
    try_one(r0, s0, c0, waves0 == 4 ? 8 : 4);
  }
  hipEventDestroy(a);
  hipEventDestroy(b);
  if (st != SIFT_OK) return st;
  if (cache_path) {
    std::ofstream f(cache_path, std::ios::app);
    if (f)
      f << key << " " << out->tile_rows << " " << out->n_streams << " " << out->blur_chain << " "
        << out->detect_waves << " " << out->ms << "\n";
  }
  return SIFT_OK;
}

}  // extern "C"
