// Replayable batches (HIP graphs of the batched launch sequence) and the
// blur chunk-height autotuner.
#include <hip/hip_runtime.h>

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
