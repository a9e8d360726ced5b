// Internal definitions of geometric verification shared by the host runtime
// and the gfx950 kernels: the on-device pair table, workspace layout and
// launch helpers.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

#include "../../include/sift.h"

namespace sift {

constexpr int kVerifySetupChunk = 16;  // pair-table entries per setup launch
constexpr int kVerifyHypPerGroup = 4;  // hypotheses per work-group (one per wave)
constexpr int kVerifyModelBlock = 64;  // hypotheses per work-group of the model kernel (one per lane)

// One pair as the kernels see it (written by the setup kernel).
struct VerifyEntry {
  const sift_keypoint* kp_a;
  const sift_keypoint* kp_b;
  const sift_match* matches;
  const int32_t* n_matches;
  double* H;
  double* score;
  int32_t* n_inliers;
  int32_t* best;
  float* weights;
  int32_t cap;
  int32_t pad;
  int64_t pts;       // double [cap][4]: normalised (xa, ya, xb, yb)
  int64_t raw;       // float4 [cap]: pixel (xa, ya, xb, yb), the keypoints' fp32 values
  int64_t norm;      // double [8]: sa, txa, tya, sb, txb, tyb, n (as double), unused
  int64_t scores;    // double [n_hyp]
  int64_t models;    // double [n_hyp][9]: each hypothesis' model (NaN when there is none)
};

struct VerifyHdr {
  char* ws;
  const VerifyEntry* table;   // [n]
  const float* samples;       // [n_hyp][4] numbers in [0, 1)
  int n_hyp;
  int hyp_groups;             // work-groups of hypotheses per pair
  double sigma_max;
  int refine_iters;
};

struct VerifySetupChunk {
  int first;
  int count;
  VerifyEntry e[kVerifySetupChunk];
};

hipError_t launch_verify_setup(const VerifyHdr& h, const VerifySetupChunk& c, hipStream_t stream);
hipError_t launch_verify_prep(const VerifyHdr& h, int n, hipStream_t stream);
hipError_t launch_verify_models(const VerifyHdr& h, int n, hipStream_t stream);
hipError_t launch_verify_hyp(const VerifyHdr& h, int n, hipStream_t stream);
hipError_t launch_verify_refine(const VerifyHdr& h, int n, hipStream_t stream);

}  // namespace sift
