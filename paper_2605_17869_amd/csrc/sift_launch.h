// Launch helpers exported by the kernel translation unit to the host runtime.
#pragma once

#include <hip/hip_runtime.h>

#include "sift_internal.h"

namespace sift {

struct SetupChunk {
  int first;
  int count;
  ImgEntry e[kSetupChunk];
};

// Each helper enqueues one kernel on `stream` and returns the launch status.
hipError_t launch_setup(const HdrPtrs& hp, const SetupChunk& c, hipStream_t stream);
hipError_t launch_finalize(const HdrPtrs& hp, int n, const DevParams& p, hipStream_t stream);
// Gaussian level: `radius` selects the instantiation; taps in a.taps[0..2R].
hipError_t launch_blur(const BlurArgs& a, int radius, int grid, hipStream_t stream);
// Chained levels lv0 .. lv0 + n_levels - 1 of one octave from the source that
// `mode` names; st as for BlurArgs.  chain_supported tells whether a kernel
// for that (mode, st, radii) run is built.
bool chain_supported(int mode, int st, int n_levels, const int* radii);
hipError_t launch_chain(const ChainArgs& a, int mode, int st, int n_levels, const int* radii,
                        int grid, hipStream_t stream);
// waves: per work-group, 4 or 8 (anything else: hipErrorInvalidValue)
hipError_t launch_detect(char* ws, const HdrPtrs& hp, int n, const DevParams& p, int waves,
                         int grid, hipStream_t stream);
hipError_t launch_band_scan(char* ws, const HdrPtrs& hp, int n, const DevParams& p,
                         hipStream_t stream);
hipError_t launch_emit(char* ws, const HdrPtrs& hp, int n, const DevParams& p, int grid,
                         hipStream_t stream);
// Per-image prefix of min(counter, limit) into the header (which = 0 candidates, 1 keypoints).
hipError_t launch_img_prefix(char* ws, const HdrPtrs& hp, int n, const DevParams& p, int which,
                             hipStream_t stream);
hipError_t launch_refine(char* ws, const HdrPtrs& hp, int n, const DevParams& p, int grid,
                         hipStream_t stream);
hipError_t launch_orient(char* ws, const HdrPtrs& hp, int n, const DevParams& p, int grid,
                         hipStream_t stream);
hipError_t launch_ori_scan(char* ws, const HdrPtrs& hp, int n, const DevParams& p,
                         hipStream_t stream);
hipError_t launch_describe(char* ws, const HdrPtrs& hp, int n, const DevParams& p, int grid,
                         hipStream_t stream);

// Bounds-check counters of the kernels of each source file (libraries
// built with -DSIFT_DEBUG_BOUNDS; hipErrorNotSupported otherwise): the count
// of out-of-range accesses since the last reset, zeroed after reading when
// `reset`.
hipError_t bounds_count_blur(unsigned long long* count, bool reset);
hipError_t bounds_count_kernels(unsigned long long* count, bool reset);
hipError_t bounds_count_match(unsigned long long* count, bool reset);
hipError_t bounds_count_verify(unsigned long long* count, bool reset);

}  // namespace sift
