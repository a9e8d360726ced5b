// Internal definitions of descriptor matching shared by the host runtime and
// the gfx950 kernels: the on-device pair table, workspace layout and launch
// helpers.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

#include "../../include/sift.h"

namespace sift {

constexpr int kMatchTile = 128;      // rows of either set per similarity tile
constexpr int kMatchColBlock = 256;  // columns per block of the column reduction
constexpr int kMatchSetupChunk = 24; // pair-table entries per setup launch

// Running nearest / second-nearest of one row or column: the best candidate
// (largest value, smallest index among equals) and the largest value among
// the others.  An empty set holds (-inf, INT32_MAX, -inf).
struct Top2 {
  float v1;
  int32_t i1;
  float v2;
  int32_t pad;
};

// One pair as the kernels see it (written by the setup kernel).
struct MatchEntry {
  const float* desc_a;
  const int32_t* count_a;
  const float* desc_b;
  const int32_t* count_b;
  sift_match* matches;
  int32_t* n_matches;
  int32_t* n_found;
  int32_t cap_a, cap_b, capacity;
  int32_t rtiles;          // row tiles of kMatchTile rows that cap_a needs
  int64_t rowbest;         // Top2 [cap_a]: a_i's nearest in b
  int64_t colbest;         // Top2 [cap_b]: b_j's nearest in a
  int64_t colpart;         // Top2 [cap_b][rtiles]: b_j's nearest within one row tile
};

// Device addresses of the header arrays (computed on the host).
struct MatchHdr {
  char* ws;
  const MatchEntry* table;   // [n]
  int* row_prefix;           // [n + 1] row tiles before each pair
  int* col_prefix;           // [n + 1] column blocks before each pair
};

struct MatchSetupChunk {
  int first;
  int count;
  MatchEntry e[kMatchSetupChunk];
  int row_prefix[kMatchSetupChunk + 1];
  int col_prefix[kMatchSetupChunk + 1];
};

hipError_t launch_match_setup(const MatchHdr& h, const MatchSetupChunk& c, int n,
                              hipStream_t stream);
hipError_t launch_match_rows(const MatchHdr& h, int n, int grid, hipStream_t stream);
hipError_t launch_match_cols(const MatchHdr& h, int n, int grid, hipStream_t stream);
hipError_t launch_match_emit(const MatchHdr& h, int n, float ratio_sq, hipStream_t stream);

}  // namespace sift
