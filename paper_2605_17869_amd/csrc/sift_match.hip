// gfx950 kernels of descriptor matching (the symmetric ratio test).
//
// Similarities come from the matrix cores: fp16 descriptors, fp32
// accumulation, V_MFMA_F32_16X16X32_F16, with every dot product summed over
// the same fixed sequence of four 32-wide MFMA steps.  Nearest neighbours are
// kept as (value, index) pairs ordered by value, then by smaller index; the
// merge of two such summaries only compares and selects, so the result does
// not depend on the order in which partial summaries meet, and no float
// atomics are used anywhere.  Built with -ffp-contract=off.
#include <hip/hip_runtime.h>

#include <math.h>

#include "sift_device.h"
#include "sift_match.h"

namespace sift {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float float4v __attribute__((ext_vector_type(4)));

constexpr int kMatchDim = 128;
constexpr int kBStride = kMatchDim + 8;   // LDS row stride of the fp16 B tile (halves)

__device__ __forceinline__ Top2 top2_empty() {
  Top2 t;
  t.v1 = -INFINITY;
  t.i1 = 0x7fffffff;
  t.v2 = -INFINITY;
  t.pad = 0;
  return t;
}

__device__ __forceinline__ bool top2_better(float va, int ia, float vb, int ib) {
  return va > vb || (va == vb && ia < ib);
}

// Add (v, i) to t, for an index larger than every index pushed into t
// before: a tie then keeps the earlier entry, so "better" is a strict
// comparison of values, and a displaced first value is never below the second.
__device__ __forceinline__ void top2_push_after(Top2& t, float v, int i) {
  const bool up = v > t.v1;
  t.v2 = up ? t.v1 : fmaxf(t.v2, v);
  t.i1 = up ? i : t.i1;
  t.v1 = up ? v : t.v1;
}

__device__ __forceinline__ Top2 top2_merge(const Top2& a, const Top2& b) {
  Top2 r = top2_empty();
  if (top2_better(a.v1, a.i1, b.v1, b.i1)) {
    r.v1 = a.v1;
    r.i1 = a.i1;
    r.v2 = fmaxf(fmaxf(a.v2, b.v1), b.v2);
  } else {
    r.v1 = b.v1;
    r.i1 = b.i1;
    r.v2 = fmaxf(fmaxf(b.v2, a.v1), a.v2);
  }
  return r;
}

__device__ __forceinline__ Top2 top2_shfl_xor(const Top2& t, int mask) {
  Top2 o;
  o.v1 = __shfl_xor(t.v1, mask, 64);
  o.i1 = __shfl_xor(t.i1, mask, 64);
  o.v2 = __shfl_xor(t.v2, mask, 64);
  o.pad = 0;
  return o;
}

__device__ __forceinline__ int rows_in_use(const int32_t* count, int cap) {
  if (!count) return cap;
  const int c = *count;
  return c < 0 ? 0 : (c < cap ? c : cap);
}

// 8 consecutive descriptor values as fp16 (round to nearest even); rows past
// the set's end read as zeros and never reach a result.
__device__ __forceinline__ half8 load_half8(const float* row, int k, bool valid) {
  half8 h;
  if (valid) {
    const float4 p = *reinterpret_cast<const float4*>(row + k);
    const float4 q = *reinterpret_cast<const float4*>(row + k + 4);
    h[0] = (_Float16)p.x; h[1] = (_Float16)p.y; h[2] = (_Float16)p.z; h[3] = (_Float16)p.w;
    h[4] = (_Float16)q.x; h[5] = (_Float16)q.y; h[6] = (_Float16)q.z; h[7] = (_Float16)q.w;
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) h[e] = (_Float16)0.0f;
  }
  return h;
}

__global__ void k_match_setup(MatchHdr h, MatchSetupChunk c, int n) {
  const int t = threadIdx.x;
  if (t < c.count) const_cast<MatchEntry*>(h.table)[c.first + t] = c.e[t];
  if (t <= c.count && c.first + t <= n) {
    h.row_prefix[c.first + t] = c.row_prefix[t];
    h.col_prefix[c.first + t] = c.col_prefix[t];
  }
}

// ---------------------------------------------------------------------------
// Similarity tiles.  One work-group (4 waves) per (pair, tile of 128 rows of
// a); it walks the tiles of 128 rows of b.  Wave w covers a rows
// 64 (w / 2) .. + 63 and b rows 64 (w % 2) .. + 63 of each tile as 4 x 4
// blocks of 16 x 16, its a fragments held in registers for the whole walk and
// the b tile staged in LDS as fp16.  Lane l supplies a row 16 ta + l % 16 and
// b row 16 tb + l % 16, 8 values each at k = 32 kk + 8 (l / 16), and receives
// s for a rows 16 ta + 4 (l / 16) + r, b row 16 tb + l % 16.
//   rows:    every lane keeps the nearest b seen so far for its 16 a rows;
//            at the end the 16 lanes of a row and the two waves of a row half
//            are merged and written to rowbest.
//   columns: per b tile, each lane summarises its 16 values of a b row, the
//            four lane groups and the two waves holding that b row are
//            merged, and the tile's summary goes to colpart[j][row tile].
__global__ __launch_bounds__(256) void k_match_rows(MatchHdr h, int n) {
  __shared__ __align__(16) _Float16 s_b[kMatchTile * kBStride];
  __shared__ Top2 s_part[2][kMatchTile];
  const int item = blockIdx.x;
  const int p = find_owner(h.row_prefix, n, item);
  const int rt = item - h.row_prefix[p];
  const MatchEntry e = h.table[p];
  const int na = rows_in_use(e.count_a, e.cap_a);
  const int nb = rows_in_use(e.count_b, e.cap_b);
  const int row0 = rt * kMatchTile;
  if (row0 >= na) return;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int li = lane & 15, gq = lane >> 4;
  const int ahalf = wv >> 1, bhalf = wv & 1;
  Top2* rowbest = reinterpret_cast<Top2*>(h.ws + e.rowbest);
  Top2* colpart = reinterpret_cast<Top2*>(h.ws + e.colpart);

  // a fragments: row row0 + 64 ahalf + 16 ta + li, k = 32 kk + 8 gq
  half8 fa[4][4];
#pragma unroll
  for (int ta = 0; ta < 4; ++ta) {
    const int ia = row0 + 64 * ahalf + 16 * ta + li;
    const float* arow = e.desc_a + (int64_t)(ia < na ? ia : 0) * kMatchDim;
    SIFT_CHECK_INDEX(ia < na ? ia : 0, e.cap_a);
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) fa[ta][kk] = load_half8(arow, 32 * kk + 8 * gq, ia < na);
  }
  Top2 rs[4][4];   // [ta][r]: a row row0 + 64 ahalf + 16 ta + 4 gq + r
#pragma unroll
  for (int ta = 0; ta < 4; ++ta)
#pragma unroll
    for (int r = 0; r < 4; ++r) rs[ta][r] = top2_empty();

  const int ctiles = (nb + kMatchTile - 1) / kMatchTile;
  for (int ct = 0; ct < ctiles; ++ct) {
    const int col0 = ct * kMatchTile;
    __syncthreads();   // the previous tile's LDS reads are done
    {
      // b tile into LDS as fp16: thread t converts 64 values of row t / 2
      const int jr = t >> 1, k0 = 64 * (t & 1);
      const int jb = col0 + jr;
      const float* brow = e.desc_b + (int64_t)(jb < nb ? jb : 0) * kMatchDim;
      SIFT_CHECK_INDEX(jb < nb ? jb : 0, e.cap_b);
#pragma unroll
      for (int q = 0; q < 8; ++q)
        *reinterpret_cast<half8*>(&s_b[jr * kBStride + k0 + 8 * q]) =
            load_half8(brow, k0 + 8 * q, jb < nb);
    }
    __syncthreads();
    float4v acc[4][4];
#pragma unroll
    for (int ta = 0; ta < 4; ++ta)
#pragma unroll
      for (int tb = 0; tb < 4; ++tb) acc[ta][tb] = float4v{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      half8 fb[4];
#pragma unroll
      for (int tb = 0; tb < 4; ++tb)
        fb[tb] = *reinterpret_cast<const half8*>(
            &s_b[(64 * bhalf + 16 * tb + li) * kBStride + 32 * kk + 8 * gq]);
#pragma unroll
      for (int ta = 0; ta < 4; ++ta)
#pragma unroll
        for (int tb = 0; tb < 4; ++tb)
          acc[ta][tb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(fa[ta][kk], fb[tb], acc[ta][tb],
                                                               0, 0, 0);
    }
    // rows: this lane's b row of each block (a lane's b rows come in
    // increasing order, over tb and over tiles)
#pragma unroll
    for (int tb = 0; tb < 4; ++tb) {
      const int jb = col0 + 64 * bhalf + 16 * tb + li;
      if (jb < nb) {
#pragma unroll
        for (int ta = 0; ta < 4; ++ta)
#pragma unroll
          for (int r = 0; r < 4; ++r) top2_push_after(rs[ta][r], acc[ta][tb][r], jb);
      }
    }
    // columns: b row 16 tb + li over this wave's 64 a rows (in increasing
    // order over ta and r)
#pragma unroll
    for (int tb = 0; tb < 4; ++tb) {
      Top2 c = top2_empty();
#pragma unroll
      for (int ta = 0; ta < 4; ++ta)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ia = row0 + 64 * ahalf + 16 * ta + 4 * gq + r;
          if (ia < na) top2_push_after(c, acc[ta][tb][r], ia);
        }
      c = top2_merge(c, top2_shfl_xor(c, 16));
      c = top2_merge(c, top2_shfl_xor(c, 32));
      if (gq == 0) s_part[ahalf][64 * bhalf + 16 * tb + li] = c;
    }
    __syncthreads();
    if (t < kMatchTile && col0 + t < nb) {
      SIFT_CHECK_INDEX((int64_t)(col0 + t) * e.rtiles + rt, (int64_t)e.cap_b * e.rtiles);
      colpart[(int64_t)(col0 + t) * e.rtiles + rt] = top2_merge(s_part[0][t], s_part[1][t]);
    }
  }
  // rows: merge the 16 lanes of each row, then the two b halves
#pragma unroll
  for (int ta = 0; ta < 4; ++ta)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      Top2 v = rs[ta][r];
#pragma unroll
      for (int m = 1; m < 16; m <<= 1) v = top2_merge(v, top2_shfl_xor(v, m));
      rs[ta][r] = v;
    }
  __syncthreads();
  if (li == 0) {
#pragma unroll
    for (int ta = 0; ta < 4; ++ta)
#pragma unroll
      for (int r = 0; r < 4; ++r) s_part[bhalf][64 * ahalf + 16 * ta + 4 * gq + r] = rs[ta][r];
  }
  __syncthreads();
  if (t < kMatchTile && row0 + t < na) {
    SIFT_CHECK_INDEX(row0 + t, e.cap_a);
    rowbest[row0 + t] = top2_merge(s_part[0][t], s_part[1][t]);
  }
}

// b_j's nearest in a: merge of its per-row-tile summaries (one thread per j).
__global__ __launch_bounds__(kMatchColBlock) void k_match_cols(MatchHdr h, int n) {
  const int item = blockIdx.x;
  const int p = find_owner(h.col_prefix, n, item);
  const int j = (item - h.col_prefix[p]) * kMatchColBlock + threadIdx.x;
  const MatchEntry e = h.table[p];
  const int na = rows_in_use(e.count_a, e.cap_a);
  const int nb = rows_in_use(e.count_b, e.cap_b);
  if (j >= nb) return;
  const Top2* colpart = reinterpret_cast<const Top2*>(h.ws + e.colpart);
  Top2 c = top2_empty();
  const int used = (na + kMatchTile - 1) / kMatchTile;
  for (int rt = 0; rt < used; ++rt) {
    SIFT_CHECK_INDEX((int64_t)j * e.rtiles + rt, (int64_t)e.cap_b * e.rtiles);
    c = top2_merge(c, colpart[(int64_t)j * e.rtiles + rt]);
  }
  SIFT_CHECK_INDEX(j, e.cap_b);
  reinterpret_cast<Top2*>(h.ws + e.colbest)[j] = c;
}

// Squared distance of unit vectors from a similarity, in fp32.
__device__ __forceinline__ float sq_dist(float s) { return fmaxf(2.0f - 2.0f * s, 0.0f); }

__device__ __forceinline__ bool ratio_pass(const Top2& t, float ratio_sq) {
  const float d1 = sq_dist(t.v1);
  const float d2 = t.v2 == -INFINITY ? 4.0f : sq_dist(t.v2);
  return d1 < ratio_sq * d2;
}

// Mutual nearest neighbours passing both ratio tests, written in ascending
// query order (one work-group per pair, a block scan per 256 rows).
__global__ __launch_bounds__(256) void k_match_emit(MatchHdr h, int n, float ratio_sq) {
  __shared__ int s_wave[4];
  const MatchEntry e = h.table[blockIdx.x];
  const int na = rows_in_use(e.count_a, e.cap_a);
  const int nb = rows_in_use(e.count_b, e.cap_b);
  const Top2* rowbest = reinterpret_cast<const Top2*>(h.ws + e.rowbest);
  const Top2* colbest = reinterpret_cast<const Top2*>(h.ws + e.colbest);
  int base = 0;
  const int rows = nb > 0 ? na : 0;
  for (int i0 = 0; i0 < rows; i0 += 256) {
    const int i = i0 + threadIdx.x;
    bool keep = false;
    Top2 rb = top2_empty();
    if (i < rows) {
      SIFT_CHECK_INDEX(i, e.cap_a);
      rb = rowbest[i];
      const int j = rb.i1;
      if (j >= 0 && j < nb) {
        SIFT_CHECK_INDEX(j, e.cap_b);
        const Top2 cb = colbest[j];
        keep = cb.i1 == i && ratio_pass(rb, ratio_sq) && ratio_pass(cb, ratio_sq);
      }
    }
    int tot;
    const int ex = block_excl_scan256(keep ? 1 : 0, s_wave, &tot);
    if (keep && base + ex < e.capacity) {
      sift_match m;
      m.query = i;
      m.train = rb.i1;
      m.similarity = rb.v1;
      m.distance = sqrtf(sq_dist(rb.v1));
      SIFT_CHECK_INDEX(base + ex, e.capacity);
      e.matches[base + ex] = m;
    }
    base += tot;
  }
  if (threadIdx.x == 0) {
    *e.n_matches = base < e.capacity ? base : e.capacity;
    if (e.n_found) *e.n_found = base;
  }
}

hipError_t launch_match_setup(const MatchHdr& h, const MatchSetupChunk& c, int n,
                              hipStream_t stream) {
  return launch(k_match_setup, dim3(1), dim3(64), stream, h, c, n);
}

hipError_t launch_match_rows(const MatchHdr& h, int n, int grid, hipStream_t stream) {
  return launch(k_match_rows, dim3(grid), dim3(256), stream, h, n);
}

hipError_t launch_match_cols(const MatchHdr& h, int n, int grid, hipStream_t stream) {
  return launch(k_match_cols, dim3(grid), dim3(kMatchColBlock), stream, h, n);
}

hipError_t launch_match_emit(const MatchHdr& h, int n, float ratio_sq, hipStream_t stream) {
  return launch(k_match_emit, dim3(n), dim3(256), stream, h, n, ratio_sq);
}

// The bounds-check counter of this file's kernels (see check_index).
hipError_t bounds_count_match(unsigned long long* count, bool reset) {
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
