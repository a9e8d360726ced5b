// Gaussian pyramid kernel of the SIFT extraction path (gfx950).
//
// Built with -ffp-contract=off: every fused multiply-add below is written out
// explicitly, so the level values are the same whatever the launch shape.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "sift_device.h"
#include "sift_launch.h"

namespace sift {

// ---------------------------------------------------------------------------
// Gaussian level: separable blur, one work-group of 256 threads per strip of
// kTileW = 192 output columns and up to `th` rows of one image.  The group
// walks down its strip in steps of B = kBlurRows rows.  Vertical pass first:
// thread t owns source column x0 - R + t (192 + 2R <= 256 of them) and keeps
// a sliding window of 2R + B source rows of that column in registers, so each
// source pixel is loaded once per strip and the next step's rows are fetched
// while the current step computes; it writes B vertically blurred values to
// an LDS block (two blocks, alternating, so one barrier per step suffices).
// Horizontal pass: 3 tasks per thread, each reading 4 + 2R values of a row
// from the block and writing 4 consecutive outputs; tasks run along the rows
// so a wave's stores cover contiguous memory.
//
// Each output is
//   acc = 0; for t = 0..2R: acc = fma(g[t], in[y - R + t], acc)
// down the column for the vertical pass and the same along the row for the
// horizontal pass, whatever the strip or chunk shape.  Levels are held
// relative to mid-grey (L - 0.5): the blur is linear with unit-sum taps, so
// this changes no difference of levels and keeps fp32 rounding error
// proportional to |L - 0.5|.
//
// Work-groups are dealt round-robin to the 8 XCDs, each with its own L2; the
// grid is a multiple of 8 and group b takes work item (b % 8) * (grid / 8) +
// b / 8, so every XCD sweeps one contiguous run of items and neighbouring
// strips find their shared halo columns in the same L2.

// LDS row stride of at least n floats with stride % 8 == 4: lanes that read
// 16 bytes each from 8 consecutive rows then touch 8 distinct bank groups.
constexpr int lds_stride4(int n) {
  return ((n + 3) / 4 * 4) % 8 == 4 ? (n + 3) / 4 * 4 : (n + 3) / 4 * 4 + 4;
}

// UP selects the source of level 0 of the upsampled octave (bilinear 2x of
// the input image); otherwise a source pixel is src[y * sp + (x << csh)] - bias.
// ST is the storage of source and destination level: 0 fp32 -> fp32, 1 fp32
// -> fp16 (the first level of the second octave under fp16 storage), 2 fp16 ->
// fp16; arithmetic is fp32 throughout, fp16 stores round to nearest even.
template <int R, bool UP, int ST>
__global__ __launch_bounds__(kBlurThreads) void k_blur(BlurArgs a) {
  constexpr int TW = kTileW;          // output columns of the strip
  constexpr int NT = kBlurThreads;
  constexpr int B = kBlurRows;        // rows per step
  constexpr int HB = 4;               // horizontal outputs per task
  constexpr int NQ = TW / HB;         // horizontal tasks per row
  constexpr int NREP = NQ * kBlurRows / kBlurThreads;   // tasks per thread
  constexpr int WI = TW + 2 * R;      // source columns of the strip
  constexpr int SS = lds_stride4(WI);
  constexpr int W = 2 * R + B;        // vertical window (rows)
  constexpr int NH = (2 * R + HB + 3) / 4;   // float4 reads per horizontal task
  static_assert(NREP * NT == NQ * B, "whole horizontal tasks per thread");
  static_assert(WI <= NT, "one source column per thread");
  static_assert(!UP || ST == 0, "the input image is fp32");
  constexpr bool S16 = ST == 2, D16 = ST >= 1;
  constexpr uint32_t ES_S = S16 ? 2u : 4u, ES_D = D16 ? 2u : 4u;   // bytes per element
  __shared__ __align__(16) float s_v[2][B * SS];

  const int* tp = a.tile_prefix;
  const int per_xcd = gridDim.x / kXcds;
  const int item = (blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds;
  if (item >= tp[a.n]) return;
  const int img = find_owner(tp, a.n, item);
  const int local = item - tp[img];
  const ImgEntry e = a.table[img];
  const LayoutCfg lc = layout_cfg(a.p);
  const int k = a.k;
  const OctView ov = octave_view(e.h, e.w, lc, k);
  const int hk = ov.h, wk = ov.w, pk = ov.pitch;
  const int strips = cdiv(wk, TW);
  const int cy = local / strips;
  const int sx = local - cy * strips;
  const int x0 = sx * TW, y0 = cy * a.th;
  const int y1 = min(y0 + a.th, hk);
  gchar* gdst = reinterpret_cast<gchar*>(as_global(level_ptr(a.ws, e, ov, a.dst_level)));
  const int t = threadIdx.x;
  const int mode = a.mode;

  // ---- the thread's source column (threads past the strip's columns repeat
  // the last one; their values are never read)
  const int xs = x0 - R + min(t, WI - 1);
  const int xc = mirror(xs, wk);
  const float* src;
  int64_t sp;          // source row pitch in bytes
  int csh;             // source column = xc << csh
  float bias = 0.0f;
  if (UP || mode == kSrcImage) {
    src = e.src;
    sp = 4 * (int64_t)e.src_pitch;
    csh = 0;
    bias = kCentre;
  } else if (mode == kSrcLevel) {
    src = level_ptr(a.ws, e, ov, a.dst_level - 1);
    sp = ES_S * (int64_t)pk;
    csh = 0;
  } else {
    // level s of the previous octave at every second row and column
    const OctView pv = octave_view(e.h, e.w, lc, k - 1);
    src = level_ptr(a.ws, e, pv, a.p.s);
    sp = 2 * ES_S * (int64_t)pv.pitch;
    csh = 1;
  }
  const gchar* gsrc = uniform_ptr(reinterpret_cast<const gchar*>(as_global(src)));
  const uint32_t bo = (uint32_t)(xc << csh) * ES_S;
  // bilinear 2x upsampling: U[y][x] = I(y/2, x/2), the sample past the last
  // row or column clamped to it; computed on centred values
  const uint32_t ua = (uint32_t)(xc >> 1) * 4u, ub = (uint32_t)min((xc >> 1) + 1, e.w - 1) * 4u;
  const bool uo = xc & 1;

  // source value of (mirrored) row y at the thread's column; loads are not
  // under a branch, so none forces an early wait
  auto fetch = [&](int y) -> float {
    if (UP) {
      const int ya = y >> 1, yb = min(ya + 1, e.h - 1);
      const gchar* r0 = uniform_ptr(gsrc + ya * sp);
      const gchar* r1 = uniform_ptr(gsrc + ((y & 1) ? yb : ya) * sp);
      const float va = load_at(r0, ua), vb = load_at(r0, ub);
      const float vc = load_at(r1, ua), vd = load_at(r1, ub);
      float top = va - bias, bot = vc - bias;
      top = uo ? (top + (vb - bias)) * 0.5f : top;
      bot = uo ? (bot + (vd - bias)) * 0.5f : bot;
      return (y & 1) ? (top + bot) * 0.5f : top;
    } else {
      const float v = load_lv<S16>(uniform_ptr(gsrc + y * sp), bo) - bias;
      // an fp32 level feeding an fp16 octave: its subsampled rows are that
      // octave's level 0, which is stored in fp16, and level 1 is blurred from
      // the stored values
      return ST == 1 ? (float)(_Float16)v : v;
    }
  };
  // n consecutive rows from image row ybase (mirrored at the borders)
  // upsampled rows ybase .. ybase + n - 1 away from the border: the
  // horizontally interpolated source rows h(j) are loaded once each
  // (2 loads, not 4 per output row) and combined as fetch() does
  auto fetch_rows_up = [&](float* dst, int ybase, auto n_c, auto odd_c) {
    constexpr int n = decltype(n_c)::value;
    constexpr int odd = decltype(odd_c)::value;   // parity of ybase
    constexpr int NS = n / 2 + 2;
    const int s0 = ybase >> 1;
    float hrow[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const gchar* rp = uniform_ptr(gsrc + min(s0 + i, e.h - 1) * sp);
      const float va = load_at(rp, ua), vb = load_at(rp, ub);
      const float top = va - bias;
      hrow[i] = uo ? (top + (vb - bias)) * 0.5f : top;
    }
#pragma unroll
    for (int r = 0; r < n; ++r) {
      const int ia = (r + odd) >> 1;          // (ybase + r) / 2 - s0
      dst[r] = ((r + odd) & 1) ? (hrow[ia] + hrow[ia + 1]) * 0.5f : hrow[ia];
    }
  };
  auto fetch_rows = [&](float* dst, int ybase, auto n_c) {
    constexpr int n = decltype(n_c)::value;
    if (ybase >= 0 && ybase + n <= hk) {
      if (UP) {
        if (ybase & 1)
          fetch_rows_up(dst, ybase, n_c, std::integral_constant<int, 1>());
        else
          fetch_rows_up(dst, ybase, n_c, std::integral_constant<int, 0>());
      } else {
#pragma unroll
        for (int r = 0; r < n; ++r) dst[r] = fetch(ybase + r);
      }
    } else {
#pragma unroll
      for (int r = 0; r < n; ++r) dst[r] = fetch(mirror(ybase + r, hk));
    }
  };

  // window w[i] = source row y0 + m B - R + i of the thread's column
  float w[W];
  float pre[B];
  fetch_rows(w, y0 - R, std::integral_constant<int, W>());
  gchar* l0 = nullptr;
  if (!UP && mode == kSrcDown)
    l0 = uniform_ptr(reinterpret_cast<gchar*>(as_global(level_ptr(a.ws, e, ov, 0))));
  const bool own_col = t >= R && t < R + TW && xs < wk;
  const int64_t pkb = ES_D * (int64_t)pk;
  const int M = cdiv(y1 - y0, B);     // steps

  for (int m = 0; m < M; ++m) {
    const int yb = y0 + m * B;
    if (m + 1 < M) fetch_rows(pre, yb + B + R, std::integral_constant<int, B>());
    if (!UP && mode == kSrcDown && own_col) {
      // the subsampled base is this octave's level 0: written by the chunk
      // that owns the row and the strip that owns the column
#pragma unroll
      for (int r = 0; r < B; ++r)
        if (yb + r < y1) store_lv<D16>(uniform_ptr(l0 + (yb + r) * pkb), (uint32_t)xs * ES_D, w[R + r]);
    }
    // vertical pass into LDS block m & 1 (threads past the strip's source
    // columns have nothing to write: their row offset would run past SS)
    float* blk = s_v[m & 1];
    if (t < WI) {
#pragma unroll
      for (int r = 0; r < B; ++r) {
        float acc = 0.0f;
#pragma unroll
        for (int q = 0; q <= 2 * R; ++q) acc = __fmaf_rn(a.taps[q], w[r + q], acc);
        blk[r * SS + t] = acc;
      }
    }
    __syncthreads();
    // horizontal pass: tasks of 4 consecutive outputs, numbered along the
    // rows so that consecutive lanes write consecutive 16-byte pieces
#pragma unroll
    for (int rep = 0; rep < NREP; ++rep) {
      const int task = rep * NT + t;
      const int hr = task / NQ, hq = task - (task / NQ) * NQ;
      const float4* in = reinterpret_cast<const float4*>(&blk[hr * SS + hq * HB]);
      float acc[HB];
#pragma unroll
      for (int j = 0; j < HB; ++j) acc[j] = 0.0f;
#pragma unroll
      for (int j4 = 0; j4 < NH; ++j4) {
        const float4 q = in[j4];
        const float qv[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int jj = 4 * j4 + u;
#pragma unroll
          for (int j = 0; j < HB; ++j) {
            const int tt = jj - j;
            if (tt >= 0 && tt <= 2 * R) acc[j] = __fmaf_rn(a.taps[tt], qv[u], acc[j]);
          }
        }
      }
      const int y = yb + hr;
      const int xo = x0 + hq * HB;
      if (y < y1) {
        gchar* row = gdst + y * pkb;   // rows differ across the wave
        if (xo + HB <= wk) {
          // consecutive dwords: the compiler merges them into one wide store
#pragma unroll
          for (int j = 0; j < HB; ++j) store_lv<D16>(row, (uint32_t)(xo + j) * ES_D, acc[j]);
        } else {
#pragma unroll
          for (int j = 0; j < HB; ++j)
            if (xo + j < wk) store_lv<D16>(row, (uint32_t)(xo + j) * ES_D, acc[j]);
        }
      }
    }
    // slide the window by B rows
#pragma unroll
    for (int i = 0; i < 2 * R; ++i) w[i] = w[i + B];
#pragma unroll
    for (int r = 0; r < B; ++r) w[2 * R + r] = pre[r];
  }
}

typedef void (*BlurKernel)(BlurArgs);

#define SIFT_BLUR_CASE(RR)                                                   \
  case RR:                                                                   \
    return up ? k_blur<RR, true, 0>                                          \
              : (st == 0 ? k_blur<RR, false, 0>                              \
                         : (st == 1 ? k_blur<RR, false, 1> : k_blur<RR, false, 2>));

static BlurKernel blur_kernel(int radius, bool up, int st) {
  switch (radius) {
    SIFT_BLUR_CASE(1) SIFT_BLUR_CASE(2) SIFT_BLUR_CASE(3) SIFT_BLUR_CASE(4)
    SIFT_BLUR_CASE(5) SIFT_BLUR_CASE(6) SIFT_BLUR_CASE(7) SIFT_BLUR_CASE(8)
    SIFT_BLUR_CASE(9) SIFT_BLUR_CASE(10) SIFT_BLUR_CASE(11) SIFT_BLUR_CASE(12)
    SIFT_BLUR_CASE(13) SIFT_BLUR_CASE(14) SIFT_BLUR_CASE(15) SIFT_BLUR_CASE(16)
    SIFT_BLUR_CASE(17) SIFT_BLUR_CASE(18) SIFT_BLUR_CASE(19) SIFT_BLUR_CASE(20)
    SIFT_BLUR_CASE(21) SIFT_BLUR_CASE(22) SIFT_BLUR_CASE(23) SIFT_BLUR_CASE(24)
    default: return nullptr;
  }
}
#undef SIFT_BLUR_CASE

hipError_t launch_blur(const BlurArgs& a, int radius, int grid, hipStream_t stream) {
  if (a.st < 0 || a.st > 2 || (a.st != 0 && (a.mode == kSrcUpsample || a.mode == kSrcImage)))
    return hipErrorInvalidValue;
  BlurKernel fn = blur_kernel(radius, a.mode == kSrcUpsample, a.st);
  if (!fn || a.th % kBlurRows != 0) return hipErrorInvalidValue;
  return launch(fn, dim3(grid), dim3(kBlurThreads), stream, a);
}

}  // namespace sift
