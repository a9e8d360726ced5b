// Gaussian pyramid kernel of the SIFT extraction path (gfx950).
//
// Built with -ffp-contract=off: every fused multiply-add below is written out
// explicitly, so the level values are the same whatever the launch shape.
#include <hip/hip_runtime.h>

#include "sift_device.h"
#include "sift_launch.h"

namespace sift {

// ---------------------------------------------------------------------------
// Gaussian level: separable blur, one work-group per strip of kTileW columns
// and up to `th` rows of one image.  The group walks down its strip in steps
// of B = kBlurRows rows: it stages B source rows (plus an R-column mirrored
// halo) in LDS, runs the horizontal pass over them into a ring of horizontally
// blurred rows, and runs the vertical pass over the ring to emit B output
// rows.  Each source row is staged once per strip and each horizontal result
// computed once, so apart from the 2R-row lead-in at the top of a chunk there
// is no halo recomputation.  Source rows of the next step are fetched into
// registers while the current step computes.
//
// Each output is
//   acc = 0; for t = 0..2R: acc = fma(g[t], in[x - R + t], acc)
// for the horizontal pass and the same along columns for the vertical pass,
// whatever the strip or chunk shape.  Levels are held relative to mid-grey
// (L - 0.5): the blur is linear with unit-sum taps, so this changes no
// difference of levels and keeps fp32 rounding error proportional to |L - 0.5|.
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
// the input image); otherwise a source pixel is src[y * sp + x * sx] - bias.
template <int R, bool UP>
__global__ __launch_bounds__(kTileW) void k_blur(BlurArgs a) {
  constexpr int TW = kTileW;          // output columns; one thread per column
  constexpr int B = kBlurRows;        // rows per step
  constexpr int HB = 16;              // horizontal outputs per thread
  constexpr int WI = TW + 2 * R;      // staged source columns
  constexpr int SS = lds_stride4(WI);
  constexpr int RS = lds_stride4(TW);
  constexpr int NB = (2 * R + B - 1) / B + 1;   // ring blocks of B rows
  constexpr int NH = (2 * R + HB + 3) / 4;      // float4 reads per horizontal task
  static_assert((TW / HB) * B == TW, "one horizontal task per thread");
  static_assert(TW + 2 * R <= 2 * TW, "two staged columns per thread");
  __shared__ __align__(16) float s_in[B * SS];
  __shared__ __align__(16) float s_ring[NB * B * RS];

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

  // ---- per-thread source columns (staged columns t and t + TW)
  const bool has1 = t + TW < WI;
  const int xc0 = mirror(x0 - R + t, wk);
  const int xc1 = has1 ? mirror(x0 - R + t + TW, wk) : xc0;
  const float* src;
  int64_t sp;          // source row pitch in bytes
  int csh;             // source column = staged column << csh
  float bias = 0.0f;
  if (UP || mode == kSrcImage) {
    src = e.src;
    sp = 4 * (int64_t)e.src_pitch;
    csh = 0;
    bias = kCentre;
  } else if (mode == kSrcLevel) {
    src = level_ptr(a.ws, e, ov, a.dst_level - 1);
    sp = 4 * (int64_t)pk;
    csh = 0;
  } else {
    // level s of the previous octave at every second row and column
    const OctView pv = octave_view(e.h, e.w, lc, k - 1);
    src = level_ptr(a.ws, e, pv, a.p.s);
    sp = 8 * (int64_t)pv.pitch;
    csh = 1;
  }
  const gchar* gsrc = uniform_ptr(reinterpret_cast<const gchar*>(as_global(src)));
  const uint32_t bo0 = (uint32_t)(xc0 << csh) * 4u, bo1 = (uint32_t)(xc1 << csh) * 4u;
  // bilinear 2x upsampling: U[y][x] = I(y/2, x/2), the sample past the last
  // row or column clamped to it; computed on centred values
  const uint32_t ua0 = (uint32_t)(xc0 >> 1) * 4u, ub0 = (uint32_t)min((xc0 >> 1) + 1, e.w - 1) * 4u;
  const uint32_t ua1 = (uint32_t)(xc1 >> 1) * 4u, ub1 = (uint32_t)min((xc1 >> 1) + 1, e.w - 1) * 4u;
  const bool uo0 = xc0 & 1, uo1 = xc1 & 1;

  // H-row h (h = 0 is image row y0 - R) belongs to block h / B
  const int M = cdiv(y1 - y0, B);     // output steps
  const int NBLK = M + NB - 1;        // horizontal blocks
  float v0[B], v1[B];
  // Loads are issued unconditionally (lanes without a second column reload
  // their first) and blended afterwards, so no load sits under a branch that
  // would force an early wait for it.
  auto fetch_row = [&](int y, int r) {
    if (UP) {
      const int ya = y >> 1, yb = min(ya + 1, e.h - 1);
      const gchar* r0 = uniform_ptr(gsrc + ya * sp);
      const gchar* r1 = uniform_ptr(gsrc + ((y & 1) ? yb : ya) * sp);
      const float a0 = load_at(r0, ua0), b0 = load_at(r0, ub0);
      const float c0 = load_at(r1, ua0), d0 = load_at(r1, ub0);
      const float a1 = load_at(r0, ua1), b1 = load_at(r0, ub1);
      const float c1 = load_at(r1, ua1), d1 = load_at(r1, ub1);
      float top0 = a0 - bias, bot0 = c0 - bias, top1 = a1 - bias, bot1 = c1 - bias;
      top0 = uo0 ? (top0 + (b0 - bias)) * 0.5f : top0;
      bot0 = uo0 ? (bot0 + (d0 - bias)) * 0.5f : bot0;
      top1 = uo1 ? (top1 + (b1 - bias)) * 0.5f : top1;
      bot1 = uo1 ? (bot1 + (d1 - bias)) * 0.5f : bot1;
      v0[r] = (y & 1) ? (top0 + bot0) * 0.5f : top0;
      v1[r] = (y & 1) ? (top1 + bot1) * 0.5f : top1;
    } else {
      const gchar* row = uniform_ptr(gsrc + y * sp);
      v0[r] = load_at(row, bo0) - bias;
      v1[r] = load_at(row, bo1) - bias;
    }
  };
  auto load_block = [&](int beta) {
    const int ybase = y0 - R + beta * B;
    if (ybase >= 0 && ybase + B <= hk) {
#pragma unroll
      for (int r = 0; r < B; ++r) fetch_row(ybase + r, r);
    } else {
#pragma unroll
      for (int r = 0; r < B; ++r) fetch_row(mirror(ybase + r, hk), r);
    }
  };
  gchar* l0 = nullptr;
  if (!UP && mode == kSrcDown)
    l0 = uniform_ptr(reinterpret_cast<gchar*>(as_global(level_ptr(a.ws, e, ov, 0))));
  const int xend = min(x0 + TW, wk);
  const int64_t pkb = 4 * (int64_t)pk;
  auto store_block = [&](int beta) {
#pragma unroll
    for (int r = 0; r < B; ++r) {
      s_in[r * SS + t] = v0[r];
      if (has1) s_in[r * SS + t + TW] = v1[r];
    }
    if (!UP && mode == kSrcDown) {
      // the subsampled base is this octave's level 0: written by the chunk
      // that owns the row and the strip that owns the column
      const int xa = x0 - R + t, xb = xa + TW;
      for (int r = 0; r < B; ++r) {
        const int y = y0 - R + beta * B + r;
        if (y >= y0 && y < y1) {
          gchar* row = uniform_ptr(l0 + y * pkb);
          if (xa >= x0 && xa < xend) store_at(row, (uint32_t)xa * 4u, v0[r]);
          if (has1 && xb < xend) store_at(row, (uint32_t)xb * 4u, v1[r]);
        }
      }
    }
  };

  // horizontal pass of the staged block into ring slot `slot`
  const int hr = t % B, hq = t / B;
  auto hpass = [&](int slot) {
    const float4* in = reinterpret_cast<const float4*>(&s_in[hr * SS + hq * HB]);
    float acc[HB];
#pragma unroll
    for (int m = 0; m < HB; ++m) acc[m] = 0.0f;
#pragma unroll
    for (int j4 = 0; j4 < NH; ++j4) {
      const float4 q = in[j4];
      const float qv[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int j = 4 * j4 + u;
#pragma unroll
        for (int m = 0; m < HB; ++m) {
          const int tt = j - m;
          if (tt >= 0 && tt <= 2 * R) acc[m] = __fmaf_rn(a.taps[tt], qv[u], acc[m]);
        }
      }
    }
    float4* out = reinterpret_cast<float4*>(&s_ring[(slot * B + hr) * RS + hq * HB]);
#pragma unroll
    for (int m = 0; m < HB / 4; ++m)
      out[m] = make_float4(acc[4 * m], acc[4 * m + 1], acc[4 * m + 2], acc[4 * m + 3]);
  };

  // vertical pass: output rows y0 + mB .. + B - 1 at column x0 + t; H-row
  // mB + j lives in block m + j / B, i.e. ring slot (m + j / B) % NB
  const bool col_ok = x0 + t < wk;
  auto vpass = [&](int m) {
    const float* base[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) base[q] = &s_ring[((m + q) % NB) * B * RS + t];
    float acc[B];
#pragma unroll
    for (int i = 0; i < B; ++i) acc[i] = 0.0f;
#pragma unroll
    for (int j = 0; j < B + 2 * R; ++j) {
      const float v = base[j / B][(j % B) * RS];
#pragma unroll
      for (int i = 0; i < B; ++i) {
        const int tt = j - i;
        if (tt >= 0 && tt <= 2 * R) acc[i] = __fmaf_rn(a.taps[tt], v, acc[i]);
      }
    }
    if (col_ok) {
      const int yb = y0 + m * B;
      const uint32_t off = (uint32_t)(x0 + t) * 4u;
#pragma unroll
      for (int i = 0; i < B; ++i)
        if (yb + i < y1) store_at(uniform_ptr(gdst + (yb + i) * pkb), off, acc[i]);
    }
  };

  // lead-in: blocks 0 .. NB - 2 hold H-rows y0 - R .. y0 - R + (NB - 1) B - 1
  load_block(0);
  for (int beta = 0; beta < NB - 1; ++beta) {
    if (beta > 0) __syncthreads();     // previous horizontal pass done with s_in
    store_block(beta);
    __syncthreads();
    load_block(beta + 1);              // NBLK >= NB, so block beta + 1 exists
    hpass(beta);
  }
  // step m: block m + NB - 1 into slot (m + NB - 1) % NB, then outputs of step m
  for (int m = 0; m < M; ++m) {
    const int beta = m + NB - 1;
    __syncthreads();                   // s_in free; ring slot of block m - 1 free
    store_block(beta);
    __syncthreads();
    if (beta + 1 < NBLK) load_block(beta + 1);
    hpass(beta % NB);
    __syncthreads();
    vpass(m);
  }
}

typedef void (*BlurKernel)(BlurArgs);

#define SIFT_BLUR_CASE(RR) \
  case RR: return up ? k_blur<RR, true> : k_blur<RR, false>;

static BlurKernel blur_kernel(int radius, bool up) {
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
  BlurKernel fn = blur_kernel(radius, a.mode == kSrcUpsample);
  if (!fn || a.th % kBlurRows != 0) return hipErrorInvalidValue;
  return launch(fn, dim3(grid), dim3(kTileW), stream, a);
}

}  // namespace sift
