// Gaussian pyramid kernels of the SIFT extraction path (gfx950).
//
// Built with -ffp-contract=off: every fused multiply-add below is written out
// explicitly, so the level values are the same whatever the launch shape.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "sift_device.h"
#include "sift_launch.h"

namespace sift {

// ---------------------------------------------------------------------------
// Tap arithmetic.  Every blurred value, in either pass and in either kernel
// below, is formed from its 2R + 1 inputs x[-R..R] in one fixed order,
// outermost pair first:
//   acc = 0; for t = R..1: acc = fma(g_t, x[-t] + x[t], acc); acc = fma(g_0, x[0], acc)
// Addition is commutative, so the value at a position mirrored across an
// image border (reflect-101, the border rule of every level) is bit-identical
// to the value at the position itself once its inputs are mirrored too.  A
// pass may therefore compute rows and columns beyond the image from mirrored
// source data and obtain exactly the values the border rule assigns there;
// the chained kernel computes its halo that way.
//
// gt(t): tap at distance t; x(j), j = 0..2R: the inputs, centre at j = R.
template <int R, typename GT, typename X>
__device__ __forceinline__ float gauss_pairs(GT gt, X x) {
  float acc = 0.0f;
#pragma unroll
  for (int t = R; t >= 1; --t) acc = __fmaf_rn(gt(t), x(R - t) + x(R + t), acc);
  return __fmaf_rn(gt(0), x(R), acc);
}

// LDS row stride of at least n floats with stride % 8 == 4: lanes that read
// 16 bytes each from 8 consecutive rows then touch 8 distinct bank groups.
constexpr int lds_stride4(int n) {
  return ((n + 3) / 4 * 4) % 8 == 4 ? (n + 3) / 4 * 4 : (n + 3) / 4 * 4 + 4;
}

// ---------------------------------------------------------------------------
// Source of a launch's first vertical pass, one column per thread: the input
// image (bilinearly upsampled 2x when UP), the previous level of the octave,
// or level s of the previous octave at every second row and column (the
// octave's level 0).  Values are centred (L - 0.5, the input shifted by
// kCentre): the blur is linear with unit-sum taps, so this changes no
// difference of levels and keeps fp32 rounding error proportional to
// |L - 0.5|.  ST is the storage of source and destination level: 0 fp32 ->
// fp32, 1 fp32 -> fp16 (the first level of the second octave under fp16
// storage), 2 fp16 -> fp16.  With ST = 1 the source values are rounded to
// fp16 as they are read: they form that octave's level 0, which is stored in
// fp16, and the next level is blurred from the stored values.
template <bool UP, int ST>
struct BlurSource {
  static constexpr bool S16 = ST == 2;
  static constexpr uint32_t ES_S = S16 ? 2u : 4u;   // bytes per source element
  const gchar* gsrc;
  int64_t sp;        // source row pitch, bytes
  uint32_t bo;       // byte offset of the thread's column within a source row
  uint32_t ua, ub;   // upsampling: byte offsets of the two input columns
  bool uo;           // upsampling: odd output column
  float bias;
  int in_h;          // input rows (upsampling)
  int hk;            // rows of the octave (mirroring)
#ifdef SIFT_DEBUG_BOUNDS
  Span span;         // the memory the source lies in (bounds checks)
#endif

  // xc: the thread's column of the octave, already mirrored into [0, wk)
  __device__ __forceinline__ void init(char* ws, const ImgEntry& e, const LayoutCfg& lc,
                                       const OctView& ov, int k, int first_level, int mode,
                                       int s, int xc) {
    const float* src;
    int csh = 0;   // source column = xc << csh
    bias = 0.0f;
#ifdef SIFT_DEBUG_BOUNDS
    span = (UP || mode == kSrcImage) ? input_span(e) : region_span(ws, e, lc);
#endif
    if (UP || mode == kSrcImage) {
      src = e.src;
      sp = 4 * (int64_t)e.src_pitch;
      bias = kCentre;
    } else if (mode == kSrcLevel) {
      src = level_ptr(ws, e, ov, first_level - 1);
      sp = ES_S * (int64_t)ov.pitch;
    } else {
      const OctView pv = octave_view(e.h, e.w, lc, k - 1);
      src = level_ptr(ws, e, pv, s);
      sp = 2 * ES_S * (int64_t)pv.pitch;
      csh = 1;
    }
    gsrc = uniform_ptr(reinterpret_cast<const gchar*>(as_global(src)));
    bo = (uint32_t)(xc << csh) * ES_S;
    // bilinear 2x upsampling: U[y][x] = I(y/2, x/2), the sample past the last
    // row or column clamped to it; computed on centred values
    ua = (uint32_t)(xc >> 1) * 4u;
    ub = (uint32_t)min((xc >> 1) + 1, e.w - 1) * 4u;
    uo = xc & 1;
    in_h = e.h;
    hk = ov.h;
  }

  // source value of row y (in [0, hk)) at the thread's column; loads are not
  // under a branch, so none forces an early wait
  __device__ __forceinline__ float fetch(int y) const {
    if constexpr (UP) {
      const int ya = y >> 1, yb = min(ya + 1, in_h - 1);
      const gchar* r0 = uniform_ptr(gsrc + ya * sp);
      const gchar* r1 = uniform_ptr(gsrc + ((y & 1) ? yb : ya) * sp);
      SIFT_CHECK_IN(span, r0 + ua, 4);
      SIFT_CHECK_IN(span, r1 + ub, 4);
      const float va = load_at(r0, ua), vb = load_at(r0, ub);
      const float vc = load_at(r1, ua), vd = load_at(r1, ub);
      float top = va - bias, bot = vc - bias;
      top = uo ? (top + (vb - bias)) * 0.5f : top;
      bot = uo ? (bot + (vd - bias)) * 0.5f : bot;
      return (y & 1) ? (top + bot) * 0.5f : top;
    } else {
      SIFT_CHECK_IN(span, gsrc + y * sp + bo, ES_S);
      const float v = load_lv<S16>(uniform_ptr(gsrc + y * sp), bo) - bias;
      return ST == 1 ? round_f16(v) : v;
    }
  }

  // upsampled rows ybase .. ybase + n - 1 away from the border: the
  // horizontally interpolated input rows are loaded once each (2 loads, not 4
  // per output row) and combined as fetch() does; ODD is the parity of ybase
  template <int n, int ODD>
  __device__ __forceinline__ void rows_up(float* dst, int ybase) const {
    constexpr int NS = n / 2 + 2;
    const int s0 = ybase >> 1;
    float hrow[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const gchar* rp = uniform_ptr(gsrc + min(s0 + i, in_h - 1) * sp);
      SIFT_CHECK_IN(span, rp + ua, 4);
      SIFT_CHECK_IN(span, rp + ub, 4);
      const float va = load_at(rp, ua), vb = load_at(rp, ub);
      const float top = va - bias;
      hrow[i] = uo ? (top + (vb - bias)) * 0.5f : top;
    }
#pragma unroll
    for (int r = 0; r < n; ++r) {
      const int ia = (r + ODD) >> 1;          // (ybase + r) / 2 - s0
      dst[r] = ((r + ODD) & 1) ? (hrow[ia] + hrow[ia + 1]) * 0.5f : hrow[ia];
    }
  }

  // n consecutive rows from octave row ybase (mirrored at the borders)
  template <int n>
  __device__ __forceinline__ void rows(float* dst, int ybase) const {
    if (ybase >= 0 && ybase + n <= hk) {
      if constexpr (UP) {
        if (ybase & 1)
          rows_up<n, 1>(dst, ybase);
        else
          rows_up<n, 0>(dst, ybase);
      } else {
#pragma unroll
        for (int r = 0; r < n; ++r) dst[r] = fetch(ybase + r);
      }
    } else {
#pragma unroll
      for (int r = 0; r < n; ++r) dst[r] = fetch(mirror(ybase + r, hk));
    }
  }
};

// ---------------------------------------------------------------------------
// One Gaussian level: separable blur, one work-group of 256 threads per strip
// of kTileW = 192 output columns and up to `th` rows of one image.  The group
// walks down its strip in steps of B = kBlurRows rows.  Vertical pass first:
// thread t owns source column x0 - R + t (192 + 2R <= 256 of them) and keeps
// a sliding window of 2R + B source rows of that column in registers, so each
// source pixel is loaded once per strip and the next step's rows are fetched
// while the current step computes; it writes B vertically blurred values to
// an LDS block (two blocks, alternating, so one barrier per step suffices).
// Horizontal pass: 3 tasks per thread, each reading 4 + 2R values of a row
// from the block and writing 4 consecutive outputs; tasks run along the rows
// so a wave's stores cover contiguous memory.  Both passes use the tap order
// of gauss_pairs.
//
// Work-groups are dealt round-robin to the 8 XCDs, each with its own L2; the
// grid is a multiple of 8 and group b takes work item (b % 8) * (grid / 8) +
// b / 8, so every XCD sweeps one contiguous run of items and neighbouring
// strips find their shared halo columns in the same L2.
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
  constexpr bool D16 = ST >= 1;
  constexpr uint32_t ES_D = D16 ? 2u : 4u;   // bytes per destination element
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

  // the thread's source column (threads past the strip's columns repeat the
  // last one; their values are never read)
  const int xs = x0 - R + min(t, WI - 1);
  BlurSource<UP, ST> src;
  src.init(a.ws, e, lc, ov, k, a.dst_level, mode, a.p.s, mirror(xs, wk));
  SIFT_SPAN(rs, region_span(a.ws, e, lc));
  auto gt = [&](int q) { return a.taps[R + q]; };

  // window w[i] = source row y0 + m B - R + i of the thread's column
  float w[W];
  float pre[B];
  src.template rows<W>(w, y0 - R);
  gchar* l0 = nullptr;
  if (!UP && mode == kSrcDown)
    l0 = uniform_ptr(reinterpret_cast<gchar*>(as_global(level_ptr(a.ws, e, ov, 0))));
  const bool own_col = t >= R && t < R + TW && xs < wk;
  const int64_t pkb = ES_D * (int64_t)pk;
  const int M = cdiv(y1 - y0, B);     // steps

  for (int m = 0; m < M; ++m) {
    const int yb = y0 + m * B;
    if (m + 1 < M) src.template rows<B>(pre, yb + B + R);
    if (!UP && mode == kSrcDown && own_col) {
      // the subsampled base is this octave's level 0: written by the chunk
      // that owns the row and the strip that owns the column
#pragma unroll
      for (int r = 0; r < B; ++r)
        if (yb + r < y1) {
          SIFT_CHECK_IN(rs, l0 + (yb + r) * pkb + (uint32_t)xs * ES_D, ES_D);
          store_lv<D16>(uniform_ptr(l0 + (yb + r) * pkb), (uint32_t)xs * ES_D, w[R + r]);
        }
    }
    // vertical pass into LDS block m & 1 (threads past the strip's source
    // columns have nothing to write: their row offset would run past SS)
    float* blk = s_v[m & 1];
    if (t < WI) {
#pragma unroll
      for (int r = 0; r < B; ++r)
        blk[r * SS + t] = gauss_pairs<R>(gt, [&](int j) { return w[r + j]; });
    }
    __syncthreads();
    // horizontal pass: tasks of 4 consecutive outputs, numbered along the
    // rows so that consecutive lanes write consecutive 16-byte pieces
#pragma unroll
    for (int rep = 0; rep < NREP; ++rep) {
      const int task = rep * NT + t;
      const int hr = task / NQ, hq = task - (task / NQ) * NQ;
      const float4* in = reinterpret_cast<const float4*>(&blk[hr * SS + hq * HB]);
      float vv[4 * NH];
#pragma unroll
      for (int j4 = 0; j4 < NH; ++j4) {
        const float4 q = in[j4];
        vv[4 * j4] = q.x;
        vv[4 * j4 + 1] = q.y;
        vv[4 * j4 + 2] = q.z;
        vv[4 * j4 + 3] = q.w;
      }
      float acc[HB];
#pragma unroll
      for (int j = 0; j < HB; ++j) acc[j] = gauss_pairs<R>(gt, [&](int q) { return vv[j + q]; });
      const int y = yb + hr;
      const int xo = x0 + hq * HB;
      if (y < y1) {
        gchar* row = gdst + y * pkb;   // rows differ across the wave
        if (xo + HB <= wk) {
          // xo is a multiple of 4 and rows start 256-byte aligned
          SIFT_CHECK_IN(rs, row + (uint32_t)xo * ES_D, HB * ES_D);
          store4_lv<D16>(row, (uint32_t)xo * ES_D, acc);
        } else {
#pragma unroll
          for (int j = 0; j < HB; ++j)
            if (xo + j < wk) {
              SIFT_CHECK_IN(rs, row + (uint32_t)(xo + j) * ES_D, ES_D);
              store_lv<D16>(row, (uint32_t)(xo + j) * ES_D, acc[j]);
            }
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

// ---------------------------------------------------------------------------
// Chained levels: N consecutive levels of an octave, each of radius R_i <=
// B / 2 (B = kChainB rows per step), in one pass over a strip of kTileW
// output columns, so the levels between the first and the last are never read
// back from memory.  Per level the thread keeps two B-row blocks of its
// input column in registers, the newest rows and the B rows before them;
// with 2 R_i <= B they hold every row a block of B outputs needs, and the
// window slides by swapping the roles of the blocks (the step loop is
// unrolled by two), without register moves.
//
// Rows.  In step g level i produces rows A_i(g) .. A_i(g) + B - 1,
// A_i(g) = y0 - Q + Lag_i + g B with Lag_i = R_{i+1} + ... + R_{N-1}: every
// level runs Lag_i rows ahead of the last, so the rows it has just produced
// are exactly the newest block of the next level's window.  Level i's output
// is valid from step i on (both blocks of its window valid), and
// Q = max_i (2 Lag_i + i B) puts level i's first valid row at or above
// y0 - Lag_i, the first row the levels after it use.  Rows outside the chunk
// are computed but not stored; rows outside the image come from mirrored
// source rows and, by the tap order of gauss_pairs, equal the mirrored values
// bit for bit.
//
// Columns.  Thread t owns column x0 - HS + t in every level.  Level i produces
// columns [x0 - HL_i, x0 + kTileW + HL_i), with HL_{N-1} = 0 and HL_{i-1} =
// HL_i + R_i rounded up to a multiple of 4 (every horizontal task writes 4
// aligned columns), and HS = HL_0 + R_0 rounded up likewise.
//
// Per level and step: vertical pass from the window into s_v (at an offset
// that makes every horizontal task's float4 reads aligned), barrier,
// horizontal pass from s_v with its rows stored to the level and, for all but
// the last level, written to s_h, barrier; each thread then appends its
// column of s_h to the next level's window.  Every value is the one the
// one-level kernel computes (same tap order, same passes, and the same fp16
// rounding of what the next level reads under fp16 storage).
template <int... Rs>
struct ChainGeom {
  static constexpr int N = sizeof...(Rs);
  static constexpr int r(int i) {
    constexpr int v[] = {Rs...};
    return v[i];
  }
  static constexpr int lag(int i) {
    int s = 0;
    for (int j = i + 1; j < N; ++j) s += r(j);
    return s;
  }
  static constexpr int hl(int i) {
    int h = 0;
    for (int j = N - 1; j > i; --j) h = (h + r(j) + 3) / 4 * 4;
    return h;
  }
  static constexpr int halo() { return (hl(0) + r(0) + 3) / 4 * 4; }
  static constexpr int q() {
    int m = 0;
    for (int i = 0; i < N; ++i) {
      const int v = 2 * lag(i) + i * kChainB;
      m = v > m ? v : m;
    }
    return m;
  }
  static constexpr bool fits() {
    for (int i = 0; i < N; ++i)
      if (r(i) < 1 || r(i) > kChainMaxR || 2 * r(i) > kChainB) return false;
    return N >= 2 && N <= kChainMaxLevels && kTileW + 2 * halo() <= kBlurThreads;
  }
};

template <int MODE, int ST, int... Rs>
__global__ __launch_bounds__(kBlurThreads, 2) void k_chain(ChainArgs a) {
  using Geo = ChainGeom<Rs...>;
  constexpr int N = Geo::N;
  constexpr int B = kChainB;
  constexpr int TW = kTileW;
  constexpr int NT = kBlurThreads;
  constexpr int HS = Geo::halo();
  constexpr int Q = Geo::q();
  constexpr int SS = lds_stride4(NT + 8);   // the V offset (< 4) and float4 over-read fit
  constexpr bool UP = MODE == kSrcUpsample;
  constexpr bool D16 = ST >= 1;
  constexpr uint32_t ES_D = D16 ? 2u : 4u;
  static_assert(Geo::fits(), "chain radii or halo out of range");
  static_assert(!UP || ST == 0, "the input image is fp32");
  __shared__ __align__(16) float s_v[B * SS];   // vertical-pass results
  __shared__ __align__(16) float s_h[B * SS];   // a level's rows for the next level

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
  const int t = threadIdx.x;
  const int xs = x0 - HS + t;          // the thread's column in every level
  BlurSource<UP, ST> src;
  src.init(a.ws, e, lc, ov, k, a.lv0, MODE, a.p.s, mirror(xs, wk));
  SIFT_SPAN(rs, region_span(a.ws, e, lc));
  const int64_t pkb = ES_D * (int64_t)pk;
  const bool own_col = xs >= x0 && xs < x0 + TW && xs < wk;
  gchar* l0 = nullptr;
  if (MODE == kSrcDown)
    l0 = uniform_ptr(reinterpret_cast<gchar*>(as_global(level_ptr(a.ws, e, ov, 0))));
  gchar* dst[N];
#pragma unroll
  for (int i = 0; i < N; ++i)
    dst[i] = uniform_ptr(reinterpret_cast<gchar*>(as_global(level_ptr(a.ws, e, ov, a.lv0 + i))));

  // win[i][b]: the two blocks of level i's input column; in step g block
  // g & 1 holds the newest rows
  float win[N][2][B];
  {
    const int a0 = y0 - Q + Geo::lag(0);   // A_0(0)
    src.template rows<B>(win[0][1], a0 + Geo::r(0) - B);
    src.template rows<B>(win[0][0], a0 + Geo::r(0));
  }
  const int G = (y1 - y0 + Q + B - 1) / B;   // steps: the last level reaches y1 - 1

  auto level = [&](auto i_c, auto p_c, int g) {
    constexpr int I = decltype(i_c)::value;
    constexpr int P = decltype(p_c)::value;   // block of the newest rows
    constexpr int R = Geo::r(I);
    constexpr int HL = Geo::hl(I);
    constexpr int NQ = (TW + 2 * HL) / 4;       // horizontal tasks per row
    constexpr int NREP = (B * NQ + NT - 1) / NT;
    constexpr int SH = R & 3;                   // s_v offset: aligned task reads
    constexpr int NH = (2 * R + 4 + 3) / 4;     // float4 reads per task
    // every LDS access stays in its row and the columns each level reads were
    // produced by the level before it (or fetched, for the first)
    static_assert((HS - HL - R + SH) >= 0 && (HS - HL - R + SH) % 4 == 0, "aligned task reads");
    static_assert(HS - HL - R + SH + 4 * (NQ - 1) + 4 * NH <= SS, "task reads inside a row");
    static_assert(NT - 1 + SH < SS, "vertical-pass writes inside a row");
    static_assert((HS - HL) % 4 == 0 && HS - HL + 4 * NQ <= SS, "handed-over rows inside a row");
    static_assert(HS + TW + HL + R <= NT, "input columns are threads' columns");
    static_assert(I == 0 || Geo::hl(I == 0 ? 0 : I - 1) >= HL + R, "input columns were produced");
    static_assert(Q >= 2 * Geo::lag(I) + I * B, "first valid row at or above y0 - Lag");
    const int ai = y0 - Q + Geo::lag(I) + g * B;   // A_I(g)
    if constexpr (I > 0) {
      if (g < I - 1) return;   // level I - 1 produced nothing valid yet
      // the rows level I - 1 produced in this step: the newest block
#pragma unroll
      for (int r = 0; r < B; ++r) win[I][P][r] = s_h[r * SS + t];
      if (g < I) return;       // the older block is not valid yet
    }
    auto gt = [&](int q) { return a.g[I][q]; };
    // vertical pass: output row ai + r uses rows ai + r - R .. ai + r + R,
    // window positions B - 2R + r .. B + r (the older block first)
#pragma unroll
    for (int r = 0; r < B; ++r) {
      s_v[r * SS + t + SH] = gauss_pairs<R>(gt, [&](int j) {
        const int c = B - 2 * R + r + j;
        return c < B ? win[I][P ^ 1][c] : win[I][P][c - B];
      });
    }
    if constexpr (I == 0) {
      if (MODE == kSrcDown && own_col) {
        // the newest source rows are the octave's level 0 (the subsampled
        // base): each row is newest in exactly one step
#pragma unroll
        for (int r = 0; r < B; ++r) {
          const int y = ai + R + r;
          if (y >= y0 && y < y1) {
            SIFT_CHECK_IN(rs, l0 + y * pkb + (uint32_t)xs * ES_D, ES_D);
            store_lv<D16>(uniform_ptr(l0 + y * pkb), (uint32_t)xs * ES_D, win[0][P][r]);
          }
        }
      }
      // the next step's newest rows, into the block this step has retired
      if (g + 1 < G) src.template rows<B>(win[0][P ^ 1], ai + B + R);
    }
    __syncthreads();
    // horizontal pass: tasks of 4 aligned columns along the rows
#pragma unroll
    for (int rep = 0; rep < NREP; ++rep) {
      const int task = rep * NT + t;
      if (task < B * NQ) {
        const int hr = task / NQ, hq = task - (task / NQ) * NQ;
        const float4* in =
            reinterpret_cast<const float4*>(&s_v[hr * SS + HS - HL - R + SH + 4 * hq]);
        float vv[4 * NH];
#pragma unroll
        for (int j4 = 0; j4 < NH; ++j4) {
          const float4 q = in[j4];
          vv[4 * j4] = q.x;
          vv[4 * j4 + 1] = q.y;
          vv[4 * j4 + 2] = q.z;
          vv[4 * j4 + 3] = q.w;
        }
        float acc[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] = gauss_pairs<R>(gt, [&](int q) { return vv[j + q]; });
        const int y = ai + hr;
        const int xo = x0 - HL + 4 * hq;
        if (y >= y0 && y < y1 && xo >= x0 && xo < x0 + TW) {
          gchar* row = dst[I] + y * pkb;
          if (xo + 4 <= wk) {
            SIFT_CHECK_IN(rs, row + (uint32_t)xo * ES_D, 4 * ES_D);
            store4_lv<D16>(row, (uint32_t)xo * ES_D, acc);   // aligned: xo % 4 == 0
          } else {
#pragma unroll
            for (int j = 0; j < 4; ++j)
              if (xo + j < wk) {
                SIFT_CHECK_IN(rs, row + (uint32_t)(xo + j) * ES_D, ES_D);
                store_lv<D16>(row, (uint32_t)(xo + j) * ES_D, acc[j]);
              }
          }
        }
        if constexpr (I + 1 < N) {
          // what the next level reads is the stored value
          float4 hv;
          hv.x = D16 ? round_f16(acc[0]) : acc[0];
          hv.y = D16 ? round_f16(acc[1]) : acc[1];
          hv.z = D16 ? round_f16(acc[2]) : acc[2];
          hv.w = D16 ? round_f16(acc[3]) : acc[3];
          *reinterpret_cast<float4*>(&s_h[hr * SS + HS - HL + 4 * hq]) = hv;
        }
      }
    }
    __syncthreads();
  };
  auto step = [&](auto p_c, int g) {
    level(std::integral_constant<int, 0>(), p_c, g);
    if constexpr (N > 1) level(std::integral_constant<int, 1>(), p_c, g);
    if constexpr (N > 2) level(std::integral_constant<int, 2>(), p_c, g);
    if constexpr (N > 3) level(std::integral_constant<int, 3>(), p_c, g);
  };
  for (int g = 0; g < G; g += 2) {
    step(std::integral_constant<int, 0>(), g);
    if (g + 1 < G) step(std::integral_constant<int, 1>(), g + 1);
  }
}

// ---------------------------------------------------------------------------
// Launch helpers

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

// The chains built: the radius runs of the default settings (sigma0 1.6,
// s = 3, sigma_in 0.5): the upsampled first octave (5, 5, 7, 8), the first
// octave without upsampling (7, 5, 7, 8), the later octaves (5, 7, 8), and
// their prefixes and the runs that start inside an octave.
typedef void (*ChainKernel)(ChainArgs);
struct ChainEntry {
  int mode, st, n, r[kChainMaxLevels];
  ChainKernel fn;
};

#define SIFT_CHAIN_ST(M, S)                                                    \
  {M, S, 3, {5, 7, 8, 0}, k_chain<M, S, 5, 7, 8>},                             \
  {M, S, 2, {5, 7, 0, 0}, k_chain<M, S, 5, 7>}

static const ChainEntry kChains[] = {
    {kSrcUpsample, 0, 4, {5, 5, 7, 8}, k_chain<kSrcUpsample, 0, 5, 5, 7, 8>},
    {kSrcUpsample, 0, 3, {5, 5, 7, 0}, k_chain<kSrcUpsample, 0, 5, 5, 7>},
    {kSrcUpsample, 0, 2, {5, 5, 0, 0}, k_chain<kSrcUpsample, 0, 5, 5>},
    {kSrcImage, 0, 4, {7, 5, 7, 8}, k_chain<kSrcImage, 0, 7, 5, 7, 8>},
    {kSrcImage, 0, 3, {7, 5, 7, 0}, k_chain<kSrcImage, 0, 7, 5, 7>},
    {kSrcImage, 0, 2, {7, 5, 0, 0}, k_chain<kSrcImage, 0, 7, 5>},
    SIFT_CHAIN_ST(kSrcDown, 0),
    SIFT_CHAIN_ST(kSrcDown, 1),
    SIFT_CHAIN_ST(kSrcDown, 2),
    SIFT_CHAIN_ST(kSrcLevel, 0),
    SIFT_CHAIN_ST(kSrcLevel, 2),
    {kSrcLevel, 0, 2, {7, 8, 0, 0}, k_chain<kSrcLevel, 0, 7, 8>},
    {kSrcLevel, 2, 2, {7, 8, 0, 0}, k_chain<kSrcLevel, 2, 7, 8>},
};
#undef SIFT_CHAIN_ST

static ChainKernel chain_kernel(int mode, int st, int n, const int* radii) {
  for (const ChainEntry& c : kChains) {
    if (c.mode != mode || c.st != st || c.n != n) continue;
    bool same = true;
    for (int i = 0; i < n; ++i) same = same && c.r[i] == radii[i];
    if (same) return c.fn;
  }
  return nullptr;
}

bool chain_supported(int mode, int st, int n_levels, const int* radii) {
  return n_levels >= 2 && n_levels <= kChainMaxLevels && chain_kernel(mode, st, n_levels, radii);
}

hipError_t launch_chain(const ChainArgs& a, int mode, int st, int n_levels, const int* radii,
                        int grid, hipStream_t stream) {
  if (n_levels < 2 || n_levels > kChainMaxLevels) return hipErrorInvalidValue;
  ChainKernel fn = chain_kernel(mode, st, n_levels, radii);
  if (!fn) return hipErrorInvalidValue;
  return launch(fn, dim3(grid), dim3(kBlurThreads), stream, a);
}

// The bounds-check counter of this file's kernels (see check_in).
hipError_t bounds_count_blur(unsigned long long* count, bool reset) {
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
