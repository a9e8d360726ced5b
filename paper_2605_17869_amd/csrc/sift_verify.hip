// gfx950 kernels of geometric verification: homography hypotheses from
// minimal samples, scored by the noise-scale-marginalised inlier likelihood,
// the best one refined by reweighted least squares.  All arithmetic is fp64;
// every sum runs in an order fixed by the code (per-lane partial sums in index
// order, then a fixed butterfly and a fixed order over waves), so results are
// bit-identical from run to run.  Built with -ffp-contract=off.
#include <hip/hip_runtime.h>

#include <math.h>

#include "sift_device.h"
#include "sift_verify.h"

namespace sift {

// sqrt(2 ln 100): the 0.99 quantile of the unit Rayleigh distribution
constexpr double kTau = 3.034854258770293;
constexpr double kErfTau = 0.9975934805411772;    // erf(kTau / sqrt 2)
constexpr double kSqrtHalfPi = 1.2533141373155001;
constexpr double kSqrt2 = 1.4142135623730951;
constexpr double kPivotEps = 1e-12;

// Marginal likelihood of residual r (pixels) over sigma uniform on (0, smax]
// of a Rayleigh residual truncated at tau * sigma; 0 at and beyond tau * smax.
__device__ __forceinline__ double marginal_w(double r, double smax) {
  if (!(r < kTau * smax)) return 0.0;
  return kSqrtHalfPi / smax * (kErfTau - erf(r / (kSqrt2 * smax)));
}

__device__ __forceinline__ int verify_count(const VerifyEntry& e) {
  if (!e.n_matches) return e.cap;
  const int c = *e.n_matches;
  return c < 0 ? 0 : (c < e.cap ? c : e.cap);
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = v + __shfl_xor(v, d, 64);
  return v;
}

// Block sum of one double per thread (blockDim 256): wave butterflies, then
// the four wave totals in wave order.  Every thread gets the same bits.
__device__ __forceinline__ double block_sum_d(double v, double* s4) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum_d(v);
  __syncthreads();
  if (lane == 0) s4[wave] = v;
  __syncthreads();
  return ((s4[0] + s4[1]) + s4[2]) + s4[3];
}

// Homography x -> H x of a normalised-coordinate solution h (h33 = 1) moved
// back to pixels: H = Tb^-1 Hn Ta, scaled to h33 = 1.  nrm: sa, txa, tya,
// sb, txb, tyb (T = [[s, 0, tx], [0, s, ty], [0, 0, 1]]).
__device__ __forceinline__ bool denormalise(const double* h, const double* nrm, double* H) {
  const double Hn[9] = {h[0], h[1], h[2], h[3], h[4], h[5], h[6], h[7], 1.0};
  const double Ta[9] = {nrm[0], 0.0, nrm[1], 0.0, nrm[0], nrm[2], 0.0, 0.0, 1.0};
  const double ib = 1.0 / nrm[3];
  const double Tbi[9] = {ib, 0.0, -nrm[4] * ib, 0.0, ib, -nrm[5] * ib, 0.0, 0.0, 1.0};
  double M[9], R[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      M[3 * i + j] = (Hn[3 * i] * Ta[j] + Hn[3 * i + 1] * Ta[3 + j]) + Hn[3 * i + 2] * Ta[6 + j];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      R[3 * i + j] = (Tbi[3 * i] * M[j] + Tbi[3 * i + 1] * M[3 + j]) + Tbi[3 * i + 2] * M[6 + j];
  bool ok = true;
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    H[q] = R[q] / R[8];
    ok = ok && isfinite(H[q]);
  }
  return ok;
}

// Solve the 8 x 8 system held as an augmented 8 x 9 matrix in LDS (row r at
// A[9 r]) by Gaussian elimination with partial pivoting (first largest
// pivot); lane r < 8 owns row r during elimination, lane 0 pivots and
// back-substitutes.  Returns false (on every lane) when a pivot falls below
// kPivotEps of the largest entry of the coefficient block.  Wave-level.
__device__ bool solve8_wave(double* A, double* h) {
  const int lane = threadIdx.x & 63;
  double scale = 0.0;
#pragma unroll
  for (int r = 0; r < 8; ++r)
#pragma unroll
    for (int c = 0; c < 8; ++c) scale = fmax(scale, fabs(A[9 * r + c]));
  bool ok = scale > 0.0;
  for (int col = 0; col < 8 && ok; ++col) {
    // pivot row: the first of the largest |A[r][col]|, r >= col
    int piv = col;
    double best = fabs(A[9 * col + col]);
    for (int r = col + 1; r < 8; ++r) {
      const double v = fabs(A[9 * r + col]);
      if (v > best) {
        best = v;
        piv = r;
      }
    }
    if (best < kPivotEps * scale) {
      ok = false;
      break;
    }
    wave_lds_sync();
    if (piv != col && lane < 9) {
      const double t = A[9 * col + lane];
      A[9 * col + lane] = A[9 * piv + lane];
      A[9 * piv + lane] = t;
    }
    wave_lds_sync();
    if (lane > col && lane < 8) {
      const double f = A[9 * lane + col] / A[9 * col + col];
      for (int j = col; j < 9; ++j) A[9 * lane + j] = A[9 * lane + j] - f * A[9 * col + j];
    }
    wave_lds_sync();
  }
  if (!ok) return false;
  for (int row = 7; row >= 0; --row) {
    double acc = A[9 * row + 8];
    for (int j = row + 1; j < 8; ++j) acc = acc - A[9 * row + j] * h[j];
    h[row] = acc / A[9 * row + row];
  }
  return true;
}

// Rows of the DLT system of correspondence (x, y) -> (u, v), h33 = 1.
__device__ __forceinline__ void dlt_rows(double x, double y, double u, double v, double* r1,
                                         double* r2) {
  r1[0] = x; r1[1] = y; r1[2] = 1.0; r1[3] = 0.0; r1[4] = 0.0; r1[5] = 0.0;
  r1[6] = -u * x; r1[7] = -u * y; r1[8] = u;
  r2[0] = 0.0; r2[1] = 0.0; r2[2] = 0.0; r2[3] = x; r2[4] = y; r2[5] = 1.0;
  r2[6] = -v * x; r2[7] = -v * y; r2[8] = v;
}

// Weight of correspondence (ax, ay) -> (bx, by) under H: marginal_w of the
// residual r = |(x / w - bx, y / w - by)|, (x, y, w) = H (ax, ay, 1); 0 when
// w <= 0 (the point maps to or behind the line at infinity).  The cut
// r < tau * smax is first tested without divisions, on
// |(x, y) - (bx, by) w|^2 < (tau smax w)^2 relaxed by 1e-9 (far more than the
// rounding that separates the two forms); only where that admits the
// correspondence is r formed, and marginal_w's exact test and weight decide,
// so the filter changes no result.
__device__ __forceinline__ double weight_at(const double* H, double ax, double ay, double bx,
                                            double by, double smax) {
  const double x = (ax * H[0] + ay * H[1]) + H[2];
  const double y = (ax * H[3] + ay * H[4]) + H[5];
  const double w = (ax * H[6] + ay * H[7]) + H[8];
  if (!(w > 0.0)) return 0.0;
  const double ex = x - bx * w, ey = y - by * w, lim = kTau * smax * w;
  if (!(ex * ex + ey * ey < (lim * lim) * (1.0 + 1e-9))) return 0.0;
  const double dx = x / w - bx, dy = y / w - by;
  return marginal_w(sqrt(dx * dx + dy * dy), smax);
}

// Pixel positions of correspondence i (stored as the keypoints' fp32 values).
struct RawPt {
  double ax, ay, bx, by;
};
__device__ __forceinline__ RawPt raw_at(const float4* raw, int i) {
  const float4 v = raw[i];
  return RawPt{(double)v.x, (double)v.y, (double)v.z, (double)v.w};
}

// solve8_wave for one lane: the same steps in the same order on a system in
// this lane's registers (A[r][c], augmented column 8), row swaps by selects.
__device__ __forceinline__ bool solve8_lane(double (&A)[8][9], double* h) {
  double scale = 0.0;
#pragma unroll
  for (int r = 0; r < 8; ++r)
#pragma unroll
    for (int c = 0; c < 8; ++c) scale = fmax(scale, fabs(A[r][c]));
  bool ok = scale > 0.0;
#pragma unroll
  for (int col = 0; col < 8; ++col) {
    // pivot row: the first of the largest |A[r][col]|, r >= col
    int piv = col;
    double best = fabs(A[col][col]);
#pragma unroll
    for (int r = col + 1; r < 8; ++r) {
      const double v = fabs(A[r][col]);
      const bool up = v > best;
      best = up ? v : best;
      piv = up ? r : piv;
    }
    ok = ok && !(best < kPivotEps * scale);
#pragma unroll
    for (int r = col + 1; r < 8; ++r) {
      const bool sw = r == piv;
#pragma unroll
      for (int j = 0; j < 9; ++j) {
        const double t = A[col][j];
        A[col][j] = sw ? A[r][j] : t;
        A[r][j] = sw ? t : A[r][j];
      }
    }
#pragma unroll
    for (int r = col + 1; r < 8; ++r) {
      const double f = A[r][col] / A[col][col];
#pragma unroll
      for (int j = col; j < 9; ++j) A[r][j] = A[r][j] - f * A[col][j];
    }
  }
#pragma unroll
  for (int row = 7; row >= 0; --row) {
    double acc = A[row][8];
#pragma unroll
    for (int j = row + 1; j < 8; ++j) acc = acc - A[row][j] * h[j];
    h[row] = acc / A[row][row];
  }
  return ok;
}

// The model of every minimal sample, one lane per hypothesis: sample k takes
// correspondences floor(u[k][j] n) (at most n - 1), j = 0..3; repeated
// indices give no model, else the DLT rows of the four normalised
// correspondences are solved (solve8_lane) and the solution moved back to
// pixels.  Stored for the scoring and refinement kernels; NaN where a sample
// gives no model.
__global__ __launch_bounds__(kVerifyModelBlock) void k_verify_models(VerifyHdr hd, int n_pairs) {
  const int groups = (hd.n_hyp + kVerifyModelBlock - 1) / kVerifyModelBlock;
  const int p = blockIdx.x / groups;
  const int k = (blockIdx.x - p * groups) * kVerifyModelBlock + threadIdx.x;
  if (k >= hd.n_hyp) return;
  const VerifyEntry e = hd.table[p];
  const int n = verify_count(e);
  SIFT_CHECK_INDEX(k, hd.n_hyp);
  double* out = reinterpret_cast<double*>(hd.ws + e.models) + 9 * (int64_t)k;
  double H[9];
  bool ok = n >= 4;
  if (ok) {
    const double* pts = reinterpret_cast<const double*>(hd.ws + e.pts);
    const double* nrm = reinterpret_cast<const double*>(hd.ws + e.norm);
    int idx[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      SIFT_CHECK_INDEX(4 * k + j, 4 * (int64_t)hd.n_hyp);
      const double u = (double)hd.samples[4 * k + j];
      const int q = (int)floor(u * (double)n);
      idx[j] = q < n - 1 ? q : n - 1;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = i + 1; j < 4; ++j) ok = ok && idx[i] != idx[j];
    if (ok) {
      double A[8][9];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const double* q = pts + 4 * (int64_t)idx[i];
        dlt_rows(q[0], q[1], q[2], q[3], A[2 * i], A[2 * i + 1]);
      }
      double h[8];
      ok = solve8_lane(A, h) && denormalise(h, nrm, H);
    }
  }
#pragma unroll
  for (int q = 0; q < 9; ++q) out[q] = ok ? H[q] : NAN;
}

__global__ void k_verify_setup(VerifyHdr hd, VerifySetupChunk c) {
  const int t = threadIdx.x;
  if (t < c.count) const_cast<VerifyEntry*>(hd.table)[c.first + t] = c.e[t];
}

// Per pair: gather the matched points (pixels), the normalising similarity of
// each set (mean to 0, mean distance to sqrt 2) and the normalised points.
__global__ __launch_bounds__(256) void k_verify_prep(VerifyHdr hd, int n_pairs) {
  __shared__ double s4[4];
  const VerifyEntry e = hd.table[blockIdx.x];
  const int n = verify_count(e);
  float4* raw = reinterpret_cast<float4*>(hd.ws + e.raw);
  double* pts = reinterpret_cast<double*>(hd.ws + e.pts);
  double* nrm = reinterpret_cast<double*>(hd.ws + e.norm);
  double sx[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < n; i += 256) {
    SIFT_CHECK_INDEX(i, e.cap);
    const sift_match m = e.matches[i];
    const sift_keypoint ka = e.kp_a[m.query], kb = e.kp_b[m.train];
    raw[i] = make_float4(ka.x, ka.y, kb.x, kb.y);
    const double v[4] = {(double)ka.x, (double)ka.y, (double)kb.x, (double)kb.y};
#pragma unroll
    for (int q = 0; q < 4; ++q) sx[q] += v[q];
  }
  double c[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) c[q] = block_sum_d(sx[q], s4) / (double)(n > 0 ? n : 1);
  __syncthreads();
  double da = 0.0, db = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    SIFT_CHECK_INDEX(i, e.cap);
    const RawPt q = raw_at(raw, i);
    const double xa = q.ax - c[0], ya = q.ay - c[1], xb = q.bx - c[2], yb = q.by - c[3];
    da += sqrt(xa * xa + ya * ya);
    db += sqrt(xb * xb + yb * yb);
  }
  const double ma = block_sum_d(da, s4) / (double)(n > 0 ? n : 1);
  const double mb = block_sum_d(db, s4) / (double)(n > 0 ? n : 1);
  const double sa = ma > 0.0 ? kSqrt2 / ma : 1.0, sb = mb > 0.0 ? kSqrt2 / mb : 1.0;
  const double t[6] = {sa, -sa * c[0], -sa * c[1], sb, -sb * c[2], -sb * c[3]};
  if (threadIdx.x < 6) nrm[threadIdx.x] = t[threadIdx.x];
  for (int i = threadIdx.x; i < n; i += 256) {
    SIFT_CHECK_INDEX(i, e.cap);
    const RawPt q = raw_at(raw, i);
    double* o = pts + 4 * (int64_t)i;
    o[0] = sa * q.ax + t[1];
    o[1] = sa * q.ay + t[2];
    o[2] = sb * q.bx + t[4];
    o[3] = sb * q.by + t[5];
  }
}

// One wave per hypothesis: its score, the sum over the pair's correspondences
// of the marginal likelihood of the residual under its stored model.
__global__ __launch_bounds__(64 * kVerifyHypPerGroup) void k_verify_hyp(VerifyHdr hd, int n_pairs) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p = blockIdx.x / hd.hyp_groups;
  const int k = (blockIdx.x - p * hd.hyp_groups) * kVerifyHypPerGroup + wave;
  if (k >= hd.n_hyp) return;
  const VerifyEntry e = hd.table[p];
  const int n = verify_count(e);
  double* scores = reinterpret_cast<double*>(hd.ws + e.scores);
  SIFT_CHECK_INDEX(k, hd.n_hyp);
  const double* model = reinterpret_cast<const double*>(hd.ws + e.models) + 9 * (int64_t)k;
  double H[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) H[q] = model[q];
  if (isnan(H[0])) {
    if (lane == 0) scores[k] = -INFINITY;
    return;
  }
  const float4* raw = reinterpret_cast<const float4*>(hd.ws + e.raw);
  double acc = 0.0;
  for (int i = lane; i < n; i += 64) {
    SIFT_CHECK_INDEX(i, e.cap);
    const RawPt q = raw_at(raw, i);
    acc += weight_at(H, q.ax, q.ay, q.bx, q.by, hd.sigma_max);
  }
  acc = wave_sum_d(acc);
  if (lane == 0) scores[k] = acc;
}

// Per pair: the best hypothesis (largest score, first among equals), then
// reweighted least squares on the normalised DLT rows, each step kept only
// if it raises the score; outputs the model, score, inlier count, weights.
__global__ __launch_bounds__(256) void k_verify_refine(VerifyHdr hd, int n_pairs) {
  __shared__ double s4[4];
  __shared__ double s_a[72];
  __shared__ double s_ne[4][44];
  __shared__ double s_h[9];
  __shared__ int s_flag;
  __shared__ double s_bv[4];
  __shared__ int s_bi[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const VerifyEntry e = hd.table[blockIdx.x];
  const int n = verify_count(e);
  const double* scores = reinterpret_cast<const double*>(hd.ws + e.scores);
  const float4* raw = reinterpret_cast<const float4*>(hd.ws + e.raw);
  const double* pts = reinterpret_cast<const double*>(hd.ws + e.pts);
  const double* nrm = reinterpret_cast<const double*>(hd.ws + e.norm);

  // best hypothesis
  double bv = -INFINITY;
  int bi = 0x7fffffff;
  if (n >= 4) {
    for (int k = threadIdx.x; k < hd.n_hyp; k += 256) {
      const double v = scores[k];
      if (v > bv || (v == bv && k < bi)) {
        bv = v;
        bi = k;
      }
    }
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const double ov = __shfl_xor(bv, d, 64);
    const int oi = __shfl_xor(bi, d, 64);
    if (ov > bv || (ov == bv && oi < bi)) {
      bv = ov;
      bi = oi;
    }
  }
  if (lane == 0) {
    s_bv[wave] = bv;
    s_bi[wave] = bi;
  }
  __syncthreads();
  bv = s_bv[0];
  bi = s_bi[0];
  for (int w = 1; w < 4; ++w)
    if (s_bv[w] > bv || (s_bv[w] == bv && s_bi[w] < bi)) {
      bv = s_bv[w];
      bi = s_bi[w];
    }
  if (!(bv > -INFINITY)) {
    // no hypothesis: NaN model, zero score and inliers
    if (threadIdx.x < 9) e.H[threadIdx.x] = NAN;
    if (threadIdx.x == 0) {
      *e.score = 0.0;
      *e.n_inliers = 0;
      if (e.best) *e.best = -1;
    }
    if (e.weights)
      for (int i = threadIdx.x; i < e.cap; i += 256) e.weights[i] = 0.0f;
    return;
  }
  // the best hypothesis' model, as stored
  double H[9];
  {
    SIFT_CHECK_INDEX(bi, hd.n_hyp);
    const double* model = reinterpret_cast<const double*>(hd.ws + e.models) + 9 * (int64_t)bi;
#pragma unroll
    for (int q = 0; q < 9; ++q) H[q] = model[q];
  }
  double Q = bv;
  for (int it = 0; it < hd.refine_iters; ++it) {
    // weighted normal equations of the DLT rows (upper triangle + rhs)
    double ne[44];
#pragma unroll
    for (int q = 0; q < 44; ++q) ne[q] = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
      SIFT_CHECK_INDEX(i, e.cap);
      const RawPt r = raw_at(raw, i);
      const double w = weight_at(H, r.ax, r.ay, r.bx, r.by, hd.sigma_max);
      const double* p = pts + 4 * (int64_t)i;
      double r1[9], r2[9];
      dlt_rows(p[0], p[1], p[2], p[3], r1, r2);
      int q = 0;
#pragma unroll
      for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = a; b < 8; ++b) {
          ne[q] = ne[q] + r1[a] * (w * r1[b]);
          ne[q] = ne[q] + r2[a] * (w * r2[b]);
          ++q;
        }
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        ne[q] = ne[q] + r1[a] * (w * r1[8]);
        ne[q] = ne[q] + r2[a] * (w * r2[8]);
        ++q;
      }
    }
#pragma unroll
    for (int q = 0; q < 44; ++q) ne[q] = wave_sum_d(ne[q]);
    __syncthreads();
    if (lane == 0)
#pragma unroll
      for (int q = 0; q < 44; ++q) s_ne[wave][q] = ne[q];
    __syncthreads();
    if (wave == 0) {
      // the system in LDS (lanes 0..43 each sum one entry over the waves)
      if (lane < 44) {
        const double v = ((s_ne[0][lane] + s_ne[1][lane]) + s_ne[2][lane]) + s_ne[3][lane];
        if (lane < 36) {
          int a = 0, rem = lane;
          while (rem >= 8 - a) {
            rem -= 8 - a;
            ++a;
          }
          const int b = a + rem;
          s_a[9 * a + b] = v;
          s_a[9 * b + a] = v;
        } else {
          s_a[9 * (lane - 36) + 8] = v;
        }
      }
      wave_lds_sync();
      double h[8], H2[9];
      bool ok = solve8_wave(s_a, h);
      if (ok) ok = denormalise(h, nrm, H2);
      if (lane == 0) {
        s_flag = ok ? 1 : 0;
        for (int q = 0; q < 9; ++q) s_h[q] = ok ? H2[q] : 0.0;
      }
    }
    __syncthreads();
    if (!s_flag) break;
    double H2[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) H2[q] = s_h[q];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
      SIFT_CHECK_INDEX(i, e.cap);
      const RawPt r = raw_at(raw, i);
      acc += weight_at(H2, r.ax, r.ay, r.bx, r.by, hd.sigma_max);
    }
    const double Q2 = block_sum_d(acc, s4);
    if (!(Q2 > Q)) break;
#pragma unroll
    for (int q = 0; q < 9; ++q) H[q] = H2[q];
    Q = Q2;
  }
  // outputs
  double cnt = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    SIFT_CHECK_INDEX(i, e.cap);
    const RawPt r = raw_at(raw, i);
    const double w = weight_at(H, r.ax, r.ay, r.bx, r.by, hd.sigma_max);
    cnt += w > 0.0 ? 1.0 : 0.0;
    SIFT_CHECK_INDEX(i, e.cap);
    if (e.weights) e.weights[i] = (float)w;
  }
  if (e.weights)
    for (int i = n + threadIdx.x; i < e.cap; i += 256) e.weights[i] = 0.0f;
  const double inl = block_sum_d(cnt, s4);
  if (threadIdx.x < 9) e.H[threadIdx.x] = H[threadIdx.x];
  if (threadIdx.x == 0) {
    *e.score = Q;
    *e.n_inliers = (int)inl;
    if (e.best) *e.best = bi;
  }
}

hipError_t launch_verify_setup(const VerifyHdr& h, const VerifySetupChunk& c, hipStream_t stream) {
  return launch(k_verify_setup, dim3(1), dim3(64), stream, h, c);
}

hipError_t launch_verify_prep(const VerifyHdr& h, int n, hipStream_t stream) {
  return launch(k_verify_prep, dim3(n), dim3(256), stream, h, n);
}

hipError_t launch_verify_models(const VerifyHdr& h, int n, hipStream_t stream) {
  const int groups = (h.n_hyp + kVerifyModelBlock - 1) / kVerifyModelBlock;
  return launch(k_verify_models, dim3(n * groups), dim3(kVerifyModelBlock), stream, h, n);
}

hipError_t launch_verify_hyp(const VerifyHdr& h, int n, hipStream_t stream) {
  return launch(k_verify_hyp, dim3(n * h.hyp_groups), dim3(64 * kVerifyHypPerGroup), stream, h, n);
}

hipError_t launch_verify_refine(const VerifyHdr& h, int n, hipStream_t stream) {
  return launch(k_verify_refine, dim3(n), dim3(256), stream, h, n);
}

// The bounds-check counter of this file's kernels (see check_index).
hipError_t bounds_count_verify(unsigned long long* count, bool reset) {
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
