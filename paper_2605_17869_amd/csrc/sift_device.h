// Device helpers shared by the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "sift_internal.h"

namespace sift {

constexpr float kTwoPi = 6.28318530717958647692f;

// ---------------------------------------------------------------------------
// Common device helpers

// Reflect-101 border: ... c b | a b c ... (index -1 -> 1), repeated with
// period 2(n-1) for indices far outside; n == 1 maps everything to 0.
__device__ __forceinline__ int mirror(int i, int n) {
  if (i >= 0 && i < n) return i;
  if (n == 1) return 0;
  const int period = 2 * (n - 1);
  i = i < 0 ? -i : i;
  i %= period;
  return i >= n ? period - i : i;
}

// Largest idx in [0, n) with prefix[idx] <= item (prefix has n + 1 entries).
__device__ __forceinline__ int find_owner(const int* prefix, int n, int item) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid] <= item) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int* counters_of(char* ws, const ImgEntry& e) {
  return reinterpret_cast<int*>(ws + e.region);
}

// ---------------------------------------------------------------------------
// Bounds checks.  A library built with -DSIFT_DEBUG_BOUNDS counts every
// checked access that falls outside the memory it belongs to (the image's
// workspace region, its input image, its output arrays, an LDS array) in a
// counter of each source file, which sift_bounds_violations reads; the
// access itself still happens.  Without the flag the checks compile to
// nothing.
#ifdef SIFT_DEBUG_BOUNDS
static __device__ unsigned long long g_bounds_violations;
#endif
struct Span {
  uint64_t lo, hi;   // byte addresses [lo, hi)
};
__device__ __forceinline__ Span region_span(const char* ws, const ImgEntry& e, const LayoutCfg& lc) {
  const uint64_t lo = reinterpret_cast<uint64_t>(ws) + (uint64_t)e.region;
  return Span{lo, lo + (uint64_t)region_tail(e.h, e.w, lc).bytes};
}
// the input image: h rows of pitch floats, the last one w wide
__device__ __forceinline__ Span input_span(const ImgEntry& e) {
  const uint64_t lo = reinterpret_cast<uint64_t>(e.src);
  return Span{lo, lo + 4u * ((uint64_t)(e.h - 1) * (uint64_t)e.src_pitch + (uint64_t)e.w)};
}
template <typename T>
__device__ __forceinline__ void check_in(const Span& s, T* p, uint32_t bytes) {
#ifdef SIFT_DEBUG_BOUNDS
  const uint64_t a = (uint64_t)(p);
  if (a < s.lo || a + bytes > s.hi) atomicAdd(&g_bounds_violations, 1ull);
#endif
}
__device__ __forceinline__ void check_index(int64_t i, int64_t n) {
#ifdef SIFT_DEBUG_BOUNDS
  if (i < 0 || i >= n) atomicAdd(&g_bounds_violations, 1ull);
#endif
}
// The kernels use these forms, which leave no trace (not even an unused
// address computation) in a normal build.
#ifdef SIFT_DEBUG_BOUNDS
#define SIFT_SPAN(name, expr) const ::sift::Span name = (expr)
#define SIFT_SPAN_VALUE(expr) (expr)
#define SIFT_CHECK_IN(span, p, bytes) ::sift::check_in((span), (p), (bytes))
#define SIFT_CHECK_INDEX(i, n) ::sift::check_index((i), (n))
#else
#define SIFT_SPAN(name, expr) ((void)0)
#define SIFT_SPAN_VALUE(expr) (::sift::Span{0, 0})
#define SIFT_CHECK_IN(span, p, bytes) ((void)0)
#define SIFT_CHECK_INDEX(i, n) ((void)0)
#endif

__device__ __forceinline__ const float* level_ptr(char* ws, const ImgEntry& e, const OctView& ov,
                                                  int level) {
  return reinterpret_cast<const float*>(ws + e.region + ov.level0 + (int64_t)level * ov.plane);
}

// Element idx of a level stored as fp32 (H16 false) or fp16 (H16 true).
template <bool H16>
__device__ __forceinline__ float lv_at(const void* base, int64_t idx) {
  if (H16) return (float)reinterpret_cast<const _Float16*>(base)[idx];
  return reinterpret_cast<const float*>(base)[idx];
}
// The same with the storage known only at run time.
__device__ __forceinline__ float lv_at(const void* base, int64_t idx, bool h16) {
  return h16 ? lv_at<true>(base, idx) : lv_at<false>(base, idx);
}

// Inclusive sum of an int over the 64 lanes of a wave (exact, any order).
__device__ __forceinline__ int wave_incl_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  return v;
}

// Butterfly sum over the 64 lanes.  Each step adds the partner's value; the
// two partners add the same two operands, so every lane ends with the same
// bits and the association order is fixed by the code.
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = v + __shfl_xor(v, d, 64);
  return v;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = fmaxf(v, __shfl_xor(v, d, 64));
  return v;
}

// Gradient orientation atan2(y, x) in (-pi, pi]: octant reduction to
// a = min(|x|, |y|) / max(|x|, |y|) and atan(a) = a * P(a^2), a degree-7
// polynomial fitted by weighted least squares (csrc/fit_atan.py; maximum
// error 1.4e-7 rad in fp32).  atan2(0, 0) = 0.
__device__ __forceinline__ float atan2_poly(float y, float x) {
  constexpr float c[8] = {0.999999344f, -0.333298594f, 0.199465662f, -0.139086306f,
                          0.0964219868f, -0.0559123345f, 0.0218629558f, -0.00405456498f};
  const float ax = fabsf(x), ay = fabsf(y);
  const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
  const float a = mx > 0.0f ? mn * __builtin_amdgcn_rcpf(mx) : 0.0f;
  const float s = a * a;
  float r = c[7];
#pragma unroll
  for (int j = 6; j >= 0; --j) r = __fmaf_rn(r, s, c[j]);
  r = r * a;
  if (ay > ax) r = 1.57079632679489662f - r;
  if (x < 0.0f) r = 3.14159265358979324f - r;
  return y < 0.0f ? -r : r;
}

// exp(x) through the hardware base-2 exponential (a few ulp).
__device__ __forceinline__ float exp_fast(float x) {
  return __builtin_amdgcn_exp2f(x * 1.44269504088896341f);
}

// Value of lane l - 1 (lane 0 keeps its own) and of lane l + 1 (lane 63
// keeps its own): whole-wave DPP shifts, no LDS round trip.
__device__ __forceinline__ float lane_prev(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v),
                                                    0x138 /* wave_shr:1 */, 0xf, 0xf, false));
}
__device__ __forceinline__ float lane_next(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v),
                                                    0x130 /* wave_shl:1 */, 0xf, 0xf, false));
}

// Lanes below this one in the wave.
__device__ __forceinline__ uint64_t lanemask_lt() {
  return (1ull << (threadIdx.x & 63)) - 1ull;
}

// Sends v to lane `dest` (a permutation of the wave's lanes).
__device__ __forceinline__ int lane_send(int dest, int v) {
  return __builtin_amdgcn_ds_permute(dest << 2, v);
}
__device__ __forceinline__ float lane_send(int dest, float v) {
  return __int_as_float(__builtin_amdgcn_ds_permute(dest << 2, __float_as_int(v)));
}

// Make this wave's LDS writes visible to its other lanes before they read.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Block-wide exclusive scan of ints (blockDim.x == 256).  Returns the
// exclusive prefix of v; *total receives the block sum.
__device__ __forceinline__ int block_excl_scan256(int v, int* s_wave, int* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int incl = wave_incl_scan(v);
  if (lane == 63) s_wave[wave] = incl;
  __syncthreads();
  int base = 0, sum = 0;
#pragma unroll
  for (int wv = 0; wv < 4; ++wv) {
    const int t = s_wave[wv];
    if (wv < wave) base += t;
    sum += t;
  }
  __syncthreads();
  *total = sum;
  return base + incl - v;
}

// Pointers into device memory that the compiler must treat as global (a
// pointer read from the image table would otherwise be accessed as flat,
// whose completion the LDS wait counter also tracks).
typedef __attribute__((address_space(1))) float gfloat;
typedef __attribute__((address_space(1))) char gchar;
__device__ __forceinline__ gfloat* as_global(const float* p) { return (gfloat*)(p); }

// A pointer every lane holds the same value of, moved to scalar registers so
// that loads and stores use the scalar-base + 32-bit vector-offset form.
__device__ __forceinline__ gchar* uniform_ptr(const gchar* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v >> 32));
  return reinterpret_cast<gchar*>((static_cast<uint64_t>(hi) << 32) | lo);
}
__device__ __forceinline__ float load_at(const gchar* row, uint32_t byte_off) {
  return *reinterpret_cast<const gfloat*>(row + byte_off);
}
__device__ __forceinline__ void store_at(gchar* row, uint32_t byte_off, float v) {
  *reinterpret_cast<gfloat*>(row + byte_off) = v;
}
typedef __attribute__((address_space(1))) _Float16 ghalf;
// fp16 of an fp32 value, nearest even.  The empty register constraint keeps
// the compiler from folding the conversion into the instruction that made x
// (a mixed-precision fma rounds the exact product-sum to fp16 once, which
// differs from rounding the fp32 result at fp16 ties).
__device__ __forceinline__ _Float16 f16_rn(float x) {
  __asm__("" : "+v"(x));
  return (_Float16)x;
}
// x rounded to fp16 and back
__device__ __forceinline__ float round_f16(float x) { return (float)f16_rn(x); }
// fp32 or fp16 (H16) element at a byte offset; stores round to nearest even
template <bool H16>
__device__ __forceinline__ float load_lv(const gchar* row, uint32_t byte_off) {
  if (H16) return (float)*reinterpret_cast<const ghalf*>(row + byte_off);
  return *reinterpret_cast<const gfloat*>(row + byte_off);
}
// Level stores are marked non-temporal: a level is read back by a later
// launch, after far more data than the caches hold has passed through them.
template <bool H16>
__device__ __forceinline__ void store_lv(gchar* row, uint32_t byte_off, float v) {
  if (H16) __builtin_nontemporal_store(f16_rn(v), reinterpret_cast<ghalf*>(row + byte_off));
  else __builtin_nontemporal_store(v, reinterpret_cast<gfloat*>(row + byte_off));
}
// Four consecutive elements at a byte offset aligned to their total size (16
// bytes fp32, 8 bytes fp16): one wide store.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
template <bool H16>
__device__ __forceinline__ void store4_lv(gchar* row, uint32_t byte_off, const float* v) {
  if (H16) {
    typedef __attribute__((address_space(1))) u32x2 gu32x2;
    const uint32_t lo = (uint32_t)__builtin_bit_cast(uint16_t, f16_rn(v[0])) |
                        ((uint32_t)__builtin_bit_cast(uint16_t, f16_rn(v[1])) << 16);
    const uint32_t hi = (uint32_t)__builtin_bit_cast(uint16_t, f16_rn(v[2])) |
                        ((uint32_t)__builtin_bit_cast(uint16_t, f16_rn(v[3])) << 16);
    u32x2 q;
    q.x = lo;
    q.y = hi;
    __builtin_nontemporal_store(q, reinterpret_cast<gu32x2*>(row + byte_off));
  } else {
    typedef __attribute__((address_space(1))) f32x4 gf32x4;
    f32x4 q;
    q.x = v[0];
    q.y = v[1];
    q.z = v[2];
    q.w = v[3];
    __builtin_nontemporal_store(q, reinterpret_cast<gf32x4*>(row + byte_off));
  }
}

// ---------------------------------------------------------------------------
// Launch helpers: hipLaunchKernel returns the launch status directly (the
// thread's last-error slot may hold another library's stale error).

template <typename... Args>
inline hipError_t launch(void (*kernel)(Args...), dim3 grid, dim3 block, hipStream_t stream,
                         Args... args) {
  void* ptrs[] = {static_cast<void*>(&args)...};
  return hipLaunchKernel(reinterpret_cast<const void*>(kernel), grid, block, ptrs, 0, stream);
}

}  // namespace sift
