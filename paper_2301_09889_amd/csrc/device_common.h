// Device helpers shared by the HIP sources: FP64 complex arithmetic on double2,
// wavefront-scope synchronisation and reductions.
#pragma once

#include "chanenv_internal.h"

#define HD __host__ __device__ __forceinline__

namespace chanenv {

// Complex helpers (double2 as re, im).  Named functions only: HIP's vector operators
// on double2 are component-wise, not complex.
HD cplx cz() { return make_double2(0.0, 0.0); }
HD cplx cadd(cplx a, cplx b) { return make_double2(a.x + b.x, a.y + b.y); }
HD cplx csub(cplx a, cplx b) { return make_double2(a.x - b.x, a.y - b.y); }
HD cplx cscale(cplx a, double s) { return make_double2(a.x * s, a.y * s); }
HD cplx cmul(cplx a, cplx b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
HD cplx cconj(cplx a) { return make_double2(a.x, -a.y); }
// i * a
HD cplx cmuli(cplx a) { return make_double2(-a.y, a.x); }
// acc + s * a
HD cplx caxpy(cplx acc, double s, cplx a) {
  return make_double2(fma(s, a.x, acc.x), fma(s, a.y, acc.y));
}

// ---- cross-lane moves without LDS (gfx950 DPP and permlane swaps) ----
// A row is 16 lanes.  DPP controls used here:
constexpr int DPP_ROW_SHL = 0x100;        // + d: lane k of a row reads lane k + d of that row
constexpr int DPP_ROW_SHR = 0x110;        // + d: lane k reads lane k - d
constexpr int DPP_WAVE_SHL1 = 0x130;      // lane l reads lane l + 1
constexpr int DPP_WAVE_SHR1 = 0x138;      // lane l reads lane l - 1
constexpr int DPP_ROW_MIRROR = 0x140;     // lane k reads lane 15 - k
constexpr int DPP_ROW_HALF_MIRROR = 0x141;  // within 8 lanes: k reads 7 - k
constexpr int DPP_ROW_BCAST = 0x150;      // + k: every lane of a row reads lane k of the row
constexpr int DPP_QUAD_XOR1 = 0xB1;       // quad_perm [1, 0, 3, 2]
constexpr int DPP_QUAD_XOR2 = 0x4E;       // quad_perm [2, 3, 0, 1]

// x moved by the DPP pattern CTRL; a lane whose source lies outside the row (or the wave)
// reads 0.
template <int CTRL>
__device__ __forceinline__ double dmov(double x) {
  return __builtin_amdgcn_update_dpp(0.0, x, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ cplx cmov(cplx v) {
  return make_double2(dmov<CTRL>(v.x), dmov<CTRL>(v.y));
}
__device__ __forceinline__ unsigned lo32(double x) { return (unsigned)(unsigned long long)__double_as_longlong(x); }
__device__ __forceinline__ unsigned hi32(double x) {
  return (unsigned)((unsigned long long)__double_as_longlong(x) >> 32);
}
__device__ __forceinline__ double join32(unsigned l, unsigned h) {
  return __longlong_as_double((long long)(((unsigned long long)h << 32) | l));
}
// Both results of v_permlane16_swap on (x, y): a holds rows (x0, y0, x2, y2), b holds rows
// (x1, y1, x3, y3).  Using both (instead of selecting one per row) costs no VALU merge.
struct Pair {
  double a, b;
};
__device__ __forceinline__ Pair row_swap(double x, double y) {
  const auto l = __builtin_amdgcn_permlane16_swap(lo32(x), lo32(y), false, false);
  const auto h = __builtin_amdgcn_permlane16_swap(hi32(x), hi32(y), false, false);
  return {join32(l[0], h[0]), join32(l[1], h[1])};
}
// Both results of v_permlane32_swap on (x, y): a holds halves (x_lo, y_lo), b (x_hi, y_hi).
__device__ __forceinline__ Pair half_swap(double x, double y) {
  const auto l = __builtin_amdgcn_permlane32_swap(lo32(x), lo32(y), false, false);
  const auto h = __builtin_amdgcn_permlane32_swap(hi32(x), hi32(y), false, false);
  return {join32(l[0], h[0]), join32(l[1], h[1])};
}
// Rows 0 and 2 receive x's rows 1 and 3; rows 1 and 3 read 0.
__device__ __forceinline__ double from_odd_rows(double x) { return row_swap(x, 0.0).b; }
__device__ __forceinline__ cplx from_odd_rows(cplx v) { return make_double2(from_odd_rows(v.x), from_odd_rows(v.y)); }
// Rows 1 and 3 receive x's rows 0 and 2; rows 0 and 2 read 0.
__device__ __forceinline__ double from_even_rows(double x) { return row_swap(0.0, x).a; }
__device__ __forceinline__ cplx from_even_rows(cplx v) {
  return make_double2(from_even_rows(v.x), from_even_rows(v.y));
}
// Lanes l < 32 receive lo's lane l + 32, lanes l >= 32 receive hi's lane l - 32.
__device__ __forceinline__ double cross_halves(double lo, double hi, bool low) {
  const auto a = __builtin_amdgcn_permlane32_swap(lo32(lo), lo32(hi), false, false);
  const auto b = __builtin_amdgcn_permlane32_swap(hi32(lo), hi32(hi), false, false);
  return low ? join32(a[1], b[1]) : join32(a[0], b[0]);
}
__device__ __forceinline__ double readlane_d(double x, int l) {
  return join32(__builtin_amdgcn_readlane(lo32(x), l), __builtin_amdgcn_readlane(hi32(x), l));
}
__device__ __forceinline__ cplx readlane_c(cplx v, int l) { return make_double2(readlane_d(v.x, l), readlane_d(v.y, l)); }
__device__ __forceinline__ cplx shfl_c(cplx v, int src) {
  return make_double2(__shfl(v.x, src, 64), __shfl(v.y, src, 64));
}
// A cross-lane result used only under a per-lane condition: the empty volatile asm keeps the
// permlane or DPP move that made it out of the conditional code, where lanes switched off by
// EXEC would not supply their values (the compiler otherwise sinks it into one arm of a select).
__device__ __forceinline__ double pin(double x) {
  asm volatile("" : "+v"(x));
  return x;
}

// Sums whose every step adds two values that are already identical within their groups, so
// that every lane of the group receives the bitwise-same result.
__device__ __forceinline__ double row_sum(double x) {
  x += dmov<DPP_QUAD_XOR1>(x);
  x += dmov<DPP_QUAD_XOR2>(x);
  x += dmov<DPP_ROW_HALF_MIRROR>(x);
  x += dmov<DPP_ROW_MIRROR>(x);
  return x;
}
__device__ __forceinline__ double half_sum(double x) {
  const Pair r = row_swap(row_sum(x), row_sum(x));
  return r.a + r.b;  // (row 0 + row 1) or (row 2 + row 3), in that order on every lane
}
__device__ __forceinline__ cplx half_sum(cplx v) { return make_double2(half_sum(v.x), half_sum(v.y)); }
__device__ __forceinline__ double lane_sum(double x) {
  const double h = half_sum(x);
  const Pair r = half_swap(h, h);
  return r.a + r.b;  // low half + high half on every lane
}
__device__ __forceinline__ cplx lane_sum(cplx v) { return make_double2(lane_sum(v.x), lane_sum(v.y)); }

// Sum over the 64 lanes (all active); every lane receives the bitwise-same total.  Pinned, so
// that a total used by one lane only is still formed with every lane taking part.
__device__ __forceinline__ double wave_sum(double v) { return pin(lane_sum(v)); }
__device__ __forceinline__ cplx wave_sum(cplx v) { return make_double2(wave_sum(v.x), wave_sum(v.y)); }

// Workgroups go to the eight XCDs in turn (workgroup b to XCD b mod 8), each XCD with its own
// L2.  Logical block of workgroup b of G: every XCD takes one contiguous range, so neighbouring
// columns, which share the cache lines of the node-major fields, meet in one L2.  A bijection
// of [0, G) for any G (the first G mod 8 XCDs take one block more).
__device__ __forceinline__ int xcd_block(int b, int G) {
  const int x = b & 7, i = b >> 3, q = G >> 3, r = G & 7;
  return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Wave-scope barrier for LDS data exchanged between lanes of one wavefront.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace chanenv
