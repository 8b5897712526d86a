// Device helpers shared by the HIP sources: FP64 complex arithmetic on double2,
// wavefront-scope synchronisation and reductions, and small in-register DFTs.
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


// cos and sin of 2 pi m / 48, m = 0..47: every root of unity the small DFTs below use
// (orders 2, 3, 4, 6, 8, 12, 16, 24, 48) is one of these.
constexpr double C48[48] = {1.0, 0.9914448613738104111446, 0.9659258262890682867497, 0.9238795325112867561282, 0.8660254037844386467637, 0.7933533402912351645798, 0.7071067811865475244008, 0.6087614290087206394161, 0.5, 0.3826834323650897717285, 0.2588190451025207623489, 0.1305261922200515915484, 2.06703210982639882365e-43, -0.1305261922200515915484, -0.2588190451025207623489, -0.3826834323650897717285, -0.5, -0.6087614290087206394161, -0.7071067811865475244008, -0.7933533402912351645798, -0.8660254037844386467637, -0.9238795325112867561282, -0.9659258262890682867497, -0.9914448613738104111446, -1.0, -0.9914448613738104111446, -0.9659258262890682867497, -0.9238795325112867561282, -0.8660254037844386467637, -0.7933533402912351645798, -0.7071067811865475244008, -0.6087614290087206394161, -0.5, -0.3826834323650897717285, -0.2588190451025207623489, -0.1305261922200515915484, 2.233876440654988324292e-41, 0.1305261922200515915484, 0.2588190451025207623489, 0.3826834323650897717285, 0.5, 0.6087614290087206394161, 0.7071067811865475244008, 0.7933533402912351645798, 0.8660254037844386467637, 0.9238795325112867561282, 0.9659258262890682867497, 0.9914448613738104111446};
constexpr double S48[48] = {0.0, 0.1305261922200515915484, 0.2588190451025207623489, 0.3826834323650897717285, 0.5, 0.6087614290087206394161, 0.7071067811865475244008, 0.7933533402912351645798, 0.8660254037844386467637, 0.9238795325112867561282, 0.9659258262890682867497, 0.9914448613738104111446, 1.0, 0.9914448613738104111446, 0.9659258262890682867497, 0.9238795325112867561282, 0.8660254037844386467637, 0.7933533402912351645798, 0.7071067811865475244008, 0.6087614290087206394161, 0.5, 0.3826834323650897717285, 0.2588190451025207623489, 0.1305261922200515915484, 4.134064219652797647299e-43, -0.1305261922200515915484, -0.2588190451025207623489, -0.3826834323650897717285, -0.5, -0.6087614290087206394161, -0.7071067811865475244008, -0.7933533402912351645798, -0.8660254037844386467637, -0.9238795325112867561282, -0.9659258262890682867497, -0.9914448613738104111446, -1.0, -0.9914448613738104111446, -0.9659258262890682867497, -0.9238795325112867561282, -0.8660254037844386467637, -0.7933533402912351645798, -0.7071067811865475244008, -0.6087614290087206394161, -0.5, -0.3826834323650897717285, -0.2588190451025207623489, -0.1305261922200515915484};

// exp(SG * 2 pi i m / R) for a root of order R dividing 48 (SG = -1 forward, +1 inverse).
template <int R, int SG>
HD cplx root(int m) {
  const int k = ((48 / R) * m) % 48;
  return make_double2(C48[k], SG * S48[k]);
}

// a * exp(SG * 2 pi i m / R), with the multiplications by 1 and +-i written out.
template <int R, int SG>
HD cplx rotate(cplx a, int m) {
  const int k = ((48 / R) * m) % 48;
  if (k == 0) return a;
  if (k == 12) return SG > 0 ? cmuli(a) : make_double2(a.y, -a.x);
  if (k == 24) return make_double2(-a.x, -a.y);
  if (k == 36) return SG > 0 ? make_double2(a.y, -a.x) : cmuli(a);
  return cmul(a, root<R, SG>(m));
}

// Small DFTs in registers: X[k] = sum_n x[n] exp(SG 2 pi i n k / R), in place.
template <int R, int SG>
struct Dft;

template <int SG>
struct Dft<1, SG> {
  static HD void run(cplx* x) {}
};

template <int SG>
struct Dft<2, SG> {
  static HD void run(cplx* x) {
    const cplx a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  }
};

template <int SG>
struct Dft<3, SG> {
  static HD void run(cplx* x) {
    const double h = 0.8660254037844386467637232;  // sqrt(3)/2
    const cplx t1 = cadd(x[1], x[2]), t2 = csub(x[1], x[2]);
    const cplx m = make_double2(x[0].x - 0.5 * t1.x, x[0].y - 0.5 * t1.y);
    const cplx r = make_double2(-SG * h * t2.y, SG * h * t2.x);  // SG i h t2
    x[0] = cadd(x[0], t1);
    x[1] = cadd(m, r);
    x[2] = csub(m, r);
  }
};

template <int SG>
struct Dft<4, SG> {
  static HD void run(cplx* x) {
    const cplx a = cadd(x[0], x[2]), b = csub(x[0], x[2]);
    const cplx c = cadd(x[1], x[3]), d = csub(x[1], x[3]);
    const cplx id = make_double2(-SG * d.y, SG * d.x);  // SG i d
    x[0] = cadd(a, c);
    x[2] = csub(a, c);
    x[1] = cadd(b, id);
    x[3] = csub(b, id);
  }
};

// R = R1 R2 by one Cooley--Tukey split (n = R2 n1 + n2, k = k1 + R1 k2).
template <int R1, int R2, int SG>
struct DftSplit {
  static HD void run(cplx* x) {
    constexpr int R = R1 * R2;
    cplx y[R];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
      cplx t[R1];
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) t[n1] = x[R2 * n1 + n2];
      Dft<R1, SG>::run(t);
#pragma unroll
      for (int k1 = 0; k1 < R1; ++k1) y[n2 * R1 + k1] = rotate<R, SG>(t[k1], n2 * k1);
    }
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      cplx t[R2];
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2) t[n2] = y[n2 * R1 + k1];
      Dft<R2, SG>::run(t);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) x[k1 + R1 * k2] = t[k2];
    }
  }
};

template <int SG> struct Dft<6, SG> : DftSplit<3, 2, SG> {};
template <int SG> struct Dft<8, SG> : DftSplit<4, 2, SG> {};
template <int SG> struct Dft<12, SG> : DftSplit<3, 4, SG> {};
template <int SG> struct Dft<16, SG> : DftSplit<4, 4, SG> {};

}  // namespace chanenv
