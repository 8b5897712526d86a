// Column pass for N <= 64 (N_y <= 65): one wavefront per wavenumber pair, with the
// Chebyshev coefficients in parity-major lane order.
//
// Lane l < 32 holds the even coefficient n = 2l, lane 32 + i the odd coefficient
// n = 2i + 1, and n = N (even) is a "tail" value that every lane carries.  The Chebyshev
// operators then map onto half-wave scans:
//   * D:  b_n = (2/c_n) sum_{p > n, p + n odd} p a_p is a suffix sum over the other
//         parity's half; D^2 is D applied twice.
//   * the tau systems (D^2 - lam) X = f (Gottlieb & Orszag 1977, even/odd
//     quasi-tridiagonal form) need the two first-order recurrences
//         e_i = w_i R_i - u_i e_{i+1}   (bottom-up),   E_i = e_i + f_i E_{i-1}   (top-down),
//     with w, u, f, F precomputed per pair and operator; both are affine scans across
//     the 32 lanes of a half, five steps each, instead of 33 serial steps.
// Node values are in the same parity-major order (lane l < 32: node 2l, lane 32 + i: node
// 2i + 1, node N the tail).  Every cross-lane exchange is a DPP move, a row broadcast or a
// permlane swap, except the gather that folds the coefficients for the inverse DCT.
//
// The tau rows T (rows n >= 2 of the quasi-tridiagonal form) invert D^2 exactly on
// polynomials of degree <= N: (T D^2 a)_n = a_n.  The right-hand side of each implicit
// stage, T[-lam0 X - ab (D^2 - k^2) X - gb h - zb h'], is therefore formed as
// T[(ab k^2 - lam0) X - gb h - zb h'] - ab X, which never forms D^2 phi or D^2 omega_y.
//
// Per stage the kernel takes the plane pass output H = u x omega at the nodes, forms
// h_v, h_g, the RK3/CN right-hand sides, solves for phi_p, omega_y and v_p, applies the
// 2x2 influence correction, and then prepares the next stage: reconstruction of
// (u, v, w, omega_x, omega_y, omega_z) and their inverse DCT-I.  The (0, 0) pair solves
// the mean flow with the constant-flow-rate pressure gradient.
//
// Geometry: every operator acts on the Chebyshev variable xi, with d/dy = ys d/dxi (closed
// channel ys = 1, open channel ys = 2).  The solve works in xi throughout: wavenumbers scaled
// by 1/ys, the explicit term h_v scaled by 1/ys^2 (phi is carried as (D_xi^2 - k^2/ys^2) v),
// the stage constants built with the viscosity nu ys^2.  The reconstruction returns physical
// y-derivatives.  ys is a power of two, so all these scalings are exact.  In the open channel
// the influence correction imposes d^2v/dxi^2 = 0 at the surface instead of dv/dxi = 0, and
// omega_y and the mean flow are corrected with the top-unit homogeneous solution phi_+ so
// that their xi-derivative vanishes there.
#include <utility>

#include "device_common.h"

namespace chanenv {

namespace {

constexpr int CWAVES = 4;  // columns (wavefronts) per block of the pressure kernel


// Compile-time loops: fn(integral_constant<int, D>) for D = 1, 2, 4, 8 below LIMIT, and for
// K = 0 .. 15.
template <int LIMIT, class Fn>
__device__ __forceinline__ void for_pow2(Fn&& fn) {
  if constexpr (LIMIT > 1) fn(std::integral_constant<int, 1>{});
  if constexpr (LIMIT > 2) fn(std::integral_constant<int, 2>{});
  if constexpr (LIMIT > 4) fn(std::integral_constant<int, 4>{});
  if constexpr (LIMIT > 8) fn(std::integral_constant<int, 8>{});
}
template <class Fn, int... K>
__device__ __forceinline__ void for_each_k(Fn&& fn, std::integer_sequence<int, K...>) {
  (fn(std::integral_constant<int, K>{}), ...);
}
template <class Fn>
__device__ __forceinline__ void for_16(Fn&& fn) {
  for_each_k(fn, std::make_integer_sequence<int, 16>{});
}

// Parity-major bookkeeping of one lane.
template <int N>
struct Lane {
  static constexpr int H = N / 2;
  int l, i, odd, n, rk;
  bool ok, even_row, low;
  __device__ explicit Lane(int lane) {
    l = lane;
    odd = lane >= 32;
    i = lane & 31;
    n = odd ? 2 * i + 1 : 2 * i;
    ok = i < H;
    rk = lane & 15;
    even_row = ((lane >> 4) & 1) == 0;
    low = !odd;
  }
  // (-1)^odd and [even]: parity choices as exact multiplications instead of per-lane selects
  // (recomputed where used rather than held in registers)
  __device__ double sgn() const { return odd ? -1.0 : 1.0; }
  __device__ double evenf() const { return odd ? 0.0 : 1.0; }
};

// Suffix sum over this lane's half: lane i receives sum_{i' >= i} x_{i'} (lanes beyond the
// valid range hold zeros).
template <int H>
__device__ __forceinline__ cplx half_suffix(const cplx x0) {
  cplx x = x0;
  for_pow2<(H < 16 ? H : 16)>([&](auto dc) { x = cadd(x, cmov<DPP_ROW_SHL + decltype(dc)::value>(x)); });
  if constexpr (H > 16) {  // add the second row's total to the first row
    x = cadd(x, from_odd_rows(cmov<DPP_ROW_BCAST + 0>(x)));  // odd rows add 0
  }
  return x;
}

// D: b_n = (2/c_n) sum_{p > n, p + n odd} p a_p.  x: this lane's coefficient, xt: a_N.
// Returns b (b_N = 0).
template <int N>
__device__ __forceinline__ cplx cheb_d(const Lane<N>& L, cplx x, cplx xt) {
  constexpr int H = N / 2;
  const cplx S = half_suffix<H>(L.ok ? cscale(x, (double)L.n) : cz());
  // even n = 2l: odd p >= 2l + 1  -> S at lane 32 + l
  // odd n = 2i + 1: even p >= 2i + 2 -> S at lane i + 1, plus the tail p = N
  const cplx Sn = cmov<DPP_WAVE_SHL1>(S);
  cplx g = make_double2(cross_halves(S.x, Sn.x, L.low), cross_halves(S.y, Sn.y, L.low));
  if (L.odd && L.i + 1 >= H) g = cz();
  const cplx b = caxpy(g, 1.0 - L.evenf(), cscale(xt, (double)N));  // odd lanes add the tail
  const double c = (L.n == 0) ? 1.0 : 2.0;
  return L.ok ? cscale(b, c) : cz();
}

// This lane's tau-row coefficients (rc1, rc2, rc3 and rc1 of the tail row N).
struct RowCoef {
  double r1, r2, r3, rt;
};
template <int N>
__device__ __forceinline__ RowCoef load_rc(const Lane<N>& L, const double* __restrict__ rc) {
  RowCoef t;
  t.r1 = rc[L.l];
  t.r2 = rc[PM_ENTRIES + L.l];
  t.r3 = rc[2 * PM_ENTRIES + L.l];
  t.rt = rc[64];
  return t;
}

// Tau right-hand side rows R_n = rc1 f_{n-2} - rc2 f_n + rc3 f_{n+2} + cx x_n (n >= 2);
// returns the lane's row, and the tail row R_N through rt.
template <int N>
__device__ __forceinline__ cplx tau_rows_pm(const Lane<N>& L, cplx f, cplx ft, const RowCoef& rc, double cx,
                                            cplx x, cplx xt, cplx& rt) {
  constexpr int H = N / 2;
  cplx fm2 = cmov<DPP_WAVE_SHR1>(f);
  if (L.i == 0) fm2 = cz();
  cplx fp2 = cmov<DPP_WAVE_SHL1>(f);
  if (L.i == 31) fp2 = cz();
  if (!L.odd && L.i == H - 1) fp2 = ft;  // n + 2 = N
  cplx r = cscale(fm2, rc.r1);
  r = caxpy(r, -rc.r2, f);
  r = caxpy(r, rc.r3, fp2);
  r = caxpy(r, cx, x);
  // R_N = rc1_N f_{N-2} + cx x_N: f_{N-2} is the even lane H - 1
  const cplx fN2 = readlane_c(f, H - 1);
  rt = caxpy(cscale(fN2, rc.rt), cx, xt);
  return (L.ok && L.n >= 2) ? r : cz();
}

// One operator's elimination record as this lane needs it (w, u, f, F at its index, the
// even tail's w, f, F and the two 1/sum F).
struct TauRec {
  double w, u, fr, F, wt, frt, Ft, isf, isf_even;
};
template <int N>
__device__ __forceinline__ TauRec load_rec(const Lane<N>& L, const double* __restrict__ rec) {
  constexpr int P = PM_ENTRIES;
  TauRec t;
  t.w = rec[L.l];
  t.u = rec[P + L.l];
  t.fr = rec[2 * P + L.l];
  t.F = rec[3 * P + L.l];
  t.wt = rec[64];
  t.frt = rec[2 * P + 64];
  t.Ft = rec[3 * P + 64];
  t.isf = rec[4 * P + L.odd];
  t.isf_even = rec[4 * P];
  return t;
}

// Solve (D^2 - lam) X = f for NR right-hand sides sharing one operator record (w, u, f,
// F, 1/sum F, parity-major), with X(+1) = gt, X(-1) = gb per right-hand side.
template <int N, int NR>
__device__ __forceinline__ void tau_solve_pm(const Lane<N>& L, const cplx* R, const cplx* Rt, const TauRec& tr,
                                             const cplx* gt, const cplx* gb, cplx* X, cplx* Xt) {
  constexpr int H = N / 2;
  const double w = tr.w, u = tr.u, fr = tr.fr, F = tr.F;
  const double wt = tr.wt, frt = tr.frt, Ft = tr.Ft;
  const double isf = tr.isf;
  const double isf_even = tr.isf_even;
  // bottom-up: e_i = A_i + B_i e_{i+1}
  cplx A[NR], et[NR];
  double B = -u;
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    A[k] = cscale(R[k], w);
    et[k] = cscale(Rt[k], wt);  // even tail e_{N/2} = w R_N
  }
  if (L.i == H - 1) {
    if (!L.odd) {
#pragma unroll
      for (int k = 0; k < NR; ++k) A[k] = caxpy(A[k], B, et[k]);
    }
    B = 0.0;
  }
  if (!L.ok || L.i == 0) {
#pragma unroll
    for (int k = 0; k < NR; ++k) A[k] = cz();
    B = 0.0;
  }
  for_pow2<(H < 16 ? H : 16)>([&](auto dc) {
    constexpr int d = decltype(dc)::value;
    const double oB = dmov<DPP_ROW_SHL + d>(B);
    cplx oA[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) oA[k] = cmov<DPP_ROW_SHL + d>(A[k]);
    if (L.rk + d < 16) {
#pragma unroll
      for (int k = 0; k < NR; ++k) A[k] = caxpy(A[k], B, oA[k]);
      B = B * oB;
    }
  });
  if constexpr (H > 16) {  // first row: e_i = A_i + B_i e_16
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const cplx e16 = from_odd_rows(cmov<DPP_ROW_BCAST + 0>(A[k]));  // 0 on the second row
      A[k] = caxpy(A[k], B, e16);
    }
  }
  // top-down: E_i = e_i + f_i E_{i-1}, E_0 = 0
  double C = (L.ok && L.i > 0) ? fr : 0.0;
  for_pow2<(H < 16 ? H : 16)>([&](auto dc) {
    constexpr int d = decltype(dc)::value;
    const double oC = dmov<DPP_ROW_SHR + d>(C);
    cplx oA[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) oA[k] = cmov<DPP_ROW_SHR + d>(A[k]);
    if (L.rk >= d) {
#pragma unroll
      for (int k = 0; k < NR; ++k) A[k] = caxpy(A[k], C, oA[k]);
      C = C * oC;
    }
  });
  if constexpr (H > 16) {  // second row: E_i = A_i + C_i E_15
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const cplx e15 = from_even_rows(cmov<DPP_ROW_BCAST + 15>(A[k]));  // 0 on the first row
      A[k] = caxpy(A[k], C, e15);
    }
  }
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    // even tail E_{N/2} = e_{N/2} + f_{N/2} E_{N/2-1}
    const cplx Elast = readlane_c(A[k], H - 1);
    const cplx Et = caxpy(et[k], frt, Elast);
    cplx sum = half_sum(A[k]);
    const cplx sum_even = readlane_c(sum, 0);
    sum = caxpy(sum, L.evenf(), Et);                            // even lanes: + E_{N/2}
    const cplx g = cscale(caxpy(gt[k], L.sgn(), gb[k]), 0.5);   // (g_t +- g_b) / 2
    const cplx x0 = cscale(csub(g, sum), isf);
    X[k] = L.ok ? caxpy(A[k], F, x0) : cz();
    const cplx ge = cscale(cadd(gt[k], gb[k]), 0.5);
    const cplx x0e = cscale(csub(ge, cadd(sum_even, Et)), isf_even);
    Xt[k] = caxpy(Et, Ft, x0e);
    // The boundary rows to rounding.  x0 comes from 1/sum F and sum E, which cancel heavily
    // when lam is large (the wall layer lives in the top coefficients), so X(+-1) = g holds
    // only to eps sum |E|.  One refinement of x0 per parity removes the row residual
    // r = sum_i X_{2i+s} - g_s along the homogeneous solution F (dx0 = -r / sum F), which
    // leaves the other tau rows as they were and every coefficient to rounding.
    cplx rs = half_sum(X[k]);
    rs = caxpy(rs, L.evenf(), Xt[k]);                           // even lanes: + X_N
    const cplx dx0 = cscale(csub(rs, g), -isf);
    X[k] = L.ok ? caxpy(X[k], F, dx0) : cz();
    Xt[k] = caxpy(Xt[k], Ft, readlane_c(dx0, 0));
  }
}

// acc[g] += c * (lane KK of this lane's row of q[g]) for G = 6 or 12 real vectors, as fused DPP
// FMAs (src0 broadcast from a row lane; the only DPP pattern the FP64 ALU takes).  The leading
// s_nop 4 covers the DPP read-after-VALU-write (2) and EXEC-write (5) wait states, whatever
// the compiler places before the block.
template <int KK, int G>
__device__ __forceinline__ void fmac_row(double (&acc)[G], const double (&q)[G], double c) {
  static_assert(G == 6 || G == 12, "row FMA blocks take 6 or 12 vectors");
  if constexpr (G == 12) {
    asm volatile(
      "s_nop 4\n\t"
      "v_fmac_f64_dpp %0, %12, %24 row_newbcast:%c25 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %1, %13, %24 row_newbcast:%c25 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %2, %14, %24 row_newbcast:%c25 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %3, %15, %24 row_newbcast:%c25 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %4, %16, %24 row_newbcast:%c25 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %5, %17, %24 row_newbcast:%c25 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %6, %18, %24 row_newbcast:%c25 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %7, %19, %24 row_newbcast:%c25 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %8, %20, %24 row_newbcast:%c25 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %9, %21, %24 row_newbcast:%c25 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %10, %22, %24 row_newbcast:%c25 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %11, %23, %24 row_newbcast:%c25 row_mask:0xf bank_mask:0xf"
      : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3]), "+v"(acc[4]), "+v"(acc[5]), "+v"(acc[6]),
        "+v"(acc[7]), "+v"(acc[8]), "+v"(acc[9]), "+v"(acc[10]), "+v"(acc[11])
      : "v"(q[0]), "v"(q[1]), "v"(q[2]), "v"(q[3]), "v"(q[4]), "v"(q[5]), "v"(q[6]), "v"(q[7]), "v"(q[8]),
        "v"(q[9]), "v"(q[10]), "v"(q[11]), "v"(c), "n"(KK));
  } else {
    asm volatile(
      "s_nop 4\n\t"
      "v_fmac_f64_dpp %0, %6, %12 row_newbcast:%c13 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %1, %7, %12 row_newbcast:%c13 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %2, %8, %12 row_newbcast:%c13 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %3, %9, %12 row_newbcast:%c13 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %4, %10, %12 row_newbcast:%c13 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %5, %11, %12 row_newbcast:%c13 row_mask:0xf bank_mask:0xf"
      : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3]), "+v"(acc[4]), "+v"(acc[5])
      : "v"(q[0]), "v"(q[1]), "v"(q[2]), "v"(q[3]), "v"(q[4]), "v"(q[5]), "v"(c), "n"(KK));
  }
}

// Forward DCT-I of F fields, a_n = (2 / (N cb_n)) sum_j f_j cos(pi j n / N) / cb_j, read straight
// from memory (load(g, j): node j of field g).  Folded: g_j = f_j / cb_j, S_j = g_j + g_{N-j},
// D_j = g_j - g_{N-j} (j < N/2); even n need S, odd n need D, and g_{N/2} enters both.  Rows
// 0, 1 (even coefficients) hold S_{16m+k}, rows 2, 3 (odd) hold D_{16m+k} in register group m
// at row position k, so each term of the matvec is a row broadcast (no LDS).  Returns
// parity-major coefficients a (this lane) and the tail a_N.
// CHUNK: request the cosines of each group of 16 terms just before its FMA blocks instead of
// all at once (fewer live registers; the same arithmetic in the same order).
template <int N, int F, bool CHUNK, class Load, class Cos>
__device__ __forceinline__ void dct_fwd_pm(const Lane<N>& L, Load load, Cos cosv, cplx* a, cplx* at) {
  constexpr int H = N / 2;
  constexpr int NQ = (H + 15) / 16;
  const int lane = L.l;
  const bool srow = L.l < 32;
  // this lane's cosines, all requested before the first use (the FMA blocks below are
  // ordering points for memory operations)
  double cf[H + 1];
  if constexpr (!CHUNK) {
#pragma unroll
    for (int j = 0; j <= H; ++j) cf[j] = cosv(j);
  }
  double Q[NQ][2 * F];  // (re, im) of each field
  cplx gh[F];
#pragma unroll
  for (int g = 0; g < F; ++g) {
    gh[g] = load(g, H);
#pragma unroll
    for (int m = 0; m < NQ; ++m) {
      const int j = 16 * m + L.rk;
      cplx q = cz();
      if (j < H) {
        cplx x = load(g, j), y = load(g, N - j);
        if (j == 0) {
          x = cscale(x, 0.5);
          y = cscale(y, 0.5);
        }
        q = srow ? cadd(x, y) : csub(x, y);
      }
      Q[m][2 * g] = q.x;
      Q[m][2 * g + 1] = q.y;
    }
  }
  double acc[2 * F];
#pragma unroll
  for (int g = 0; g < 2 * F; ++g) acc[g] = 0.0;
  auto term = [&](auto kk_c, auto m_c) {
    constexpr int kk = decltype(kk_c)::value;
    constexpr int m = decltype(m_c)::value;
    if constexpr (16 * m + kk < H) fmac_row<kk, 2 * F>(acc, Q[m], cf[16 * m + kk]);
  };
  for_each_k(
      [&](auto m_c) {
        constexpr int m = decltype(m_c)::value;
        if constexpr (CHUNK) {
#pragma unroll
          for (int kk = 0; kk < 16; ++kk)
            if (16 * m + kk < H) cf[16 * m + kk] = cosv(16 * m + kk);
        }
        for_16([&](auto kk_c) { term(kk_c, m_c); });
      },
      std::make_integer_sequence<int, NQ>{});
  if constexpr (CHUNK) cf[H] = cosv(H);
  const double ch = cf[H];
  const double sc = (L.n == 0) ? (1.0 / N) : (2.0 / N);
#pragma unroll
  for (int g = 0; g < F; ++g) {
    a[g] = L.ok ? cscale(caxpy(make_double2(acc[2 * g], acc[2 * g + 1]), ch, gh[g]), sc) : cz();
    // a_N = (1/N) [sum_{j < N/2} (-1)^j S_j + (-1)^{N/2} g_{N/2}]; row 0 holds the S_j
    cplx part = cz();
#pragma unroll
    for (int m = 0; m < NQ; ++m) part = cadd(part, make_double2(Q[m][2 * g], Q[m][2 * g + 1]));
    if (L.rk & 1) part = cscale(part, -1.0);
    const cplx rs = readlane_c(make_double2(row_sum(part.x), row_sum(part.y)), 0);
    at[g] = cscale(caxpy(rs, (H & 1) ? -1.0 : 1.0, gh[g]), 1.0 / N);
  }
}

// Inverse DCT-I: parity-major coefficients (this lane, tail) -> node values in parity-major
// node order (lane l < 32: node 2l, lane 32 + i: node 2i + 1; tail: node N).
// f_j = sum_n a_n cos(pi n j / N), folded with P_n = a_n + a_{N-n}, M_n = a_n - a_{N-n}
// (n < N/2; even nodes need P, odd nodes M) and a_{N/2} in both; the node-N tail is
// sum_n (-1)^n a_n.
template <int N, int F, bool CHUNK, class Cos>
__device__ __forceinline__ void dct_inv_pm(const Lane<N>& L, const cplx* a, const cplx* at, Cos cosv, cplx* f,
                                           cplx* ft) {
  constexpr int H = N / 2;
  constexpr int NQ = (H + 15) / 16;
  constexpr int SH = (H & 1) ? 32 + (H >> 1) : (H >> 1);  // lane of a_{N/2}
  const int lane = L.l;
  double cf[H + 1];  // this lane's cosines, requested up front (or per group of 16, CHUNK)
  if constexpr (!CHUNK) {
#pragma unroll
    for (int n = 0; n <= H; ++n) cf[n] = cosv(n);
  }
  double Q[NQ][2 * F];  // (re, im) of each field
  cplx ah[F];
#pragma unroll
  for (int m = 0; m < NQ; ++m) {
    const int n = 16 * m + L.rk;
    const int n2 = N - n;
    const int s1 = (n & 1) ? 32 + (n >> 1) : (n >> 1);
    const int s2 = (n2 & 1) ? 32 + (n2 >> 1) : (n2 >> 1);
#pragma unroll
    for (int g = 0; g < F; ++g) {
      const cplx x = shfl_c(a[g], s1 & 63);
      cplx y = shfl_c(a[g], s2 & 63);
      if (n == 0) y = at[g];
      const cplx qv = (n < H) ? caxpy(x, L.sgn(), y) : cz();  // P_n (rows 0-1) or M_n (rows 2-3)
      Q[m][2 * g] = qv.x;
      Q[m][2 * g + 1] = qv.y;
    }
  }
#pragma unroll
  for (int g = 0; g < F; ++g) ah[g] = readlane_c(a[g], SH);
  double acc[2 * F];
#pragma unroll
  for (int g = 0; g < 2 * F; ++g) acc[g] = 0.0;
  auto term = [&](auto kk_c, auto m_c) {
    constexpr int kk = decltype(kk_c)::value;
    constexpr int m = decltype(m_c)::value;
    if constexpr (16 * m + kk < H) fmac_row<kk, 2 * F>(acc, Q[m], cf[16 * m + kk]);
  };
  for_each_k(
      [&](auto m_c) {
        constexpr int m = decltype(m_c)::value;
        if constexpr (CHUNK) {
#pragma unroll
          for (int kk = 0; kk < 16; ++kk)
            if (16 * m + kk < H) cf[16 * m + kk] = cosv(16 * m + kk);
        }
        for_16([&](auto kk_c) { term(kk_c, m_c); });
      },
      std::make_integer_sequence<int, NQ>{});
  if constexpr (CHUNK) cf[H] = cosv(H);
  const double ch = cf[H];
#pragma unroll
  for (int g = 0; g < F; ++g) {
    f[g] = L.ok ? caxpy(make_double2(acc[2 * g], acc[2 * g + 1]), ch, ah[g]) : cz();
    const cplx part = L.ok ? cscale(a[g], L.sgn()) : cz();
    ft[g] = cadd(lane_sum(part), at[g]);
  }
}

// Sum over the coefficients of weight(n) x_n, with the tail.
template <int N>
__device__ __forceinline__ cplx coef_sum(const Lane<N>& L, cplx x, cplx xt, double w_lane, double w_tail) {
  cplx part = L.ok ? cscale(x, w_lane) : cz();
  return caxpy(lane_sum(part), w_tail, xt);
}

// Parts of the column pass: the implicit solve of a stage, the reconstruction with the
// inverse DCT that feeds the next plane pass (from the stored state: after the last stage of
// an env step and for set_state), or both in one launch with the solved state kept in
// registers (every other stage).
constexpr int PART_SOLVE = 0, PART_RECON = 1, PART_BOTH = 2;

// Time fraction at the end of RK stage r (c_end of the stage).
__device__ __forceinline__ double stage_end(int r) { return r == 0 ? 8.0 / 15.0 : (r == 1 ? 2.0 / 3.0 : 1.0); }

// One column of a block: wave `wave` of the block takes column c = (p, q).  H at the nodes is
// read from the block's LDS tile Hin ([g][column][node]), and the six reconstructed fields are
// written into its tile Fout ([f][column][node]) for the block's coalesced store.  ctab: the
// block's LDS copy of cos(pi k / N), k < 2N (LDS_COS); the DCTs' cosine cos(pi j n / N) of this
// lane's index n is entry (j n) mod 2N of it, or entry j of the lane's column of the 64-lane table
// in memory (the same double).
template <int N, int PART, bool CHUNK, int CW, bool LDS_COS>
__device__ __forceinline__ void column_body(const ColChan& A, const ColStage& S, int c, int p, int q, int wave,
                                            int status0, const cplx* Hin, cplx* Fout, const double* ctab) {
  constexpr int NY = N + 1;
  const int lane = threadIdx.x & 63;
  const int nz = A.nz;
  const int ln = Lane<N>(lane).n;
  auto cosv = [&](int j) { return LDS_COS ? ctab[(j * ln) & (2 * N - 1)] : A.kfwd[j * 64 + lane]; };
  const bool mean = (c == 0);
  const int partner = (p == 0 && q > 0) ? (nz - q) : -1;
  // the per-column operator tables depend on k^2 only: (p, q) and (p, N_z - q) share them
  const int crec = p * nz + (q > nz / 2 ? nz - q : q);
  const Lane<N> L(lane);
  const double al = A.alpha[p], be = A.beta[q];
  const double k2 = al * al + be * be;
  const size_t col = (size_t)c * NY;
  const int nl = (L.ok ? L.n : 0);  // this lane's coefficient index (for loads)
  const double dn = (double)L.n, dN = (double)N;

  cplx v, om, vt, omt;  // state after this call (mean: v = U + i W, om = 0)

  if constexpr (PART != PART_RECON) {
    const int r = S.stage;
    const double lam0 = A.lam0[r], ab = A.ab[r], gb = A.gb[r], zb = A.zb[r];
    // H1, H2, H3 at node j of this column; the mean flow sees the real parts of H1, H3 only
    auto loadH = [&](int g, int j) {
      cplx x = Hin[(g * CW + wave) * NY + j];
      if (mean && g != 1) x.y = 0.0;
      return x;
    };
    cplx hc[3], hct[3];
    dct_fwd_pm<N, 3, true>(L, loadH, cosv, hc, hct);
    if (status0 & STATUS_BAD_ACTION) return;
    // state (v, omega_y; mean: X = U + i W) and the previous stage's explicit terms
    // (h_v, h_g; mean: h_u + i h_w)
    cplx x0, x0t, y0 = cz(), y0t = cz();
    cplx hp0 = cz(), hp0t = cz(), hp1 = cz(), hp1t = cz();
    cplx* hist_v = A.hist + col;
    cplx* hist_g = A.hist + (size_t)A.ncol * NY + col;
    if (!mean) {
      x0 = L.ok ? A.vS[col + nl] : cz();
      x0t = A.vS[col + N];
      y0 = L.ok ? A.oS[col + nl] : cz();
      y0t = A.oS[col + N];
      if (r > 0) {
        hp0 = L.ok ? hist_v[nl] : cz();
        hp1 = L.ok ? hist_g[nl] : cz();
        hp0t = hist_v[N];
        hp1t = hist_g[N];
      }
    } else {
      x0 = L.ok ? make_double2(A.meanS[nl], A.meanS[NY + nl]) : cz();
      x0t = make_double2(A.meanS[N], A.meanS[NY + N]);
      if (r > 0) {
        if (L.ok) hp0 = make_double2(A.meanH[nl], A.meanH[NY + nl]);
        hp0t = make_double2(A.meanH[N], A.meanH[NY + N]);
      }
    }
    const RowCoef rcf = load_rc<N>(L, A.rc_pm);
    const TauRec rs = load_rec<N>(L, A.op_pm + ((size_t)crec * NOPS + r) * PM_OPSZ);
    TauRec rv = rs;
    cplx vw = cz();
    double mi0 = 0.0, mi1 = 0.0, mi2 = 0.0, mi3 = 0.0, tv = 0.0, tvt = 0.0;
    double iw = 0.0, iwt = 0.0, upl = 0.0, upt = 0.0, iiu = 0.0;
    if (!mean) {
      rv = load_rec<N>(L, A.op_pm + ((size_t)crec * NOPS + 3) * PM_OPSZ);
      if (!A.ext) {
        vw = A.vw_opp[c];
      } else {  // wall velocity ramped from the old to the new action (or the new one held)
        const double s_ramp = A.hold ? 1.0 : (S.m + stage_end(r)) / (double)S.n_sub;
        const cplx o = A.vw_old[c], nn = A.vw_new[c];
        vw = caxpy(o, s_ramp, csub(nn, o));
      }
      const double* mi = A.minv + ((size_t)crec * 3 + r) * 4;
      mi0 = mi[0];
      mi1 = mi[1];
      mi2 = mi[2];
      mi3 = mi[3];
      const double* vtab = A.vt_pm + ((size_t)crec * 3 + r) * PM_ENTRIES;
      tv = vtab[lane];
      tvt = vtab[64];
    } else {
      iw = L.ok ? A.intw_pm[lane] : 0.0;
      iwt = A.intw_pm[64];
      const double* up = A.up_pm + (size_t)r * PM_ENTRIES;
      upl = L.ok ? up[lane] : 0.0;
      upt = up[64];
      iiu = A.inv_int_up[r];
    }

    // wavenumbers in xi (k2s = k^2/ys^2)
    const double als = al * A.ysi, bes = be * A.ysi;
    const double k2s = als * als + bes * bes;
    // tau rows of the implicit stage: T[cx X - gb h - zb h'] - ab X, cx = ab k^2 - lam0
    const double cx = ab * k2s - lam0;
    auto comb = [&](cplx x, cplx h, cplx hp) { return caxpy(caxpy(cscale(x, cx), -gb, h), -zb, hp); };
    if (!mean) {
      // explicit terms: h_v = -k^2 H2 - D(i al H1 + i be H3), h_g = i be H1 - i al H3
      // (h_v / ys^2 in xi: the wavenumbers of the D term and k^2 are the scaled ones)
      const cplx T = cmuli(make_double2(als * hc[0].x + bes * hc[2].x, als * hc[0].y + bes * hc[2].y));
      const cplx Tt = cmuli(make_double2(als * hct[0].x + bes * hct[2].x, als * hct[0].y + bes * hct[2].y));
      // phi0 = (D^2 - k^2) v, independent of the explicit terms
      const cplx dv = cheb_d<N>(L, x0, x0t);
      const cplx dT = cheb_d<N>(L, T, Tt);
      const cplx d2v = cheb_d<N>(L, dv, cz());
      const cplx phi0 = caxpy(d2v, -k2s, x0), phi0t = cscale(x0t, -k2s);
      const cplx hv = csub(cscale(hc[1], -k2s), dT);
      const cplx hvt = cscale(hct[1], -k2s);
      const cplx hg = cmuli(make_double2(be * hc[0].x - al * hc[2].x, be * hc[0].y - al * hc[2].y));
      const cplx hgt = cmuli(make_double2(be * hct[0].x - al * hct[2].x, be * hct[0].y - al * hct[2].y));
      if (r < 2) {
        if (L.ok) {
          hist_v[nl] = hv;
          hist_g[nl] = hg;
        }
        if (lane == 0) {
          hist_v[N] = hvt;
          hist_g[N] = hgt;
        }
      }
      cplx R[2], Rt[2];
      R[0] = tau_rows_pm<N>(L, comb(phi0, hv, hp0), comb(phi0t, hvt, hp0t), rcf, -ab, phi0, phi0t, Rt[0]);
      R[1] = tau_rows_pm<N>(L, comb(y0, hg, hp1), comb(y0t, hgt, hp1t), rcf, -ab, y0, y0t, Rt[1]);
      const cplx zero2[2] = {cz(), cz()};
      cplx X[2], Xt[2];
      tau_solve_pm<N, 2>(L, R, Rt, rs, zero2, zero2, X, Xt);
      // v_p: (D^2 - k^2) v_p = phi_p, v_p(+1) = 0, v_p(-1) = v_w
      cplx Rv[1], Rvt[1];
      Rv[0] = tau_rows_pm<N>(L, X[0], Xt[0], rcf, 0.0, cz(), cz(), Rvt[0]);
      const cplx gtop[1] = {cz()}, gbot[1] = {vw};
      cplx vp[1], vpt[1];
      tau_solve_pm<N, 1>(L, Rv, Rvt, rv, gtop, gbot, vp, vpt);
      // influence correction: dv/dy(-1) = 0 and, at the top, dv/dy = 0 (wall) or
      // d^2v/dy^2 = 0 (surface), with v = v_p + c0 v_+ + c1 v_-
      // (T_n'(1) = n^2, T_n''(1) = n^2 (n^2 - 1)/3, an exact integer)
      const double n2 = dn * dn, N2 = dN * dN;
      const double wtop = A.open ? n2 * (n2 - 1.0) / 3.0 : n2;
      const double wtopt = A.open ? N2 * (N2 - 1.0) / 3.0 : N2;
      const cplx dtop = coef_sum<N>(L, vp[0], vpt[0], wtop, wtopt);
      const cplx dbot = coef_sum<N>(L, vp[0], vpt[0], -L.sgn() * n2, -dN * dN);
      const cplx c0 = make_double2(-(mi0 * dtop.x + mi1 * dbot.x), -(mi0 * dtop.y + mi1 * dbot.y));
      const cplx c1 = make_double2(-(mi2 * dtop.x + mi3 * dbot.x), -(mi2 * dtop.y + mi3 * dbot.y));
      v = caxpy(caxpy(vp[0], tv, c0), L.sgn() * tv, c1);
      vt = caxpy(caxpy(vpt[0], tvt, c0), tvt, c1);
      if (!L.ok) v = cz();
      om = X[1];
      omt = Xt[1];
      if (A.open) {  // d omega_y/dxi (+1) = 0: add c phi_+
        const double* ptab = A.pt_pm + ((size_t)crec * 3 + r) * PM_ENTRIES;
        const double pl = ptab[lane], plt = ptab[64];
        const cplx dw = coef_sum<N>(L, om, omt, n2, N2);
        const double pinv = A.ptinv[(size_t)crec * 3 + r];
        const cplx cw = make_double2(-dw.x * pinv, -dw.y * pinv);
        om = caxpy(om, pl, cw);
        omt = caxpy(omt, plt, cw);
      }
      cplx* vout = A.vS + col;
      cplx* oout = A.oS + col;
      if (L.ok) {
        vout[nl] = v;
        oout[nl] = om;
      }
      if (lane == 0) {
        vout[N] = vt;
        oout[N] = omt;
      }
      if (partner >= 0) {
        cplx* vpo = A.vS + (size_t)partner * NY;
        cplx* opo = A.oS + (size_t)partner * NY;
        if (L.ok) {
          vpo[nl] = cconj(v);
          opo[nl] = cconj(om);
        }
        if (lane == 0) {
          vpo[N] = cconj(vt);
          opo[N] = cconj(omt);
        }
      }
      bool ok = isfinite(v.x) && isfinite(v.y) && isfinite(om.x) && isfinite(om.y) && isfinite(vt.x) &&
                isfinite(vt.y) && isfinite(omt.x) && isfinite(omt.y);
      if (r == 2 && __any(!ok) && lane == 0) atomicOr(A.status, STATUS_NONFINITE);
    } else {
      // mean flow, packed X = U + i W; h = h_u + i h_w (k = 0)
      const cplx hm = make_double2(hc[0].x, hc[2].x), hmt = make_double2(hct[0].x, hct[2].x);
      if (r < 2) {
        if (L.ok) {
          A.meanH[nl] = hm.x;
          A.meanH[NY + nl] = hm.y;
        }
        if (lane == 0) {
          A.meanH[N] = hmt.x;
          A.meanH[NY + N] = hmt.y;
        }
      }
      cplx R[1], Rt[1];
      R[0] = tau_rows_pm<N>(L, comb(x0, hm, hp0), comb(x0t, hmt, hp0t), rcf, -ab, x0, x0t, Rt[0]);
      const cplx z1[1] = {cz()};
      cplx Xs[1], Xst[1];
      tau_solve_pm<N, 1>(L, R, Rt, rs, z1, z1, Xs, Xst);
      if (A.open) {  // dU/dxi (+1) = dW/dxi (+1) = 0: add c phi_+ (k = 0)
        const double* ptab = A.pt_pm + (size_t)r * PM_ENTRIES;
        const double pl = ptab[lane], plt = ptab[64];
        const cplx ds = coef_sum<N>(L, Xs[0], Xst[0], dn * dn, dN * dN);
        const double pinv = A.ptinv[r];
        const cplx cu = make_double2(-ds.x * pinv, -ds.y * pinv);
        Xs[0] = caxpy(Xs[0], pl, cu);
        Xst[0] = caxpy(Xst[0], plt, cu);
      }
      double flux = lane_sum(iw * Xs[0].x) + iwt * Xst[0].x;
      const double P_r = (A.forcing == 0) ? (A.ub2 - flux) * iiu : A.px;
      const double U = fma(P_r, upl, Xs[0].x);
      const double Ut = fma(P_r, upt, Xst[0].x);
      v = L.ok ? make_double2(U, Xs[0].y) : cz();
      vt = make_double2(Ut, Xst[0].y);
      om = omt = cz();
      if (L.ok) {
        A.meanS[nl] = v.x;
        A.meanS[NY + nl] = v.y;
      }
      if (lane == 0) {
        A.meanS[N] = vt.x;
        A.meanS[NY + N] = vt.y;
      }
      const double n2 = dn * dn;
      const double slope = lane_sum(L.ok ? (-L.sgn() * n2) * v.x : 0.0) - dN * dN * vt.x;
      if (r == 2 && lane == 0) A.drag_acc[0] += A.nu_wall * slope;  // drag: end of every time step
      const bool ok = isfinite(v.x) && isfinite(v.y) && isfinite(vt.x) && isfinite(vt.y);
      if (r == 2 && __any(!ok) && lane == 0) atomicOr(A.status, STATUS_NONFINITE);
    }
  } else {
    // load the state
    if (mean) {
      v = L.ok ? make_double2(A.meanS[nl], A.meanS[NY + nl]) : cz();
      vt = make_double2(A.meanS[N], A.meanS[NY + N]);
      om = omt = cz();
    } else {
      v = L.ok ? A.vS[col + nl] : cz();
      vt = A.vS[col + N];
      om = L.ok ? A.oS[col + nl] : cz();
      omt = A.oS[col + N];
    }
  }

  // ---------------- reconstruction and inverse DCT for the next stage ----------------
  if constexpr (PART == PART_SOLVE) return;
  const bool want_end = (S.stage == 2 || S.stage < 0);  // end of a time step
  cplx fld[6], fldt[6];  // (u, v, w, omega_x, omega_y, omega_z) coefficients
  cplx tau_hat;
  if (!mean) {
    const double ik2 = 1.0 / k2;
    const cplx dv = cheb_d<N>(L, v, vt);  // dv/dxi; dv/dy = ys dv/dxi
    const double aly = al * A.ys, bey = be * A.ys;
    const cplx u = cscale(cmuli(make_double2(aly * dv.x - be * om.x, aly * dv.y - be * om.y)), ik2);
    const cplx w = cscale(cmuli(make_double2(bey * dv.x + al * om.x, bey * dv.y + al * om.y)), ik2);
    const cplx ut = cscale(cmuli(make_double2(-be * omt.x, -be * omt.y)), ik2);
    const cplx wt = cscale(cmuli(make_double2(al * omt.x, al * omt.y)), ik2);
    const cplx du = cheb_d<N>(L, u, ut);
    const cplx dw = cheb_d<N>(L, w, wt);
    fld[0] = u;
    fldt[0] = ut;
    fld[1] = v;
    fldt[1] = vt;
    fld[2] = w;
    fldt[2] = wt;
    fld[3] = csub(cscale(dw, A.ys), cmuli(cscale(v, be)));
    fldt[3] = cscale(cmuli(vt), -be);
    fld[4] = om;
    fldt[4] = omt;
    fld[5] = csub(cmuli(cscale(v, al)), cscale(du, A.ys));
    fldt[5] = cscale(cmuli(vt), al);
    const double n2 = dn * dn;
    tau_hat = cscale(coef_sum<N>(L, u, ut, -L.sgn() * n2, -dN * dN), A.nu_wall);
  } else {
    const cplx dX = cheb_d<N>(L, v, vt);
    fld[0] = make_double2(v.x, 0.0);
    fldt[0] = make_double2(vt.x, 0.0);
    fld[1] = fldt[1] = cz();
    fld[2] = make_double2(v.y, 0.0);
    fldt[2] = make_double2(vt.y, 0.0);
    fld[3] = make_double2(A.ys * dX.y, 0.0);
    fldt[3] = cz();
    fld[4] = fldt[4] = cz();
    fld[5] = make_double2(-(A.ys * dX.x), 0.0);
    fldt[5] = cz();
    const double n2 = dn * dn;
    const double slope = lane_sum(L.ok ? (-L.sgn() * n2) * v.x : 0.0) - dN * dN * vt.x;
    tau_hat = make_double2(A.nu_wall * slope, 0.0);
  }
  cplx ph[6], pht[6];
  dct_inv_pm<N, 6, CHUNK>(L, fld, fldt, cosv, ph, pht);
  if (status0 & STATUS_BAD_ACTION) return;
  // the six fields at the nodes (this lane: node n; lane 0 also node N) into the block's tile
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    cplx val = ph[f], valt = pht[f];
    if (mean) {
      val.y = 0.0;
      valt.y = 0.0;
    }
    cplx* dst = Fout + (f * CW + wave) * NY;
    if (L.ok) dst[nl] = val;
    if (lane == 0) dst[N] = valt;
  }
  if (want_end) {
    // opposition target from v at the sensing node (js < N), Hermitian partner too
    if (L.ok && L.n == A.js) {
      const cplx opp = mean ? cz() : cscale(ph[1], -A.opp_alpha);
      A.vw_opp[c] = opp;
      if (partner >= 0) A.vw_opp[partner] = cconj(opp);
    }
    if (lane == 0) {
      A.tauw[c] = tau_hat;
      if (partner >= 0) A.tauw[partner] = cconj(tau_hat);
    }
  }
}

// One block of CW columns (block cb of the channel's columns): one p, CW consecutive q (CW
// divides N_z), one wavefront per column.  H of the block's columns is loaded into LDS and the
// reconstructed fields stored from LDS by the whole block with q fastest, so that a load or
// store instruction covers CW consecutive q of 64 / CW nodes instead of 64 nodes of one column
// (every node of a column lies in its own cache line of the node-major planes).  Every wave
// reaches the block's barriers: a Nyquist or partner-written column, or a rejected action,
// only skips its work and its stores.
template <int N, int PART, bool CHUNK, int CW, bool LDS_COS>
__device__ __forceinline__ void column_block(const ColChan& A, const ColStage& S, int cb, cplx* tile) {
  constexpr int NY = N + 1;
  const int wave = threadIdx.x >> 6;
  const int nz = A.nz;
  const int c0 = cb * CW;
  if (c0 >= A.ncol) return;  // whole block (N_x/2 N_z is a multiple of CW)
  const int p = c0 / nz, q0 = c0 - p * nz;
  const size_t jstride = (size_t)A.nkx * nz;
  // a rejected action skips the step: tested before every store
  const int status0 = *A.status;
  cplx* Hin = tile;                 // [g][column][node]
  cplx* Fout = tile + 3 * CW * NY;  // [f][column][node]
  double* ctab = reinterpret_cast<double*>(tile + 9 * CW * NY);  // cos(pi k / N), k < 2N
  if constexpr (LDS_COS)
    for (int t = threadIdx.x; t < 2 * N; t += 64 * CW) ctab[t] = A.ccos[t];
  if constexpr (PART != PART_RECON) {
    const cplx* src = A.H3 + (size_t)p * nz + q0;
#pragma unroll 1
    for (int t = threadIdx.x; t < 3 * NY * CW; t += 64 * CW) {
      const int qq = t % CW, gj = t / CW;
      const int g = gj / NY, j = gj - g * NY;
      Hin[(g * CW + qq) * NY + j] = src[g * A.plane + (size_t)j * jstride + qq];
    }
  }
  __syncthreads();
  const int q = q0 + wave;
  const int c = __builtin_amdgcn_readfirstlane(c0 + wave);
  // Nyquist columns are never stored; (0, q > N_z/2) is written by its Hermitian partner (0, -q)
  if (q != nz / 2 && !(p == 0 && q > nz / 2))
    column_body<N, PART, CHUNK, CW, LDS_COS>(A, S, c, p, q, wave, status0, Hin, Fout, ctab);
  if constexpr (PART == PART_SOLVE) return;
  __syncthreads();
  if (status0 & STATUS_BAD_ACTION) return;
  cplx* dst = A.F6 + (size_t)p * nz + q0;
#pragma unroll 1
  for (int t = threadIdx.x; t < 6 * NY * CW; t += 64 * CW) {
    const int qq = t % CW, fj = t / CW;
    const int f = fj / NY, j = fj - f * NY;
    const int qc = q0 + qq;
    if (qc == nz / 2 || (p == 0 && qc > nz / 2)) continue;
    const cplx val = Fout[(f * CW + qq) * NY + j];
    const size_t o = f * A.plane + (size_t)j * jstride;
    dst[o + qq] = val;
    if (p == 0 && qc > 0) A.F6[o + (nz - qc)] = cconj(val);  // Hermitian partner (0, -q)
  }
}

// Many channels: channel blockIdx.x / bpc of the device array.  With many columns resident,
// occupancy hides load latency: the reconstruction requests its cosines per group of 16
// terms, which keeps the reconstruction and the fused launch within three waves per SIMD
// (138 and 164 VGPRs at N = 64; all cosines up front needs more than 170).
// CW columns per block, chosen per grid shape by the batch's tuner (2 or 4: the 16x65x16 channels
// of a large batch run about 3 % faster two per block, the 32x65x32 ones as fast four per block).
template <int N, int PART, int CW>
__global__ __launch_bounds__(64 * CW, 3) void k_column_pm(const ColChan* __restrict__ chans, ColStage S, int bpc) {
  // contiguous block ranges per XCD: 23.8 -> 20.6 ms of column launches per env step of the
  // 256-channel batch (the one-channel launch below, all blocks resident at once, is 2 % slower
  // with the same mapping)
  __shared__ double tile[9 * CW * (N + 1) * 2];
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int ch = b / bpc;
  column_block<N, PART, PART != PART_SOLVE, CW, false>(chans[ch], S, b - ch * bpc, reinterpret_cast<cplx*>(tile));
}

// One channel, its arguments by value (preloaded with the kernel arguments instead of read
// through a pointer); the same column code as the batched kernel.  CW columns per block: few
// columns spread over more CUs in small blocks (the minimal channel, 120 columns, steps about
// 5 % faster with one per block), many fill the CUs better in blocks of four (the larger
// channel, 1984 columns, 8 % slower with one per block).
template <int N, int PART, int CW>
__global__ __launch_bounds__(64 * CW, 2) void k_column_pm1(ColChan A, ColStage S) {
  __shared__ double tile[9 * CW * (N + 1) * 2 + 2 * N];
  // contiguous block ranges per XCD: neighbouring blocks share the cache lines of their tiles
  column_block<N, PART, false, CW, true>(A, S, xcd_block(blockIdx.x, gridDim.x), reinterpret_cast<cplx*>(tile));
}

// Columns per block of the single-channel launch for ncol columns.
inline int single_channel_cw(int ncol) { return ncol <= 256 ? 1 : (ncol <= 1024 ? 2 : 4); }

template <int N, int CW>
int launch_pm1(const ColChan& A, int ncol, const ColStage& S, bool solve, bool recon, hipStream_t st,
               KernelTimer* tm) {
  const dim3 grid((ncol + CW - 1) / CW), block(64 * CW);
  if (solve && recon) {
    timed_launch(tm, KC_FUSED, k_column_pm1<N, PART_BOTH, CW>, grid, block, 0, st, A, S);
    return hipGetLastError() == hipSuccess ? 0 : -1;
  }
  if (solve) {
    timed_launch(tm, KC_COLUMN, k_column_pm1<N, PART_SOLVE, CW>, grid, block, 0, st, A, S);
    if (hipGetLastError() != hipSuccess) return -1;
  }
  if (recon) {
    timed_launch(tm, KC_RECON, k_column_pm1<N, PART_RECON, CW>, grid, block, 0, st, A, S);
    if (hipGetLastError() != hipSuccess) return -1;
  }
  return 0;
}

template <int N, int CW>
int launch_pmb(const ColChan* d_col, int nch, int ncol, const ColStage& S, bool solve, bool recon, hipStream_t st,
               KernelTimer* tm) {
  const int bpc = (ncol + CW - 1) / CW;
  const dim3 grid(bpc * nch), block(64 * CW);
  if (solve && recon) {
    timed_launch(tm, KC_FUSED, k_column_pm<N, PART_BOTH, CW>, grid, block, 0, st, d_col, S, bpc);
    return hipGetLastError() == hipSuccess ? 0 : -1;
  }
  if (solve) {
    timed_launch(tm, KC_COLUMN, k_column_pm<N, PART_SOLVE, CW>, grid, block, 0, st, d_col, S, bpc);
    if (hipGetLastError() != hipSuccess) return -1;
  }
  if (recon) {
    timed_launch(tm, KC_RECON, k_column_pm<N, PART_RECON, CW>, grid, block, 0, st, d_col, S, bpc);
    if (hipGetLastError() != hipSuccess) return -1;
  }
  return 0;
}

template <int N>
int launch_pm(const ColChan* d_col, const ColChan* h_col, int nch, int ncol, const ColStage& S, bool solve,
              bool recon, hipStream_t st, KernelTimer* tm, int batch_cw) {
  // Both parts in one launch: the solved state stays in registers for the reconstruction,
  // which saves a kernel boundary and the state's reload.  (Every stage of every batch takes
  // this path, so a channel's arithmetic does not depend on the batch it is in; neither does
  // it depend on the block shape.)
  if (nch == 1 && h_col != nullptr) {
    switch (single_channel_cw(ncol)) {
      case 1: return launch_pm1<N, 1>(h_col[0], ncol, S, solve, recon, st, tm);
      case 2: return launch_pm1<N, 2>(h_col[0], ncol, S, solve, recon, st, tm);
      default: return launch_pm1<N, 4>(h_col[0], ncol, S, solve, recon, st, tm);
    }
  }
  switch (batch_cw) {
    case 2: return launch_pmb<N, 2>(d_col, nch, ncol, S, solve, recon, st, tm);
    case 4: return launch_pmb<N, 4>(d_col, nch, ncol, S, solve, recon, st, tm);
    default: return -1;
  }
}

// Pressure on the observation planes (the observable p - <p>_plane; end of an env step, after a
// plane pass of the end-of-step state filled H3).  With P = p + |u|^2/2, per pair k != 0:
//   (D^2 - k^2) P = i al H1 + D H2 + i be H3,   dP/dy = H2 + nu (D^2 - k^2) v - dv/dt at both
// boundaries (dv/dt: the lower wall's velocity rate, a ramped external action's slope).  In xi:
// (D_xi^2 - k^2/ys^2) P = (i (al H1 + be H3)/ys + D_xi H2)/ys, dP/dxi = (dP/dy)/ys.  Tau
// solution with zero values, plus c_+ phi_+ + c_- phi_- for the two Neumann conditions; P is
// then evaluated at each plane's node.  The (0, 0) pair (plane means) is set to zero.
template <int N>
__device__ __forceinline__ void pressure_block(const ColChan& A, const ColStage& S, int cb) {
  constexpr int NY = N + 1;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c = __builtin_amdgcn_readfirstlane(cb * CWAVES + wave);
  if (c >= A.ncol || A.n_pplanes <= 0) return;
  const int nz = A.nz;
  const int p = c / nz, q = c - p * nz;
  if (q == nz / 2) return;
  if (p == 0 && q > nz / 2) return;
  const int partner = (p == 0 && q > 0) ? (nz - q) : -1;
  const size_t pstride = (size_t)A.nkx * nz;
  cplx* pout = A.pbuf;
  if (c == 0) {
    if (lane < A.n_pplanes) pout[(size_t)lane * pstride] = cz();
    return;
  }
  const Lane<N> L(lane);
  const double al = A.alpha[p], be = A.beta[q];
  const double als = al * A.ysi, bes = be * A.ysi;
  const double k2s = als * als + bes * bes;
  const double dn = (double)L.n, dN = (double)N;
  // H1, H2, H3 at the nodes of this column -> Chebyshev coefficients
  const cplx* h3 = A.H3 + (size_t)p * nz + q;
  const size_t jstride = (size_t)A.nkx * nz;
  auto loadH = [&](int g, int j) { return h3[g * A.plane + (size_t)j * jstride]; };
  cplx hc[3], hct[3];
  dct_fwd_pm<N, 3, false>(L, loadH, [&](int j) { return A.kfwd[j * 64 + lane]; }, hc, hct);
  const int nl = (L.ok ? L.n : 0);
  const size_t col = (size_t)c * NY;
  const cplx v = L.ok ? A.vS[col + nl] : cz();
  const cplx vt = A.vS[col + N];
  // right-hand side in xi
  const cplx dH2 = cheb_d<N>(L, hc[1], hct[1]);
  const cplx ab = cmuli(make_double2(als * hc[0].x + bes * hc[2].x, als * hc[0].y + bes * hc[2].y));
  const cplx abt = cmuli(make_double2(als * hct[0].x + bes * hct[2].x, als * hct[0].y + bes * hct[2].y));
  // ab = i (al H1 + be H3)/ys already carries one 1/ys
  const cplx f = cscale(cadd(dH2, ab), A.ysi);
  const cplx ft = cscale(abt, A.ysi);
  const RowCoef rcf = load_rc<N>(L, A.rc_pm);
  const int crec = p * nz + (q > nz / 2 ? nz - q : q);  // tables shared by (p, +-q)
  const TauRec rk = load_rec<N>(L, A.op_pm + ((size_t)crec * NOPS + 3) * PM_OPSZ);
  cplx R[1], Rt[1];
  R[0] = tau_rows_pm<N>(L, f, ft, rcf, 0.0, cz(), cz(), Rt[0]);
  const cplx z1[1] = {cz()};
  cplx P[1], Pt[1];
  tau_solve_pm<N, 1>(L, R, Rt, rk, z1, z1, P, Pt);
  // Neumann data at +1 (top) and -1 (bottom), in xi
  const double n2 = dn * dn, N2 = dN * dN;
  const double w2 = n2 * (n2 - 1.0) / 3.0, w2t = N2 * (N2 - 1.0) / 3.0;  // T_n''(1)
  const cplx d2v_top = coef_sum<N>(L, v, vt, w2, w2t);
  const cplx d2v_bot = coef_sum<N>(L, v, vt, L.sgn() * w2, w2t);
  const cplx v_top = coef_sum<N>(L, v, vt, 1.0, 1.0);
  const cplx v_bot = coef_sum<N>(L, v, vt, L.sgn(), 1.0);
  const double nux = A.nu_wall * A.ys;  // nu ys^2
  const cplx H2_top = loadH(1, 0), H2_bot = loadH(1, N);
  cplx rate = cz();
  if (A.ext && !A.hold) {
    const cplx o = A.vw_old[c], nn = A.vw_new[c];
    rate = cscale(csub(nn, o), 1.0 / ((double)S.n_sub * A.dt));
  }
  // g = H2 + nu' (D_xi^2 - k'^2) v - dv/dt, then / ys
  const cplx g_top = cscale(caxpy(H2_top, nux, caxpy(d2v_top, -k2s, v_top)), A.ysi);
  const cplx g_bot = cscale(csub(caxpy(H2_bot, nux, caxpy(d2v_bot, -k2s, v_bot)), rate), A.ysi);
  const cplx dP_top = coef_sum<N>(L, P[0], Pt[0], n2, N2);
  const cplx dP_bot = coef_sum<N>(L, P[0], Pt[0], -L.sgn() * n2, -N2);
  const cplx r_top = csub(g_top, dP_top), r_bot = csub(g_bot, dP_bot);
  const double* mi = A.pkinv + (size_t)crec * 4;
  const cplx c0 = make_double2(mi[0] * r_top.x + mi[1] * r_bot.x, mi[0] * r_top.y + mi[1] * r_bot.y);
  const cplx c1 = make_double2(mi[2] * r_top.x + mi[3] * r_bot.x, mi[2] * r_top.y + mi[3] * r_bot.y);
  const double* ptab = A.pk_pm + (size_t)crec * PM_ENTRIES;
  const double pl = ptab[lane], plt = ptab[64];
  cplx Pc = caxpy(caxpy(P[0], pl, c0), L.sgn() * pl, c1);
  const cplx Pct = caxpy(caxpy(Pt[0], plt, c0), plt, c1);
  if (!L.ok) Pc = cz();
  // value at each plane's node j: sum_n P_n cos(pi n j/N); cos(pi n j/N) = (-1)^n cos(pi n (N-j)/N)
  for (int k = 0; k < A.n_pplanes; ++k) {
    const int j = A.pjs[k];
    const bool flip = j > N / 2;
    const int jj = flip ? N - j : j;
    const double cw = A.kfwd[(size_t)jj * 64 + lane] * (flip ? L.sgn() : 1.0);
    const double tail = (j & 1) ? -1.0 : 1.0;
    const cplx val = make_double2(lane_sum(cw * Pc.x) + tail * Pct.x, lane_sum(cw * Pc.y) + tail * Pct.y);
    if (lane == 0) {
      pout[(size_t)k * pstride + (size_t)p * nz + q] = val;
      if (partner >= 0) pout[(size_t)k * pstride + partner] = cconj(val);
    }
  }
}

template <int N>
__global__ __launch_bounds__(64 * CWAVES, 2) void k_pressure_pm(const ColChan* __restrict__ chans, ColStage S, int bpc) {
  const int ch = blockIdx.x / bpc;
  pressure_block<N>(chans[ch], S, blockIdx.x - ch * bpc);
}

}  // namespace

int launch_column_pm(const Dims& d, const ColChan* d_col, const ColChan* h_col, int nch, const ColStage& S,
                     bool solve, bool recon, hipStream_t st, KernelTimer* tm, int batch_cw) {
  if (nch < 1) return 0;
  switch (d.N) {
    case 16: return launch_pm<16>(d_col, h_col, nch, d.ncol, S, solve, recon, st, tm, batch_cw);
    case 32: return launch_pm<32>(d_col, h_col, nch, d.ncol, S, solve, recon, st, tm, batch_cw);
    case 64: return launch_pm<64>(d_col, h_col, nch, d.ncol, S, solve, recon, st, tm, batch_cw);
    default: return -1;
  }
}

int launch_pressure_pm(const Dims& d, const ColChan* d_col, int nch, const ColStage& S, hipStream_t st,
                       KernelTimer* tm) {
  if (nch < 1) return 0;
  const int bpc = (d.ncol + CWAVES - 1) / CWAVES;
  const dim3 grid(bpc * nch), block(64 * CWAVES);
  switch (d.N) {
    case 16: timed_launch(tm, KC_OUTPUT, k_pressure_pm<16>, grid, block, 0, st, d_col, S, bpc); break;
    case 32: timed_launch(tm, KC_OUTPUT, k_pressure_pm<32>, grid, block, 0, st, d_col, S, bpc); break;
    case 64: timed_launch(tm, KC_OUTPUT, k_pressure_pm<64>, grid, block, 0, st, d_col, S, bpc); break;
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace chanenv
