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
// Node values (for the DCT-I and the plane pass) are in plain lane order: lane j holds
// node j < N and node N is the tail.
//
// Per stage the kernel takes the plane pass output H = u x omega at the nodes, forms
// h_v, h_g, the RK3/CN right-hand sides, solves for phi_p, omega_y and v_p, applies the
// 2x2 influence correction, and then prepares the next stage: reconstruction of
// (u, v, w, omega_x, omega_y, omega_z) and their inverse DCT-I.  The (0, 0) pair solves
// the mean flow with the constant-flow-rate pressure gradient.
#include "device_common.h"

namespace chanenv {

namespace {

constexpr int CWAVES = 4;  // columns (wavefronts) per block

struct ColArgsPm {
  int nkx, nz, ncol;
  int stage;            // 0, 1, 2; -1: reconstruct only
  int wall_mode;
  double s_ramp;
  double lam0, ab, gb, zb;
  double nu, opp_alpha, ub2, px;
  int forcing, js, accumulate_drag;
  int recon;            // 0: skip the reconstruction for the next stage
  size_t plane;         // elements per field in F6 / H3 (ny nkx nz)
  cplx *vS, *oS, *hist;
  double *meanS, *meanH;
  const cplx* H3;
  cplx* F6;
  const cplx *vw_old, *vw_new;
  cplx *vw_opp, *tauw;
  const double *kfwd, *kinv, *rc_pm, *intw_pm, *op_pm, *vt_pm, *up_pm, *minv, *inv_int_up, *alpha, *beta;
  double* drag_acc;
  int* status;
};

__device__ __forceinline__ cplx shfl_c(cplx v, int src) {
  return make_double2(__shfl(v.x, src, 64), __shfl(v.y, src, 64));
}
__device__ __forceinline__ cplx shfl_down32(cplx v, int d) {
  return make_double2(__shfl_down(v.x, d, 32), __shfl_down(v.y, d, 32));
}
__device__ __forceinline__ cplx shfl_up32(cplx v, int d) {
  return make_double2(__shfl_up(v.x, d, 32), __shfl_up(v.y, d, 32));
}
// Sum over the 32 lanes of this lane's half (every lane of the half gets the same value).
__device__ __forceinline__ cplx half_sum(cplx v) {
#pragma unroll
  for (int off = 16; off > 0; off >>= 1) {
    v.x += __shfl_xor(v.x, off, 64);
    v.y += __shfl_xor(v.y, off, 64);
  }
  return v;
}

// Parity-major bookkeeping of one lane.
template <int N>
struct Lane {
  static constexpr int H = N / 2;
  int l, i, odd, n;
  bool ok;
  __device__ explicit Lane(int lane) {
    l = lane;
    odd = lane >= 32;
    i = lane & 31;
    n = odd ? 2 * i + 1 : 2 * i;
    ok = i < H;
  }
};

// D: b_n = (2/c_n) sum_{p > n, p + n odd} p a_p.  x: this lane's coefficient, xt: a_N.
// Returns b (b_N = 0).
template <int N>
__device__ __forceinline__ cplx cheb_d(const Lane<N>& L, cplx x, cplx xt) {
  constexpr int H = N / 2;
  cplx S = L.ok ? cscale(x, (double)L.n) : cz();
#pragma unroll
  for (int d = 1; d < 32; d <<= 1) {
    const cplx o = shfl_down32(S, d);
    if (L.i + d < 32) S = cadd(S, o);
  }
  // even n = 2l: odd p >= 2l + 1  -> S at lane 32 + l
  // odd n = 2i + 1: even p >= 2i + 2 -> S at lane i + 1, plus the tail p = N
  const cplx from_odd = shfl_c(S, (L.l + 32) & 63);
  cplx from_even = shfl_c(S, (L.i + 1) & 31);
  if (L.i + 1 >= H) from_even = cz();
  cplx b = L.odd ? cadd(from_even, cscale(xt, (double)N)) : from_odd;
  const double c = (L.n == 0) ? 1.0 : 2.0;
  return L.ok ? cscale(b, c) : cz();
}

// Tau right-hand side rows R_n = rc1 f_{n-2} - rc2 f_n + rc3 f_{n+2} (n >= 2); returns the
// lane's row, and the tail row R_N through rt.
template <int N>
__device__ __forceinline__ cplx tau_rows_pm(const Lane<N>& L, cplx f, cplx ft, const double* __restrict__ rc,
                                            cplx& rt) {
  constexpr int H = N / 2;
  const cplx fm2 = shfl_up32(f, 1);
  cplx fp2 = shfl_down32(f, 1);
  if (!L.odd && L.i == H - 1) fp2 = ft;  // n + 2 = N
  const double r1 = rc[L.l], r2 = rc[PM_ENTRIES + L.l], r3 = rc[2 * PM_ENTRIES + L.l];
  cplx r = cscale(fm2, r1);
  r = caxpy(r, -r2, f);
  r = caxpy(r, r3, fp2);
  // R_N = rc1_N f_{N-2}: f_{N-2} is the even lane H - 1
  const cplx fN2 = shfl_c(f, H - 1);
  rt = cscale(fN2, rc[64]);
  return (L.ok && L.n >= 2) ? r : cz();
}

// Solve (D^2 - lam) X = f for NR right-hand sides sharing one operator record (w, u, f,
// F, 1/sum F, parity-major), with X(+1) = gt, X(-1) = gb per right-hand side.
template <int N, int NR>
__device__ __forceinline__ void tau_solve_pm(const Lane<N>& L, const cplx* R, const cplx* Rt,
                                             const double* __restrict__ rec, const cplx* gt, const cplx* gb,
                                             cplx* X, cplx* Xt) {
  constexpr int H = N / 2;
  constexpr int P = PM_ENTRIES;
  const double w = rec[L.l], u = rec[P + L.l], fr = rec[2 * P + L.l], F = rec[3 * P + L.l];
  const double wt = rec[64], frt = rec[2 * P + 64], Ft = rec[3 * P + 64];
  const double isf = rec[4 * P + L.odd];
  const double isf_even = rec[4 * P];
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
#pragma unroll
  for (int d = 1; d < 32; d <<= 1) {
    const double oB = __shfl_down(B, d, 32);
    cplx oA[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) oA[k] = shfl_down32(A[k], d);
    if (L.i + d < 32) {
#pragma unroll
      for (int k = 0; k < NR; ++k) A[k] = caxpy(A[k], B, oA[k]);
      B = B * oB;
    }
  }
  // top-down: E_i = e_i + f_i E_{i-1}, E_0 = 0
  double C = (L.ok && L.i > 0) ? fr : 0.0;
#pragma unroll
  for (int d = 1; d < 32; d <<= 1) {
    const double oC = __shfl_up(C, d, 32);
    cplx oA[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) oA[k] = shfl_up32(A[k], d);
    if (L.i >= d) {
#pragma unroll
      for (int k = 0; k < NR; ++k) A[k] = caxpy(A[k], C, oA[k]);
      C = C * oC;
    }
  }
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    // even tail E_{N/2} = e_{N/2} + f_{N/2} E_{N/2-1}
    const cplx Elast = shfl_c(A[k], H - 1);
    const cplx Et = caxpy(et[k], frt, Elast);
    cplx sum = half_sum(A[k]);
    const cplx sum_even = shfl_c(sum, 0);
    if (!L.odd) sum = cadd(sum, Et);
    const cplx g = L.odd ? cscale(csub(gt[k], gb[k]), 0.5) : cscale(cadd(gt[k], gb[k]), 0.5);
    const cplx x0 = cscale(csub(g, sum), isf);
    X[k] = L.ok ? caxpy(A[k], F, x0) : cz();
    const cplx ge = cscale(cadd(gt[k], gb[k]), 0.5);
    const cplx x0e = cscale(csub(ge, cadd(sum_even, Et)), isf_even);
    Xt[k] = caxpy(Et, Ft, x0e);
  }
}

// Forward DCT-I of F node vectors (this lane's node j = lane < N, tail = node N), giving
// parity-major coefficients a (this lane) and the tail a_N.
template <int N, int F>
__device__ __forceinline__ void dct_fwd_pm(const Lane<N>& L, const cplx* f, const cplx* ft,
                                           const double* __restrict__ kfwd, cplx* Sb, cplx* a, cplx* at) {
  constexpr int H = N / 2;
  constexpr int HP = H + 1;
  const int lane = L.l;
  // fold: g_j = f_j / cb_j; S_j = g_j + g_{N-j}, D_j = g_j - g_{N-j} (j < N/2), S = D = g at N/2
  const int partner = (N - lane) & 63;
#pragma unroll
  for (int k = 0; k < F; ++k) {
    cplx g = f[k];
    if (lane == 0) g = cscale(g, 0.5);
    cplx pg = shfl_c(f[k], partner);
    if (lane == 0) pg = cscale(ft[k], 0.5);
    if (lane < H) {
      Sb[(2 * k) * HP + lane] = cadd(g, pg);
      Sb[(2 * k + 1) * HP + lane] = csub(g, pg);
    } else if (lane == H) {
      Sb[(2 * k) * HP + H] = g;
      Sb[(2 * k + 1) * HP + H] = g;
    }
  }
  wave_sync();
  cplx acc[F];
#pragma unroll
  for (int k = 0; k < F; ++k) acc[k] = cz();
  const int sel = L.odd;  // even coefficients use S, odd ones D
#pragma unroll 3
  for (int jj = 0; jj <= H; ++jj) {
    const double c = kfwd[jj * 64 + lane];
#pragma unroll
    for (int k = 0; k < F; ++k) acc[k] = caxpy(acc[k], c, Sb[(2 * k + sel) * HP + jj]);
  }
  const double sc = (L.n == 0) ? (1.0 / N) : (2.0 / N);
#pragma unroll
  for (int k = 0; k < F; ++k) {
    a[k] = L.ok ? cscale(acc[k], sc) : cz();
    // a_N = (1/N) sum_{j <= N/2} (-1)^j S_j
    cplx part = cz();
    if (lane <= H) part = cscale(Sb[(2 * k) * HP + lane], (lane & 1) ? -1.0 : 1.0);
    at[k] = cscale(wave_sum(part), 1.0 / N);
  }
}

// Inverse DCT-I: parity-major coefficients (this lane, tail) -> node values (node = lane < N,
// tail node N).  f_j = sum_n a_n cos(pi n j / N), folded with P_n = a_n + a_{N-n},
// M_n = a_n - a_{N-n} (n < N/2), P = M = a_{N/2} at n = N/2.
template <int N, int F>
__device__ __forceinline__ void dct_inv_pm(const Lane<N>& L, const cplx* a, const cplx* at,
                                           const double* __restrict__ kinv, cplx* Sb, cplx* f, cplx* ft) {
  constexpr int H = N / 2;
  constexpr int HP = H + 1;
  const int lane = L.l;
  // partner lane of N - n in the same half (n = 0 pairs with the tail)
  int partner = 0;
  if (!L.odd) partner = (H - L.i) & 63;
  else partner = 32 + ((H - 1 - L.i) & 31);
#pragma unroll
  for (int k = 0; k < F; ++k) {
    cplx pa = shfl_c(a[k], partner);
    if (!L.odd && L.i == 0) pa = at[k];
    if (L.ok && L.n < H) {
      Sb[(2 * k) * HP + L.n] = cadd(a[k], pa);
      Sb[(2 * k + 1) * HP + L.n] = csub(a[k], pa);
    } else if (L.ok && L.n == H) {
      Sb[(2 * k) * HP + H] = a[k];
      Sb[(2 * k + 1) * HP + H] = a[k];
    }
  }
  wave_sync();
  cplx acc[F];
#pragma unroll
  for (int k = 0; k < F; ++k) acc[k] = cz();
  const int sel = lane & 1;  // even nodes use P, odd nodes M
#pragma unroll 3
  for (int n = 0; n <= H; ++n) {
    const double c = kinv[n * 64 + lane];
#pragma unroll
    for (int k = 0; k < F; ++k) acc[k] = caxpy(acc[k], c, Sb[(2 * k + sel) * HP + n]);
  }
#pragma unroll
  for (int k = 0; k < F; ++k) {
    f[k] = (lane < N) ? acc[k] : cz();
    cplx part = cz();
    if (lane <= H) part = cscale(Sb[(2 * k) * HP + lane], (lane & 1) ? -1.0 : 1.0);
    ft[k] = wave_sum(part);
  }
}

// Sum over the coefficients of weight(n) x_n, with the tail.
template <int N>
__device__ __forceinline__ cplx coef_sum(const Lane<N>& L, cplx x, cplx xt, double w_lane, double w_tail) {
  cplx part = L.ok ? cscale(x, w_lane) : cz();
  return caxpy(wave_sum(part), w_tail, xt);
}

template <int N>
__global__ __launch_bounds__(64 * CWAVES) void k_column_pm(ColArgsPm A) {
  constexpr int NY = N + 1;
  constexpr int H = N / 2;
  constexpr int HP = H + 1;
  constexpr int SB = 12 * HP;  // complex scratch per wave: 6 fields x (P, M)
  extern __shared__ double dyn_lds[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c = blockIdx.x * CWAVES + wave;
  if (c >= A.ncol) return;
  if (*A.status & STATUS_BAD_ACTION) return;
  const int nz = A.nz;
  const int p = c / nz, q = c - p * nz;
  if (q == nz / 2) return;            // Nyquist: never stored
  if (p == 0 && q > nz / 2) return;   // written by its Hermitian partner (0, -q)
  const bool mean = (c == 0);
  const int partner = (p == 0 && q > 0) ? (nz - q) : -1;
  cplx* Sb = reinterpret_cast<cplx*>(dyn_lds) + (size_t)wave * SB;
  const Lane<N> L(lane);
  const double al = A.alpha[p], be = A.beta[q];
  const double k2 = al * al + be * be;
  const size_t col = (size_t)c * NY;
  const int nl = (L.ok ? L.n : 0);  // this lane's coefficient index (for loads)
  const double dn = (double)L.n, dN = (double)N;

  cplx v, om, vt, omt;  // state after this call (mean: v = U + i W, om = 0)

  if (A.stage >= 0) {
    const int r = A.stage;
    // H1, H2, H3 at the nodes (lane j < N, tail N)
    cplx hn[3], hnt[3];
#pragma unroll
    for (int g = 0; g < 3; ++g) {
      const size_t o = ((size_t)(lane < N ? lane : 0) * A.nkx + p) * nz + q;
      const size_t ot = ((size_t)N * A.nkx + p) * nz + q;
      hn[g] = (lane < N) ? A.H3[g * A.plane + o] : cz();
      hnt[g] = A.H3[g * A.plane + ot];
      if (mean && g != 1) {  // the mean flow sees the real parts of H1, H3 only
        hn[g].y = 0.0;
        hnt[g].y = 0.0;
      }
    }
    cplx hc[3], hct[3];
    dct_fwd_pm<N, 3>(L, hn, hnt, A.kfwd, Sb, hc, hct);
    wave_sync();
    if (!mean) {
      // explicit terms: h_v = -k^2 H2 - D(i al H1 + i be H3), h_g = i be H1 - i al H3
      const cplx T = cmuli(make_double2(al * hc[0].x + be * hc[2].x, al * hc[0].y + be * hc[2].y));
      const cplx Tt = cmuli(make_double2(al * hct[0].x + be * hct[2].x, al * hct[0].y + be * hct[2].y));
      const cplx dT = cheb_d<N>(L, T, Tt);
      const cplx hv = csub(cscale(hc[1], -k2), dT);
      const cplx hvt = cscale(hct[1], -k2);
      const cplx hg = cmuli(make_double2(be * hc[0].x - al * hc[2].x, be * hc[0].y - al * hc[2].y));
      const cplx hgt = cmuli(make_double2(be * hct[0].x - al * hct[2].x, be * hct[0].y - al * hct[2].y));
      cplx hvp = cz(), hgp = cz(), hvpt = cz(), hgpt = cz();
      cplx* hist_v = A.hist + col;
      cplx* hist_g = A.hist + (size_t)A.ncol * NY + col;
      if (r > 0) {
        hvp = L.ok ? hist_v[nl] : cz();
        hgp = L.ok ? hist_g[nl] : cz();
        hvpt = hist_v[N];
        hgpt = hist_g[N];
      }
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
      // phi0 = (D^2 - k^2) v, psi = (D^2 - k^2) phi0, chi = (D^2 - k^2) omega_y
      const cplx v0 = L.ok ? A.vS[col + nl] : cz(), v0t = A.vS[col + N];
      const cplx o0 = L.ok ? A.oS[col + nl] : cz(), o0t = A.oS[col + N];
      const cplx dv = cheb_d<N>(L, v0, v0t);
      const cplx d2v = cheb_d<N>(L, dv, cz());
      const cplx phi0 = caxpy(d2v, -k2, v0), phi0t = cscale(v0t, -k2);
      const cplx dphi = cheb_d<N>(L, phi0, phi0t);
      const cplx d2phi = cheb_d<N>(L, dphi, cz());
      const cplx psi = caxpy(d2phi, -k2, phi0), psit = cscale(phi0t, -k2);
      const cplx dom = cheb_d<N>(L, o0, o0t);
      const cplx d2om = cheb_d<N>(L, dom, cz());
      const cplx chi = caxpy(d2om, -k2, o0), chit = cscale(o0t, -k2);
      // right-hand sides of (D^2 - lam) X = rhs with lam = k^2 + lam0
      auto rhs = [&](cplx x, cplx y, cplx h, cplx hp) {
        cplx t = cscale(x, -A.lam0);
        t = caxpy(t, -A.ab, y);
        t = caxpy(t, -A.gb, h);
        return caxpy(t, -A.zb, hp);
      };
      const cplx rp = rhs(phi0, psi, hv, hvp), rpt = rhs(phi0t, psit, hvt, hvpt);
      const cplx ro = rhs(o0, chi, hg, hgp), rot = rhs(o0t, chit, hgt, hgpt);
      cplx R[2], Rt[2];
      R[0] = tau_rows_pm<N>(L, rp, rpt, A.rc_pm, Rt[0]);
      R[1] = tau_rows_pm<N>(L, ro, rot, A.rc_pm, Rt[1]);
      const double* rec = A.op_pm + ((size_t)c * NOPS + r) * PM_OPSZ;
      const cplx zero2[2] = {cz(), cz()};
      cplx X[2], Xt[2];
      tau_solve_pm<N, 2>(L, R, Rt, rec, zero2, zero2, X, Xt);
      // v_p: (D^2 - k^2) v_p = phi_p, v_p(+1) = 0, v_p(-1) = v_w
      cplx vw;
      if (A.wall_mode == WALL_OPP) {
        vw = A.vw_opp[c];
      } else {
        const cplx o = A.vw_old[c], nn = A.vw_new[c];
        vw = caxpy(o, A.s_ramp, csub(nn, o));
      }
      cplx Rv[1], Rvt[1];
      Rv[0] = tau_rows_pm<N>(L, X[0], Xt[0], A.rc_pm, Rvt[0]);
      const double* recv = A.op_pm + ((size_t)c * NOPS + 3) * PM_OPSZ;
      const cplx gtop[1] = {cz()}, gbot[1] = {vw};
      cplx vp[1], vpt[1];
      tau_solve_pm<N, 1>(L, Rv, Rvt, recv, gtop, gbot, vp, vpt);
      // influence correction: dv/dy(+-1) = 0 with v = v_p + c0 v_+ + c1 v_-
      const double n2 = dn * dn;
      const cplx dtop = coef_sum<N>(L, vp[0], vpt[0], n2, dN * dN);
      const cplx dbot = coef_sum<N>(L, vp[0], vpt[0], L.odd ? n2 : -n2, -dN * dN);
      const double* mi = A.minv + ((size_t)c * 3 + r) * 4;
      const cplx c0 = make_double2(-(mi[0] * dtop.x + mi[1] * dbot.x), -(mi[0] * dtop.y + mi[1] * dbot.y));
      const cplx c1 = make_double2(-(mi[2] * dtop.x + mi[3] * dbot.x), -(mi[2] * dtop.y + mi[3] * dbot.y));
      const double* vtab = A.vt_pm + ((size_t)c * 3 + r) * PM_ENTRIES;
      const double tv = vtab[lane], tvt = vtab[64];
      v = caxpy(caxpy(vp[0], tv, c0), L.odd ? -tv : tv, c1);
      vt = caxpy(caxpy(vpt[0], tvt, c0), tvt, c1);
      if (!L.ok) v = cz();
      om = X[1];
      omt = Xt[1];
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
      // mean flow, packed X = U + i W; h = h_u + i h_w
      const cplx hm = make_double2(hc[0].x, hc[2].x), hmt = make_double2(hct[0].x, hct[2].x);
      cplx hmp = cz(), hmpt = cz();
      if (r > 0) {
        if (L.ok) hmp = make_double2(A.meanH[nl], A.meanH[NY + nl]);
        hmpt = make_double2(A.meanH[N], A.meanH[NY + N]);
      }
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
      const cplx X0 = L.ok ? make_double2(A.meanS[nl], A.meanS[NY + nl]) : cz();
      const cplx X0t = make_double2(A.meanS[N], A.meanS[NY + N]);
      const cplx d2X = cheb_d<N>(L, cheb_d<N>(L, X0, X0t), cz());
      auto rhs = [&](cplx x, cplx y, cplx h, cplx hp) {
        cplx t = cscale(x, -A.lam0);
        t = caxpy(t, -A.ab, y);
        t = caxpy(t, -A.gb, h);
        return caxpy(t, -A.zb, hp);
      };
      const cplx rr = rhs(X0, d2X, hm, hmp), rrt = rhs(X0t, cz(), hmt, hmpt);
      cplx R[1], Rt[1];
      R[0] = tau_rows_pm<N>(L, rr, rrt, A.rc_pm, Rt[0]);
      const double* rec = A.op_pm + ((size_t)0 * NOPS + r) * PM_OPSZ;
      const cplx z1[1] = {cz()};
      cplx Xs[1], Xst[1];
      tau_solve_pm<N, 1>(L, R, Rt, rec, z1, z1, Xs, Xst);
      double flux = wave_sum(L.ok ? A.intw_pm[lane] * Xs[0].x : 0.0) + A.intw_pm[64] * Xst[0].x;
      const double P_r = (A.forcing == 0) ? (A.ub2 - flux) * A.inv_int_up[r] : A.px;
      const double* up = A.up_pm + (size_t)r * PM_ENTRIES;
      const double U = fma(P_r, L.ok ? up[lane] : 0.0, Xs[0].x);
      const double Ut = fma(P_r, up[64], Xst[0].x);
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
      const double slope = wave_sum(L.ok ? (L.odd ? n2 : -n2) * v.x : 0.0) - dN * dN * vt.x;
      if (A.accumulate_drag && lane == 0) A.drag_acc[0] += A.nu * slope;
      const bool ok = isfinite(v.x) && isfinite(v.y) && isfinite(vt.x) && isfinite(vt.y);
      if (r == 2 && __any(!ok) && lane == 0) atomicOr(A.status, STATUS_NONFINITE);
    }
  } else {
    // reconstruct only: load the state
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
  if (!A.recon) return;
  const bool want_end = (A.stage == 2 || A.stage < 0);
  cplx fld[6], fldt[6];  // (u, v, w, omega_x, omega_y, omega_z) coefficients
  cplx tau_hat;
  if (!mean) {
    const double ik2 = 1.0 / k2;
    const cplx dv = cheb_d<N>(L, v, vt);
    const cplx u = cscale(cmuli(make_double2(al * dv.x - be * om.x, al * dv.y - be * om.y)), ik2);
    const cplx w = cscale(cmuli(make_double2(be * dv.x + al * om.x, be * dv.y + al * om.y)), ik2);
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
    fld[3] = csub(dw, cmuli(cscale(v, be)));
    fldt[3] = cscale(cmuli(vt), -be);
    fld[4] = om;
    fldt[4] = omt;
    fld[5] = csub(cmuli(cscale(v, al)), du);
    fldt[5] = cscale(cmuli(vt), al);
    const double n2 = dn * dn;
    tau_hat = cscale(coef_sum<N>(L, u, ut, L.odd ? n2 : -n2, -dN * dN), A.nu);
  } else {
    const cplx dX = cheb_d<N>(L, v, vt);
    fld[0] = make_double2(v.x, 0.0);
    fldt[0] = make_double2(vt.x, 0.0);
    fld[1] = fldt[1] = cz();
    fld[2] = make_double2(v.y, 0.0);
    fldt[2] = make_double2(vt.y, 0.0);
    fld[3] = make_double2(dX.y, 0.0);
    fldt[3] = cz();
    fld[4] = fldt[4] = cz();
    fld[5] = make_double2(-dX.x, 0.0);
    fldt[5] = cz();
    const double n2 = dn * dn;
    const double slope = wave_sum(L.ok ? (L.odd ? n2 : -n2) * v.x : 0.0) - dN * dN * vt.x;
    tau_hat = make_double2(A.nu * slope, 0.0);
  }
  cplx ph[6], pht[6];
  dct_inv_pm<N, 6>(L, fld, fldt, A.kinv, Sb, ph, pht);
  // write the six fields at the nodes (and the Hermitian partner column)
  const size_t o = ((size_t)(lane < N ? lane : 0) * A.nkx + p) * nz + q;
  const size_t ot = ((size_t)N * A.nkx + p) * nz + q;
  const size_t o2 = ((size_t)(lane < N ? lane : 0) * A.nkx + p) * nz + (partner >= 0 ? partner : 0);
  const size_t ot2 = ((size_t)N * A.nkx + p) * nz + (partner >= 0 ? partner : 0);
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    cplx val = ph[f], valt = pht[f];
    if (mean) {
      val.y = 0.0;
      valt.y = 0.0;
    }
    if (lane < N) {
      A.F6[(size_t)f * A.plane + o] = val;
      if (partner >= 0) A.F6[(size_t)f * A.plane + o2] = cconj(val);
    }
    if (lane == 0) {
      A.F6[(size_t)f * A.plane + ot] = valt;
      if (partner >= 0) A.F6[(size_t)f * A.plane + ot2] = cconj(valt);
    }
  }
  if (want_end) {
    // opposition target from v at the sensing node (js < N), Hermitian partner too
    if (lane == A.js) {
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

template <int N>
int launch_pm(const ColArgsPm& A, hipStream_t st, KernelTimer* tm) {
  const int blocks = (A.ncol + CWAVES - 1) / CWAVES;
  const size_t shm = (size_t)CWAVES * 12 * (N / 2 + 1) * sizeof(cplx);
  if (tm) (void)tm->begin(A.stage < 0 ? KC_RECON : KC_COLUMN, st);
  hipLaunchKernelGGL(k_column_pm<N>, dim3(blocks), dim3(64 * CWAVES), shm, st, A);
  if (tm) (void)tm->end(st);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace

int launch_column_pass_pm(const Dims& d, DeviceState& s, const PhysParams& ph, int stage, const StageConsts& sc,
                          int wall_mode, double s_ramp, int js, double opp_alpha, bool accumulate_drag,
                          bool recon, hipStream_t st, KernelTimer* tm) {
  ColArgsPm A;
  A.recon = recon ? 1 : 0;
  A.nkx = d.nkx;
  A.nz = d.nz;
  A.ncol = d.ncol;
  A.stage = stage;
  A.wall_mode = wall_mode;
  A.s_ramp = s_ramp;
  A.lam0 = sc.lam0;
  A.ab = sc.ab;
  A.gb = sc.gb;
  A.zb = sc.zb;
  A.nu = ph.nu;
  A.opp_alpha = opp_alpha;
  A.ub2 = 2.0 * ph.ub;
  A.px = ph.px;
  A.forcing = ph.forcing;
  A.js = js;
  A.accumulate_drag = accumulate_drag ? 1 : 0;
  A.plane = (size_t)d.ny * d.nkx * d.nz;
  A.vS = s.vS;
  A.oS = s.oS;
  A.hist = s.hist;
  A.meanS = s.meanS;
  A.meanH = s.meanH;
  A.H3 = s.H3;
  A.F6 = s.F6;
  A.vw_old = s.vw_old;
  A.vw_new = s.vw_new;
  A.vw_opp = s.vw_opp;
  A.tauw = s.tauw;
  A.kfwd = s.kfwd;
  A.kinv = s.kinv;
  A.rc_pm = s.rc_pm;
  A.intw_pm = s.intw_pm;
  A.op_pm = s.op_pm;
  A.vt_pm = s.vt_pm;
  A.up_pm = s.up_pm;
  A.minv = s.minv;
  A.inv_int_up = s.inv_int_up;
  A.alpha = s.alpha;
  A.beta = s.beta;
  A.drag_acc = s.drag_acc;
  A.status = s.status;
  switch (d.N) {
    case 16: return launch_pm<16>(A, st, tm);
    case 32: return launch_pm<32>(A, st, tm);
    case 64: return launch_pm<64>(A, st, tm);
    default: return -1;
  }
}

}  // namespace chanenv
