// FP64 HIP kernels of the channel-flow DNS step, written for gfx950 (CDNA4).
//
// One time step is three RK3/CN stages; each stage is a plane pass (plane_pass.hip)
// followed by a column pass:
//
//   column pass  one wavefront per wavenumber pair (alpha, beta) owns the whole
//                wall-normal column: forward DCT-I of H, the explicit terms h_v, h_g,
//                the RK3/CN right-hand sides, the Chebyshev-tau solves (quasi-
//                tridiagonal even/odd recurrences on a few lanes), the 2x2
//                influence-matrix correction, and then the reconstruction of
//                (u, v, w, omega_x, omega_y, omega_z) and their inverse DCT-I for the
//                next stage.  The (0, 0) pair carries the mean flow and the constant-
//                flow-rate pressure gradient.
//
// Small kernels ingest the action (clip, 2-D FFT, zero net flux) and produce the
// observation plane and the wall-shear field (inverse 2-D FFTs).
//
// Everything is FP64 (the method is chaotic and the tau systems are stiff); nothing is
// a dense contraction, so there is no MFMA here.

#include <cstring>

#include "device_common.h"

namespace chanenv {

hipError_t KernelTimer::next(int c, hipEvent_t* start, hipEvent_t* stop) {
  *start = *stop = nullptr;
  if (!on) return hipSuccess;
  if (2 * (used + 1) > pool.size()) {
    for (int k = 0; k < 2; ++k) {
      hipEvent_t ev;
      const hipError_t err = hipEventCreate(&ev);
      if (err != hipSuccess) return err;
      pool.push_back(ev);
    }
  }
  if (cls.size() < used + 1) cls.resize(used + 1);
  cls[used] = c;
  *start = pool[2 * used];
  *stop = pool[2 * used + 1];
  ++used;
  return hipSuccess;
}

// Launch timed by the optional timer (argument order of hipLaunchKernelGGL after the class).
#define TIMED_LAUNCH(tm, cls, st, kernel, grid, block, shm, st2, ...) \
  timed_launch((tm), (cls), kernel, grid, block, shm, st2, __VA_ARGS__)

// ----------------------------------------------------------------------------
// Batched Stockham FFT in LDS (radix 3, 4, 2), used by all (x, z) transforms.
// Sequence b of the batch lives at src + b*ld, length L (L = 2^a or 3*2^a).
// tw[k] = exp(-2 pi i k / L).  inv selects the +i sign (no 1/L scaling).
// Must be called by every thread of the block.  Returns the buffer holding the
// result (src or dst).
// ----------------------------------------------------------------------------
__device__ cplx* fft_batch(cplx* src, cplx* dst, int L, int nb_seq, int ld,
                           const cplx* __restrict__ tw, bool inv) {
  const int tid = threadIdx.x, nthr = blockDim.x;
  const double sg = inv ? 1.0 : -1.0;
  int Ns = 1;
  while (Ns < L) {
    const int rem = L / Ns;
    const int R = (rem % 3 == 0) ? 3 : ((rem % 4 == 0) ? 4 : 2);
    const int nb = L / R;
    const int tstep = L / (Ns * R);
    for (int t = tid; t < nb_seq * nb; t += nthr) {
      const int b = t / nb;
      const int j = t - b * nb;
      const int k = j % Ns;
      const cplx* s = src + b * ld;
      cplx x0 = s[j], x1 = s[j + nb], x2 = cz(), x3 = cz();
      if (R >= 3) x2 = s[j + 2 * nb];
      if (R == 4) x3 = s[j + 3 * nb];
      if (k != 0) {
        cplx w1 = tw[k * tstep];
        if (inv) w1.y = -w1.y;
        x1 = cmul(x1, w1);
        if (R >= 3) {
          cplx w2 = tw[2 * k * tstep];
          if (inv) w2.y = -w2.y;
          x2 = cmul(x2, w2);
        }
        if (R == 4) {
          cplx w3 = tw[3 * k * tstep];
          if (inv) w3.y = -w3.y;
          x3 = cmul(x3, w3);
        }
      }
      cplx y0, y1, y2, y3;
      if (R == 2) {
        y0 = cadd(x0, x1);
        y1 = csub(x0, x1);
      } else if (R == 4) {
        const cplx a = cadd(x0, x2), b2 = csub(x0, x2);
        const cplx c = cadd(x1, x3), d = csub(x1, x3);
        // sg * i * d
        const cplx id = make_double2(-sg * d.y, sg * d.x);
        y0 = cadd(a, c);
        y2 = csub(a, c);
        y1 = cadd(b2, id);
        y3 = csub(b2, id);
      } else {  // R == 3
        const double h = 0.86602540378443864676;  // sqrt(3)/2
        const cplx t1 = cadd(x1, x2), t2 = csub(x1, x2);
        y0 = cadd(x0, t1);
        const cplx m = make_double2(x0.x - 0.5 * t1.x, x0.y - 0.5 * t1.y);
        // sg * i * h * t2
        const cplx r = make_double2(-sg * h * t2.y, sg * h * t2.x);
        y1 = cadd(m, r);
        y2 = csub(m, r);
      }
      cplx* dd = dst + b * ld + (j / Ns) * Ns * R + k;
      dd[0] = y0;
      dd[Ns] = y1;
      if (R >= 3) dd[2 * Ns] = y2;
      if (R == 4) dd[3 * Ns] = y3;
    }
    __syncthreads();
    cplx* tmp = src;
    src = dst;
    dst = tmp;
    Ns *= R;
  }
  return src;
}

// ----------------------------------------------------------------------------
// Column pass.
// ----------------------------------------------------------------------------
template <int N>
struct CP {
  static constexpr int NY = N + 1;
  static constexpr int NS = (NY + 63) / 64;  // element slots per lane
  static constexpr int ML = N / 2 + 1;
  static constexpr int OPSZ = 4 * ML + 2;
  static constexpr int NB = 6;               // complex work vectors per wave
  static constexpr int NYP = NY + 1;
  // LDS per wave: the work vectors and 32 doubles of small scalars.  The operator records are
  // read from the table in global memory where they are used: staged in LDS as well, a wave took
  // 16 KB at N = 96 and five two-wave blocks filled a CU (2.5 waves per SIMD).  Six work vectors
  // (no phase needs more) take 9.4 KB at N = 96, so that 16 waves (four per SIMD) fit a CU.
  static constexpr int WAVE_DOUBLES = NB * NYP * 2 + 32;
};

// wavefronts (columns) per block: four for N <= 64, two above (LDS per block < 64 KiB)
template <int N>
constexpr int wpb() { return N <= 64 ? 4 : 2; }

// Waves per SIMD the general column kernel asks the compiler for: four at N = 96 and three at
// N = 128, which their registers allow without spilling (116, 161) and the LDS of six work
// vectors too (at N = 128 four would spill 63 registers); the compiler's own choice otherwise.
template <int N>
constexpr int col_waves() { return N == 96 ? 4 : (N == 128 ? 3 : 1); }

struct ColArgs {
  int nkx, nz, ncol;
  int stage;            // 0, 1, 2; -1: reconstruct only (after reset / set_state)
  int wall_mode;
  double s_ramp;
  double lam0, ab, gb, zb;       // built with nu' = nu ys^2 (the Chebyshev variable's)
  double nu, opp_alpha, ub2, px; // nu: nu ys, the wall-shear factor of d/dxi
  int forcing, js, accumulate_drag;
  int open;                      // free-slip top: phi_+ corrections and the d^2v row
  double ys, ysi;                // d/dy = ys d/dxi
  int recon;            // 0: skip the reconstruction for the next stage
  size_t plane;         // elements per field in F6 / H3 (ny * nkx * nz)
  cplx *vS, *oS, *hist;
  double *meanS, *meanH;
  const cplx* H3;
  cplx* F6;
  const cplx *vw_old, *vw_new;
  cplx *vw_opp, *tauw;
  const double *cosk, *rc, *optab, *vt, *minv, *up, *inv_int_up, *alpha, *beta;
  const double *pt, *ptinv;      // open channel: phi_+ per pair and stage [c][r][n], 1/dphi_+/dxi(+1)
  double* drag_acc;
  int* status;
};

// D on coefficients held in registers, element e = lane + 64 s in slot s (zero above N):
//   b_e = (2/c_e) sum_{p > e, p + e odd} p a_p = (2/c_e) W(e + 1),  W(e) = sum_{k >= 0} y_{e+2k},
// y_p = p a_p.  W is a stride-2 suffix sum, done without LDS: within each row of 16 lanes by DPP
// row shifts of 2, 4 and 8 (each lane keeps its parity); then the same-parity totals of the rows
// above in the slot (each row's total broadcast in its row and exchanged by permlane swaps: row 0
// adds T1 + (T2 + T3), row 1 T2 + T3, row 2 T3); then those of the higher slots (lanes 0 and 1
// of a slot hold its totals); b_e takes W of lane e + 1 by the wave-wide one-lane shift.
// b_N = 0.  Wave-uniform.
template <int N>
__device__ __forceinline__ void cheb_d1_reg(const cplx* x, cplx* out, int lane) {
  constexpr int NS = CP<N>::NS;
  const bool odd = lane & 1;
  const bool even_row = ((lane >> 4) & 1) == 0, low = lane < 32;
  cplx w[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int e = lane + 64 * s;
    cplx v = (e <= N) ? cscale(x[s], (double)e) : cz();
    v = cadd(v, cmov<DPP_ROW_SHL + 2>(v));
    v = cadd(v, cmov<DPP_ROW_SHL + 4>(v));
    v = cadd(v, cmov<DPP_ROW_SHL + 8>(v));
    const double t0x = pin(dmov<DPP_ROW_BCAST + 0>(v.x)), t0y = pin(dmov<DPP_ROW_BCAST + 0>(v.y));
    const double t1x = pin(dmov<DPP_ROW_BCAST + 1>(v.x)), t1y = pin(dmov<DPP_ROW_BCAST + 1>(v.y));
    const cplx T = make_double2(odd ? t1x : t0x, odd ? t1y : t0y);  // this parity's total of the row
    const Pair rx = row_swap(T.x, T.x), ry = row_swap(T.y, T.y);  // a: T0 T0 T2 T2, b: T1 T1 T3 T3
    const double px = rx.a + rx.b, py = ry.a + ry.b;   // T0 + T1 (rows 0, 1), T2 + T3 (rows 2, 3)
    const double nx = pin(rx.b), ny = pin(ry.b);
    const double hx = pin(half_swap(px, px).b), hy = pin(half_swap(py, py).b);  // T2 + T3 everywhere
    const cplx carry = make_double2((even_row ? nx : 0.0) + (low ? hx : 0.0), (even_row ? ny : 0.0) + (low ? hy : 0.0));
    w[s] = cadd(v, carry);
  }
  // every cross-lane value below is read by all lanes before any per-lane choice
  cplx up = cz();
#pragma unroll
  for (int s = NS - 1; s >= 0; --s) {
    const double ex = pin(readlane_d(w[s].x, 0)), ey = pin(readlane_d(w[s].y, 0));
    const double ox = pin(readlane_d(w[s].x, 1)), oy = pin(readlane_d(w[s].y, 1));
    const cplx tot = make_double2(odd ? ox : ex, odd ? oy : ey);
    w[s] = cadd(w[s], up);
    up = cadd(up, tot);
  }
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const double zx = pin(dmov<DPP_WAVE_SHL1>(w[s].x)), zy = pin(dmov<DPP_WAVE_SHL1>(w[s].y));
    double nx = 0.0, ny = 0.0;
    if (s + 1 < NS) {
      nx = pin(readlane_d(w[s + 1 < NS ? s + 1 : s].x, 0));
      ny = pin(readlane_d(w[s + 1 < NS ? s + 1 : s].y, 0));
    }
    const cplx z = make_double2(lane == 63 ? nx : zx, lane == 63 ? ny : zy);
    const int e = lane + 64 * s;
    out[s] = (e < N) ? cscale(z, e == 0 ? 1.0 : 2.0) : cz();
  }
}

typedef double dbl4 __attribute__((ext_vector_type(4)));

// DCT-I matvecs of F folded vectors on the matrix cores (N/2 a multiple of 16).  After the
// even/odd fold, even outputs 2i take the S values X[f][0..N/2] and odd outputs 2i+1 the D
// values X[f][N-k], k < N/2 (the middle term's cosine vanishes for odd outputs), with the
// cosines cosk[k (N+1) + e] of both transforms.  Each is a product of a (N/2 x terms) cosine
// matrix and a (terms x 2F) matrix of the fields' real and imaginary parts, done as 16 x 16
// output tiles of v_mfma_f64_16x16x4_f64 (A: 16 outputs x 4 terms, B: 4 terms x 16 columns):
// lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and holds D[4r + l / 16][l % 16],
// r < 4.  The 2F <= 16 columns are (field, re/im) pairs; lanes of unused columns supply zeros.
// The results are written back over X (after every lane's reads) and returned in the lanes'
// element order, as the loops below do; top: the last output (a_N or the node N value).
template <int N, int F>
__device__ __forceinline__ void dct_mfma(cplx* const* X, const double* __restrict__ cosk, int lane,
                                         cplx (*out)[CP<N>::NS], const cplx* top, double sc0, double sc) {
  static_assert((N / 2) % 16 == 0 && 2 * F <= 16, "matrix-core DCT shape");
  constexpr int H = N / 2, T = H / 16, KE = (H + 4) / 4, KO = H / 4;
  const int col = lane & 15, kq = lane >> 4;
  const int f = col >> 1, part = col & 1;
  double* xf = nullptr;
#pragma unroll
  for (int g = 0; g < F; ++g)
    if (g == f) xf = reinterpret_cast<double*>(X[g]);
  dbl4 de[T], dd[T];
#pragma unroll
  for (int t = 0; t < T; ++t) de[t] = dd[t] = dbl4{0.0, 0.0, 0.0, 0.0};
  // The cosines of step ks + 1 are requested before the products of step ks, so that their
  // load overlaps the matrix instructions instead of stalling each step (the same operands in
  // the same order).  Steps ks < H/4 have every term k = 4 ks + kq below H; the one after it
  // (k = H for kq = 0 only) is done last on its own.
  constexpr int KEF = H / 4;
  static_assert(KE == KEF + 1 && KO == KEF, "step counts");
  double an[T];
#pragma unroll
  for (int t = 0; t < T; ++t) an[t] = cosk[kq * (N + 1) + 2 * (16 * t + col)];
#pragma unroll 2
  for (int ks = 0; ks < KEF; ++ks) {
    const int k = 4 * ks + kq;
    double a[T];
#pragma unroll
    for (int t = 0; t < T; ++t) a[t] = an[t];
    const int kn = (ks + 1 < KEF) ? k + 4 : k;  // the last step reloads its own (unused)
#pragma unroll
    for (int t = 0; t < T; ++t) an[t] = cosk[kn * (N + 1) + 2 * (16 * t + col)];
    const double b = xf ? xf[2 * k + part] : 0.0;
#pragma unroll
    for (int t = 0; t < T; ++t) de[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], b, de[t], 0, 0, 0);
  }
  {
    const int k = 4 * KEF + kq;
    const bool in = k <= H;
    const double b = (xf && in) ? xf[2 * k + part] : 0.0;
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const double a = in ? cosk[k * (N + 1) + 2 * (16 * t + col)] : 0.0;
      de[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, de[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < T; ++t) an[t] = cosk[kq * (N + 1) + 2 * (16 * t + col) + 1];
#pragma unroll 2
  for (int ks = 0; ks < KO; ++ks) {
    const int k = 4 * ks + kq;
    double a[T];
#pragma unroll
    for (int t = 0; t < T; ++t) a[t] = an[t];
    const int kn = (ks + 1 < KO) ? k + 4 : k;
#pragma unroll
    for (int t = 0; t < T; ++t) an[t] = cosk[kn * (N + 1) + 2 * (16 * t + col) + 1];
    const double b = xf ? xf[2 * (N - k) + part] : 0.0;
#pragma unroll
    for (int t = 0; t < T; ++t) dd[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], b, dd[t], 0, 0, 0);
  }
  wave_sync();
  if (xf) {
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * t + 4 * r + kq;
        xf[2 * (2 * i) + part] = de[t][r];
        xf[2 * (2 * i + 1) + part] = dd[t][r];
      }
  }
  wave_sync();
#pragma unroll
  for (int s = 0; s < CP<N>::NS; ++s) {
    const int e = lane + 64 * s;
#pragma unroll
    for (int g = 0; g < F; ++g) out[g][s] = (e < N) ? cscale(X[g][e], e == 0 ? sc0 : sc) : cz();
  }
#pragma unroll
  for (int g = 0; g < F; ++g)
    if (lane == (N % 64)) out[g][N / 64] = top[g];
}

// Forward DCT-I of F nodal vectors X[f][0..N] (overwritten by the even/odd fold):
// a_n = 2/(N cb_n) sum_j f_j cos(pi n j/N)/cb_j.  Result in out[f][slot].
template <int N, int F>
__device__ __forceinline__ void dct_forward(cplx* const* X, const double* __restrict__ cosk, int lane,
                                            cplx (*out)[CP<N>::NS]) {
  constexpr int H = N / 2;
  for (int j = lane; j < H; j += 64) {
#pragma unroll
    for (int f = 0; f < F; ++f) {
      cplx a = X[f][j], b = X[f][N - j];
      if (j == 0) {
        a = cscale(a, 0.5);
        b = cscale(b, 0.5);
      }
      X[f][j] = cadd(a, b);
      X[f][N - j] = csub(a, b);
    }
  }
  wave_sync();
  if constexpr (H % 16 == 0 && 2 * F <= 16) {
    // a_N = (1/N) sum_{j <= N/2} (-1)^j S_j, from the folded values before they are replaced
    cplx top[F];
#pragma unroll
    for (int f = 0; f < F; ++f) {
      cplx part = cz();
      for (int j = lane; j <= H; j += 64) part = caxpy(part, (j & 1) ? -1.0 : 1.0, X[f][j]);
      top[f] = cscale(wave_sum(part), 1.0 / N);
    }
    dct_mfma<N, F>(X, cosk, lane, out, top, 1.0 / N, 2.0 / N);
    return;
  }
#pragma unroll
  for (int s = 0; s < CP<N>::NS; ++s) {
    const int e = lane + 64 * s;
    cplx acc[F];
#pragma unroll
    for (int f = 0; f < F; ++f) acc[f] = cz();
    if (e < N) {
      const bool odd = e & 1;
#pragma unroll 4
      for (int jj = 0; jj <= H; ++jj) {
        const double cs = cosk[jj * (N + 1) + e];
        const int idx = odd ? (jj < H ? N - jj : H) : jj;
#pragma unroll
        for (int f = 0; f < F; ++f) acc[f] = caxpy(acc[f], cs, X[f][idx]);
      }
    }
    const double sc = (e == 0) ? (1.0 / N) : (2.0 / N);
#pragma unroll
    for (int f = 0; f < F; ++f) out[f][s] = cscale(acc[f], sc);
  }
  // a_N = (1/N) sum_{j <= N/2} (-1)^j S_j
#pragma unroll
  for (int f = 0; f < F; ++f) {
    cplx part = cz();
    for (int j = lane; j <= H; j += 64) part = caxpy(part, (j & 1) ? -1.0 : 1.0, X[f][j]);
    const cplx tot = wave_sum(part);
    if (lane == (N % 64)) out[f][N / 64] = cscale(tot, 1.0 / N);
  }
}

// Inverse DCT-I of F coefficient vectors X[f][0..N] (overwritten by the fold):
// f_j = sum_n a_n cos(pi n j / N).  Result in out[f][slot] for node e = lane + 64 slot.
template <int N, int F>
__device__ __forceinline__ void dct_inverse(cplx* const* X, const double* __restrict__ cosk, int lane,
                                            cplx (*out)[CP<N>::NS]) {
  constexpr int H = N / 2;
  for (int n = lane; n < H; n += 64) {
#pragma unroll
    for (int f = 0; f < F; ++f) {
      const cplx a = X[f][n], b = X[f][N - n];
      X[f][n] = cadd(a, b);
      X[f][N - n] = csub(a, b);
    }
  }
  wave_sync();
  if constexpr (H % 16 == 0 && 2 * F <= 16) {
    // f_N = sum_{n <= N/2} (-1)^n S_n, from the folded values before they are replaced
    cplx top[F];
#pragma unroll
    for (int f = 0; f < F; ++f) {
      cplx part = cz();
      for (int n = lane; n <= H; n += 64) part = caxpy(part, (n & 1) ? -1.0 : 1.0, X[f][n]);
      top[f] = wave_sum(part);
    }
    dct_mfma<N, F>(X, cosk, lane, out, top, 1.0, 1.0);
    return;
  }
#pragma unroll
  for (int s = 0; s < CP<N>::NS; ++s) {
    const int e = lane + 64 * s;
    cplx acc[F];
#pragma unroll
    for (int f = 0; f < F; ++f) acc[f] = cz();
    if (e < N) {
      const bool odd = e & 1;
#pragma unroll 4
      for (int n = 0; n <= H; ++n) {
        const double cs = cosk[n * (N + 1) + e];
        const int idx = odd ? (n < H ? N - n : H) : n;
#pragma unroll
        for (int f = 0; f < F; ++f) acc[f] = caxpy(acc[f], cs, X[f][idx]);
      }
    }
#pragma unroll
    for (int f = 0; f < F; ++f) out[f][s] = acc[f];
  }
#pragma unroll
  for (int f = 0; f < F; ++f) {
    cplx part = cz();
    for (int n = lane; n <= H; n += 64) part = caxpy(part, (n & 1) ? -1.0 : 1.0, X[f][n]);
    const cplx tot = wave_sum(part);
    if (lane == (N % 64)) out[f][N / 64] = tot;
  }
}

// Right-hand side rows of the quasi-tridiagonal tau system (n = 2..N):
// R_n = rc1_n f_{n-2} - rc2_n f_n + rc3_n f_{n+2}.
template <int N>
__device__ __forceinline__ cplx tau_rows(const cplx* f, const double* __restrict__ rc, int n) {
  constexpr int NY = N + 1;
  if (n < 2) return cz();
  cplx r = cscale(f[n - 2], rc[n]);
  r = caxpy(r, -rc[NY + n], f[n]);
  if (n + 2 <= N) r = caxpy(r, rc[2 * NY + n], f[n + 2]);
  return r;
}

// The tau-row coefficients of the lane's elements e = lane + 64 s, requested together (an
// element past N reads row N and does not use it), so that a loop over the lane's elements
// waits for memory once.
template <int N>
struct RcLane {
  double c0[CP<N>::NS], c1[CP<N>::NS], c2[CP<N>::NS];
  __device__ __forceinline__ RcLane(const double* __restrict__ rc, int lane) {
    constexpr int NY = N + 1;
#pragma unroll
    for (int s = 0; s < CP<N>::NS; ++s) {
      const int n = min(lane + 64 * s, N);
      c0[s] = rc[n];
      c1[s] = rc[NY + n];
      c2[s] = rc[2 * NY + n];
    }
  }
  // tau_rows of element n = lane + 64 s (n <= N) with these coefficients
  __device__ __forceinline__ cplx rows(const cplx* f, int s, int n) const {
    if (n < 2) return cz();
    cplx r = cscale(f[n - 2], c0[s]);
    r = caxpy(r, -c1[s], f[n]);
    if (n + 2 <= N) r = caxpy(r, c2[s], f[n + 2]);
    return r;
  }
};

// x moved by the DPP pattern CTRL; a lane whose source lies outside its row keeps id (the
// identity of the composition being scanned).
template <int CTRL>
__device__ __forceinline__ double dmov_id(double x, double id) {
  return __builtin_amdgcn_update_dpp(id, x, CTRL, 0xF, 0xF, false);
}

// Affine compositions over the 64 lanes, without LDS.  Suffix: lane l holds (a_l, b_l) with
// e_l = a_l + b_l e_{l+1} (e_64 = 0); returns e_l for every a[k] (one multiplier chain b shared
// by the K right-hand sides).  Prefix: E_l = c_l + g_l E_{l-1} (E_{-1} = 0).  Each takes four
// DPP steps within the rows of 16 lanes (a source outside the row reads the identity (0, 1)),
// then the composition with the rows further along in the scan's direction: each row's
// composite is broadcast in its row and exchanged by permlane swaps (suffix: row 2 takes row
// 3's, row 1 the composite of rows 2-3, row 0 that of rows 1-3; prefix mirrored).
template <int K>
__device__ __forceinline__ void affine_suffix(cplx* a, double b, int lane) {
  const int row = lane >> 4;
  const bool even_row = (row & 1) == 0, low = lane < 32;
  auto step = [&](auto dc) {
    constexpr int D = decltype(dc)::value;
#pragma unroll
    for (int k = 0; k < K; ++k)
      a[k] = caxpy(a[k], b, make_double2(dmov_id<DPP_ROW_SHL + D>(a[k].x, 0.0), dmov_id<DPP_ROW_SHL + D>(a[k].y, 0.0)));
    b *= dmov_id<DPP_ROW_SHL + D>(b, 1.0);
  };
  step(std::integral_constant<int, 1>{});
  step(std::integral_constant<int, 2>{});
  step(std::integral_constant<int, 4>{});
  step(std::integral_constant<int, 8>{});
  const double RB = dmov<DPP_ROW_BCAST + 0>(b);
  const double foB = pin(row_swap(RB, RB).b);  // rows 0, 2: the next row's multiplier
#pragma unroll
  for (int k = 0; k < K; ++k) {
    cplx carry;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const double x = c ? a[k].y : a[k].x;
      const double RA = dmov<DPP_ROW_BCAST + 0>(x);
      const double foA = pin(row_swap(RA, RA).b);    // rows 0, 2: the next row's composite
      const double V = fma(RB, foA, RA);              // row 2: e at the first lane of row 2
      const double W = row_swap(V, V).a;              // rows 2, 3: row 2's V
      const double X = pin(cross_halves(W, W, low));  // rows 0, 1 take it from rows 2, 3
      const double cv = row == 3 ? 0.0 : row == 2 ? foA : row == 1 ? X : fma(foB, X, foA);
      if (c) carry.y = cv; else carry.x = cv;
    }
    a[k] = caxpy(a[k], b, carry);
  }
}

template <int K>
__device__ __forceinline__ void affine_prefix(cplx* c, double g, int lane) {
  const int row = lane >> 4;
  const bool even_row = (row & 1) == 0, low = lane < 32;
  auto step = [&](auto dc) {
    constexpr int D = decltype(dc)::value;
#pragma unroll
    for (int k = 0; k < K; ++k)
      c[k] = caxpy(c[k], g, make_double2(dmov_id<DPP_ROW_SHR + D>(c[k].x, 0.0), dmov_id<DPP_ROW_SHR + D>(c[k].y, 0.0)));
    g *= dmov_id<DPP_ROW_SHR + D>(g, 1.0);
  };
  step(std::integral_constant<int, 1>{});
  step(std::integral_constant<int, 2>{});
  step(std::integral_constant<int, 4>{});
  step(std::integral_constant<int, 8>{});
  const double RG = dmov<DPP_ROW_BCAST + 15>(g);
  const double feG = pin(row_swap(RG, RG).a);  // rows 1, 3: the previous row's multiplier
#pragma unroll
  for (int k = 0; k < K; ++k) {
    cplx carry;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const double x = q ? c[k].y : c[k].x;
      const double RC = dmov<DPP_ROW_BCAST + 15>(x);
      const double feC = pin(row_swap(RC, RC).a);    // rows 1, 3: the previous row's composite
      const double V = fma(RG, feC, RC);              // row 1: E at the last lane of row 1
      const double W = row_swap(V, V).b;              // rows 0, 1: row 1's V
      const double X = pin(cross_halves(W, W, low));  // rows 2, 3 take it from rows 0, 1
      const double cv = row == 0 ? 0.0 : row == 1 ? feC : row == 2 ? X : fma(feG, X, feC);
      if (q) carry.y = cv; else carry.x = cv;
    }
    c[k] = caxpy(c[k], g, carry);
  }
}

// Even/odd elimination of both parities of K tau systems that share one operator record
// {w, u, f, F, 1/sum F} per parity, on the whole wavefront: lane l takes index i = l + 1
// (i <= m = (N - s)/2 <= 64).  The bottom-up recurrence e_i = w_i R_{2i+s} - u_i e_{i+1}
// (e_{m+1} = 0) is the affine suffix composition of (w_i R_{2i+s}, -u_i), the top-down one
// E_i = e_i + f_i E_{i-1} (E_0 = 0) the affine prefix composition of (e_i, f_i); lanes past m
// hold (0, 0), which ends the chains there.
// Writes E_i to E[k][2i+s] and x0[2k+s] = (g[2k+s] - sum_i E_i) / sum F_i.
template <int N, int K>
__device__ __forceinline__ void tau_chain_wave(cplx* const* R, const double* TAB, const cplx* g, cplx* const* E,
                                               cplx* x0, int lane) {
  constexpr int ML = N / 2 + 1;
  constexpr int OPSZ = 4 * ML + 2;
  static_assert(N / 2 <= 64, "one lane per elimination index");
  const int i = lane + 1;
  // both parities' coefficients requested up front (lanes past m read row m and discard it), so
  // that their loads overlap instead of following each parity's scans
  double tw[2], tu[2], tf[2], tsc[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const double* tab = TAB + s * OPSZ;
    const int ic = min(i, (N - s) / 2);
    tw[s] = tab[ic];
    tu[s] = tab[ML + ic];
    tf[s] = tab[2 * ML + ic];
    tsc[s] = tab[4 * ML];
  }
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int m = (N - s) / 2;
    const bool act = i <= m;
    const double w = act ? tw[s] : 0.0, u = act ? tu[s] : 0.0, f = act ? tf[s] : 0.0;
    cplx a[K];
#pragma unroll
    for (int k = 0; k < K; ++k) a[k] = act ? cscale(R[k][2 * i + s], w) : cz();
    affine_suffix<K>(a, act ? -u : 0.0, lane);   // a[k] = e_i
    affine_prefix<K>(a, act ? f : 0.0, lane);    // a[k] = E_i
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (act) E[k][2 * i + s] = a[k];
      const cplx sum = wave_sum(act ? a[k] : cz());
      x0[2 * k + s] = cscale(csub(g[2 * k + s], sum), tsc[s]);
    }
  }
}

template <int N>
__device__ __forceinline__ cplx tau_value(const cplx* E, const double* TAB, const cplx* x0, int e) {
  constexpr int ML = N / 2 + 1;
  constexpr int OPSZ = 4 * ML + 2;
  const int i = e >> 1, s = e & 1;
  const cplx base = (i == 0) ? cz() : E[e];
  return caxpy(base, TAB[s * OPSZ + 3 * ML + i], x0[s]);
}

// The homogeneous solutions F of the lane's elements e = lane + 64 s in an operator record,
// requested together (an element past N reads element N); tau_value with them.
template <int N>
struct TauF {
  double f[CP<N>::NS];
  __device__ __forceinline__ TauF(const double* TAB, int lane) {
    constexpr int ML = N / 2 + 1;
    constexpr int OPSZ = 4 * ML + 2;
#pragma unroll
    for (int s = 0; s < CP<N>::NS; ++s) {
      const int e = min(lane + 64 * s, N);
      f[s] = TAB[(e & 1) * OPSZ + 3 * ML + (e >> 1)];
    }
  }
  __device__ __forceinline__ cplx value(const cplx* E, const cplx* x0, int s, int e) const {
    const cplx base = ((e >> 1) == 0) ? cz() : E[e];
    return caxpy(base, f[s], x0[e & 1]);
  }
};

// The Dirichlet rows x(+1) = g_t, x(-1) = g_b of a tau solution held in registers (element
// e = lane + 64 slot), to rounding.  x0 = (g - sum E) / sum F cancels heavily when lam is large
// (the wall layer lives in the top coefficients), so the rows hold only to eps sum |E|.  One
// refinement of x0 per parity removes the row residual r_s = sum_i x_{2i+s} - g_s along the
// homogeneous solution F_i of that parity (x_{2i+s} -= F_i r_s / sum F), which leaves the other
// tau rows as they were and every coefficient to rounding; g_e, g_o = (g_t +- g_b)/2.  TAB holds
// the operator record the solution was computed with.
template <int N>
__device__ __forceinline__ void refine_rows(cplx* xs, const double* TAB, cplx ge, cplx go, int lane) {
  constexpr int NS = CP<N>::NS;
  constexpr int ML = N / 2 + 1;
  constexpr int OPSZ = 4 * ML + 2;
  // the record's values requested before the sums they follow (elements past N read element N)
  const double re = TAB[4 * ML], ro = TAB[OPSZ + 4 * ML];
  double fw[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int ec = min(lane + 64 * s, N);
    fw[s] = TAB[(ec & 1) * OPSZ + 3 * ML + (ec >> 1)];
  }
  cplx se = cz(), so = cz();
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int e = lane + 64 * s;
    if (e <= N) {
      if (e & 1) so = cadd(so, xs[s]);
      else se = cadd(se, xs[s]);
    }
  }
  se = wave_sum(se);
  so = wave_sum(so);
  const cplx de = cscale(csub(se, ge), -re);
  const cplx dodd = cscale(csub(so, go), -ro);
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int e = lane + 64 * s;
    if (e <= N) xs[s] = caxpy(xs[s], fw[s], (e & 1) ? dodd : de);
  }
}

template <int N>
__global__ __launch_bounds__(64 * wpb<N>()) __attribute__((amdgpu_waves_per_eu(col_waves<N>())))
void k_column(ColArgs A) {
  constexpr int WPB = wpb<N>();
  using P = CP<N>;
  constexpr int NY = P::NY;
  constexpr int NS = P::NS;
  constexpr int H = N / 2;
  extern __shared__ double dyn_lds[];
  double* smem = dyn_lds;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // contiguous column ranges per XCD: 317 -> 293 us per launch at 128x97x128
  const int c = xcd_block(blockIdx.x, gridDim.x) * WPB + wave;
  if (c >= A.ncol) return;
  if (*A.status & STATUS_BAD_ACTION) return;
  const int nz = A.nz;
  const int p = c / nz, q = c - p * nz;
  if (q == nz / 2) return;            // Nyquist: never stored
  if (p == 0 && q > nz / 2) return;   // written by its Hermitian partner (0, -q)
  const bool mean = (c == 0);
  const int partner = (p == 0 && q > 0) ? (nz - q) : -1;
  // the per-column operator tables depend on k^2 only: (p, q) and (p, N_z - q) share them
  const int crec = p * nz + (q > nz / 2 ? nz - q : q);

  double* wb = smem + (size_t)wave * P::WAVE_DOUBLES;
  cplx* B[P::NB];
#pragma unroll
  for (int k = 0; k < P::NB; ++k) B[k] = reinterpret_cast<cplx*>(wb + (size_t)k * P::NYP * 2);
  const double* TAB = nullptr;                                            // operator record
  cplx* SC = reinterpret_cast<cplx*>(wb + (size_t)P::NB * P::NYP * 2);  // small scalars

  const double al = A.alpha[p], be = A.beta[q];
  const double k2 = al * al + be * be;
  // the solve works in xi: wavenumbers / ys (exact, ys a power of two)
  const double als = al * A.ysi, bes = be * A.ysi;
  const double k2s = als * als + bes * bes;
  const size_t col = (size_t)c * NY;

  cplx vv[NS], oo[NS];  // state after this call (v, omega_y) or (U + iW, 0) for the mean

  if (A.stage >= 0) {
    // ---------------- solve part ----------------
    const int r = A.stage;
    // (a) H1, H2, H3 at the nodes
    for (int e = lane; e < NY; e += 64) {
      const size_t o = ((size_t)e * A.nkx + p) * nz + q;
      cplx h0 = A.H3[o], h1 = A.H3[A.plane + o], h2 = A.H3[2 * A.plane + o];
      if (mean) {  // the mean flow sees the real parts of H1, H3 only
        h0.y = 0.0;
        h2.y = 0.0;
      }
      B[0][e] = h0;
      B[1][e] = h1;
      B[2][e] = h2;
    }
    wave_sync();
    cplx hc[3][NS];
    dct_forward<N, 3>(B, A.cosk, lane, hc);
    wave_sync();
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int e = lane + 64 * s;
      if (e <= N) {
        B[0][e] = hc[0][s];
        B[1][e] = hc[1][s];
        B[2][e] = hc[2][s];
      }
    }
    wave_sync();
    if (!mean) {
      // (b) explicit terms h_v = -k^2 H2 - D(i al H1 + i be H3), h_g = i be H1 - i al H3
      for (int e = lane; e <= N; e += 64) {
        const cplx h1 = B[0][e], h3 = B[2][e];
        B[3][e] = cmuli(make_double2(als * h1.x + bes * h3.x, als * h1.y + bes * h3.y));
      }
      wave_sync();
      cplx hv[NS], hg[NS], hvp[NS], hgp[NS], tT[NS], dTs[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int e = lane + 64 * s;
        tT[s] = (e <= N) ? B[3][e] : cz();
      }
      cheb_d1_reg<N>(tT, dTs, lane);
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int e = lane + 64 * s;
        hv[s] = hg[s] = hvp[s] = hgp[s] = cz();
        if (e <= N) {
          const cplx dT = dTs[s];
          const cplx h1 = B[0][e], h2 = B[1][e], h3 = B[2][e];
          hv[s] = csub(cscale(h2, -k2s), dT);
          hg[s] = cmuli(make_double2(be * h1.x - al * h3.x, be * h1.y - al * h3.y));
          if (r > 0) {
            hvp[s] = A.hist[col + e];
            hgp[s] = A.hist[(size_t)A.ncol * NY + col + e];
          }
          if (r < 2) {
            A.hist[col + e] = hv[s];
            A.hist[(size_t)A.ncol * NY + col + e] = hg[s];
          }
        }
      }
      // (c) phi0 = (D^2 - k^2) v, psi = (D^2 - k^2) phi0, chi = (D^2 - k^2) omega_y
      for (int e = lane; e <= N; e += 64) {
        B[4][e] = A.vS[col + e];
        B[5][e] = A.oS[col + e];
      }
      wave_sync();
      cplx phi0[NS], chi[NS], xv[NS], xo[NS], d1[NS], d2v[NS], d2o[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int e = lane + 64 * s;
        xv[s] = (e <= N) ? B[4][e] : cz();
        xo[s] = (e <= N) ? B[5][e] : cz();
      }
      cheb_d1_reg<N>(xv, d1, lane);
      cheb_d1_reg<N>(d1, d2v, lane);
      cheb_d1_reg<N>(xo, d1, lane);
      cheb_d1_reg<N>(d1, d2o, lane);
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int e = lane + 64 * s;
        phi0[s] = chi[s] = cz();
        if (e <= N) {
          phi0[s] = caxpy(d2v[s], -k2s, xv[s]);
          chi[s] = caxpy(d2o[s], -k2s, xo[s]);
        }
      }
      cplx d2p[NS];
      cheb_d1_reg<N>(phi0, d1, lane);
      cheb_d1_reg<N>(d1, d2p, lane);
      // (d) right-hand sides of the two Helmholtz problems with lam = k^2 + lam0
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int e = lane + 64 * s;
        if (e <= N) {
          const cplx psi = caxpy(d2p[s], -k2s, phi0[s]);
          cplx rp = cscale(phi0[s], -A.lam0);
          rp = caxpy(rp, -A.ab, psi);
          rp = caxpy(rp, -A.gb, hv[s]);
          rp = caxpy(rp, -A.zb, hvp[s]);
          const cplx om = B[5][e];
          cplx ro = cscale(om, -A.lam0);
          ro = caxpy(ro, -A.ab, chi[s]);
          ro = caxpy(ro, -A.gb, hg[s]);
          ro = caxpy(ro, -A.zb, hgp[s]);
          B[0][e] = rp;
          B[1][e] = ro;
        }
      }
      // operator record of D^2 - lam for this column and stage (read where used)
      TAB = A.optab + ((size_t)crec * NOPS + r) * 2 * P::OPSZ;
      const TauF<N> tf1(TAB, lane);
      {
        const RcLane<N> rq(A.rc, lane);
        wave_sync();
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const int e = lane + 64 * s;
          if (e <= N) {
            B[2][e] = rq.rows(B[0], s, e);
            B[3][e] = rq.rows(B[1], s, e);
          }
        }
      }
      wave_sync();
      // (e) phi_p and omega_y: both parities of both systems as wave-wide scans
      {
        cplx* const Rs[2] = {B[2], B[3]};
        cplx* const Es[2] = {B[4], B[5]};
        const cplx g0[4] = {cz(), cz(), cz(), cz()};
        cplx x0[4];
        tau_chain_wave<N, 2>(Rs, TAB, g0, Es, x0, lane);
        if (lane == 0)
          for (int t = 0; t < 4; ++t) SC[t] = x0[t];
      }
      wave_sync();
      {
        cplx xp[NS], xw[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const int e = lane + 64 * s;
          xp[s] = xw[s] = cz();
          if (e <= N) {
            xp[s] = tf1.value(B[4], SC, s, e);
            xw[s] = tf1.value(B[5], SC + 2, s, e);
          }
        }
        refine_rows<N>(xp, TAB, cz(), cz(), lane);
        refine_rows<N>(xw, TAB, cz(), cz(), lane);
#pragma unroll
        for (int s = 0; s < NS; ++s) {  // over the chain's inputs, no longer needed
          const int e = lane + 64 * s;
          if (e <= N) {
            B[2][e] = xp[s];  // phi_p
            B[3][e] = xw[s];  // omega_y
          }
        }
      }
      wave_sync();
      // (f) v_p: (D^2 - k^2) v_p = phi_p, v_p(+1) = 0, v_p(-1) = v_w
      cplx vw;
      if (A.wall_mode == WALL_OPP) {
        vw = A.vw_opp[c];
      } else {
        const cplx o = A.vw_old[c], nn = A.vw_new[c];
        vw = caxpy(o, A.s_ramp, csub(nn, o));
      }
      TAB = A.optab + ((size_t)crec * NOPS + 3) * 2 * P::OPSZ;
      const TauF<N> tf3(TAB, lane);
      {
        const RcLane<N> rq(A.rc, lane);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const int e = lane + 64 * s;
          if (e <= N) B[0][e] = rq.rows(B[2], s, e);
        }
      }
      wave_sync();
      {
        // even part (g_top + g_bot)/2, odd part (g_top - g_bot)/2 with g_top = 0, g_bot = v_w
        cplx* const Rs[1] = {B[0]};
        cplx* const Es[1] = {B[1]};
        const cplx gv[2] = {cscale(vw, 0.5), cscale(vw, -0.5)};
        cplx x0[2];
        tau_chain_wave<N, 1>(Rs, TAB, gv, Es, x0, lane);
        if (lane == 0) {
          SC[4] = x0[0];
          SC[5] = x0[1];
        }
      }
      wave_sync();
      // (g) influence-matrix correction: Dv(+1) = Dv(-1) = 0
      cplx vp[NS];
      cplx dtop = cz(), dbot = cz();
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int e = lane + 64 * s;
        vp[s] = (e <= N) ? tf3.value(B[1], SC + 4, s, e) : cz();
      }
      refine_rows<N>(vp, TAB, cscale(vw, 0.5), cscale(vw, -0.5), lane);
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int e = lane + 64 * s;
        if (e <= N) {
          const double n2 = (double)e * (double)e;
          // top row: dv/dxi(+1) (wall) or d^2v/dxi^2(+1) = sum n^2 (n^2 - 1)/3 v_n (surface)
          dtop = caxpy(dtop, A.open ? n2 * (n2 - 1.0) / 3.0 : n2, vp[s]);
          dbot = caxpy(dbot, (e & 1) ? n2 : -n2, vp[s]);
        }
      }
      dtop = wave_sum(dtop);
      dbot = wave_sum(dbot);
      const double* mi = A.minv + ((size_t)crec * 3 + r) * 4;
      const cplx c0 = make_double2(-(mi[0] * dtop.x + mi[1] * dbot.x), -(mi[0] * dtop.y + mi[1] * dbot.y));
      const cplx c1 = make_double2(-(mi[2] * dtop.x + mi[3] * dbot.x), -(mi[2] * dtop.y + mi[3] * dbot.y));
      const double* vt = A.vt + ((size_t)crec * 3 + r) * NY;
      // free-slip top: omega_y += c phi_+ with c = -(domega/dxi)(+1) / (dphi_+/dxi)(+1)
      cplx cw = cz();
      const double* ptc = A.open ? A.pt + ((size_t)crec * 3 + r) * NY : nullptr;
      if (A.open) {
        cplx dw = cz();
        for (int e = lane; e <= N; e += 64) dw = caxpy(dw, (double)e * (double)e, B[3][e]);
        dw = wave_sum(dw);
        const double pinv = A.ptinv[(size_t)crec * 3 + r];
        cw = make_double2(-dw.x * pinv, -dw.y * pinv);
      }
      bool ok = true;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int e = lane + 64 * s;
        vv[s] = oo[s] = cz();
        if (e <= N) {
          const double t = vt[e];
          const double b = (e & 1) ? -t : t;
          vv[s] = caxpy(caxpy(vp[s], t, c0), b, c1);
          oo[s] = A.open ? caxpy(B[3][e], ptc[e], cw) : B[3][e];
          A.vS[col + e] = vv[s];
          A.oS[col + e] = oo[s];
          if (partner >= 0) {
            A.vS[(size_t)partner * NY + e] = cconj(vv[s]);
            A.oS[(size_t)partner * NY + e] = cconj(oo[s]);
          }
          ok = ok && isfinite(vv[s].x) && isfinite(vv[s].y) && isfinite(oo[s].x) && isfinite(oo[s].y);
        }
      }
      if (r == 2 && __any(!ok) && lane == 0) atomicOr(A.status, STATUS_NONFINITE);
    } else {
      // ---------------- mean flow (0, 0), packed as X = U + i W ----------------
      cplx hm[NS], hmp[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int e = lane + 64 * s;
        hm[s] = hmp[s] = cz();
        if (e <= N) {
          hm[s] = make_double2(B[0][e].x, B[2][e].x);  // h_u + i h_w
          if (r > 0) hmp[s] = make_double2(A.meanH[e], A.meanH[NY + e]);
          if (r < 2) {
            A.meanH[e] = hm[s].x;
            A.meanH[NY + e] = hm[s].y;
          }
        }
      }
      for (int e = lane; e <= N; e += 64) B[4][e] = make_double2(A.meanS[e], A.meanS[NY + e]);
      TAB = A.optab + ((size_t)crec * NOPS + r) * 2 * P::OPSZ;
      wave_sync();
      cplx xm[NS], dm1[NS], dm2[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int e = lane + 64 * s;
        xm[s] = (e <= N) ? B[4][e] : cz();
      }
      cheb_d1_reg<N>(xm, dm1, lane);
      cheb_d1_reg<N>(dm1, dm2, lane);
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int e = lane + 64 * s;
        if (e <= N) {
          const cplx X = xm[s];
          cplx rr = cscale(X, -A.lam0);
          rr = caxpy(rr, -A.ab, dm2[s]);
          rr = caxpy(rr, -A.gb, hm[s]);
          rr = caxpy(rr, -A.zb, hmp[s]);
          B[0][e] = rr;
        }
      }
      const TauF<N> tfm(TAB, lane);
      {
        const RcLane<N> rq(A.rc, lane);
        wave_sync();
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const int e = lane + 64 * s;
          if (e <= N) B[2][e] = rq.rows(B[0], s, e);
        }
      }
      wave_sync();
      {
        cplx* const Rs[1] = {B[2]};
        cplx* const Es[1] = {B[3]};
        const cplx g0[2] = {cz(), cz()};
        cplx x0[2];
        tau_chain_wave<N, 1>(Rs, TAB, g0, Es, x0, lane);
        if (lane == 0) {
          SC[0] = x0[0];
          SC[1] = x0[1];
        }
      }
      wave_sync();
      cplx xs[NS];
      double flux = 0.0;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int e = lane + 64 * s;
        xs[s] = cz();
        if (e <= N) xs[s] = tfm.value(B[3], SC, s, e);
      }
      refine_rows<N>(xs, TAB, cz(), cz(), lane);
      if (A.open) {  // dU/dxi(+1) = dW/dxi(+1) = 0: add c phi_+ (k = 0)
        cplx ds = cz();
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const int e = lane + 64 * s;
          if (e <= N) ds = caxpy(ds, (double)e * (double)e, xs[s]);
        }
        ds = wave_sum(ds);
        const double pinv = A.ptinv[r];
        const cplx cu = make_double2(-ds.x * pinv, -ds.y * pinv);
        const double* pt0 = A.pt + (size_t)r * NY;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const int e = lane + 64 * s;
          if (e <= N) xs[s] = caxpy(xs[s], pt0[e], cu);
        }
      }
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int e = lane + 64 * s;
        if (e <= N && !(e & 1)) flux = fma(2.0 / (1.0 - (double)e * (double)e), xs[s].x, flux);
      }
      flux = wave_sum(flux);
      const double P_r = (A.forcing == 0) ? (A.ub2 - flux) * A.inv_int_up[r] : A.px;
      const double* up = A.up + (size_t)r * NY;
      double slope = 0.0;
      bool ok = true;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int e = lane + 64 * s;
        vv[s] = oo[s] = cz();
        if (e <= N) {
          const double U = fma(P_r, up[e], xs[s].x);
          vv[s] = make_double2(U, xs[s].y);  // U + i W
          A.meanS[e] = U;
          A.meanS[NY + e] = xs[s].y;
          const double n2 = (double)e * (double)e;
          slope = fma((e & 1) ? n2 : -n2, U, slope);
          ok = ok && isfinite(U) && isfinite(xs[s].y);
        }
      }
      slope = wave_sum(slope);
      if (A.accumulate_drag && lane == 0) A.drag_acc[0] += A.nu * slope;
      if (r == 2 && __any(!ok) && lane == 0) atomicOr(A.status, STATUS_NONFINITE);
    }
    wave_sync();
  } else {
    // ---------------- reconstruct-only: load the state ----------------
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int e = lane + 64 * s;
      vv[s] = oo[s] = cz();
      if (e <= N) {
        if (mean) {
          vv[s] = make_double2(A.meanS[e], A.meanS[NY + e]);
        } else {
          vv[s] = A.vS[col + e];
          oo[s] = A.oS[col + e];
        }
      }
    }
  }

  // ---------------- reconstruction and inverse DCT for the next stage ----------------
  if (!A.recon) return;
  const bool want_end = (A.stage == 2 || A.stage < 0);
  cplx tau_hat = cz();
  if (!mean) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int e = lane + 64 * s;
      if (e <= N) B[0][e] = vv[s];
    }
    wave_sync();
    // u = (i al Dv - i be om)/k^2, w = (i be Dv + i al om)/k^2
    const double ik2 = 1.0 / k2;
    cplx uu[NS], ww[NS], dvs[NS];
    cheb_d1_reg<N>(vv, dvs, lane);  // dv/dxi; dv/dy = ys dv/dxi
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int e = lane + 64 * s;
      uu[s] = ww[s] = cz();
      if (e <= N) {
        const cplx dv = dvs[s];
        const cplx om = oo[s];
        const double aly = al * A.ys, bey = be * A.ys;
        uu[s] = cscale(cmuli(make_double2(aly * dv.x - be * om.x, aly * dv.y - be * om.y)), ik2);
        ww[s] = cscale(cmuli(make_double2(bey * dv.x + al * om.x, bey * dv.y + al * om.y)), ik2);
        const double n2 = (double)e * (double)e;
        tau_hat = caxpy(tau_hat, (e & 1) ? n2 : -n2, uu[s]);
      }
    }
    tau_hat = cscale(wave_sum(tau_hat), A.nu);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int e = lane + 64 * s;
      if (e <= N) {
        B[2][e] = uu[s];
        B[3][e] = ww[s];
      }
    }
    wave_sync();
    // omega_x = Dw - i be v, omega_z = i al v - Du
    cplx dus[NS], dws[NS];
    cheb_d1_reg<N>(uu, dus, lane);
    cheb_d1_reg<N>(ww, dws, lane);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int e = lane + 64 * s;
      if (e <= N) {
        const cplx du = dus[s];
        const cplx dw = dws[s];
        const cplx v = vv[s];
        B[4][e] = csub(cscale(dw, A.ys), cmuli(cscale(v, be)));
        B[5][e] = csub(cmuli(cscale(v, al)), cscale(du, A.ys));
        B[1][e] = oo[s];
      }
    }
    wave_sync();
  } else {
    // mean: u = U, w = W, omega_x = DW, omega_z = -DU, v = omega_y = 0
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int e = lane + 64 * s;
      if (e <= N) B[0][e] = vv[s];
    }
    wave_sync();
    double slope = 0.0;
    cplx dXs[NS];
    cheb_d1_reg<N>(vv, dXs, lane);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int e = lane + 64 * s;
      if (e <= N) {
        const cplx X = vv[s];
        const cplx dX = dXs[s];
        const double n2 = (double)e * (double)e;
        slope = fma((e & 1) ? n2 : -n2, X.x, slope);
        B[2][e] = make_double2(X.x, 0.0);
        B[3][e] = make_double2(X.y, 0.0);
        B[4][e] = make_double2(A.ys * dX.y, 0.0);
        B[5][e] = make_double2(-(A.ys * dX.x), 0.0);
        B[1][e] = cz();
      }
    }
    tau_hat = make_double2(A.nu * wave_sum(slope), 0.0);
    wave_sync();
    for (int e = lane; e <= N; e += 64) B[0][e] = cz();
    wave_sync();
  }
  // fields in order (u, v, w, omega_x, omega_y, omega_z)
  cplx* X6[6] = {B[2], B[0], B[3], B[4], B[1], B[5]};
  cplx ph[6][NS];
  dct_inverse<N, 6>(X6, A.cosk, lane, ph);
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int e = lane + 64 * s;
    if (e <= N) {
      const size_t o = ((size_t)e * A.nkx + p) * nz + q;
      const size_t o2 = ((size_t)e * A.nkx + p) * nz + (partner >= 0 ? partner : 0);
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        cplx val = ph[f][s];
        if (mean) val.y = 0.0;
        A.F6[(size_t)f * A.plane + o] = val;
        if (partner >= 0) A.F6[(size_t)f * A.plane + o2] = cconj(val);
      }
      if (want_end && e == A.js) {
        const cplx opp = mean ? cz() : cscale(ph[1][s], -A.opp_alpha);
        A.vw_opp[c] = opp;
        if (partner >= 0) A.vw_opp[partner] = cconj(opp);
      }
    }
  }
  if (want_end && lane == 0) {
    A.tauw[c] = tau_hat;
    if (partner >= 0) A.tauw[partner] = cconj(tau_hat);
  }
}

// Pressure on the observation planes, general column kernel (one wavefront per pair, column
// data in LDS): the same Poisson problem as the parity-major pressure kernel,
//   (D_xi^2 - k^2/ys^2) P = (i (al H1 + be H3)/ys + D_xi H2)/ys,
//   dP/dxi(+-1) = (H2 + nu ys^2 (D_xi^2 - k^2/ys^2) v - [lower wall] dv_w/dt)/ys,
// solved as the zero-value tau solution plus c_+ phi_+ + c_- phi_-, then evaluated at each
// plane's node.  The pair (0, 0) is set to zero.
struct PressGenArgs {
  int nkx, nz, ncol, n_pplanes;
  int pjs[MAX_PLANES];
  int ramp;                 // ramped external action: its slope enters the lower-wall condition
  double rate_scale;        // 1 / (n_sub dt)
  double ys, ysi, nu_xi;    // nu_xi = nu ys^2
  size_t plane;
  const cplx *H3, *vS, *vw_old, *vw_new;
  cplx* pbuf;
  const double *cosk, *rc, *optab, *alpha, *beta, *pk, *pkinv;
};

template <int N>
__global__ __launch_bounds__(64 * wpb<N>()) void k_pressure_gen(PressGenArgs A) {
  constexpr int WPB = wpb<N>();
  using P = CP<N>;
  constexpr int NY = P::NY;
  constexpr int NS = P::NS;
  constexpr int H = N / 2;
  extern __shared__ double dyn_lds[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c = blockIdx.x * WPB + wave;
  if (c >= A.ncol) return;
  const int nz = A.nz;
  const int p = c / nz, q = c - p * nz;
  if (q == nz / 2) return;
  if (p == 0 && q > nz / 2) return;
  const int partner = (p == 0 && q > 0) ? (nz - q) : -1;
  const int crec = p * nz + (q > nz / 2 ? nz - q : q);  // tables shared by (p, +-q)
  const size_t pstride = (size_t)A.nkx * nz;
  if (c == 0) {
    if (lane < A.n_pplanes) A.pbuf[(size_t)lane * pstride] = cz();
    return;
  }
  double* wb = dyn_lds + (size_t)wave * P::WAVE_DOUBLES;
  cplx* B[P::NB];
#pragma unroll
  for (int k = 0; k < P::NB; ++k) B[k] = reinterpret_cast<cplx*>(wb + (size_t)k * P::NYP * 2);
  const double* TAB = nullptr;                                            // operator record
  cplx* SC = reinterpret_cast<cplx*>(wb + (size_t)P::NB * P::NYP * 2);  // small scalars
  const double al = A.alpha[p], be = A.beta[q];
  const double als = al * A.ysi, bes = be * A.ysi;
  const double k2s = als * als + bes * bes;
  for (int e = lane; e < NY; e += 64) {
    const size_t o = ((size_t)e * A.nkx + p) * nz + q;
    B[0][e] = A.H3[o];
    B[1][e] = A.H3[A.plane + o];
    B[2][e] = A.H3[2 * A.plane + o];
  }
  wave_sync();
  const cplx H2_top = B[1][0], H2_bot = B[1][N];  // node values at y = +1 and -1
  wave_sync();
  cplx hc[3][NS];
  dct_forward<N, 3>(B, A.cosk, lane, hc);
  wave_sync();
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int e = lane + 64 * s;
    if (e <= N) {
      B[0][e] = hc[0][s];
      B[1][e] = hc[1][s];
      B[2][e] = hc[2][s];
    }
  }
  wave_sync();
  cplx dH2s[NS];
  cheb_d1_reg<N>(hc[1], dH2s, lane);
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int e = lane + 64 * s;
    if (e <= N) {
      const cplx h1 = hc[0][s], h3 = hc[2][s];
      const cplx ab = cmuli(make_double2(als * h1.x + bes * h3.x, als * h1.y + bes * h3.y));
      B[3][e] = cscale(cadd(dH2s[s], ab), A.ysi);
    }
  }
  TAB = A.optab + ((size_t)crec * NOPS + 3) * 2 * P::OPSZ;
  wave_sync();
  for (int e = lane; e <= N; e += 64) B[4][e] = tau_rows<N>(B[3], A.rc, e);
  wave_sync();
  {
    cplx* const Rs[1] = {B[4]};
    cplx* const Es[1] = {B[5]};
    const cplx g0[2] = {cz(), cz()};
    cplx x0[2];
    tau_chain_wave<N, 1>(Rs, TAB, g0, Es, x0, lane);
    if (lane == 0) {
      SC[0] = x0[0];
      SC[1] = x0[1];
    }
  }
  wave_sync();
  cplx Pd[NS];
  cplx dPt = cz(), dPb = cz(), d2vt = cz(), d2vb = cz(), vt0 = cz(), vb0 = cz();
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int e = lane + 64 * s;
    Pd[s] = cz();
    if (e <= N) {
      Pd[s] = tau_value<N>(B[5], TAB, SC, e);
      const double n2 = (double)e * (double)e;
      const double sg = (e & 1) ? -1.0 : 1.0;
      const double w2 = n2 * (n2 - 1.0) / 3.0;  // T_n''(1)
      const cplx v = A.vS[(size_t)c * NY + e];
      dPt = caxpy(dPt, n2, Pd[s]);
      dPb = caxpy(dPb, -sg * n2, Pd[s]);
      d2vt = caxpy(d2vt, w2, v);
      d2vb = caxpy(d2vb, sg * w2, v);
      vt0 = cadd(vt0, v);
      vb0 = caxpy(vb0, sg, v);
    }
  }
  dPt = wave_sum(dPt);
  dPb = wave_sum(dPb);
  d2vt = wave_sum(d2vt);
  d2vb = wave_sum(d2vb);
  vt0 = wave_sum(vt0);
  vb0 = wave_sum(vb0);
  cplx rate = cz();
  if (A.ramp) rate = cscale(csub(A.vw_new[c], A.vw_old[c]), A.rate_scale);
  const cplx g_top = cscale(caxpy(H2_top, A.nu_xi, caxpy(d2vt, -k2s, vt0)), A.ysi);
  const cplx g_bot = cscale(csub(caxpy(H2_bot, A.nu_xi, caxpy(d2vb, -k2s, vb0)), rate), A.ysi);
  const cplx r_top = csub(g_top, dPt), r_bot = csub(g_bot, dPb);
  const double* mi = A.pkinv + (size_t)crec * 4;
  const cplx c0 = make_double2(mi[0] * r_top.x + mi[1] * r_bot.x, mi[0] * r_top.y + mi[1] * r_bot.y);
  const cplx c1 = make_double2(mi[2] * r_top.x + mi[3] * r_bot.x, mi[2] * r_top.y + mi[3] * r_bot.y);
  const double* pk = A.pk + (size_t)crec * NY;
  for (int k = 0; k < A.n_pplanes; ++k) {
    const int j = A.pjs[k];
    const bool flip = j > H;
    const int jj = flip ? N - j : j;
    cplx part = cz();
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int e = lane + 64 * s;
      if (e <= N) {
        const double sg = (e & 1) ? -1.0 : 1.0;
        const cplx Pe = caxpy(caxpy(Pd[s], pk[e], c0), sg * pk[e], c1);
        part = caxpy(part, A.cosk[(size_t)jj * (N + 1) + e] * (flip ? sg : 1.0), Pe);
      }
    }
    const cplx val = wave_sum(part);
    if (lane == 0) {
      A.pbuf[(size_t)k * pstride + (size_t)p * nz + q] = val;
      if (partner >= 0) A.pbuf[(size_t)k * pstride + partner] = cconj(val);
    }
  }
}

template <int N>
static int launch_pgen(const PressGenArgs& A, hipStream_t st, KernelTimer* tm) {
  constexpr int WPB = wpb<N>();
  const int blocks = (A.ncol + WPB - 1) / WPB;
  const size_t shm = (size_t)WPB * CP<N>::WAVE_DOUBLES * sizeof(double);
  TIMED_LAUNCH(tm, KC_OUTPUT, st, k_pressure_gen<N>, dim3(blocks), dim3(64 * WPB), shm, st, A);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_pressure_generic(const Dims& d, const DeviceState& s, const PhysParams& ph, int n_planes,
                            const int* js_planes, bool ramp, int n_sub, hipStream_t st, KernelTimer* tm) {
  PressGenArgs A;
  std::memset(&A, 0, sizeof(A));
  A.nkx = d.nkx;
  A.nz = d.nz;
  A.ncol = d.ncol;
  A.n_pplanes = n_planes;
  for (int k = 0; k < n_planes && k < MAX_PLANES; ++k) A.pjs[k] = js_planes[k];
  A.ramp = ramp ? 1 : 0;
  A.rate_scale = 1.0 / ((double)n_sub * ph.dt);
  A.ys = ph.ys;
  A.ysi = 1.0 / ph.ys;
  A.nu_xi = ph.nu_xi();
  A.plane = (size_t)d.ny * d.nkx * d.nz;
  A.H3 = s.H3;
  A.vS = s.vS;
  A.vw_old = s.vw_old;
  A.vw_new = s.vw_new;
  A.pbuf = s.pbuf;
  A.cosk = s.cosk;
  A.rc = s.rc;
  A.optab = s.optab;
  A.alpha = s.alpha;
  A.beta = s.beta;
  A.pk = s.pk;
  A.pkinv = s.pkinv;
  switch (d.N) {
    case 16: return launch_pgen<16>(A, st, tm);
    case 32: return launch_pgen<32>(A, st, tm);
    case 64: return launch_pgen<64>(A, st, tm);
    case 96: return launch_pgen<96>(A, st, tm);
    case 128: return launch_pgen<128>(A, st, tm);
    default: return -1;
  }
}

template <int N>
static int launch_col(const ColArgs& A, hipStream_t st, KernelTimer* tm) {
  constexpr int WPB = wpb<N>();
  const int blocks = (A.ncol + WPB - 1) / WPB;
  const size_t shm = (size_t)WPB * CP<N>::WAVE_DOUBLES * sizeof(double);
  TIMED_LAUNCH(tm, A.stage < 0 ? KC_RECON : KC_COLUMN, st, k_column<N>, dim3(blocks), dim3(64 * WPB), shm, st, A);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}


int launch_column_pass(const Dims& d, DeviceState& s, const PhysParams& ph, int stage,
                       const StageConsts& sc, int wall_mode, double s_ramp, int js,
                       double opp_alpha, bool accumulate_drag, bool recon, hipStream_t st, KernelTimer* tm) {
  ColArgs A;
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
  A.nu = ph.nu * ph.ys;
  A.open = ph.open;
  A.ys = ph.ys;
  A.ysi = 1.0 / ph.ys;
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
  A.cosk = s.cosk;
  A.rc = s.rc;
  A.optab = s.optab;
  A.vt = s.vt;
  A.minv = s.minv;
  A.pt = s.pt;
  A.ptinv = s.ptinv;
  A.up = s.up;
  A.inv_int_up = s.inv_int_up;
  A.alpha = s.alpha;
  A.beta = s.beta;
  A.drag_acc = s.drag_acc;
  A.status = s.status;
  switch (d.N) {
    case 16: return launch_col<16>(A, st, tm);
    case 32: return launch_col<32>(A, st, tm);
    case 64: return launch_col<64>(A, st, tm);
    case 96: return launch_col<96>(A, st, tm);
    case 128: return launch_col<128>(A, st, tm);
    default: return -1;
  }
}

// ----------------------------------------------------------------------------
// Small kernels: step bookkeeping, action ingest, observation and wall shear.
// ----------------------------------------------------------------------------
// ----------------------------------------------------------------------------
// Per-env-step kernels.  Each covers every channel of a step call (blockIdx.y = channel),
// whatever its grid: sizes come from the channel's StepChan, LDS is sized by the launcher
// for the largest channel, and blocks beyond a channel's own extent return at once.
// ----------------------------------------------------------------------------

// Start of an env step: clear the status word and the drag accumulator; v_w,new := 0 when
// an external-action channel gets no action.
__global__ void k_begin_step(const StepChan* __restrict__ chans) {
  const StepChan C = chans[blockIdx.y];
  const int t = threadIdx.x;
  if (t == 0) {
    C.status[0] = C.skip ? STATUS_BAD_ACTION : 0;
    C.drag_acc[0] = 0.0;
  }
  if (C.zero_vw && !C.skip) {
    for (int i = t; i < C.ncol; i += blockDim.x) C.vw_new[i] = cz();
  }
}

int launch_begin_step(const StepChan* d_step, int nch, hipStream_t st, KernelTimer* tm) {
  if (nch < 1) return 0;
  timed_launch(tm, KC_BOOK, k_begin_step, dim3(1, nch), dim3(256), 0, st, d_step);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Rows of the action: finiteness check, clip, forward FFT along x; keeps p < nx/2.
__global__ void k_ingest_rows(const StepChan* __restrict__ chans) {
  extern __shared__ double dyn_lds[];
  const StepChan C = chans[blockIdx.y];
  const int k = blockIdx.x;
  if (C.action == nullptr || C.skip || k >= C.nz) return;
  const int nx = C.nx, nkx = C.nkx;
  cplx* a = reinterpret_cast<cplx*>(dyn_lds);
  cplx* b = a + nx;
  int bad = 0;
  for (int i = threadIdx.x; i < nx; i += blockDim.x) {
    double v = C.action[(size_t)k * nx + i];
    if (!isfinite(v)) bad = 1;
    if (C.clip > 0.0) v = fmin(fmax(v, -C.clip), C.clip);
    a[i] = make_double2(v, 0.0);
  }
  if (__syncthreads_or(bad)) {
    if (threadIdx.x == 0) atomicOr(C.status, STATUS_BAD_ACTION);
    return;
  }
  cplx* r = fft_batch(a, b, nx, 1, nx, C.twnx, false);
  for (int pidx = threadIdx.x; pidx < nkx; pidx += blockDim.x) C.tmp2d[(size_t)k * nkx + pidx] = r[pidx];
}

// Columns: forward FFT along z, 1/(nx nz), Nyquist and mean removed, Hermitian fix.
__global__ void k_ingest_cols(const StepChan* __restrict__ chans) {
  extern __shared__ double dyn_lds[];
  const StepChan C = chans[blockIdx.y];
  const int p = blockIdx.x;
  if (C.action == nullptr || p >= C.nkx) return;
  if (*C.status & STATUS_BAD_ACTION) return;
  const int nx = C.nx, nz = C.nz, nkx = C.nkx;
  cplx* a = reinterpret_cast<cplx*>(dyn_lds);
  cplx* b = a + nz;
  for (int k = threadIdx.x; k < nz; k += blockDim.x) a[k] = C.tmp2d[(size_t)k * nkx + p];
  __syncthreads();
  cplx* r = fft_batch(a, b, nz, 1, nz, C.twnz, false);
  const double sc = 1.0 / ((double)nx * (double)nz);
  const int h = nz / 2;
  for (int q = threadIdx.x; q < nz; q += blockDim.x) {
    cplx v = cz();
    if (q != h && !(p == 0 && q == 0)) {
      v = (p == 0 && q > h) ? cconj(r[nz - q]) : r[q];
      v = cscale(v, sc);
    }
    C.vw_new[(size_t)p * nz + q] = v;
  }
}

int launch_ingest(const StepChan* d_step, int nch, int max_nx, int max_nz, int max_nkx, hipStream_t st,
                  KernelTimer* tm) {
  if (nch < 1) return 0;
  timed_launch(tm, KC_INGEST, k_ingest_rows, dim3(max_nz, nch), dim3(64), (size_t)2 * max_nx * sizeof(cplx), st,
               d_step);
  timed_launch(tm, KC_INGEST, k_ingest_cols, dim3(max_nkx, nch), dim3(64), (size_t)2 * max_nz * sizeof(cplx), st,
               d_step);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Output transforms, slot = blockIdx.z (tau_w, then per observation plane u, v, w and P into
// the observation and u, v, w into the pressure scratch).
// Source spectra are [p][q].  Columns: inverse FFT along z.
__global__ void k_out_cols(const StepChan* __restrict__ chans) {
  extern __shared__ double dyn_lds[];
  const StepChan& C = chans[blockIdx.y];  // read in place: a copy indexed by slot lives in scratch
  const int p = blockIdx.x, f = blockIdx.z;
  const cplx* src = C.out_src[f];
  if (src == nullptr || C.out_dst[f] == nullptr || C.skip || p >= C.nkx) return;
  const int nz = C.nz, nkx = C.nkx;
  cplx* a = reinterpret_cast<cplx*>(dyn_lds);
  cplx* b = a + nz;
  const cplx* s = src + (size_t)p * nz;
  const int h = nz / 2;
  for (int q = threadIdx.x; q < nz; q += blockDim.x) a[q] = (q == h) ? cz() : s[q];
  __syncthreads();
  cplx* r = fft_batch(a, b, nz, 1, nz, C.twnz, true);
  for (int k = threadIdx.x; k < nz; k += blockDim.x) C.tmp2d[((size_t)f * nz + k) * nkx + p] = r[k];
}

// Rows: Hermitian extension along x (real part of p = 0), inverse FFT, real part out.
__global__ void k_out_rows(const StepChan* __restrict__ chans) {
  extern __shared__ double dyn_lds[];
  const StepChan& C = chans[blockIdx.y];
  const int k = blockIdx.x, f = blockIdx.z;
  double* out = C.out_dst[f];
  if (C.out_src[f] == nullptr || out == nullptr || C.skip || k >= C.nz) return;
  const int nx = C.nx, nz = C.nz, nkx = C.nkx;
  cplx* a = reinterpret_cast<cplx*>(dyn_lds);
  cplx* b = a + nx;
  const cplx* row = C.tmp2d + ((size_t)f * nz + k) * nkx;
  for (int i = threadIdx.x; i < nx; i += blockDim.x) {
    cplx v = cz();
    if (i == 0) {
      v = make_double2(row[0].x, 0.0);
    } else if (i < nkx) {
      v = row[i];
    } else if (i > nx - nkx) {
      v = cconj(row[nx - i]);
    }
    a[i] = v;
  }
  __syncthreads();
  cplx* r = fft_batch(a, b, nx, 1, nx, C.twnx, true);
  for (int i = threadIdx.x; i < nx; i += blockDim.x) out[(size_t)k * nx + i] = r[i].x;
}

// Static pressure on plane blockIdx.y of channel blockIdx.x: the output transforms left P (the
// pair (0, 0) excluded) in the observation and u, v, w in the scratch; p = P - (|u|^2/2 minus
// its plane mean), pointwise on the N_z x N_x grid, in place.  Fixed-order block reduction.
__global__ __launch_bounds__(256) void k_pressure_finish(const StepChan* __restrict__ chans) {
  __shared__ double red[256];
  const StepChan& C = chans[blockIdx.x];
  const int base = 1 + SLOTS_PER_PLANE * (int)blockIdx.y;
  auto pr = C.out_dst[base + 3];
  if (C.skip || pr == nullptr || C.out_src[base + 3] == nullptr) return;  // uniform per block
  auto u = C.out_dst[base + 4];
  auto v = C.out_dst[base + 5];
  auto w = C.out_dst[base + 6];
  const int n = C.nx * C.nz;
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc += 0.5 * (u[i] * u[i] + v[i] * v[i] + w[i] * w[i]);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  const double mean = red[0] / (double)n;
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    pr[i] = pr[i] - (0.5 * (u[i] * u[i] + v[i] * v[i] + w[i] * w[i]) - mean);
}

int launch_pressure_finish(const StepChan* d_step, int nch, hipStream_t st, KernelTimer* tm) {
  if (nch < 1) return 0;
  timed_launch(tm, KC_OUTPUT, k_pressure_finish, dim3(nch, MAX_PLANES), dim3(256), 0, st, d_step);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_outputs(const StepChan* d_step, int nch, int max_nx, int max_nz, int max_nkx, int nslots, hipStream_t st,
                   KernelTimer* tm) {
  if (nch < 1) return 0;
  if (nslots < 1 || nslots > OUT_SLOTS) return -1;
  const size_t shz = (size_t)2 * max_nz * sizeof(cplx), shx = (size_t)2 * max_nx * sizeof(cplx);
  timed_launch(tm, KC_OUTPUT, k_out_cols, dim3(max_nkx, nch, nslots), dim3(64), shz, st, d_step);
  timed_launch(tm, KC_OUTPUT, k_out_rows, dim3(max_nz, nch, nslots), dim3(64), shx, st, d_step);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// End of an env step: drag = accumulated / n, v_w,old := v_w,new (unless the action was
// rejected), and the channel's status into the batch-wide status array.
__global__ void k_finish_step(const StepChan* __restrict__ chans) {
  const StepChan C = chans[blockIdx.y];
  const int t = threadIdx.x;
  const int status = *C.status;
  if (t == 0) C.status_out[0] = status;
  if (status & STATUS_BAD_ACTION) return;
  if (t == 0 && C.drag_out) C.drag_out[0] = C.drag_acc[0] / (double)C.n_sub;
  if (C.copy_vw) {
    for (int i = t; i < C.ncol; i += blockDim.x) C.vw_old[i] = C.vw_new[i];
  }
}

int launch_finish_step(const StepChan* d_step, int nch, hipStream_t st, KernelTimer* tm) {
  if (nch < 1) return 0;
  timed_launch(tm, KC_BOOK, k_finish_step, dim3(1, nch), dim3(256), 0, st, d_step);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace chanenv
