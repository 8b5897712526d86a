// Host precompute of the operator tables, FP64 (done once per env).
//
// * cos(pi a b / N) for the folded DCT-I, a <= N/2, b <= N.
// * The three-term rows of the quasi-tridiagonal tau form (Gottlieb & Orszag 1977;
//   Canuto et al.): for a polynomial X of degree N with b = D^2 X,
//     X_n = c_{n-2} b_{n-2} / (4n(n-1)) - b_n / (2(n^2-1)) + b_{n+2} / (4n(n+1)),
//   n = 2..N, b_m = 0 for m >= N-1.  With the tau equations b_m = lam X_m + f_m
//   (m <= N-2) this is, for each parity of n, a tridiagonal system closed by the
//   boundary row sum_i X_{2i+s} = g_s.
// * For every wavenumber pair and each of the operators D^2 - lam (the three RK
//   stages' lam = k^2 + 1/(b_r nu dt), and lam = k^2 for v) and each parity: the
//   bottom-up elimination coefficients w_i = 1/den_i, u_i = U_i/den_i,
//   f_i = -L_i/den_i with den_i = D_i + U_i f_{i+1}, the products F_i = f_1..f_i and
//   1/sum F_i.  The device then solves any right-hand side with two first-order
//   recurrences.
// * Per pair and stage, the homogeneous solution v_+ of the influence-matrix method
//   (Kim, Moin & Moser 1987): (D^2 - lam) phi_+ = 0, phi_+(+1) = 1, phi_+(-1) = 0;
//   (D^2 - k^2) v_+ = phi_+, v_+(+-1) = 0; v_- is its mirror image
//   (v_-)_n = (-1)^n (v_+)_n, and the inverse of the 2x2 matrix of dv_+-/dy at
//   the walls.
// * Mean flow: the unit-pressure-gradient response U_P of each stage and 1/int U_P.
// * Geometry: every operator acts on the Chebyshev variable xi, d/dy = ys d/dxi (ys = 1 closed
//   channel, 2 open channel), so the Helmholtz operators are built for k^2/ys^2 and the
//   viscosity nu ys^2.  In the open channel the influence matrix imposes d^2v/dxi^2 = 0 at
//   the surface instead of dv/dxi = 0, and omega_y and the mean flow take d/dxi = 0 there:
//   their Dirichlet solutions are corrected with phi_+ (the top-unit homogeneous solution),
//   which is stored with 1/(dphi_+/dxi)(+1) for every pair and stage (the mean flow's at
//   k = 0).
// * FFT twiddles exp(-2 pi i k / L) for the padded and unpadded lengths, and the
//   wavenumbers.
#include <cmath>

#include "chanenv_internal.h"

namespace chanenv {

namespace {

// Solve (D^2 - lam) X = f (tau rows 0..N-2) with X(+1) = gt, X(-1) = gb, real data,
// using the packed elimination records rec (two parities).
void host_tau_solve(const Dims& d, const double* rec, const double* rc, const double* f, double gt,
                    double gb, double* x) {
  const int N = d.N, NY = d.ny, ML = d.ml;
  std::vector<double> R(NY, 0.0), E(NY, 0.0);
  for (int n = 2; n <= N; ++n) {
    double r = rc[n] * f[n - 2] - rc[NY + n] * f[n];
    if (n + 2 <= N) r += rc[2 * NY + n] * f[n + 2];
    R[n] = r;
  }
  for (int s = 0; s < 2; ++s) {
    const double* t = rec + (size_t)s * d.opsz;
    const double *w = t, *u = t + ML, *fr = t + 2 * ML, *F = t + 3 * ML;
    const int m = (N - s) / 2;
    const double g = (s == 0) ? 0.5 * (gt + gb) : 0.5 * (gt - gb);
    double e = 0.0;
    for (int i = m; i >= 1; --i) {
      e = w[i] * R[2 * i + s] - u[i] * e;
      E[2 * i + s] = e;
    }
    double Ei = 0.0, sum = 0.0;
    for (int i = 1; i <= m; ++i) {
      Ei = E[2 * i + s] + fr[i] * Ei;
      E[2 * i + s] = Ei;
      sum += Ei;
    }
    const double x0 = (g - sum) * t[4 * ML];
    for (int i = 0; i <= m; ++i) x[2 * i + s] = (i == 0 ? 0.0 : E[2 * i + s]) + F[i] * x0;
    // one refinement of x0: the boundary-row residual removed along the homogeneous solution
    double r = -g;
    for (int i = 0; i <= m; ++i) r += x[2 * i + s];
    const double dx0 = -r * t[4 * ML];
    for (int i = 0; i <= m; ++i) x[2 * i + s] += F[i] * dx0;
  }
}

void fill_record(const Dims& d, double lam, double* rec) {
  const int N = d.N, ML = d.ml;
  for (int s = 0; s < 2; ++s) {
    double* t = rec + (size_t)s * d.opsz;
    double *w = t, *u = t + ML, *f = t + 2 * ML, *F = t + 3 * ML;
    for (int k = 0; k < d.opsz; ++k) t[k] = 0.0;
    const int m = (N - s) / 2;
    double fnext = 0.0;
    for (int i = m; i >= 1; --i) {
      const int n = 2 * i + s;
      const double cm2 = (n == 2) ? 2.0 : 1.0;
      const double en = (n <= N - 2) ? 1.0 : 0.0;
      const double en2 = (n + 2 <= N - 2) ? 1.0 : 0.0;
      const double Li = -cm2 * lam / (4.0 * n * (n - 1.0));
      const double Di = 1.0 + en * lam / (2.0 * ((double)n * n - 1.0));
      const double Ui = -en2 * lam / (4.0 * n * (n + 1.0));
      const double den = Di + Ui * fnext;
      w[i] = 1.0 / den;
      u[i] = Ui / den;
      f[i] = -Li / den;
      fnext = f[i];
    }
    F[0] = 1.0;
    double sum = 1.0;
    for (int i = 1; i <= m; ++i) {
      F[i] = f[i] * F[i - 1];
      sum += F[i];
    }
    t[4 * ML] = 1.0 / sum;
  }
}

}  // namespace

static const double RK_ALPHA[3] = {4.0 / 15.0, 1.0 / 15.0, 1.0 / 6.0};
static const double RK_BETA[3] = {4.0 / 15.0, 1.0 / 15.0, 1.0 / 6.0};

// Position of Chebyshev index n in the parity-major order (lane, or 64 for n = N), or -1.
static int pm_slot(int N, int n) {
  if (n == N) return 64;
  if (n % 2 == 0) return n / 2;
  return 32 + (n - 1) / 2;
}

// Copies of the natural-order tables in parity-major order for the N <= 64 column kernel.
static void fill_parity_major(const Dims& d, std::vector<double>& T, const TableLayout& L) {
  const int N = d.N, NY = d.ny, H = N / 2, ML = d.ml;
  const long double PI = 3.141592653589793238462643383279502884L;
  auto lane_n = [&](int l) { return l < 32 ? 2 * l : 2 * (l - 32) + 1; };
  auto lane_ok = [&](int l) { return (l < 32 ? l : l - 32) < H; };
  for (int jj = 0; jj <= H; ++jj)
    for (int l = 0; l < 64; ++l) {
      const int n = lane_n(l);
      T[L.kfwd + (size_t)jj * 64 + l] = lane_ok(l) ? (double)cosl(PI * (long double)((jj * n) % (2 * N)) / N) : 0.0;
    }
  // the distinct entries of that table: cos(pi k / N), k < 2N (the same expression, so a lookup
  // at k = (jj n) mod 2N gives the same double)
  for (int k = 0; k < 2 * N; ++k) T[L.ccos + k] = (double)cosl(PI * (long double)k / N);
  for (int n = 0; n <= N; ++n) {
    const int sl = pm_slot(N, n);
    for (int k = 0; k < 3; ++k) T[L.rc_pm + (size_t)k * PM_ENTRIES + sl] = T[L.rc + (size_t)k * NY + n];
    T[L.intw_pm + sl] = (n % 2 == 0) ? 2.0 / (1.0 - (double)n * n) : 0.0;
    for (int r = 0; r < 3; ++r) T[L.up_pm + (size_t)r * PM_ENTRIES + sl] = T[L.up + (size_t)r * NY + n];
  }
  for (int c = 0; c < d.ncol; ++c) {
    for (int op = 0; op < NOPS; ++op) {
      const double* src = &T[L.optab + ((size_t)c * NOPS + op) * 2 * d.opsz];
      double* dst = &T[L.op_pm + ((size_t)c * NOPS + op) * PM_OPSZ];
      for (int s = 0; s < 2; ++s) {
        const double* rec = src + (size_t)s * d.opsz;
        const int m = (N - s) / 2;
        for (int i = 0; i <= m; ++i) {
          const int sl = pm_slot(N, 2 * i + s);
          for (int a = 0; a < 4; ++a) dst[(size_t)a * PM_ENTRIES + sl] = rec[(size_t)a * ML + i];
        }
        dst[4 * PM_ENTRIES + s] = rec[4 * ML];
      }
    }
    for (int r = 0; r < 3; ++r)
      for (int n = 0; n <= N; ++n)
        T[L.vt_pm + ((size_t)c * 3 + r) * PM_ENTRIES + pm_slot(N, n)] = T[L.vt + ((size_t)c * 3 + r) * NY + n];
  }
}

void precompute_tables(const Dims& d, const PhysParams& ph, HostTables* out) {
  const int N = d.N, NY = d.ny, H = N / 2;
  TableLayout& L = out->L;
  size_t o = 0;
  auto take = [&](size_t n) {
    size_t r = o;
    o += (n + 1) & ~size_t(1);  // keep every table 16-byte aligned
    return r;
  };
  L.cosk = take((size_t)(H + 1) * NY);
  L.rc = take((size_t)3 * NY);
  L.optab = take((size_t)d.ncol * NOPS * 2 * d.opsz);
  L.vt = take((size_t)d.ncol * 3 * NY);
  L.minv = take((size_t)d.ncol * 3 * 4);
  L.up = take((size_t)3 * NY);
  L.inv_int_up = take(4);
  L.twz = take((size_t)2 * d.mz);
  L.twx = take((size_t)2 * d.mx);
  L.twnx = take((size_t)2 * d.nx);
  L.twnz = take((size_t)2 * d.nz);
  L.alpha = take(d.nkx);
  L.beta = take(d.nz);
  const bool pm = d.N <= 64;
  L.kfwd = take(pm ? (size_t)(H + 1) * 64 : 0);
  L.ccos = take(pm ? (size_t)2 * N : 0);
  L.rc_pm = take(pm ? (size_t)3 * PM_ENTRIES : 0);
  L.intw_pm = take(pm ? (size_t)PM_ENTRIES : 0);
  L.op_pm = take(pm ? (size_t)d.ncol * NOPS * PM_OPSZ : 0);
  L.vt_pm = take(pm ? (size_t)d.ncol * 3 * PM_ENTRIES : 0);
  L.up_pm = take(pm ? (size_t)3 * PM_ENTRIES : 0);
  const bool open = ph.open;
  L.pt_pm = take(open && pm ? (size_t)d.ncol * 3 * PM_ENTRIES : 0);
  L.ptinv = take(open ? (size_t)d.ncol * 3 : 0);
  // natural order, for the general kernel (which CHANENV_GENERIC_COLUMN can select at any N)
  L.pt = take(open ? (size_t)d.ncol * 3 * NY : 0);
  L.pk_pm = take(pm ? (size_t)d.ncol * PM_ENTRIES : 0);
  L.pkinv = take((size_t)d.ncol * 4);
  L.pk = take((size_t)d.ncol * NY);
  L.total = o;
  std::vector<double>& T = out->data;
  T.assign(L.total, 0.0);

  const long double PI = 3.141592653589793238462643383279502884L;
  for (int a = 0; a <= H; ++a)
    for (int b = 0; b <= N; ++b) {
      const int k = (a * b) % (2 * N);
      T[L.cosk + (size_t)a * NY + b] = (double)cosl(PI * (long double)k / (long double)N);
    }
  double* rc = &T[L.rc];
  for (int n = 2; n <= N; ++n) {
    const double cm2 = (n == 2) ? 2.0 : 1.0;
    rc[n] = cm2 / (4.0 * n * (n - 1.0));
    rc[NY + n] = (n <= N - 2) ? 1.0 / (2.0 * ((double)n * n - 1.0)) : 0.0;
    rc[2 * NY + n] = (n + 2 <= N - 2) ? 1.0 / (4.0 * n * (n + 1.0)) : 0.0;
  }
  double* alpha = &T[L.alpha];
  double* beta = &T[L.beta];
  for (int p = 0; p < d.nkx; ++p) alpha[p] = 2.0 * M_PI * p / ph.lx;
  for (int q = 0; q < d.nz; ++q) {
    const int qs = (q < d.nz / 2) ? q : q - d.nz;
    beta[q] = (q == d.nz / 2) ? 0.0 : 2.0 * M_PI * qs / ph.lz;
  }
  // operators in xi: nu' = nu ys^2, k'^2 = k^2 / ys^2 (exact: ys is a power of two)
  const double nux = ph.nu_xi(), iys2 = 1.0 / (ph.ys * ph.ys);
  double lam0[3];
  for (int r = 0; r < 3; ++r) lam0[r] = 1.0 / (RK_BETA[r] * nux * ph.dt);
  // dX/dxi (+1) of a coefficient vector
  auto slope_top = [&](const double* x) {
    double a = 0.0;
    for (int n = 0; n <= N; ++n) a += (double)n * n * x[n];
    return a;
  };

  std::vector<double> phi(NY), v(NY), zero(NY, 0.0);
  // Columns (p, q) and (p, N_z - q) have the same k^2 and so the same tables: only q < N_z/2
  // is filled, and the kernels read the tables of (p, N_z - q) for q > N_z/2.
  for (int c = 0; c < d.ncol; ++c) {
    const int p = c / d.nz, q = c % d.nz;
    if (q >= d.nz / 2) continue;
    const double k2 = (alpha[p] * alpha[p] + beta[q] * beta[q]) * iys2;
    double* base = &T[L.optab + (size_t)c * NOPS * 2 * d.opsz];
    for (int r = 0; r < 3; ++r) fill_record(d, k2 + lam0[r], base + (size_t)r * 2 * d.opsz);
    fill_record(d, k2, base + (size_t)3 * 2 * d.opsz);
    if (c > 0) {
      // pressure: phi_+ of (D^2 - k'^2), phi_+(+1) = 1, phi_+(-1) = 0, and the inverse of the
      // Neumann matrix [dphi_+(+1), dphi_-(+1); dphi_+(-1), dphi_-(-1)] (phi_- its mirror)
      host_tau_solve(d, base + (size_t)3 * 2 * d.opsz, rc, zero.data(), 1.0, 0.0, phi.data());
      double a = 0.0, b = 0.0;  // dphi_+/dxi at +1 and -1
      for (int n = 0; n <= N; ++n) {
        const double n2 = (double)n * n;
        a += n2 * phi[n];
        b += ((n & 1) ? n2 : -n2) * phi[n];
      }
      const double det = b * b - a * a;
      double* mi = &T[L.pkinv + (size_t)c * 4];
      mi[0] = -a / det;
      mi[1] = b / det;
      mi[2] = -b / det;
      mi[3] = a / det;
      for (int n = 0; n <= N; ++n) {
        if (pm) T[L.pk_pm + (size_t)c * PM_ENTRIES + pm_slot(N, n)] = phi[n];
        T[L.pk + (size_t)c * NY + n] = phi[n];
      }
    }
    for (int r = 0; r < 3; ++r) {
      // phi_+: (D^2 - lam) phi = 0, phi(+1) = 1, phi(-1) = 0
      host_tau_solve(d, base + (size_t)r * 2 * d.opsz, rc, zero.data(), 1.0, 0.0, phi.data());
      if (open) {
        for (int n = 0; n <= N; ++n) {
          if (pm) T[L.pt_pm + ((size_t)c * 3 + r) * PM_ENTRIES + pm_slot(N, n)] = phi[n];
          T[L.pt + ((size_t)c * 3 + r) * NY + n] = phi[n];
        }
        T[L.ptinv + (size_t)c * 3 + r] = 1.0 / slope_top(phi.data());
      }
      if (c == 0) continue;
      host_tau_solve(d, base + (size_t)3 * 2 * d.opsz, rc, phi.data(), 0.0, 0.0, v.data());
      // influence matrix M = [top row of v_+, of v_-; dv/dxi(-1) of v_+, of v_-], with
      // v_- the mirror image of v_+; top row dv/dxi(+1) (wall) or d^2v/dxi^2(+1) (surface)
      double a11 = 0.0, a12 = 0.0, a21 = 0.0, a22 = 0.0;
      for (int n = 0; n <= N; ++n) {
        const double n2 = (double)n * n;
        const double sgn = (n & 1) ? -1.0 : 1.0;
        const double wt = ph.open ? n2 * (n2 - 1.0) / 3.0 : n2;
        a11 += wt * v[n];
        a12 += wt * sgn * v[n];
        a21 += -sgn * n2 * v[n];
        a22 += -n2 * v[n];
      }
      const double det = a11 * a22 - a12 * a21;
      double* mi = &T[L.minv + ((size_t)c * 3 + r) * 4];
      mi[0] = a22 / det;
      mi[1] = -a12 / det;
      mi[2] = -a21 / det;
      mi[3] = a11 / det;
      for (int n = 0; n <= N; ++n) T[L.vt + ((size_t)c * 3 + r) * NY + n] = v[n];
    }
  }
  // mean flow: (D^2 - lam0_r) U_P = -(a_r + b_r)/(b_r nu'), U_P = 0 at the wall(s); at a
  // free-slip top dU_P/dxi = 0 (the Dirichlet solution plus a multiple of phi_+ at k = 0)
  {
    const double* base = &T[L.optab];
    std::vector<double> f(NY, 0.0);
    for (int r = 0; r < 3; ++r) {
      f[0] = -(RK_ALPHA[r] + RK_BETA[r]) / (RK_BETA[r] * nux);
      double* up = &T[L.up + (size_t)r * NY];
      host_tau_solve(d, base + (size_t)r * 2 * d.opsz, rc, f.data(), 0.0, 0.0, up);
      if (open) {
        host_tau_solve(d, base + (size_t)r * 2 * d.opsz, rc, zero.data(), 1.0, 0.0, phi.data());
        const double cu = -slope_top(up) / slope_top(phi.data());
        for (int n = 0; n <= N; ++n) up[n] += cu * phi[n];
      }
      double integ = 0.0;
      for (int n = 0; n <= N; n += 2) integ += 2.0 / (1.0 - (double)n * n) * up[n];
      T[L.inv_int_up + r] = 1.0 / integ;
    }
  }
  if (pm) fill_parity_major(d, T, L);
  auto twiddles = [&](size_t off, int len) {
    for (int k = 0; k < len; ++k) {
      const long double ang = -2.0L * PI * (long double)k / (long double)len;
      T[off + 2 * k] = (double)cosl(ang);
      T[off + 2 * k + 1] = (double)sinl(ang);
    }
  };
  twiddles(L.twz, d.mz);
  twiddles(L.twx, d.mx);
  twiddles(L.twnx, d.nx);
  twiddles(L.twnz, d.nz);
}

}  // namespace chanenv
