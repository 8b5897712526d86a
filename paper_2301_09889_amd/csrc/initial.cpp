// Seeded synthetic initial condition (host, FP64, built with -ffp-contract=off).
//
// The paper starts each episode from stored turbulent fields (§3.3, §4.2) that are not
// part of this library; a reproducible synthetic field stands in:
//   mean:   laminar U = 1.5 U_b (1 - r^2), r the distance from the closed channel's
//           centreline (r = xi) or from the open channel's surface (r = (1 - xi)/2), or
//           Reichardt's law of the wall in d+ = d/nu, d the distance from the nearest wall,
//           scaled so that the integral over xi is 2 U_b;
//   perturbation on 0 < k, p <= 3, |q| <= 6 (inside the resolved modes):
//           v = E_v(xi) sum_{m<8} c_m T_m(xi),   omega_y = E_o(xi) sum_{m<8} d_m T_m(xi),
//           closed channel E_v = (1 - xi^2)^2, E_o = 1 - xi^2 (v = dv/dy = omega_y = 0 at
//           both walls); open channel E_v = (1 + xi)^2 (1 - xi)^3, E_o = (1 + xi)(1 - xi)^2
//           (wall conditions at the bottom; v = v'' = omega_y' = 0 at the surface);
//           divergence-free by construction of the v--omega_y form; Re and Im of c_m, d_m are 2U - 1
//           with U = (x >> 11) 2^-53 from SplitMix64(seed) (Steele, Lea & Flood 2014),
//           drawn in the order q = -6..6, p, field (v, omega_y), m, Re then Im;
//   the p = 0 column is made Hermitian (the q > 0 half is kept), and the perturbation
//   is scaled so that sqrt(<u'^2 + v'^2 + w'^2>/3) = amp * 1.5 U_b, the y integral
//   being Clenshaw--Curtis quadrature on the nodes.
#include <cmath>
#include <complex>

#include "chanenv_internal.h"

namespace chanenv {

namespace {

struct SplitMix64 {
  uint64_t s;
  uint64_t next() {
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return (double)(next() >> 11) * 0x1.0p-53; }
};

typedef std::complex<double> cd;

// a_n = 2/(N cb_n) sum_j f_j cos(pi n j/N) / cb_j
template <class T>
void dct_fwd(int N, const T* f, T* a) {
  for (int n = 0; n <= N; ++n) {
    T acc = T(0);
    for (int j = 0; j <= N; ++j) {
      const double cbj = (j == 0 || j == N) ? 2.0 : 1.0;
      acc += f[j] * std::cos(M_PI * (double)((n * j) % (2 * N)) / N) / cbj;
    }
    const double cbn = (n == 0 || n == N) ? 2.0 : 1.0;
    a[n] = acc * (2.0 / (N * cbn));
  }
}

template <class T>
void dct_inv(int N, const T* a, T* f) {
  for (int j = 0; j <= N; ++j) {
    T acc = T(0);
    for (int n = 0; n <= N; ++n) acc += a[n] * std::cos(M_PI * (double)((n * j) % (2 * N)) / N);
    f[j] = acc;
  }
}

void deriv(int N, const cd* a, cd* b) {
  for (int n = 0; n <= N; ++n) {
    cd acc = 0.0;
    for (int p = n + 1; p <= N; p += 2) acc += (double)p * a[p];
    b[n] = acc * (n == 0 ? 1.0 : 2.0);
  }
}

double reichardt(double dp) {
  const double kappa = 0.41;
  return std::log1p(kappa * dp) / kappa + 7.8 * (1.0 - std::exp(-dp / 11.0) - (dp / 11.0) * std::exp(-dp / 3.0));
}

}  // namespace

void initial_condition(const Dims& d, const PhysParams& ph, int profile, double amp, uint64_t seed,
                       std::vector<double>* flat) {
  const int N = d.N, NY = d.ny, nz = d.nz, nkx = d.nkx;
  std::vector<double> y(NY);
  for (int j = 0; j <= N; ++j) y[j] = std::cos(M_PI * j / N);
  std::vector<double> intw(NY, 0.0);
  for (int n = 0; n <= N; n += 2) intw[n] = 2.0 / (1.0 - (double)n * n);

  // mean profile (y[] holds the Chebyshev variable xi)
  std::vector<double> U(NY), Uv(NY);
  if (profile == 1) {
    for (int j = 0; j <= N; ++j) {
      const double dist = ph.open ? (1.0 + y[j]) / 2.0 : std::fmin(1.0 + y[j], 1.0 - y[j]);
      Uv[j] = reichardt(dist / ph.nu);
    }
    dct_fwd(N, Uv.data(), U.data());
    double q = 0.0;
    for (int n = 0; n <= N; ++n) q += intw[n] * U[n];
    for (int n = 0; n <= N; ++n) U[n] *= 2.0 * ph.ub / q;
  } else {
    for (int j = 0; j <= N; ++j) {
      const double r = ph.open ? (1.0 - y[j]) / 2.0 : y[j];
      Uv[j] = 1.5 * ph.ub * (1.0 - r * r);
    }
    dct_fwd(N, Uv.data(), U.data());
  }

  // perturbation, layout [q][p][n]
  const size_t nspec = (size_t)nz * nkx * NY;
  std::vector<cd> v(nspec, 0.0), om(nspec, 0.0);
  SplitMix64 rng{seed};
  const int pmax = std::min(3, nkx - 1), qmax = std::min(6, nz / 2 - 1);
  std::vector<cd> vals(NY), coef(NY);
  for (int qs = -qmax; qs <= qmax; ++qs) {
    for (int p = 0; p <= pmax; ++p) {
      if (p == 0 && qs == 0) continue;
      const int qi = ((qs % nz) + nz) % nz;
      for (int field = 0; field < 2; ++field) {
        cd c[8];
        for (int m = 0; m < 8; ++m) {
          const double re = 2.0 * rng.uniform() - 1.0;
          const double im = 2.0 * rng.uniform() - 1.0;
          c[m] = cd(re, im);
        }
        for (int j = 0; j <= N; ++j) {
          cd s = 0.0;
          for (int m = 0; m < 8; ++m) s += c[m] * std::cos(M_PI * (double)((m * j) % (2 * N)) / N);
          double env;
          if (ph.open) {
            const double bp = 1.0 + y[j], bm = 1.0 - y[j];
            env = field == 0 ? bp * bp * (bm * bm * bm) : bp * (bm * bm);
          } else {
            const double e1 = 1.0 - y[j] * y[j];
            env = field == 0 ? e1 * e1 : e1;
          }
          vals[j] = s * env;
        }
        dct_fwd(N, vals.data(), coef.data());
        cd* dst = (field == 0 ? v.data() : om.data()) + ((size_t)qi * nkx + p) * NY;
        for (int n = 0; n <= N; ++n) dst[n] = coef[n];
      }
    }
  }
  for (int q = 1; q < nz / 2; ++q)
    for (int n = 0; n <= N; ++n) {
      v[((size_t)(nz - q) * nkx) * NY + n] = std::conj(v[((size_t)q * nkx) * NY + n]);
      om[((size_t)(nz - q) * nkx) * NY + n] = std::conj(om[((size_t)q * nkx) * NY + n]);
    }

  // rms of the fluctuation: Parseval in (x, z), Clenshaw--Curtis in y
  double total = 0.0;
  std::vector<cd> Dv(NY), uu(NY), ww(NY), fv(NY), g(NY), gc(NY);
  for (int q = 0; q < nz; ++q) {
    if (q == nz / 2) continue;
    const int qs = (q < nz / 2) ? q : q - nz;
    const double be = 2.0 * M_PI * qs / ph.lz;
    for (int p = 0; p < nkx; ++p) {
      if (p == 0 && q == 0) continue;
      const double al = 2.0 * M_PI * p / ph.lx;
      const double k2 = al * al + be * be;
      const cd* vp = &v[((size_t)q * nkx + p) * NY];
      const cd* op = &om[((size_t)q * nkx + p) * NY];
      deriv(N, vp, Dv.data());
      for (int n = 0; n <= N; ++n) Dv[n] *= ph.ys;  // d/dy = ys d/dxi
      const cd I(0.0, 1.0);
      for (int n = 0; n <= N; ++n) {
        uu[n] = (I * al * Dv[n] - I * be * op[n]) / k2;
        ww[n] = (I * be * Dv[n] + I * al * op[n]) / k2;
      }
      const double mult = (p == 0) ? 1.0 : 2.0;
      const cd* fields[3] = {uu.data(), vp, ww.data()};
      for (int f = 0; f < 3; ++f) {
        dct_inv(N, fields[f], fv.data());
        std::vector<double> m2(NY), m2c(NY);
        for (int j = 0; j <= N; ++j) m2[j] = std::norm(fv[j]);
        dct_fwd(N, m2.data(), m2c.data());
        double integ = 0.0;
        for (int n = 0; n <= N; ++n) integ += intw[n] * m2c[n];
        total += mult * integ;
      }
    }
  }
  const double rms = std::sqrt(total / 2.0 / 3.0);
  const double scale = (rms > 0.0) ? amp * 1.5 * ph.ub / rms : 0.0;

  const size_t total_doubles = 4 * nspec + 2 * (size_t)NY + 2 * (size_t)nz * nkx + 2;
  flat->assign(total_doubles, 0.0);
  double* o = flat->data();
  for (size_t i = 0; i < nspec; ++i) {
    o[2 * i] = v[i].real() * scale;
    o[2 * i + 1] = v[i].imag() * scale;
  }
  o += 2 * nspec;
  for (size_t i = 0; i < nspec; ++i) {
    o[2 * i] = om[i].real() * scale;
    o[2 * i + 1] = om[i].imag() * scale;
  }
  o += 2 * nspec;
  for (int n = 0; n <= N; ++n) o[n] = U[n];
  // W, old action, t and the step counter stay zero
}

}  // namespace chanenv
