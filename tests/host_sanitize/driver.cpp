// Host-side checks of the library's validation, operator precompute, initial condition and
// plane-pass tiling, built host-only with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_host_sanitize.py.  No GPU call succeeds here (there is no device); every device
// path ends at its first HIP call with CHAN_EDEVICE, after the host work it does first.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "chanenv.h"
#include "chanenv_internal.h"

using namespace chanenv;

static int failures = 0;

#define CHECK(cond, ...)                                \
  do {                                                  \
    if (!(cond)) {                                      \
      ++failures;                                       \
      std::fprintf(stderr, "FAILED %s: ", #cond);       \
      std::fprintf(stderr, __VA_ARGS__);                \
      std::fprintf(stderr, "\n");                       \
    }                                                   \
  } while (0)

static chan_grid_t grid(int nx, int ny, int nz) {
  chan_grid_t g;
  g.nx = nx;
  g.ny = ny;
  g.nz = nz;
  g.lx = 2.67;
  g.lz = 0.8;
  g.re_tau = 180.0;
  g.dt_plus = 0.05;
  g.obs_y_plus = 15.0;
  return g;
}

static Dims dims(int nx, int ny, int nz) {
  Dims d;
  d.nx = nx;
  d.ny = ny;
  d.nz = nz;
  d.N = ny - 1;
  d.nkx = nx / 2;
  d.mx = 3 * nx / 2;
  d.mz = 3 * nz / 2;
  d.ncol = d.nkx * nz;
  d.ml = d.N / 2 + 1;
  d.opsz = 4 * d.ml + 2;
  return d;
}

static PhysParams phys(bool open, double re_tau) {
  PhysParams ph;
  ph.nu = 1.0 / re_tau;
  ph.dt = 0.05 / re_tau;
  ph.ub = 15.66;
  ph.forcing = 0;
  ph.px = 0.0;
  ph.lx = 2.67;
  ph.lz = 0.8;
  ph.open = open ? 1 : 0;
  ph.ys = open ? 2.0 : 1.0;
  return ph;
}

// Every supported grid: footprint > 0, and creation gets past validation and the host
// precompute (then stops at the missing device, or succeeds where there is one).
static void valid_grids() {
  const int nys[] = {17, 33, 65, 97, 129};
  const int nxs[] = {4, 16, 128};
  for (int ny : nys)
    for (int nx : nxs)
      for (int top = 0; top < 2; ++top) {
        chan_grid_t g = grid(nx, ny, nx == 128 ? 8 : nx);
        chan_opts_t o;
        chan_opts_default(&o);
        o.top_bc = top ? CHAN_TOP_FREESLIP : CHAN_TOP_WALL;
        o.obs_mask = CHAN_OBS_U | CHAN_OBS_V | CHAN_OBS_P;
        o.n_extra_planes = 1;
        o.extra_obs_y_plus[0] = 5.0;
        const size_t fp = chan_env_footprint_bytes(&g, &o);
        CHECK(fp > 0, "footprint of %dx%dx%d top %d", g.nx, g.ny, g.nz, top);
        chan_env* e = nullptr;
        const int rc = chan_env_create(&g, &o, nullptr, &e);
        CHECK(rc == CHAN_OK || rc == CHAN_EDEVICE, "create %dx%dx%d top %d: %d (%s)", g.nx, g.ny, g.nz, top, rc,
              chan_last_error());
        if (rc == CHAN_OK) chan_env_destroy(e);
        else CHECK(e == nullptr, "*out written on failure");
      }
}

// Every invalid grid or option: footprint 0, creation refused with CHAN_EINVAL and *out
// untouched, without any device call.
static void invalid_inputs() {
  const double nan = std::nan("");
  std::vector<chan_grid_t> bad;
  chan_grid_t g = grid(16, 65, 16);
  auto push = [&](chan_grid_t x) { bad.push_back(x); };
  { chan_grid_t x = g; x.nx = 3; push(x); }
  { chan_grid_t x = g; x.nx = 256; push(x); }
  { chan_grid_t x = g; x.nz = 2; push(x); }
  { chan_grid_t x = g; x.ny = 64; push(x); }
  { chan_grid_t x = g; x.ny = 257; push(x); }
  { chan_grid_t x = g; x.lx = 0.0; push(x); }
  { chan_grid_t x = g; x.lz = INFINITY; push(x); }
  { chan_grid_t x = g; x.re_tau = -1.0; push(x); }
  { chan_grid_t x = g; x.re_tau = nan; push(x); }
  { chan_grid_t x = g; x.dt_plus = 0.0; push(x); }
  { chan_grid_t x = g; x.obs_y_plus = 1e6; push(x); }   // above the channel
  { chan_grid_t x = g; x.obs_y_plus = nan; push(x); }
  for (const chan_grid_t& x : bad) {
    CHECK(chan_env_footprint_bytes(&x, nullptr) == 0, "footprint of an invalid grid (%d %d %d)", x.nx, x.ny, x.nz);
    chan_env* e = reinterpret_cast<chan_env*>(0x1);
    CHECK(chan_env_create(&x, nullptr, nullptr, &e) == CHAN_EINVAL, "create accepted an invalid grid");
    CHECK(e == reinterpret_cast<chan_env*>(0x1), "*out written for an invalid grid");
  }
  std::vector<chan_opts_t> bado;
  chan_opts_t o;
  chan_opts_default(&o);
  { chan_opts_t x = o; x.top_bc = 2; bado.push_back(x); }
  { chan_opts_t x = o; x.forcing = -1; bado.push_back(x); }
  { chan_opts_t x = o; x.controller = 7; bado.push_back(x); }
  { chan_opts_t x = o; x.action_mode = 2; bado.push_back(x); }
  { chan_opts_t x = o; x.obs_mask = 16; bado.push_back(x); }
  { chan_opts_t x = o; x.ub_plus = INFINITY; bado.push_back(x); }
  { chan_opts_t x = o; x.clip = nan; bado.push_back(x); }
  { chan_opts_t x = o; x.n_extra_planes = CHAN_MAX_EXTRA_PLANES + 1; bado.push_back(x); }
  { chan_opts_t x = o; x.n_extra_planes = -1; bado.push_back(x); }
  { chan_opts_t x = o; x.n_extra_planes = 2; x.extra_obs_y_plus[0] = 5.0; x.extra_obs_y_plus[1] = -3.0; bado.push_back(x); }
  { chan_opts_t x = o; x.n_extra_planes = 1; x.extra_obs_y_plus[0] = 1e6; bado.push_back(x); }
  for (const chan_opts_t& x : bado) {
    CHECK(chan_env_footprint_bytes(&g, &x) == 0, "footprint with invalid options");
    chan_env* e = nullptr;
    CHECK(chan_env_create(&g, &x, nullptr, &e) == CHAN_EINVAL, "create accepted invalid options");
    CHECK(e == nullptr, "*out written for invalid options");
  }
  CHECK(chan_env_create(nullptr, nullptr, nullptr, nullptr) == CHAN_EINVAL, "null arguments");
  double state[4] = {0, 0, 0, 0};
  CHECK(chan_step_static(&bad[0], nullptr, nullptr, state, nullptr, 1, nullptr, nullptr, nullptr) == CHAN_EINVAL,
        "static step accepted an invalid grid");
  CHECK(chan_batch_create(0, nullptr, nullptr) == CHAN_EINVAL, "empty batch");
  // captured steps and the tuning query refuse missing arguments without touching a device
  chan_graph* gr = reinterpret_cast<chan_graph*>(0x1);
  CHECK(chan_batch_capture(nullptr, 1, nullptr, nullptr, 1, nullptr, nullptr, nullptr, &gr) == CHAN_EINVAL,
        "capture without a batch");
  CHECK(gr == nullptr, "capture without a batch leaves *out null");
  CHECK(chan_env_capture(nullptr, nullptr, 1, nullptr, nullptr, nullptr, nullptr) == CHAN_EINVAL, "env capture");
  chan_call* call = reinterpret_cast<chan_call*>(0x1);
  CHECK(chan_graph_launch(nullptr, nullptr, &call) == CHAN_EINVAL, "launch without a graph");
  CHECK(call == nullptr, "launch without a graph leaves *out null");
  chan_graph_destroy(nullptr);
  int32_t rec[7];  // one tuning record
  CHECK(chan_batch_tuning(nullptr, 1, rec) == CHAN_EINVAL, "tuning of no batch");
  for (int code = -8; code <= 0; ++code) CHECK(chan_strerror(code) != nullptr, "strerror(%d)", code);
  CHECK(chan_last_error() != nullptr, "last error");
}

// The homogeneous solutions of the influence-matrix method meet their Dirichlet rows to rounding
// (the tau solve's x0 refinement): v_+(+1) = v_+(-1) = 0 for every pair and stage, and in the
// open channel phi_+(+1) = 1, phi_+(-1) = 0.  Residuals relative to sum |x_n|; the scan alone
// (without the refinement) leaves them at eps times its much larger intermediate sums.
static void boundary_rows(const Dims& d, const HostTables& t, bool open, double* worst) {
  const int N = d.N, NY = d.ny;
  for (int c = 1; c < d.ncol; ++c) {
    const int q = c % d.nz;
    if (q >= d.nz / 2) continue;
    for (int r = 0; r < 3; ++r) {
      const double* v = &t.data[t.L.vt + ((size_t)c * 3 + r) * NY];
      double top = 0.0, bot = 0.0, mag = 0.0;
      for (int n = 0; n <= N; ++n) {
        top += v[n];
        bot += (n & 1) ? -v[n] : v[n];
        mag += std::fabs(v[n]);
      }
      *worst = std::fmax(*worst, std::fmax(std::fabs(top), std::fabs(bot)) / mag);
      if (open) {
        const double* ph = &t.data[t.L.pt + ((size_t)c * 3 + r) * NY];
        double pt = -1.0, pb = 0.0, pm = 0.0;
        for (int n = 0; n <= N; ++n) {
          pt += ph[n];
          pb += (n & 1) ? -ph[n] : ph[n];
          pm += std::fabs(ph[n]);
        }
        *worst = std::fmax(*worst, std::fmax(std::fabs(pt), std::fabs(pb)) / pm);
      }
    }
  }
}

// The operator tables of every supported N, closed and open, at two Reynolds numbers: every
// entry finite, and the homogeneous solutions on their boundary rows.
static void tables() {
  const int nys[] = {17, 33, 65, 97, 129};
  for (int ny : nys)
    for (int open = 0; open < 2; ++open)
      for (double re : {180.0, 1000.0}) {
        const Dims d = dims(16, ny, 8);
        HostTables t;
        precompute_tables(d, phys(open != 0, re), &t);
        CHECK(!t.data.empty(), "empty tables N=%d", ny - 1);
        size_t bad = 0;
        for (double v : t.data) bad += std::isfinite(v) ? 0 : 1;
        CHECK(bad == 0, "%zu non-finite table entries N=%d open=%d re=%g", bad, ny - 1, open, re);
        double worst = 0.0;
        boundary_rows(d, t, open != 0, &worst);
        CHECK(worst <= 1e-14, "boundary rows of v_+ / phi_+ off by %.2e (N=%d open=%d re=%g)", worst, ny - 1, open, re);
        std::printf("boundary rows N=%d open=%d re=%g: %.2e\n", ny - 1, open, re, worst);
      }
}

// The seeded initial condition: finite, the documented length, the same for the same seed,
// different for another seed, and the (0, 0) pair of v and omega_y zero.
static void initial() {
  const Dims d = dims(16, 65, 16);
  const size_t nspec = (size_t)d.nz * d.nkx * d.ny * 2;
  const size_t expect = 2 * nspec + 2 * (size_t)d.ny + (size_t)d.nz * d.nkx * 2 + 2;
  for (int open = 0; open < 2; ++open)
    for (int profile = 0; profile < 2; ++profile) {
      std::vector<double> a, b, c;
      initial_condition(d, phys(open != 0, 180.0), profile, 0.1, 7, &a);
      initial_condition(d, phys(open != 0, 180.0), profile, 0.1, 7, &b);
      initial_condition(d, phys(open != 0, 180.0), profile, 0.1, 8, &c);
      CHECK(a.size() == expect, "state length %zu vs %zu", a.size(), expect);
      size_t bad = 0;
      for (double v : a) bad += std::isfinite(v) ? 0 : 1;
      CHECK(bad == 0, "non-finite initial condition");
      CHECK(a == b, "initial condition not reproducible");
      CHECK(a != c, "seed has no effect");
      double m = 0.0;
      for (int n = 0; n < d.ny; ++n) m += std::fabs(a[2 * n]) + std::fabs(a[2 * n + 1]) +
                                         std::fabs(a[nspec + 2 * n]) + std::fabs(a[nspec + 2 * n + 1]);
      CHECK(m == 0.0, "(0, 0) pair of v or omega_y not zero");
    }
}

static void tilings() {
  const int ns[] = {4, 8, 16, 32, 64, 128};
  for (int nx : ns)
    for (int nz : ns) {
      std::vector<PlaneTiles> c;
      const int rc = plane_tile_candidates(dims(nx, 33, nz), &c);
      CHECK(rc == 0 && !c.empty(), "no plane tiling for %d x %d", nx, nz);
      // the fused z inverse and x rows exist exactly for padded lengths 48 and 96 (N = 32, 64)
      const bool fusable = (nx == 32 || nx == 64) && (nz == 32 || nz == 64);
      int nfused = 0;
      for (const PlaneTiles& t : c) nfused += t.fused ? 1 : 0;
      CHECK((nfused > 0) == fusable, "fused candidates for %d x %d: %d", nx, nz, nfused);
      std::vector<PlaneTiles> split, fused;
      CHECK(plane_tile_candidates(dims(nx, 33, nz), &split, 1) == 0, "split tilings %d x %d", nx, nz);
      for (const PlaneTiles& t : split) CHECK(!t.fused, "split form lists a fused tiling");
      const int rf = plane_tile_candidates(dims(nx, 33, nz), &fused, 2);
      CHECK((rf == 0 && !fused.empty()) == fusable, "fused-only tilings %d x %d", nx, nz);
      for (const PlaneTiles& t : fused) CHECK(t.fused == 1, "fused form lists a split tiling");
      CHECK(split.size() + fused.size() == c.size(), "forms do not partition the tilings");
    }
}

int main() {
  valid_grids();
  invalid_inputs();
  tables();
  initial();
  tilings();
  if (failures) {
    std::fprintf(stderr, "%d host checks failed\n", failures);
    return 1;
  }
  std::printf("host checks passed\n");
  return 0;
}
