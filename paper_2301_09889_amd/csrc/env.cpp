// C ABI of the channel-flow environment: validation, device allocation, the stage
// loop and the state exchange.  All numerical work of a step is queued as HIP
// kernels (kernels.hip); the host only sequences launches.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>

#include "../../include/chanenv.h"
#include "chanenv_internal.h"

using namespace chanenv;

struct chan_env {
  chan_grid_t grid;
  chan_opts_t opts;
  Dims d;
  PhysParams ph;
  int js;
  double y_plus_node;
  hipStream_t stream;
  int device;
  DeviceState s;
  void* dev_block;       // single device allocation holding every buffer
  size_t dev_bytes;
  int* host_status;      // pinned
  bool have_flow, poisoned;
  double t;
  int64_t nstep;
  StageConsts sc[3];
  KernelTimer timer;
  bool force_generic;   // CHANENV_GENERIC_COLUMN=1: use the general column kernel for every N
  double timing_ms[KC_COUNT];
  int64_t timing_launches[KC_COUNT];
};

namespace {

const double RK_ALPHA[3] = {4.0 / 15.0, 1.0 / 15.0, 1.0 / 6.0};
const double RK_BETA[3] = {4.0 / 15.0, 1.0 / 15.0, 1.0 / 6.0};
const double RK_GAMMA[3] = {8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0};
const double RK_ZETA[3] = {0.0, -17.0 / 60.0, -5.0 / 12.0};
const double RK_C_END[3] = {8.0 / 15.0, 2.0 / 3.0, 1.0};

bool pow2_in(int v, int lo, int hi) {
  if (v < lo || v > hi) return false;
  return (v & (v - 1)) == 0;
}

bool valid_grid(const chan_grid_t* g) {
  if (!g) return false;
  if (!pow2_in(g->nx, 4, 128) || !pow2_in(g->nz, 4, 128)) return false;
  const int N = g->ny - 1;
  if (!(N == 16 || N == 32 || N == 64 || N == 96 || N == 128)) return false;
  if (!(g->lx > 0) || !(g->lz > 0) || !std::isfinite(g->lx) || !std::isfinite(g->lz)) return false;
  if (!(g->re_tau > 0) || !std::isfinite(g->re_tau)) return false;
  if (!(g->dt_plus > 0) || !std::isfinite(g->dt_plus)) return false;
  if (!(g->obs_y_plus > 0) || !std::isfinite(g->obs_y_plus)) return false;
  return true;
}

bool valid_opts(const chan_opts_t* o) {
  if (o->top_bc != CHAN_TOP_WALL) return false;
  if (o->forcing != CHAN_CFR && o->forcing != CHAN_CPG) return false;
  if (o->controller != CHAN_CTRL_EXTERNAL && o->controller != CHAN_CTRL_OPPOSITION) return false;
  if (o->action_mode != CHAN_RAMP && o->action_mode != CHAN_HOLD) return false;
  if (o->ic_profile != CHAN_IC_LAMINAR && o->ic_profile != CHAN_IC_REICHARDT) return false;
  if (o->obs_mask & ~7u) return false;
  const double vals[] = {o->ub_plus, o->px, o->nu_override, o->dt_override, o->opp_alpha, o->clip, o->ic_amp};
  for (double v : vals)
    if (!std::isfinite(v)) return false;
  return true;
}

Dims make_dims(const chan_grid_t* g) {
  Dims d;
  d.nx = g->nx;
  d.ny = g->ny;
  d.nz = g->nz;
  d.N = g->ny - 1;
  d.nkx = g->nx / 2;
  d.mx = 3 * g->nx / 2;
  d.mz = 3 * g->nz / 2;
  d.ncol = d.nkx * d.nz;
  d.ml = d.N / 2 + 1;
  d.opsz = 4 * d.ml + 2;
  return d;
}

PhysParams make_phys(const chan_grid_t* g, const chan_opts_t* o) {
  PhysParams p;
  p.nu = o->nu_override > 0 ? o->nu_override : 1.0 / g->re_tau;
  p.dt = o->dt_override > 0 ? o->dt_override : g->dt_plus / g->re_tau;
  p.ub = o->ub_plus > 0 ? o->ub_plus : 15.66 * std::pow(g->re_tau / 180.0, 1.0 / 7.0);
  p.forcing = o->forcing;
  p.px = o->px;
  p.lx = g->lx;
  p.lz = g->lz;
  return p;
}

// Sensing node: the first Chebyshev node at or above obs_y_plus from the lower wall.
int sensing_node(const Dims& d, double nu, double yplus, double* node_yplus) {
  int js = -1;
  for (int j = 0; j <= d.N; ++j) {
    const double dist = 1.0 + std::cos(M_PI * j / d.N);
    if (dist / nu >= yplus) js = j;
  }
  if (js >= 0) *node_yplus = (1.0 + std::cos(M_PI * js / d.N)) / nu;
  return js;
}

struct Sizes {
  size_t spec, plane6, z6, w3, h3, wall, tmp2d, tab, total;
};

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

Sizes buffer_sizes(const Dims& d, size_t tab_doubles) {
  Sizes z;
  const size_t C = sizeof(cplx);
  z.spec = align256((size_t)d.ncol * d.ny * C);
  z.plane6 = align256((size_t)6 * d.ny * d.nkx * d.nz * C);
  z.z6 = align256((size_t)6 * d.ny * d.mz * d.nkx * C);
  z.w3 = align256((size_t)3 * d.ny * d.mz * d.nkx * C);
  z.h3 = align256((size_t)3 * d.ny * d.nkx * d.nz * C);
  z.wall = align256((size_t)d.ncol * C);
  z.tmp2d = align256((size_t)3 * d.nz * d.nkx * C);
  z.tab = align256(tab_doubles * sizeof(double));
  z.total = 4 * z.spec + align256((size_t)4 * d.ny * sizeof(double)) + z.plane6 + z.z6 + z.w3 + z.h3 +
            4 * z.wall + z.tmp2d + z.tab + 256 + 256;
  return z;
}

size_t table_doubles(const Dims& d) {
  // mirrors precompute_tables' layout (with per-table rounding to even counts)
  auto r2 = [](size_t n) { return (n + 1) & ~size_t(1); };
  const int NY = d.ny, H = d.N / 2;
  const bool pm = d.N <= 64;
  size_t t = r2((size_t)(H + 1) * NY) + r2((size_t)3 * NY) + r2((size_t)d.ncol * NOPS * 2 * d.opsz) +
             r2((size_t)d.ncol * 3 * NY) + r2((size_t)d.ncol * 12) + r2((size_t)3 * NY) + r2(4) + r2(2 * d.mz) +
             r2(2 * d.mx) + r2(2 * d.nx) + r2(2 * d.nz) + r2(d.nkx) + r2(d.nz);
  if (pm)
    t += 2 * r2((size_t)(H + 1) * 64) + r2((size_t)3 * PM_ENTRIES) + r2(PM_ENTRIES) +
         r2((size_t)d.ncol * NOPS * PM_OPSZ) + r2((size_t)d.ncol * 3 * PM_ENTRIES) + r2((size_t)3 * PM_ENTRIES);
  return t;
}

thread_local std::string g_last_error;

int fail(int code, const char* what, hipError_t err = hipSuccess) {
  g_last_error = what;
  if (err != hipSuccess) {
    g_last_error += ": ";
    g_last_error += hipGetErrorString(err);
  }
  return code;
}

#define HIPCHECK(x)                                        \
  do {                                                     \
    hipError_t err_ = (x);                                 \
    if (err_ != hipSuccess) return fail(CHAN_EDEVICE, #x, err_); \
  } while (0)

// The column pass: the parity-major kernel for N <= 64, the general one above.
int column_pass(chan_env* e, int stage, const StageConsts& sc, int mode, double s_ramp, bool drag, bool recon,
                KernelTimer* tm) {
  if (e->d.N <= 64 && !e->force_generic)
    return launch_column_pass_pm(e->d, e->s, e->ph, stage, sc, mode, s_ramp, e->js, e->opts.opp_alpha, drag,
                                 recon, e->stream, tm);
  return launch_column_pass(e->d, e->s, e->ph, stage, sc, mode, s_ramp, e->js, e->opts.opp_alpha, drag, recon,
                            e->stream, tm);
}

int prime(chan_env* e) {
  // Fill the plane-pass inputs, the opposition wall velocity and the wall shear from
  // the state just loaded (column pass in reconstruct-only mode).
  StageConsts sc = e->sc[0];
  if (launch_begin_step(e->d, e->s, false, e->stream, nullptr))
    return fail(CHAN_EDEVICE, "launch begin_step", hipGetLastError());
  if (column_pass(e, -1, sc, WALL_RAMP, 0.0, false, true, nullptr))
    return fail(CHAN_EDEVICE, "launch column pass", hipGetLastError());
  HIPCHECK(hipStreamSynchronize(e->stream));
  return CHAN_OK;
}

// Host-side canonicalisation of a state in the exchange layout: zero Nyquist rows and
// the (0,0) entries of v, omega_y; Hermitian p = 0 column (q > 0 half kept).
void canonicalise(const Dims& d, double* flat) {
  const int NY = d.ny, nz = d.nz, nkx = d.nkx;
  const size_t nspec2 = (size_t)2 * nz * nkx * NY;
  for (int fld = 0; fld < 2; ++fld) {
    double* f = flat + fld * nspec2;
    auto at = [&](int q, int p, int n) { return f + 2 * (((size_t)q * nkx + p) * NY + n); };
    for (int n = 0; n < NY; ++n) {
      at(0, 0, n)[0] = 0.0;
      at(0, 0, n)[1] = 0.0;
      for (int p = 0; p < nkx; ++p) {
        at(nz / 2, p, n)[0] = 0.0;
        at(nz / 2, p, n)[1] = 0.0;
      }
      for (int q = 1; q < nz / 2; ++q) {
        at(nz - q, 0, n)[0] = at(q, 0, n)[0];
        at(nz - q, 0, n)[1] = -at(q, 0, n)[1];
      }
    }
  }
  double* vw = flat + 2 * nspec2 + 2 * NY;
  auto w = [&](int q, int p) { return vw + 2 * ((size_t)q * nkx + p); };
  w(0, 0)[0] = w(0, 0)[1] = 0.0;
  for (int p = 0; p < nkx; ++p) w(nz / 2, p)[0] = w(nz / 2, p)[1] = 0.0;
  for (int q = 1; q < nz / 2; ++q) {
    w(nz - q, 0)[0] = w(q, 0)[0];
    w(nz - q, 0)[1] = -w(q, 0)[1];
  }
}

int upload_state(chan_env* e, const double* flat_in) {
  const Dims& d = e->d;
  const int NY = d.ny, nz = d.nz, nkx = d.nkx;
  const size_t n = (size_t)4 * nz * nkx * NY + 2 * (size_t)NY + 2 * (size_t)nz * nkx + 2;
  std::vector<double> flat(flat_in, flat_in + n);
  canonicalise(d, flat.data());
  // exchange layout [q][p][n] -> device column layout [p][q][n]
  const size_t nspec2 = (size_t)2 * nz * nkx * NY;
  std::vector<double> dv(nspec2), dom(nspec2), vw(2 * (size_t)d.ncol), mean(2 * (size_t)NY), zeros;
  for (int q = 0; q < nz; ++q)
    for (int p = 0; p < nkx; ++p)
      for (int k = 0; k < 2 * NY; ++k) {
        const size_t src = ((size_t)q * nkx + p) * 2 * NY + k;
        const size_t dst = ((size_t)p * nz + q) * 2 * NY + k;
        dv[dst] = flat[src];
        dom[dst] = flat[nspec2 + src];
      }
  for (int k = 0; k < 2 * NY; ++k) mean[k] = flat[2 * nspec2 + k];
  const double* vwsrc = flat.data() + 2 * nspec2 + 2 * NY;
  for (int q = 0; q < nz; ++q)
    for (int p = 0; p < nkx; ++p)
      for (int k = 0; k < 2; ++k) vw[((size_t)p * nz + q) * 2 + k] = vwsrc[((size_t)q * nkx + p) * 2 + k];
  HIPCHECK(hipMemcpyAsync(e->s.vS, dv.data(), nspec2 * sizeof(double), hipMemcpyHostToDevice, e->stream));
  HIPCHECK(hipMemcpyAsync(e->s.oS, dom.data(), nspec2 * sizeof(double), hipMemcpyHostToDevice, e->stream));
  HIPCHECK(hipMemcpyAsync(e->s.meanS, mean.data(), 2 * NY * sizeof(double), hipMemcpyHostToDevice, e->stream));
  HIPCHECK(hipMemcpyAsync(e->s.vw_old, vw.data(), vw.size() * sizeof(double), hipMemcpyHostToDevice, e->stream));
  HIPCHECK(hipMemcpyAsync(e->s.vw_new, vw.data(), vw.size() * sizeof(double), hipMemcpyHostToDevice, e->stream));
  HIPCHECK(hipStreamSynchronize(e->stream));
  e->t = flat[n - 2];
  e->nstep = (int64_t)flat[n - 1];
  e->have_flow = true;
  e->poisoned = false;
  return prime(e);
}

}  // namespace

extern "C" {

void chan_opts_default(chan_opts_t* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->top_bc = CHAN_TOP_WALL;
  o->forcing = CHAN_CFR;
  o->controller = CHAN_CTRL_EXTERNAL;
  o->opp_alpha = 1.0;
  o->action_mode = CHAN_RAMP;
  o->clip = 1.0;
  o->obs_mask = CHAN_OBS_U | CHAN_OBS_V;
  o->ic_profile = CHAN_IC_LAMINAR;
  o->ic_amp = 0.1;
}

const char* chan_last_error(void) { return g_last_error.c_str(); }

const char* chan_strerror(int code) {
  switch (code) {
    case CHAN_OK: return "ok";
    case CHAN_EINVAL: return "invalid argument";
    case CHAN_ENOMEM: return "out of memory";
    case CHAN_EDEVICE: return "HIP device error";
    case CHAN_ENONFINITE: return "non-finite action or state";
    case CHAN_ESTATE: return "no flow state (reset or set_state first) or poisoned state";
    default: return "unknown error";
  }
}

size_t chan_env_footprint_bytes(const chan_grid_t* grid, const chan_opts_t* opts) {
  chan_opts_t o;
  if (opts) o = *opts; else chan_opts_default(&o);
  if (!valid_grid(grid) || !valid_opts(&o)) return 0;
  const Dims d = make_dims(grid);
  return buffer_sizes(d, table_doubles(d)).total;
}

int chan_env_create(const chan_grid_t* grid, const chan_opts_t* opts, void* hip_stream, chan_env** out) {
  g_last_error.clear();
  if (!out || !valid_grid(grid)) return fail(CHAN_EINVAL, "grid");
  chan_opts_t o;
  if (opts) o = *opts; else chan_opts_default(&o);
  if (!valid_opts(&o)) return fail(CHAN_EINVAL, "options");
  const Dims d = make_dims(grid);
  const PhysParams ph = make_phys(grid, &o);
  if (!(ph.nu > 0) || !(ph.dt > 0)) return CHAN_EINVAL;
  double ypn = 0.0;
  const int js = sensing_node(d, ph.nu, grid->obs_y_plus, &ypn);
  if (js < 0 || js >= d.N) return CHAN_EINVAL;

  HostTables ht;
  try {
    precompute_tables(d, ph, &ht);
  } catch (const std::bad_alloc&) {
    return CHAN_ENOMEM;
  }
  if (ht.L.total != table_doubles(d)) return CHAN_EINVAL;
  for (double v : ht.data)
    if (!std::isfinite(v)) return CHAN_EINVAL;  // e.g. a singular influence matrix

  chan_env* e = new (std::nothrow) chan_env();
  if (!e) return CHAN_ENOMEM;
  e->grid = *grid;
  e->opts = o;
  e->d = d;
  e->ph = ph;
  e->js = js;
  e->y_plus_node = ypn;
  e->stream = (hipStream_t)hip_stream;
  e->have_flow = false;
  e->poisoned = false;
  {
    const char* g = std::getenv("CHANENV_GENERIC_COLUMN");
    e->force_generic = g && g[0] == '1';
  }
  e->t = 0.0;
  e->nstep = 0;
  for (int r = 0; r < 3; ++r) {
    e->sc[r].lam0 = 1.0 / (RK_BETA[r] * ph.nu * ph.dt);
    e->sc[r].ab = RK_ALPHA[r] / RK_BETA[r];
    e->sc[r].gb = RK_GAMMA[r] / (RK_BETA[r] * ph.nu);
    e->sc[r].zb = RK_ZETA[r] / (RK_BETA[r] * ph.nu);
  }
  {
    const hipError_t err = hipGetDevice(&e->device);
    if (err != hipSuccess) {
      delete e;
      return fail(CHAN_EDEVICE, "hipGetDevice", err);
    }
  }
  const Sizes z = buffer_sizes(d, ht.L.total);
  e->dev_bytes = z.total;
  {
    const hipError_t err = hipMalloc(&e->dev_block, z.total);
    if (err != hipSuccess) {
      delete e;
      return fail(CHAN_ENOMEM, "hipMalloc", err);
    }
  }
  if (hipHostMalloc((void**)&e->host_status, sizeof(int)) != hipSuccess) {
    (void)hipFree(e->dev_block);
    delete e;
    return CHAN_ENOMEM;
  }
  char* b = (char*)e->dev_block;
  auto take = [&](size_t n) {
    char* r = b;
    b += n;
    return r;
  };
  DeviceState& s = e->s;
  s.vS = (cplx*)take(z.spec);
  s.oS = (cplx*)take(z.spec);
  s.hist = (cplx*)take(2 * z.spec);
  s.meanS = (double*)take(align256((size_t)2 * d.ny * sizeof(double)));
  s.meanH = (double*)take(align256((size_t)2 * d.ny * sizeof(double)));
  s.F6 = (cplx*)take(z.plane6);
  s.Z6 = (cplx*)take(z.z6);
  s.W3 = (cplx*)take(z.w3);
  s.H3 = (cplx*)take(z.h3);
  s.vw_old = (cplx*)take(z.wall);
  s.vw_new = (cplx*)take(z.wall);
  s.vw_opp = (cplx*)take(z.wall);
  s.tauw = (cplx*)take(z.wall);
  s.tmp2d = (cplx*)take(z.tmp2d);
  s.tab = (double*)take(z.tab);
  s.drag_acc = (double*)take(256);
  s.status = (int*)take(256);
  const TableLayout& L = ht.L;
  s.cosk = s.tab + L.cosk;
  s.rc = s.tab + L.rc;
  s.optab = s.tab + L.optab;
  s.vt = s.tab + L.vt;
  s.minv = s.tab + L.minv;
  s.up = s.tab + L.up;
  s.inv_int_up = s.tab + L.inv_int_up;
  s.alpha = s.tab + L.alpha;
  s.beta = s.tab + L.beta;
  s.twz = (const cplx*)(s.tab + L.twz);
  s.twx = (const cplx*)(s.tab + L.twx);
  s.twnx = (const cplx*)(s.tab + L.twnx);
  s.twnz = (const cplx*)(s.tab + L.twnz);
  s.kfwd = s.tab + L.kfwd;
  s.kinv = s.tab + L.kinv;
  s.rc_pm = s.tab + L.rc_pm;
  s.intw_pm = s.tab + L.intw_pm;
  s.op_pm = s.tab + L.op_pm;
  s.vt_pm = s.tab + L.vt_pm;
  s.up_pm = s.tab + L.up_pm;
  {
    hipError_t err = hipMemsetAsync(e->dev_block, 0, z.total, e->stream);
    const char* what = "hipMemsetAsync";
    if (err == hipSuccess) {
      err = hipMemcpyAsync(s.tab, ht.data.data(), ht.data.size() * sizeof(double), hipMemcpyHostToDevice, e->stream);
      what = "hipMemcpyAsync(tables)";
    }
    if (err == hipSuccess) {
      err = hipStreamSynchronize(e->stream);
      what = "hipStreamSynchronize";
    }
    if (err != hipSuccess) {
      chan_env_destroy(e);
      return fail(CHAN_EDEVICE, what, err);
    }
  }
  *out = e;
  return CHAN_OK;
}

void chan_env_destroy(chan_env* e) {
  if (!e) return;
  if (e->stream) (void)hipStreamSynchronize(e->stream);
  for (hipEvent_t ev : e->timer.pool) (void)hipEventDestroy(ev);
  if (e->dev_block) (void)hipFree(e->dev_block);
  if (e->host_status) (void)hipHostFree(e->host_status);
  delete e;
}

int chan_env_reset(chan_env* e, uint64_t seed) {
  if (!e) return CHAN_EINVAL;
  std::vector<double> flat;
  try {
    initial_condition(e->d, e->ph, e->opts.ic_profile, e->opts.ic_amp, seed, &flat);
  } catch (const std::bad_alloc&) {
    return CHAN_ENOMEM;
  }
  return upload_state(e, flat.data());
}

int chan_env_set_state(chan_env* e, const double* host, size_t n_doubles) {
  if (!e || !host) return CHAN_EINVAL;
  const Dims& d = e->d;
  const size_t n = (size_t)4 * d.nz * d.nkx * d.ny + 2 * (size_t)d.ny + 2 * (size_t)d.nz * d.nkx + 2;
  if (n_doubles != n) return CHAN_EINVAL;
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(host[i])) return CHAN_ENONFINITE;
  return upload_state(e, host);
}

int chan_env_get_state(const chan_env* e, double* host, size_t n_doubles) {
  if (!e || !host) return CHAN_EINVAL;
  const Dims& d = e->d;
  const int NY = d.ny, nz = d.nz, nkx = d.nkx;
  const size_t n = (size_t)4 * nz * nkx * NY + 2 * (size_t)NY + 2 * (size_t)nz * nkx + 2;
  if (n_doubles != n) return CHAN_EINVAL;
  if (!e->have_flow) return CHAN_ESTATE;
  const size_t nspec2 = (size_t)2 * nz * nkx * NY;
  std::vector<double> dv(nspec2), dom(nspec2), vw(2 * (size_t)d.ncol), mean(2 * (size_t)NY);
  HIPCHECK(hipStreamSynchronize(e->stream));
  HIPCHECK(hipMemcpy(dv.data(), e->s.vS, nspec2 * sizeof(double), hipMemcpyDeviceToHost));
  HIPCHECK(hipMemcpy(dom.data(), e->s.oS, nspec2 * sizeof(double), hipMemcpyDeviceToHost));
  HIPCHECK(hipMemcpy(mean.data(), e->s.meanS, 2 * NY * sizeof(double), hipMemcpyDeviceToHost));
  HIPCHECK(hipMemcpy(vw.data(), e->s.vw_old, vw.size() * sizeof(double), hipMemcpyDeviceToHost));
  for (int q = 0; q < nz; ++q)
    for (int p = 0; p < nkx; ++p)
      for (int k = 0; k < 2 * NY; ++k) {
        const size_t dst = ((size_t)q * nkx + p) * 2 * NY + k;
        const size_t src = ((size_t)p * nz + q) * 2 * NY + k;
        host[dst] = dv[src];
        host[nspec2 + dst] = dom[src];
      }
  for (int k = 0; k < 2 * NY; ++k) host[2 * nspec2 + k] = mean[k];
  double* vwdst = host + 2 * nspec2 + 2 * NY;
  for (int q = 0; q < nz; ++q)
    for (int p = 0; p < nkx; ++p)
      for (int k = 0; k < 2; ++k) vwdst[((size_t)q * nkx + p) * 2 + k] = vw[((size_t)p * nz + q) * 2 + k];
  host[n - 2] = e->t;
  host[n - 1] = (double)e->nstep;
  return CHAN_OK;
}

int chan_env_query(const chan_env* e, chan_info_t* out) {
  if (!e || !out) return CHAN_EINVAL;
  std::memset(out, 0, sizeof(*out));
  const Dims& d = e->d;
  out->nx = d.nx;
  out->ny = d.ny;
  out->nz = d.nz;
  out->js = e->js;
  out->y_plus_node = e->y_plus_node;
  out->nu = e->ph.nu;
  out->dt = e->ph.dt;
  out->ub = e->ph.ub;
  out->t = e->t;
  out->nstep = e->nstep;
  out->state_doubles = (size_t)4 * d.nz * d.nkx * d.ny + 2 * (size_t)d.ny + 2 * (size_t)d.nz * d.nkx + 2;
  out->obs_doubles = (size_t)__builtin_popcount(e->opts.obs_mask) * d.nz * d.nx;
  out->footprint_bytes = e->dev_bytes;
  return CHAN_OK;
}

int chan_env_step(chan_env* e, const double* action, int32_t n_substeps, double* obs, double* tau_w,
                  double* drag) {
  if (!e) return CHAN_EINVAL;
  if (n_substeps < 1) return CHAN_EINVAL;
  if (!e->have_flow || e->poisoned) return CHAN_ESTATE;
  const Dims& d = e->d;
  const bool ext = e->opts.controller == CHAN_CTRL_EXTERNAL;
  hipStream_t st = e->stream;
  KernelTimer* tm = e->timer.on ? &e->timer : nullptr;
  g_last_error.clear();
  if (launch_begin_step(d, e->s, ext && action == nullptr, st, tm))
    return fail(CHAN_EDEVICE, "launch begin_step", hipGetLastError());
  if (ext && action != nullptr)
    if (launch_ingest(d, e->s, action, e->opts.clip, st, tm))
      return fail(CHAN_EDEVICE, "launch ingest", hipGetLastError());
  for (int m = 0; m < n_substeps; ++m) {
    for (int r = 0; r < 3; ++r) {
      int mode = WALL_OPP;
      double s = 0.0;
      if (ext) {
        mode = WALL_RAMP;
        s = (e->opts.action_mode == CHAN_HOLD) ? 1.0 : (m + RK_C_END[r]) / (double)n_substeps;
      }
      if (launch_plane_pass(d, e->s, st, tm)) return fail(CHAN_EDEVICE, "launch plane pass", hipGetLastError());
      // The last stage of the env step leaves the reconstruction to the reconstruct-only
      // pass below, so that the plane-pass input at an env-step boundary is always made
      // by the same code path as after set_state (bitwise-identical resume).
      const bool last = (m == n_substeps - 1) && (r == 2);
      if (column_pass(e, r, e->sc[r], mode, s, r == 2, !last, tm))
        return fail(CHAN_EDEVICE, "launch column pass", hipGetLastError());
    }
  }
  if (column_pass(e, -1, e->sc[0], WALL_RAMP, 0.0, false, true, tm))
    return fail(CHAN_EDEVICE, "launch column pass", hipGetLastError());
  if (launch_finish_step(d, e->s, ext, drag, n_substeps, st, tm))
    return fail(CHAN_EDEVICE, "launch finish_step", hipGetLastError());
  if (launch_outputs(d, e->s, e->js, e->opts.obs_mask, obs, tau_w, st, tm))
    return fail(CHAN_EDEVICE, "launch outputs", hipGetLastError());
  HIPCHECK(hipMemcpyAsync(e->host_status, e->s.status, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
  const int status = *e->host_status;
  if (status & STATUS_BAD_ACTION) return fail(CHAN_ENONFINITE, "non-finite action");
  e->t += n_substeps * e->ph.dt;
  e->nstep += n_substeps;
  if (status & STATUS_NONFINITE) {
    e->poisoned = true;
    return fail(CHAN_ENONFINITE, "non-finite state after the step");
  }
  return CHAN_OK;
}

static const char* const kClassNames[KC_COUNT] = {
    "column_pass", "z_inverse_fft", "x_rows_fft_product", "z_forward_fft", "action_ingest", "outputs",
    "bookkeeping", "column_reconstruct"};

const char* chan_kernel_class_name(int32_t cls) {
  if (cls < 0 || cls >= KC_COUNT) return "";
  return kClassNames[cls];
}

// Fold the recorded event pairs into the per-class accumulators.
static int drain_timer(chan_env* e) {
  KernelTimer& t = e->timer;
  if (t.used == 0) return CHAN_OK;
  HIPCHECK(hipStreamSynchronize(e->stream));
  for (size_t k = 0; k < t.used; ++k) {
    float ms = 0.0f;
    HIPCHECK(hipEventElapsedTime(&ms, t.pool[2 * k], t.pool[2 * k + 1]));
    e->timing_ms[t.cls[k]] += ms;
    e->timing_launches[t.cls[k]] += 1;
  }
  t.used = 0;
  return CHAN_OK;
}

int chan_env_set_timing(chan_env* e, int32_t enable) {
  if (!e) return CHAN_EINVAL;
  const int rc = drain_timer(e);
  if (rc != CHAN_OK) return rc;
  for (int k = 0; k < KC_COUNT; ++k) {
    e->timing_ms[k] = 0.0;
    e->timing_launches[k] = 0;
  }
  e->timer.on = enable != 0;
  return CHAN_OK;
}

int chan_env_timing_read(chan_env* e, int32_t nclass, int64_t* launches, double* ms) {
  if (!e || nclass < 0 || (nclass > 0 && (!launches || !ms))) return CHAN_EINVAL;
  const int rc = drain_timer(e);
  if (rc != CHAN_OK) return rc;
  for (int k = 0; k < nclass && k < KC_COUNT; ++k) {
    launches[k] = e->timing_launches[k];
    ms[k] = e->timing_ms[k];
  }
  return KC_COUNT;
}

}  // extern "C"
