// C ABI of the channel-flow environment: validation, device allocation, the stage
// loop and the state exchange.  All numerical work of a step is queued as HIP
// kernels (kernels.hip); the host only sequences launches.
#include <dlfcn.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "../../include/chanenv.h"
#include "chanenv_internal.h"

using namespace chanenv;

// A grid shape seen by a batch; its plane-pass tiling is tuned once and kept while the batch
// lives, also after its channels leave.
struct ShapeInfo {
  Dims d;
  bool pm;                        // N <= 64: the parity-major column kernels
  PlaneTiles tiles = {0, 0, 0};
  int col_cw = 4;                 // columns per block of the batched column launch (tuned)
};

// Launch-argument staging of one call: the pinned host arrays, their device copy and the
// per-env status words.  A call holds its slot from launch to finish, so calls in flight at the
// same time never share staging.
struct CallSlot {
  int cap = 0;
  size_t off_col = 0, off_plane = 0, off_status = 0, bytes = 0;
  char* host = nullptr;           // pinned: StepChan[cap] | ColChan[cap] | PlaneChan[cap] | int[cap]
  char* dev = nullptr;            // the same layout on the device
  hipEvent_t done = nullptr;      // recorded after the call's last command
  bool busy = false;
};

// A call's channels of one shape: one launch per kernel covers them.
struct CallGroup {
  int shape = 0;
  std::vector<chan_env*> envs;
  ColChan* d_col = nullptr;
  const ColChan* h_col = nullptr;
  PlaneChan* d_plane = nullptr;
};

// One env step of some of a batch's channels, queued on one stream (chan_batch_launch), or
// the priming pass after reset / set_state.
struct chan_call {
  chan_batch* b = nullptr;
  CallSlot* slot = nullptr;
  hipStream_t stream = nullptr;
  std::vector<chan_env*> envs;    // in call order
  std::vector<CallGroup> groups;  // in the batch's shape order
  int n_sub = 1;
  int max_nx = 0, max_nz = 0, max_nkx = 0;
};

// One env step of some of a batch's channels captured as a HIP graph (chan_batch_capture).  The
// launch arguments never change between replays, so they are staged once, before the capture,
// into a slot the graph owns (outside the batch's pool); the graph holds the kernels, the status
// read-back into that slot's pinned words, and nothing else.  A replay is an ordinary call on
// that slot (busy while it is in flight), finished by batch_finish like any other.
struct chan_graph {
  chan_batch* b = nullptr;        // null once the batch is destroyed
  std::vector<chan_env*> envs;    // in call order
  int n_sub = 1;
  CallSlot* slot = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool stale = false;             // an env left the batch or was destroyed after the capture
};

// Envs stepped together.  Members can join and leave; every call stages the launch arguments
// of its channels (per-step StepChan, and the fixed ColChan / PlaneChan grouped by shape) in a
// slot of its own and uploads them with one copy per array.  Every env owns a batch of one for
// its own steps.
struct chan_batch {
  std::vector<chan_env*> envs;    // members in order (the indices of chan_batch_step_subset)
  std::vector<ShapeInfo> shapes;
  hipStream_t stream = nullptr;   // the synchronous calls' stream: the first member's
  int device = 0;
  std::vector<CallSlot*> slots;
  std::vector<chan_call*> calls;  // launched and not yet finished
  std::vector<chan_graph*> graphs;  // captured steps of this batch's envs (chan_batch_capture)
  KernelTimer timer;
  double timing_ms[KC_COUNT];
  int64_t timing_launches[KC_COUNT];
};

struct chan_env {
  chan_grid_t grid;
  chan_opts_t opts;
  Dims d;
  PhysParams ph;
  int js;
  double y_plus_node;
  int n_planes;                     // observation planes (the sensing plane first)
  int js_planes[MAX_PLANES];
  double y_plus_planes[MAX_PLANES];
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
  bool force_generic;   // CHANENV_GENERIC_COLUMN=1: use the general column kernel for every N
  chan_batch* self;     // batch of one for chan_env_step
  ColChan col;          // the column kernels' arguments (fixed for the env's life)
  PlaneChan plane;      // the plane kernels' arguments
  chan_call* in_flight;  // the unfinished asynchronous call holding this env, if any
  std::vector<chan_batch*> member_of;  // the caller's batches that list this env
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
  if (o->top_bc != CHAN_TOP_WALL && o->top_bc != CHAN_TOP_FREESLIP) return false;
  if (o->forcing != CHAN_CFR && o->forcing != CHAN_CPG) return false;
  if (o->controller != CHAN_CTRL_EXTERNAL && o->controller != CHAN_CTRL_OPPOSITION) return false;
  if (o->action_mode != CHAN_RAMP && o->action_mode != CHAN_HOLD) return false;
  if (o->ic_profile != CHAN_IC_LAMINAR && o->ic_profile != CHAN_IC_REICHARDT) return false;
  if (o->obs_mask & ~15u) return false;
  const double vals[] = {o->ub_plus, o->px, o->nu_override, o->dt_override, o->opp_alpha, o->clip, o->ic_amp};
  for (double v : vals)
    if (!std::isfinite(v)) return false;
  if (o->n_extra_planes < 0 || o->n_extra_planes > CHAN_MAX_EXTRA_PLANES) return false;
  for (int k = 0; k < o->n_extra_planes; ++k)
    if (!(o->extra_obs_y_plus[k] > 0) || !std::isfinite(o->extra_obs_y_plus[k])) return false;
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
  p.open = o->top_bc == CHAN_TOP_FREESLIP ? 1 : 0;
  p.ys = p.open ? 2.0 : 1.0;
  return p;
}

// Sensing node: the first Chebyshev node at or above obs_y_plus from the lower wall.
// The sensing node: the first node at or above y+ from the lower wall.  The wall distance of
// node j is 1 + xi_j (closed channel) or (1 + xi_j)/2 (open channel).
int sensing_node(const Dims& d, const PhysParams& ph, double yplus, double* node_yplus) {
  int js = -1;
  for (int j = 0; j <= d.N; ++j) {
    const double dist = (1.0 + std::cos(M_PI * j / d.N)) / ph.ys;
    if (dist / ph.nu >= yplus) js = j;
  }
  if (js >= 0) *node_yplus = (1.0 + std::cos(M_PI * js / d.N)) / ph.ys / ph.nu;
  return js;
}


bool generic_forced() {
  const char* g = std::getenv("CHANENV_GENERIC_COLUMN");
  return g && g[0] == '1';
}

// Plane-pass forms the tuner may pick from (CHANENV_PLANE_FORM, read when a shape is tuned):
// "split" only the three-launch tilings, "fused" only the fused z inverse and x rows (where the
// shape has them), anything else every tiling.  The forms give bitwise the same results.
int plane_form() {
  const char* f = std::getenv("CHANENV_PLANE_FORM");
  if (f && std::strcmp(f, "split") == 0) return 1;
  if (f && std::strcmp(f, "fused") == 0) return 2;
  return 0;
}

struct Sizes {
  size_t spec, plane6, z6, w3, h3, wall, tmp2d, tab, pbuf, pscr, total;
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
  z.tmp2d = align256((size_t)OUT_SLOTS * d.nz * d.nkx * C);
  z.tab = align256(tab_doubles * sizeof(double));
  z.pbuf = align256((size_t)MAX_PLANES * d.nkx * d.nz * C);
  z.pscr = align256((size_t)MAX_PLANES * 3 * d.nz * d.nx * sizeof(double));
  z.total = 4 * z.spec + align256((size_t)4 * d.ny * sizeof(double)) + z.plane6 + z.z6 + z.w3 + z.h3 +
            4 * z.wall + z.tmp2d + z.tab + z.pbuf + z.pscr + 256 + 256;
  return z;
}

size_t table_doubles(const Dims& d, bool open) {
  // mirrors precompute_tables' layout (with per-table rounding to even counts)
  auto r2 = [](size_t n) { return (n + 1) & ~size_t(1); };
  const int NY = d.ny, H = d.N / 2;
  const bool pm = d.N <= 64;
  size_t t = r2((size_t)(H + 1) * NY) + r2((size_t)3 * NY) + r2((size_t)d.ncol * NOPS * 2 * d.opsz) +
             r2((size_t)d.ncol * 3 * NY) + r2((size_t)d.ncol * 12) + r2((size_t)3 * NY) + r2(4) + r2(2 * d.mz) +
             r2(2 * d.mx) + r2(2 * d.nx) + r2(2 * d.nz) + r2(d.nkx) + r2(d.nz);
  if (pm)
    t += r2((size_t)(H + 1) * 64) + r2((size_t)2 * d.N) + r2((size_t)3 * PM_ENTRIES) + r2(PM_ENTRIES) +
         r2((size_t)d.ncol * NOPS * PM_OPSZ) + r2((size_t)d.ncol * 3 * PM_ENTRIES) + r2((size_t)3 * PM_ENTRIES);
  if (open) t += r2((size_t)d.ncol * 3) + r2((size_t)d.ncol * 3 * NY) + (pm ? r2((size_t)d.ncol * 3 * PM_ENTRIES) : 0);
  t += r2((size_t)d.ncol * 4) + r2((size_t)d.ncol * NY) + (pm ? r2((size_t)d.ncol * PM_ENTRIES) : 0);
  return t;
}

// Every device buffer of one env, carved in a fixed order out of one block of z.total bytes
// (the env's own allocation, or the static scratch of chan_step_static).
void carve_state(const Dims& d, const Sizes& z, const TableLayout& L, char* base, DeviceState* out) {
  char* b = base;
  auto take = [&](size_t n) {
    char* r = b;
    b += n;
    return r;
  };
  DeviceState& s = *out;
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
  s.pbuf = (cplx*)take(z.pbuf);
  s.pscr = (double*)take(z.pscr);
  s.drag_acc = (double*)take(256);
  s.status = (int*)take(256);
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
  s.ccos = s.tab + L.ccos;
  s.rc_pm = s.tab + L.rc_pm;
  s.intw_pm = s.tab + L.intw_pm;
  s.op_pm = s.tab + L.op_pm;
  s.vt_pm = s.tab + L.vt_pm;
  s.up_pm = s.tab + L.up_pm;
  s.pt_pm = s.tab + L.pt_pm;
  s.ptinv = s.tab + L.ptinv;
  s.pt = s.tab + L.pt;
  s.pk_pm = s.tab + L.pk_pm;
  s.pkinv = s.tab + L.pkinv;
  s.pk = s.tab + L.pk;
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

// Validates grid and options and fills every field of *e that does not depend on its device
// buffers (the flow is absent, the device unset).
int setup_env(const chan_grid_t* grid, const chan_opts_t* opts, void* hip_stream, chan_env* e) {
  if (!valid_grid(grid)) return fail(CHAN_EINVAL, "grid");
  chan_opts_t o;
  if (opts) o = *opts; else chan_opts_default(&o);
  if (!valid_opts(&o)) return fail(CHAN_EINVAL, "options");
  const Dims d = make_dims(grid);
  const PhysParams ph = make_phys(grid, &o);
  if (!(ph.nu > 0) || !(ph.dt > 0)) return fail(CHAN_EINVAL, "viscosity or time step");
  double ypn = 0.0;
  const int js = sensing_node(d, ph, grid->obs_y_plus, &ypn);
  if (js < 0 || js >= d.N) return fail(CHAN_EINVAL, "sensing plane not inside the channel");
  int js_planes[MAX_PLANES];
  double yp_planes[MAX_PLANES];
  js_planes[0] = js;
  yp_planes[0] = ypn;
  for (int k = 0; k < o.n_extra_planes; ++k) {
    js_planes[1 + k] = sensing_node(d, ph, o.extra_obs_y_plus[k], &yp_planes[1 + k]);
    if (js_planes[1 + k] < 0 || js_planes[1 + k] >= d.N)
      return fail(CHAN_EINVAL, "extra observation plane not inside the channel");
  }
  std::memset(&e->s, 0, sizeof(e->s));
  e->grid = *grid;
  e->opts = o;
  e->d = d;
  e->ph = ph;
  e->js = js;
  e->y_plus_node = ypn;
  e->n_planes = 1 + o.n_extra_planes;
  for (int k = 0; k < MAX_PLANES; ++k) {
    e->js_planes[k] = k < e->n_planes ? js_planes[k] : -1;
    e->y_plus_planes[k] = k < e->n_planes ? yp_planes[k] : 0.0;
  }
  e->stream = (hipStream_t)hip_stream;
  e->device = -1;
  e->dev_block = nullptr;
  e->dev_bytes = 0;
  e->host_status = nullptr;
  e->have_flow = false;
  e->poisoned = false;
  e->self = nullptr;
  e->in_flight = nullptr;
  e->force_generic = generic_forced();
  e->t = 0.0;
  e->nstep = 0;
  for (int r = 0; r < 3; ++r) {
    // in the Chebyshev variable: nu' = nu ys^2 (closed channel: nu)
    const double nux = ph.nu_xi();
    e->sc[r].lam0 = 1.0 / (RK_BETA[r] * nux * ph.dt);
    e->sc[r].ab = RK_ALPHA[r] / RK_BETA[r];
    e->sc[r].gb = RK_GAMMA[r] / (RK_BETA[r] * nux);
    e->sc[r].zb = RK_ZETA[r] / (RK_BETA[r] * nux);
  }
  return CHAN_OK;
}

// Host precompute of the operator tables (FP64), checked for the expected size and finiteness.
int host_tables(const Dims& d, const PhysParams& ph, HostTables* ht) {
  try {
    precompute_tables(d, ph, ht);
  } catch (const std::bad_alloc&) {
    return fail(CHAN_ENOMEM, "host tables");
  }
  if (ht->L.total != table_doubles(d, ph.open)) return fail(CHAN_EINVAL, "table layout");
  for (double v : ht->data)
    if (!std::isfinite(v)) return fail(CHAN_EINVAL, "non-finite operator table (singular influence matrix)");
  return CHAN_OK;
}

ColChan make_col_chan(const chan_env* e) {
  ColChan c;
  std::memset(&c, 0, sizeof(c));
  const Dims& d = e->d;
  const DeviceState& s = e->s;
  c.nkx = d.nkx;
  c.nz = d.nz;
  c.ncol = d.ncol;
  c.ext = e->opts.controller == CHAN_CTRL_EXTERNAL ? 1 : 0;
  c.hold = e->opts.action_mode == CHAN_HOLD ? 1 : 0;
  c.forcing = e->ph.forcing;
  c.js = e->js;
  c.open = e->ph.open;
  for (int r = 0; r < 3; ++r) {
    c.lam0[r] = e->sc[r].lam0;
    c.ab[r] = e->sc[r].ab;
    c.gb[r] = e->sc[r].gb;
    c.zb[r] = e->sc[r].zb;
  }
  c.nu_wall = e->ph.nu * e->ph.ys;
  c.dt = e->ph.dt;
  c.n_pplanes = (e->opts.obs_mask & CHAN_OBS_P) ? e->n_planes : 0;
  for (int k = 0; k < MAX_PLANES; ++k) c.pjs[k] = k < e->n_planes ? e->js_planes[k] : 0;
  c.ys = e->ph.ys;
  c.ysi = 1.0 / e->ph.ys;
  c.opp_alpha = e->opts.opp_alpha;
  c.ub2 = 2.0 * e->ph.ub;
  c.px = e->ph.px;
  c.plane = (size_t)d.ny * d.nkx * d.nz;
  c.vS = (decltype(c.vS))(s.vS);
  c.oS = (decltype(c.oS))(s.oS);
  c.hist = (decltype(c.hist))(s.hist);
  c.meanS = (decltype(c.meanS))(s.meanS);
  c.meanH = (decltype(c.meanH))(s.meanH);
  c.H3 = (decltype(c.H3))(s.H3);
  c.F6 = (decltype(c.F6))(s.F6);
  c.vw_old = (decltype(c.vw_old))(s.vw_old);
  c.vw_new = (decltype(c.vw_new))(s.vw_new);
  c.vw_opp = (decltype(c.vw_opp))(s.vw_opp);
  c.tauw = (decltype(c.tauw))(s.tauw);
  c.kfwd = (decltype(c.kfwd))(s.kfwd);
  c.ccos = (decltype(c.ccos))(s.ccos);
  c.rc_pm = (decltype(c.rc_pm))(s.rc_pm);
  c.intw_pm = (decltype(c.intw_pm))(s.intw_pm);
  c.op_pm = (decltype(c.op_pm))(s.op_pm);
  c.vt_pm = (decltype(c.vt_pm))(s.vt_pm);
  c.up_pm = (decltype(c.up_pm))(s.up_pm);
  c.pt_pm = (decltype(c.pt_pm))(s.pt_pm);
  c.ptinv = (decltype(c.ptinv))(s.ptinv);
  c.pk_pm = (decltype(c.pk_pm))(s.pk_pm);
  c.pkinv = (decltype(c.pkinv))(s.pkinv);
  c.pbuf = (decltype(c.pbuf))(s.pbuf);
  c.minv = (decltype(c.minv))(s.minv);
  c.inv_int_up = (decltype(c.inv_int_up))(s.inv_int_up);
  c.alpha = (decltype(c.alpha))(s.alpha);
  c.beta = (decltype(c.beta))(s.beta);
  c.drag_acc = (decltype(c.drag_acc))(s.drag_acc);
  c.status = (decltype(c.status))(s.status);
  return c;
}

PlaneChan make_plane_chan(const chan_env* e) {
  PlaneChan c;
  std::memset(&c, 0, sizeof(c));
  const Dims& d = e->d;
  c.ny = d.ny;
  c.nkx = d.nkx;
  c.nz = d.nz;
  c.scale = 1.0 / ((double)d.mx * (double)d.mz);
  c.F6 = (decltype(c.F6))(e->s.F6);
  c.Z6 = (decltype(c.Z6))(e->s.Z6);
  c.W3 = (decltype(c.W3))(e->s.W3);
  c.H3 = (decltype(c.H3))(e->s.H3);
  c.twz = (decltype(c.twz))(e->s.twz);
  c.twx = (decltype(c.twx))(e->s.twx);
  c.status = (decltype(c.status))(e->s.status);
  return c;
}

bool uses_pm(const chan_env* e) { return e->d.N <= 64 && !e->force_generic; }

void free_slot(CallSlot* sl) {
  if (!sl) return;
  if (sl->done) {
    (void)hipEventSynchronize(sl->done);
    (void)hipEventDestroy(sl->done);
  }
  if (sl->dev) (void)hipFree(sl->dev);
  if (sl->host) (void)hipHostFree(sl->host);
  delete sl;
}

template <class T>
void erase_value(std::vector<T>& v, const T& x) {
  v.erase(std::remove(v.begin(), v.end(), x), v.end());
}

int batch_finish(chan_call* c, int32_t* results);

void batch_free(chan_batch* b) {
  if (!b) return;
  // calls never finished: finish them (wait, apply each env's outcome, release, free)
  for (chan_call* c : std::vector<chan_call*>(b->calls)) (void)batch_finish(c, nullptr);
  for (chan_graph* g : b->graphs) g->b = nullptr;  // the caller still destroys them
  for (chan_env* e : b->envs) erase_value(e->member_of, b);
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  for (CallSlot* sl : b->slots) free_slot(sl);
  for (hipEvent_t ev : b->timer.pool) (void)hipEventDestroy(ev);
  delete b;
}

// The per-call launch arguments of env e; status_out: the device word that receives its status.
StepChan make_step_chan_env(const chan_env* e, int* status_out, const double* action, int n_sub, double* obs,
                            double* tau_w, double* drag) {
  const Dims& d = e->d;
  const bool ext = e->opts.controller == CHAN_CTRL_EXTERNAL;
  StepChan c;
  std::memset(&c, 0, sizeof(c));
  c.nx = d.nx;
  c.nz = d.nz;
  c.nkx = d.nkx;
  c.ncol = d.ncol;
  c.n_sub = n_sub;
  c.skip = (e->have_flow && !e->poisoned) ? 0 : 1;
  c.zero_vw = (ext && action == nullptr) ? 1 : 0;
  c.copy_vw = ext ? 1 : 0;
  c.clip = e->opts.clip;
  c.action = (decltype(c.action))(ext ? action : nullptr);
  c.drag_out = (decltype(c.drag_out))(drag);
  const size_t plane = (size_t)d.ny * d.nkx * d.nz;
  if (obs) {  // [plane][component][z][x]
    const bool pres = (e->opts.obs_mask & CHAN_OBS_P) != 0;
    const size_t pl = (size_t)d.nz * d.nx;
    int slot = 0;
    for (int k = 0; k < e->n_planes; ++k) {
      const int base = 1 + SLOTS_PER_PLANE * k;
      const size_t node = (size_t)e->js_planes[k] * d.nkx * d.nz;
      for (int f = 0; f < 3; ++f) {
        if (pres)  // u, v, w on the plane for the Bernoulli term
          c.out_src[base + 4 + f] = (gptr<const cplx>)(e->s.F6 + (size_t)f * plane + node),
          c.out_dst[base + 4 + f] = (gptr<double>)(e->s.pscr + ((size_t)k * 3 + f) * pl);
        if (!(e->opts.obs_mask & (1u << f))) continue;
        c.out_src[base + f] = (gptr<const cplx>)(e->s.F6 + (size_t)f * plane + node);
        c.out_dst[base + f] = (gptr<double>)(obs + (size_t)slot * pl);
        ++slot;
      }
      if (pres) {  // P on the plane, then p = P - |u|^2/2 + its mean in place
        c.out_src[base + 3] = (gptr<const cplx>)(e->s.pbuf + (size_t)k * d.nkx * d.nz);
        c.out_dst[base + 3] = (gptr<double>)(obs + (size_t)slot * pl);
        ++slot;
      }
    }
  }
  if (tau_w) {
    c.out_src[0] = (gptr<const cplx>)(e->s.tauw);
    c.out_dst[0] = (gptr<double>)(tau_w);
  }
  c.vw_new = (decltype(c.vw_new))(e->s.vw_new);
  c.vw_old = (decltype(c.vw_old))(e->s.vw_old);
  c.tmp2d = (decltype(c.tmp2d))(e->s.tmp2d);
  c.twnx = (decltype(c.twnx))(e->s.twnx);
  c.twnz = (decltype(c.twnz))(e->s.twnz);
  c.drag_acc = (decltype(c.drag_acc))(e->s.drag_acc);
  c.status = (decltype(c.status))(e->s.status);
  c.status_out = (decltype(c.status_out))(status_out);
  return c;
}

int find_shape(const chan_batch* b, const chan_env* e) {
  for (size_t k = 0; k < b->shapes.size(); ++k) {
    const ShapeInfo& sh = b->shapes[k];
    if (sh.d.nx == e->d.nx && sh.d.ny == e->d.ny && sh.d.nz == e->d.nz && sh.pm == uses_pm(e)) return (int)k;
  }
  return -1;
}

int find_member(const chan_batch* b, const chan_env* e) {
  for (size_t k = 0; k < b->envs.size(); ++k)
    if (b->envs[k] == e) return (int)k;
  return -1;
}

bool size_slot(CallSlot* pick, int cap);

// A free slot of the batch's pool with room for n envs (grown or created if none), marked busy;
// nullptr if out of memory.
CallSlot* acquire_slot(chan_batch* b, int n) {
  CallSlot* pick = nullptr;
  for (CallSlot* sl : b->slots)
    if (!sl->busy && sl->cap >= n) return sl->busy = true, sl;
  for (CallSlot* sl : b->slots)
    if (!sl->busy) {
      pick = sl;
      break;
    }
  if (!pick) {
    pick = new (std::nothrow) CallSlot();
    if (!pick) return nullptr;
    if (hipEventCreateWithFlags(&pick->done, hipEventDisableTiming) != hipSuccess) {
      delete pick;
      return nullptr;
    }
    b->slots.push_back(pick);
  }
  if (!size_slot(pick, std::max(n, 2 * pick->cap))) return nullptr;
  pick->busy = true;
  return pick;
}

// (Re)allocates the slot's buffers for cap envs; false (slot unchanged) if an allocation fails.
bool size_slot(CallSlot* pick, int cap) {
  const size_t off_col = align256((size_t)cap * sizeof(StepChan));
  const size_t off_plane = off_col + align256((size_t)cap * sizeof(ColChan));
  const size_t off_status = off_plane + align256((size_t)cap * sizeof(PlaneChan));
  const size_t bytes = off_status + align256((size_t)cap * sizeof(int));
  char *dev = nullptr, *host = nullptr;
  if (hipMalloc((void**)&dev, bytes) != hipSuccess) return false;
  if (hipHostMalloc((void**)&host, bytes) != hipSuccess) {
    (void)hipFree(dev);
    return false;
  }
  if (pick->dev) (void)hipFree(pick->dev);
  if (pick->host) (void)hipHostFree(pick->host);
  pick->dev = dev;
  pick->host = host;
  pick->cap = cap;
  pick->off_col = off_col;
  pick->off_plane = off_plane;
  pick->off_status = off_status;
  pick->bytes = bytes;
  return true;
}

StepChan* host_step(const chan_call* c) { return (StepChan*)c->slot->host; }
StepChan* dev_step(const chan_call* c) { return (StepChan*)c->slot->dev; }
int* dev_status(const chan_call* c) { return (int*)(c->slot->dev + c->slot->off_status); }
int* host_status(const chan_call* c) { return (int*)(c->slot->host + c->slot->off_status); }

// Stages the launch arguments of the call's envs (c->envs set): step(k) gives env k's
// StepChan.  Groups the envs by shape (the batch's shape order, call order within a shape) and
// uploads the three arrays on the call's stream.
template <class StepFn>
int stage_call(chan_call* c, StepFn step) {
  chan_batch* b = c->b;
  const int na = (int)c->envs.size();
  if (!c->slot) c->slot = acquire_slot(b, na);  // a captured step brings its own
  if (!c->slot) return fail(CHAN_ENOMEM, "call staging buffers");
  StepChan* hs = host_step(c);
  ColChan* hc = (ColChan*)(c->slot->host + c->slot->off_col);
  PlaneChan* hp = (PlaneChan*)(c->slot->host + c->slot->off_plane);
  char* dbase = c->slot->dev;
  c->max_nx = c->max_nz = c->max_nkx = 0;
  for (int k = 0; k < na; ++k) {
    hs[k] = step(k);
    c->max_nx = std::max(c->max_nx, c->envs[k]->d.nx);
    c->max_nz = std::max(c->max_nz, c->envs[k]->d.nz);
    c->max_nkx = std::max(c->max_nkx, c->envs[k]->d.nkx);
  }
  c->groups.clear();
  size_t pos = 0;
  for (size_t sh = 0; sh < b->shapes.size(); ++sh) {
    CallGroup g;
    g.shape = (int)sh;
    g.d_col = (ColChan*)(dbase + c->slot->off_col) + pos;
    g.h_col = hc + pos;
    g.d_plane = (PlaneChan*)(dbase + c->slot->off_plane) + pos;
    for (chan_env* e : c->envs) {
      if (find_shape(b, e) != (int)sh) continue;
      g.envs.push_back(e);
      hc[pos] = e->col;
      hp[pos] = e->plane;
      ++pos;
    }
    if (!g.envs.empty()) c->groups.push_back(g);
  }
  HIPCHECK(hipMemcpyAsync(dbase, c->slot->host, na * sizeof(StepChan), hipMemcpyHostToDevice, c->stream));
  HIPCHECK(hipMemcpyAsync(dbase + c->slot->off_col, hc, pos * sizeof(ColChan), hipMemcpyHostToDevice, c->stream));
  HIPCHECK(hipMemcpyAsync(dbase + c->slot->off_plane, hp, pos * sizeof(PlaneChan), hipMemcpyHostToDevice, c->stream));
  return CHAN_OK;
}

void release_call(chan_call* c) {
  for (chan_env* e : c->envs)
    if (e && e->in_flight == c) e->in_flight = nullptr;
  if (c->slot) c->slot->busy = false;
  c->slot = nullptr;
}


// Column pass of one group after the plane pass of stage S.stage (or, S.stage = -1, the
// reconstruction alone).
int group_column(const chan_batch* b, const CallGroup& g, hipStream_t st, const ColStage& S, bool solve, bool recon,
                 KernelTimer* tm) {
  if (g.envs.empty()) return 0;
  const ShapeInfo& sh = b->shapes[g.shape];
  if (sh.pm) return launch_column_pm(sh.d, g.d_col, g.h_col, (int)g.envs.size(), S, solve, recon, st, tm, sh.col_cw);
  for (chan_env* e : g.envs) {
    const int r = S.stage;
    int mode = WALL_OPP;
    double s = 0.0;
    if (e->opts.controller == CHAN_CTRL_EXTERNAL) {
      mode = WALL_RAMP;
      if (r >= 0) s = (e->opts.action_mode == CHAN_HOLD) ? 1.0 : (S.m + RK_C_END[r]) / (double)S.n_sub;
    }
    if (launch_column_pass(e->d, e->s, e->ph, r, e->sc[r < 0 ? 0 : r], mode, s, e->js, e->opts.opp_alpha, r == 2,
                           recon, st, tm))
      return -1;
  }
  return 0;
}

int tune_plane(chan_batch* b, int shape, const std::vector<chan_env*>& members);
int tune_column(chan_batch* b, int shape, const std::vector<chan_env*>& members);

// Adds env to the batch (its shape's tiling tuned on it if the shape is new).
int batch_add(chan_batch* b, chan_env* e) {
  if (!e) return fail(CHAN_EINVAL, "batch: null env");
  if (e->device != b->device) return fail(CHAN_EINVAL, "batch: env on another device");
  if (find_member(b, e) >= 0) return fail(CHAN_EINVAL, "batch: env listed twice");
  if (e->in_flight) return fail(CHAN_EBUSY, "batch: env has an unfinished call");
  int sh = find_shape(b, e);
  if (sh < 0) {
    ShapeInfo info;
    info.d = e->d;
    info.pm = uses_pm(e);
    b->shapes.push_back(info);
    sh = (int)b->shapes.size() - 1;
    const int rc = tune_plane(b, sh, std::vector<chan_env*>{e});
    if (rc != CHAN_OK) {
      b->shapes.pop_back();
      return rc;
    }
  }
  b->envs.push_back(e);
  return CHAN_OK;
}

int batch_build(chan_env* const* envs, int n, chan_batch** out) {
  if (n < 1 || !envs) return fail(CHAN_EINVAL, "batch: no envs");
  for (int i = 0; i < n; ++i)
    if (!envs[i]) return fail(CHAN_EINVAL, "batch: null env");
  chan_batch* b = new (std::nothrow) chan_batch();
  if (!b) return CHAN_ENOMEM;
  b->stream = envs[0]->stream;
  b->device = envs[0]->device;
  for (int k = 0; k < KC_COUNT; ++k) {
    b->timing_ms[k] = 0.0;
    b->timing_launches[k] = 0;
  }
  // shapes first, each tuned on all of its channels together
  for (int i = 0; i < n; ++i) {
    if (envs[i]->device != b->device) {
      batch_free(b);
      return fail(CHAN_EINVAL, "batch: envs on different devices");
    }
    for (int k = 0; k < i; ++k)
      if (envs[k] == envs[i]) {
        batch_free(b);
        return fail(CHAN_EINVAL, "batch: env listed twice");
      }
    if (envs[i]->in_flight) {
      batch_free(b);
      return fail(CHAN_EBUSY, "batch: env has an unfinished call");
    }
    if (find_shape(b, envs[i]) < 0) {
      ShapeInfo info;
      info.d = envs[i]->d;
      info.pm = uses_pm(envs[i]);
      b->shapes.push_back(info);
    }
  }
  for (size_t sh = 0; sh < b->shapes.size(); ++sh) {
    std::vector<chan_env*> members;
    for (int i = 0; i < n; ++i)
      if (find_shape(b, envs[i]) == (int)sh) members.push_back(envs[i]);
    if ((size_t)b->shapes[sh].d.ny * members.size() > 65535) {
      batch_free(b);
      return fail(CHAN_EINVAL, "batch: too many channels of one shape (N_y x count > 65535)");
    }
    int rc = tune_plane(b, (int)sh, members);
    if (rc == CHAN_OK) rc = tune_column(b, (int)sh, members);
    if (rc != CHAN_OK) {
      batch_free(b);
      return rc;
    }
  }
  b->envs.assign(envs, envs + n);
  *out = b;
  return CHAN_OK;
}

// Plane-pass tiling of a shape, timed on the given channels' own buffers with every valid
// tiling; the fastest is kept.  The plane pass rewrites only its intermediates and H3 with the
// values the next plane pass writes anyway, and no tiling changes a result.  The channels must
// not be in an unfinished call.
int tune_plane(chan_batch* b, int shape, const std::vector<chan_env*>& members) {
  ShapeInfo& sh = b->shapes[shape];
  std::vector<PlaneTiles> cands;
  const int form = plane_form();
  if (form && (plane_tile_candidates(sh.d, &cands, form) || cands.empty())) cands.clear();
  if (cands.empty() && plane_tile_candidates(sh.d, &cands))
    return fail(CHAN_EINVAL, "no plane-pass tiling for this grid");
  sh.tiles = cands.back();
  if (cands.size() == 1) return CHAN_OK;
  chan_call c;
  c.b = b;
  c.stream = b->stream;
  c.envs = members;
  int rc = stage_call(&c, [&](int k) {
    return make_step_chan_env(members[k], dev_status(&c) + k, nullptr, 1, nullptr, nullptr, nullptr);
  });
  if (rc != CHAN_OK) {
    release_call(&c);
    return rc;
  }
  const CallGroup& g = c.groups[0];
  const int nm = (int)g.envs.size();
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t err = hipEventCreate(&e0);
  if (err == hipSuccess) err = hipEventCreate(&e1);
  // Every candidate is timed in each of ROUNDS sweeps over the list (reps back-to-back plane
  // passes after one warm-up) and keeps its best sweep, so that clock ramps and one-off
  // stalls do not decide the choice.  reps (4 to 64) makes a sweep last about 1 ms, from the
  // time of one pass with the last tiling: tilings a few per cent apart are not ranked on a
  // window of a hundred microseconds.
  constexpr int ROUNDS = 3;
  int reps = 4;
  if (err == hipSuccess && !launch_plane_pass(sh.d, g.d_plane, nm, cands.back(), c.stream, nullptr)) {
    float ms = 0.0f;
    err = hipEventRecord(e0, c.stream);
    if (err == hipSuccess && launch_plane_pass(sh.d, g.d_plane, nm, cands.back(), c.stream, nullptr))
      err = hipErrorLaunchFailure;
    if (err == hipSuccess) err = hipEventRecord(e1, c.stream);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    if (err == hipSuccess && ms > 0.0f) reps = std::min(64, std::max(4, (int)std::ceil(1.0f / ms)));
  }
  std::vector<float> best_ms(cands.size(), 0.0f);
  std::vector<char> ran(cands.size(), 0);
  for (int round = 0; round < ROUNDS && err == hipSuccess; ++round) {
    for (size_t k = 0; k < cands.size(); ++k) {
      const PlaneTiles& t = cands[k];
      if (launch_plane_pass(sh.d, g.d_plane, nm, t, c.stream, nullptr)) continue;  // warm-up
      err = hipEventRecord(e0, c.stream);
      for (int r = 0; r < reps && err == hipSuccess; ++r)
        if (launch_plane_pass(sh.d, g.d_plane, nm, t, c.stream, nullptr)) err = hipErrorLaunchFailure;
      if (err == hipSuccess) err = hipEventRecord(e1, c.stream);
      if (err == hipSuccess) err = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
      if (err != hipSuccess) break;
      if (!ran[k] || ms < best_ms[k]) best_ms[k] = ms;
      ran[k] = 1;
    }
  }
  bool have = false;
  float best = 0.0f;
  for (size_t k = 0; k < cands.size() && err == hipSuccess; ++k) {
    if (ran[k] && (!have || best_ms[k] < best)) {
      best = best_ms[k];
      sh.tiles = cands[k];
      have = true;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  const hipError_t sync = hipStreamSynchronize(c.stream);
  release_call(&c);
  if (err == hipSuccess) err = sync;
  if (err != hipSuccess) return fail(CHAN_EDEVICE, "plane-pass tiling", err);
  return have ? CHAN_OK : fail(CHAN_EDEVICE, "plane-pass tiling: no candidate ran", hipGetLastError());
}

// Columns per block of the batched column launch for a shape with several channels, timed with
// the launch the steps use most (solve and reconstruction of stage 0 in one launch) on shadow
// arguments: the channels' own H3 and tables, but a scratch copy of the state it writes at that
// stage (v, omega_y, the RK history, the mean profiles and the plane-pass input: the leading
// region of every env's block, up to Z6), so that no real buffer is written.  No block shape
// changes a result (each column's arithmetic is the same).  At most 1 GiB of scratch: a larger
// group is timed on its first channels.  A single channel keeps its own launch; without scratch
// memory the shape keeps 4.
int tune_column(chan_batch* b, int shape, const std::vector<chan_env*>& members) {
  ShapeInfo& sh = b->shapes[shape];
  if (!sh.pm || members.size() < 2) return CHAN_OK;
  static const int kCands[] = {4, 2};
  const size_t lead = (size_t)((char*)members[0]->s.Z6 - (char*)members[0]->s.vS);
  const int nm = (int)std::min(members.size(), std::max<size_t>(2, ((size_t)1 << 30) / lead));
  char* scratch = nullptr;
  ColChan* d_shadow = nullptr;
  if (hipMalloc((void**)&scratch, lead * nm) != hipSuccess) {
    (void)hipGetLastError();
    return CHAN_OK;
  }
  if (hipMalloc((void**)&d_shadow, nm * sizeof(ColChan)) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(scratch);
    return CHAN_OK;
  }
  std::vector<ColChan> h(nm);
  const hipStream_t st = b->stream;
  hipError_t err = hipSuccess;
  for (int k = 0; k < nm && err == hipSuccess; ++k) {
    const chan_env* e = members[k];
    char* base = scratch + (size_t)k * lead;
    auto relo = [&](const void* ptr) { return base + ((const char*)ptr - (const char*)e->s.vS); };
    h[k] = e->col;
    h[k].vS = (decltype(h[k].vS))(relo(e->s.vS));
    h[k].oS = (decltype(h[k].oS))(relo(e->s.oS));
    h[k].hist = (decltype(h[k].hist))(relo(e->s.hist));
    h[k].meanS = (decltype(h[k].meanS))(relo(e->s.meanS));
    h[k].meanH = (decltype(h[k].meanH))(relo(e->s.meanH));
    h[k].F6 = (decltype(h[k].F6))(relo(e->s.F6));
    err = hipMemcpyAsync(base, e->s.vS, lead, hipMemcpyDeviceToDevice, st);
  }
  if (err == hipSuccess) err = hipMemcpyAsync(d_shadow, h.data(), nm * sizeof(ColChan), hipMemcpyHostToDevice, st);
  if (err == hipSuccess) err = hipStreamSynchronize(st);
  const ColStage S = {0, 0, 1};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (err == hipSuccess) err = hipEventCreate(&e0);
  if (err == hipSuccess) err = hipEventCreate(&e1);
  // as for the plane tiling: ROUNDS sweeps of REPS launches after a warm-up, best sweep kept
  constexpr int REPS = 4, ROUNDS = 3;
  float best_ms[2] = {0.0f, 0.0f};
  bool ran[2] = {false, false};
  for (int round = 0; round < ROUNDS && err == hipSuccess; ++round) {
    for (int k = 0; k < 2 && err == hipSuccess; ++k) {
      if (launch_column_pm(sh.d, d_shadow, nullptr, nm, S, true, true, st, nullptr, kCands[k])) {
        err = hipErrorLaunchFailure;
        break;
      }
      err = hipEventRecord(e0, st);
      for (int r = 0; r < REPS && err == hipSuccess; ++r)
        if (launch_column_pm(sh.d, d_shadow, nullptr, nm, S, true, true, st, nullptr, kCands[k]))
          err = hipErrorLaunchFailure;
      if (err == hipSuccess) err = hipEventRecord(e1, st);
      if (err == hipSuccess) err = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
      if (err != hipSuccess) break;
      if (!ran[k] || ms < best_ms[k]) best_ms[k] = ms;
      ran[k] = true;
    }
  }
  if (err == hipSuccess && ran[0] && ran[1]) sh.col_cw = best_ms[1] < best_ms[0] ? kCands[1] : kCands[0];
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  const hipError_t sync = hipStreamSynchronize(st);
  (void)hipFree(d_shadow);
  (void)hipFree(scratch);
  if (err == hipSuccess) err = sync;
  if (err != hipSuccess) return fail(CHAN_EDEVICE, "column block tuning", err);
  return CHAN_OK;
}

// Named host ranges (roctx) around the launches of each env step and RK3 stage, so that a marker
// trace (rocprofv3 --marker-trace) shows where the host queued them.  The roctx library is
// opened at first use; without it the ranges are no-ops.
struct Roctx {
  int (*push)(const char*) = nullptr;
  int (*pop)() = nullptr;
  Roctx() {
    void* h = dlopen("librocprofiler-sdk-roctx.so.1", RTLD_NOW | RTLD_LOCAL);
    if (!h) return;
    push = reinterpret_cast<int (*)(const char*)>(dlsym(h, "roctxRangePushA"));
    pop = reinterpret_cast<int (*)()>(dlsym(h, "roctxRangePop"));
    if (!push || !pop) push = nullptr, pop = nullptr;
  }
};

const Roctx& roctx() {
  static const Roctx r;
  return r;
}

struct RoctxRange {
  const bool on;
  explicit RoctxRange(const char* msg) : on(roctx().push != nullptr) {
    if (on) roctx().push(msg);
  }
  ~RoctxRange() {
    if (on) roctx().pop();
  }
  RoctxRange(const RoctxRange&) = delete;
  RoctxRange& operator=(const RoctxRange&) = delete;
};

// Queues the launches of one env step of the call's envs (already staged), then the status
// read-back and (record_done) the completion event.
int launch_step(chan_call* c, bool any_action, KernelTimer* tm, double* const* obs, bool record_done = true) {
  chan_batch* b = c->b;
  hipStream_t st = c->stream;
  const int na = (int)c->envs.size();
  const int n_substeps = c->n_sub;
  StepChan* ds = dev_step(c);
  const RoctxRange step_range(record_done ? "chan env step" : "chan env step (captured)");
  if (launch_begin_step(ds, na, st, tm)) return fail(CHAN_EDEVICE, "launch begin_step", hipGetLastError());
  if (any_action && launch_ingest(ds, na, c->max_nx, c->max_nz, c->max_nkx, st, tm))
    return fail(CHAN_EDEVICE, "launch ingest", hipGetLastError());
  for (int m = 0; m < n_substeps; ++m) {
    for (int r = 0; r < 3; ++r) {
      // The last stage of the env step leaves its reconstruction to the reconstruction
      // below, which also serves set_state (bitwise-identical resume).
      const bool last = (m == n_substeps - 1) && (r == 2);
      const ColStage S = {r, m, n_substeps};
      static const char* const kStageName[3] = {"RK3 stage 1", "RK3 stage 2", "RK3 stage 3"};
      const RoctxRange stage_range(kStageName[r]);
      for (const CallGroup& g : c->groups) {
        const ShapeInfo& sh = b->shapes[g.shape];
        if (launch_plane_pass(sh.d, g.d_plane, (int)g.envs.size(), sh.tiles, st, tm))
          return fail(CHAN_EDEVICE, "launch plane pass", hipGetLastError());
        if (group_column(b, g, st, S, true, !last, tm)) return fail(CHAN_EDEVICE, "launch column pass", hipGetLastError());
      }
    }
  }
  const ColStage S_end = {-1, 0, n_substeps};
  for (const CallGroup& g : c->groups)
    if (group_column(b, g, st, S_end, false, true, tm)) return fail(CHAN_EDEVICE, "launch column pass", hipGetLastError());
  // pressure observed: the end-of-step state's non-linear term (a plane pass; the next step's
  // first stage recomputes the same H), then the Poisson solve per pair, before finish_step
  // replaces the old wall velocity (its rate enters the wall condition)
  int max_planes = 1;
  bool any_pressure = false;
  for (int k = 0; k < na; ++k) {
    const chan_env* e = c->envs[k];
    max_planes = std::max(max_planes, e->n_planes);
    any_pressure = any_pressure || (obs != nullptr && obs[k] != nullptr && (e->opts.obs_mask & CHAN_OBS_P));
  }
  if (any_pressure)
    for (const CallGroup& g : c->groups) {
      const ShapeInfo& sh = b->shapes[g.shape];
      bool has = false;
      for (size_t k = 0; k < g.envs.size(); ++k) has = has || g.h_col[k].n_pplanes > 0;
      if (!has) continue;
      if (launch_plane_pass(sh.d, g.d_plane, (int)g.envs.size(), sh.tiles, st, tm))
        return fail(CHAN_EDEVICE, "launch plane pass (pressure)", hipGetLastError());
      if (sh.pm) {
        if (launch_pressure_pm(sh.d, g.d_col, (int)g.envs.size(), S_end, st, tm))
          return fail(CHAN_EDEVICE, "launch pressure", hipGetLastError());
      } else {
        for (const chan_env* e : g.envs) {
          if (e->col.n_pplanes == 0) continue;
          const bool ramp = e->opts.controller == CHAN_CTRL_EXTERNAL && e->opts.action_mode == CHAN_RAMP;
          if (launch_pressure_generic(e->d, e->s, e->ph, e->n_planes, e->js_planes, ramp, n_substeps, st, tm))
            return fail(CHAN_EDEVICE, "launch pressure", hipGetLastError());
        }
      }
    }
  if (launch_finish_step(ds, na, st, tm)) return fail(CHAN_EDEVICE, "launch finish_step", hipGetLastError());
  const int nslots = any_pressure ? 1 + SLOTS_PER_PLANE * max_planes : SLOTS_PER_PLANE * max_planes - 3;
  if (launch_outputs(ds, na, c->max_nx, c->max_nz, c->max_nkx, nslots, st, tm))
    return fail(CHAN_EDEVICE, "launch outputs", hipGetLastError());
  if (any_pressure && launch_pressure_finish(ds, na, st, tm))
    return fail(CHAN_EDEVICE, "launch pressure finish", hipGetLastError());
  HIPCHECK(hipMemcpyAsync(host_status(c), dev_status(c), na * sizeof(int), hipMemcpyDeviceToHost, st));
  if (record_done) HIPCHECK(hipEventRecord(c->slot->done, st));
  return CHAN_OK;
}

// The envs of a call: members of b, each listed once, none held by an unfinished call.
int check_call_envs(const chan_batch* b, int32_t na, chan_env* const* envs) {
  if (na < 1 || na > (int32_t)b->envs.size() || !envs) return fail(CHAN_EINVAL, "batch step: bad number of envs");
  for (int k = 0; k < na; ++k) {
    if (!envs[k] || find_member(b, envs[k]) < 0) return fail(CHAN_EINVAL, "batch step: env not in the batch");
    if (envs[k]->in_flight) return fail(CHAN_EBUSY, "batch step: env has an unfinished call");
    for (int j = 0; j < k; ++j)
      if (envs[j] == envs[k]) return fail(CHAN_EINVAL, "batch step: env listed twice");
  }
  return CHAN_OK;
}

// Validates and queues one env step of envs[0..na) on stream st; on success *out holds the call
// (every env marked as held by it).
int batch_launch(chan_batch* b, hipStream_t st, int32_t na, chan_env* const* envs, const double* const* actions,
                 int32_t n_substeps, double* const* obs, double* const* tau_w, double* const* drag, chan_call** out) {
  if (n_substeps < 1) return fail(CHAN_EINVAL, "n_substeps < 1");
  const int rc0 = check_call_envs(b, na, envs);
  if (rc0 != CHAN_OK) return rc0;
  int n_ready = 0;
  for (int k = 0; k < na; ++k) n_ready += (envs[k]->have_flow && !envs[k]->poisoned) ? 1 : 0;
  if (n_ready == 0) return fail(CHAN_ESTATE, "no env with a valid flow state");
  chan_call* c = new (std::nothrow) chan_call();
  if (!c) return CHAN_ENOMEM;
  c->b = b;
  c->stream = st;
  c->n_sub = n_substeps;
  c->envs.assign(envs, envs + na);
  bool any_action = false;
  int rc = stage_call(c, [&](int k) {
    StepChan s = make_step_chan_env(c->envs[k], dev_status(c) + k, actions ? actions[k] : nullptr, n_substeps,
                                    obs ? obs[k] : nullptr, tau_w ? tau_w[k] : nullptr, drag ? drag[k] : nullptr);
    any_action = any_action || (s.action != nullptr && !s.skip);
    return s;
  });
  if (rc == CHAN_OK) rc = launch_step(c, any_action, b->timer.on ? &b->timer : nullptr, obs);
  if (rc != CHAN_OK) {
    (void)hipStreamSynchronize(st);
    release_call(c);
    delete c;
    return rc;
  }
  for (chan_env* e : c->envs) e->in_flight = c;
  b->calls.push_back(c);
  *out = c;
  return CHAN_OK;
}

// Waits for the call, applies each env's outcome (clock, step counter, poisoning), writes the
// result codes, frees the call.  Returns CHAN_OK if every env succeeded, else the first
// failing env's code.
int batch_finish(chan_call* c, int32_t* results) {
  const hipError_t err = hipEventSynchronize(c->slot->done);
  int rc = CHAN_OK;
  if (err != hipSuccess) {
    rc = fail(CHAN_EDEVICE, "hipEventSynchronize", err);
  } else {
    const StepChan* hs = host_step(c);
    const int* status = host_status(c);
    for (size_t k = 0; k < c->envs.size(); ++k) {
      chan_env* e = c->envs[k];
      int ri = CHAN_OK;
      if (!e) {  // destroyed while the call was in flight
        ri = CHAN_EINVAL;
        if (rc == CHAN_OK) fail(CHAN_EINVAL, "env destroyed before its call was finished");
      } else if (hs[k].skip) {
        ri = CHAN_ESTATE;
        if (rc == CHAN_OK) fail(CHAN_ESTATE, "env without a valid flow state (skipped)");
      } else if (status[k] & STATUS_BAD_ACTION) {
        ri = CHAN_ENONFINITE;
        if (rc == CHAN_OK) fail(CHAN_ENONFINITE, "non-finite action");
      } else {
        e->t += c->n_sub * e->ph.dt;
        e->nstep += c->n_sub;
        if (status[k] & STATUS_NONFINITE) {
          e->poisoned = true;
          ri = CHAN_ENONFINITE;
          if (rc == CHAN_OK) fail(CHAN_ENONFINITE, "non-finite state after the step");
        }
      }
      if (results) results[k] = ri;
      if (rc == CHAN_OK) rc = ri;
    }
  }
  erase_value(c->b->calls, c);
  release_call(c);
  delete c;
  return rc;
}

void graph_free(chan_graph* g) {
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  free_slot(g->slot);
  delete g;
}

// Captures one env step of envs[0..na) with these buffers: stages the launch arguments into the
// graph's own slot on a private stream, waits for them, then records the step's launches on that
// stream.  Every env must have a valid flow state (a replay steps all of them).
int batch_capture(chan_batch* b, int32_t na, chan_env* const* envs, const double* const* actions,
                  int32_t n_substeps, double* const* obs, double* const* tau_w, double* const* drag,
                  chan_graph** out) {
  if (n_substeps < 1) return fail(CHAN_EINVAL, "n_substeps < 1");
  const int rc0 = check_call_envs(b, na, envs);
  if (rc0 != CHAN_OK) return rc0;
  for (int k = 0; k < na; ++k)
    if (!envs[k]->have_flow || envs[k]->poisoned) return fail(CHAN_ESTATE, "capture: env without a valid flow state");
  chan_graph* g = new (std::nothrow) chan_graph();
  if (!g) return CHAN_ENOMEM;
  g->b = b;
  g->envs.assign(envs, envs + na);
  g->n_sub = n_substeps;
  g->slot = new (std::nothrow) CallSlot();
  if (!g->slot) {
    delete g;
    return CHAN_ENOMEM;
  }
  if (hipEventCreateWithFlags(&g->slot->done, hipEventDisableTiming) != hipSuccess) {
    g->slot->done = nullptr;
    graph_free(g);
    return fail(CHAN_EDEVICE, "hipEventCreateWithFlags");
  }
  if (!size_slot(g->slot, na)) {
    graph_free(g);
    return fail(CHAN_ENOMEM, "capture staging buffers");
  }
  hipStream_t cs = nullptr;
  hipError_t err = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (err != hipSuccess) {
    graph_free(g);
    return fail(CHAN_EDEVICE, "hipStreamCreateWithFlags", err);
  }
  chan_call c;
  c.b = b;
  c.stream = cs;
  c.slot = g->slot;
  c.envs = g->envs;
  c.n_sub = n_substeps;
  bool any_action = false;
  int rc = stage_call(&c, [&](int k) {
    StepChan s = make_step_chan_env(c.envs[k], dev_status(&c) + k, actions ? actions[k] : nullptr, n_substeps,
                                    obs ? obs[k] : nullptr, tau_w ? tau_w[k] : nullptr, drag ? drag[k] : nullptr);
    any_action = any_action || (s.action != nullptr && !s.skip);
    return s;
  });
  if (rc == CHAN_OK && (err = hipStreamSynchronize(cs)) != hipSuccess) rc = fail(CHAN_EDEVICE, "hipStreamSynchronize", err);
  if (rc == CHAN_OK) {
    err = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (err != hipSuccess) {
      rc = fail(CHAN_EDEVICE, "hipStreamBeginCapture", err);
    } else {
      rc = launch_step(&c, any_action, nullptr, obs, false);
      hipGraph_t graph = nullptr;
      err = hipStreamEndCapture(cs, &graph);
      g->graph = graph;
      if (rc == CHAN_OK && err != hipSuccess) rc = fail(CHAN_EDEVICE, "hipStreamEndCapture", err);
      if (rc == CHAN_OK && (err = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0)) != hipSuccess)
        rc = fail(CHAN_EDEVICE, "hipGraphInstantiate", err);
    }
  }
  (void)hipStreamDestroy(cs);
  if (rc != CHAN_OK) {
    graph_free(g);
    return rc;
  }
  b->graphs.push_back(g);
  *out = g;
  return CHAN_OK;
}

// Replays a captured step on stream st; *out: the call (finished by batch_finish).
int graph_launch(chan_graph* g, hipStream_t st, chan_call** out) {
  if (!g->b) return fail(CHAN_ESTATE, "graph: its batch was destroyed");
  if (g->stale) return fail(CHAN_ESTATE, "graph: an env left the batch or was destroyed after the capture");
  if (g->slot->busy) return fail(CHAN_EBUSY, "graph: its previous replay is unfinished");
  for (chan_env* e : g->envs) {
    if (e->in_flight) return fail(CHAN_EBUSY, "graph: env has an unfinished call");
    if (!e->have_flow || e->poisoned) return fail(CHAN_ESTATE, "graph: env without a valid flow state");
  }
  chan_call* c = new (std::nothrow) chan_call();
  if (!c) return CHAN_ENOMEM;
  c->b = g->b;
  c->slot = g->slot;
  c->stream = st;
  c->envs = g->envs;
  c->n_sub = g->n_sub;
  hipError_t err = hipGraphLaunch(g->exec, st);
  if (err == hipSuccess) err = hipEventRecord(g->slot->done, st);
  if (err != hipSuccess) {
    (void)hipStreamSynchronize(st);
    delete c;
    return fail(CHAN_EDEVICE, "hipGraphLaunch", err);
  }
  g->slot->busy = true;
  for (chan_env* e : c->envs) e->in_flight = c;
  g->b->calls.push_back(c);
  *out = c;
  return CHAN_OK;
}

// Finishes the graph's replay in flight (if any), then frees it.
void graph_destroy(chan_graph* g) {
  if (g->b) {
    for (chan_call* c : std::vector<chan_call*>(g->b->calls))
      if (c->slot == g->slot) (void)batch_finish(c, nullptr);
    erase_value(g->b->graphs, g);
  }
  graph_free(g);
}

// Graphs of b that step env e can no longer be replayed (e left b or is being destroyed).
void stale_graphs(chan_batch* b, const chan_env* e) {
  for (chan_graph* g : b->graphs)
    for (const chan_env* x : g->envs)
      if (x == e) g->stale = true;
}

// Synchronous env step of the batch's envs idx[0..na) (idx null: the first na) on the batch's
// stream.
int batch_step(chan_batch* b, int32_t na, const int32_t* idx, const double* const* actions, int32_t n_substeps,
               double* const* obs, double* const* tau_w, double* const* drag, int32_t* results) {
  const int n = (int)b->envs.size();
  if (na < 1 || na > n) return fail(CHAN_EINVAL, "batch step: bad number of envs");
  std::vector<chan_env*> envs(na);
  for (int k = 0; k < na; ++k) {
    const int i = idx ? idx[k] : k;
    if (i < 0 || i >= n) return fail(CHAN_EINVAL, "batch step: env index out of range or repeated");
    envs[k] = b->envs[i];
  }
  g_last_error.clear();
  chan_call* c = nullptr;
  const int rc = batch_launch(b, b->stream, na, envs.data(), actions, n_substeps, obs, tau_w, drag, &c);
  if (rc != CHAN_OK) {
    if (rc == CHAN_EINVAL && g_last_error == "batch step: env listed twice")
      g_last_error = "batch step: env index out of range or repeated";
    return rc;
  }
  return batch_finish(c, results);
}

// Plane-pass input, opposition target and wall shear from the stored state of env e (after
// reset or set_state), on its own batch of one.
int batch_prime(chan_batch* b) {
  chan_call c;
  c.b = b;
  c.stream = b->stream;
  c.envs = b->envs;
  int rc = stage_call(&c, [&](int k) {
    StepChan s = make_step_chan_env(c.envs[k], dev_status(&c) + k, nullptr, 1, nullptr, nullptr, nullptr);
    s.zero_vw = 0;
    s.skip = 0;
    return s;
  });
  if (rc == CHAN_OK && launch_begin_step(dev_step(&c), (int)c.envs.size(), c.stream, nullptr))
    rc = fail(CHAN_EDEVICE, "launch begin_step", hipGetLastError());
  const ColStage S = {-1, 0, 1};
  for (size_t k = 0; k < c.groups.size() && rc == CHAN_OK; ++k)
    if (group_column(b, c.groups[k], c.stream, S, false, true, nullptr))
      rc = fail(CHAN_EDEVICE, "launch column pass", hipGetLastError());
  const hipError_t err = hipStreamSynchronize(c.stream);
  release_call(&c);
  if (rc != CHAN_OK) return rc;
  if (err != hipSuccess) return fail(CHAN_EDEVICE, "hipStreamSynchronize", err);
  return CHAN_OK;
}

int batch_drain_timer(chan_batch* b) {
  KernelTimer& t = b->timer;
  if (t.used == 0) return CHAN_OK;
  HIPCHECK(hipDeviceSynchronize());
  for (size_t k = 0; k < t.used; ++k) {
    float ms = 0.0f;
    HIPCHECK(hipEventElapsedTime(&ms, t.pool[2 * k], t.pool[2 * k + 1]));
    b->timing_ms[t.cls[k]] += ms;
    b->timing_launches[t.cls[k]] += 1;
  }
  t.used = 0;
  return CHAN_OK;
}

int batch_set_timing(chan_batch* b, int32_t enable) {
  const int rc = batch_drain_timer(b);
  if (rc != CHAN_OK) return rc;
  for (int k = 0; k < KC_COUNT; ++k) {
    b->timing_ms[k] = 0.0;
    b->timing_launches[k] = 0;
  }
  b->timer.on = enable != 0;
  return CHAN_OK;
}

int batch_timing_read(chan_batch* b, int32_t nclass, int64_t* launches, double* ms) {
  if (nclass < 0 || (nclass > 0 && (!launches || !ms))) return CHAN_EINVAL;
  const int rc = batch_drain_timer(b);
  if (rc != CHAN_OK) return rc;
  for (int k = 0; k < nclass && k < KC_COUNT; ++k) {
    launches[k] = b->timing_launches[k];
    ms[k] = b->timing_ms[k];
  }
  return KC_COUNT;
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
  return batch_prime(e->self);
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
    case CHAN_EBUSY: return "env held by an unfinished asynchronous call";
    default: return "unknown error";
  }
}

size_t chan_env_footprint_bytes(const chan_grid_t* grid, const chan_opts_t* opts) {
  chan_opts_t o;
  if (opts) o = *opts; else chan_opts_default(&o);
  if (!valid_grid(grid) || !valid_opts(&o)) return 0;
  const Dims d = make_dims(grid);
  // the same checks as chan_env_create: a grid it would refuse has no footprint
  const PhysParams ph = make_phys(grid, &o);
  if (!(ph.nu > 0) || !(ph.dt > 0)) return 0;
  double ypn = 0.0;
  const int js = sensing_node(d, ph, grid->obs_y_plus, &ypn);
  if (js < 0 || js >= d.N) return 0;
  for (int k = 0; k < o.n_extra_planes; ++k) {
    const int jk = sensing_node(d, ph, o.extra_obs_y_plus[k], &ypn);
    if (jk < 0 || jk >= d.N) return 0;
  }
  return buffer_sizes(d, table_doubles(d, ph.open)).total;
}

int chan_env_create(const chan_grid_t* grid, const chan_opts_t* opts, void* hip_stream, chan_env** out) {
  g_last_error.clear();
  if (!out) return fail(CHAN_EINVAL, "out");
  chan_env setup;
  int rc = setup_env(grid, opts, hip_stream, &setup);
  if (rc != CHAN_OK) return rc;
  const Dims d = setup.d;
  const PhysParams ph = setup.ph;
  HostTables ht;
  rc = host_tables(d, ph, &ht);
  if (rc != CHAN_OK) return rc;

  chan_env* e = new (std::nothrow) chan_env(setup);
  if (!e) return CHAN_ENOMEM;
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
  DeviceState& s = e->s;
  carve_state(d, z, ht.L, (char*)e->dev_block, &s);
  e->col = make_col_chan(e);
  e->plane = make_plane_chan(e);
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
  {
    chan_env* one[1] = {e};
    const int rc = batch_build(one, 1, &e->self);
    if (rc != CHAN_OK) {
      const std::string why = g_last_error;
      chan_env_destroy(e);
      g_last_error = why;
      return rc;
    }
  }
  *out = e;
  return CHAN_OK;
}

void chan_env_destroy(chan_env* e) {
  if (!e) return;
  if (chan_call* c = e->in_flight) {  // wait for its call, then leave it (finishing it reports CHAN_EINVAL here)
    if (c->slot) (void)hipEventSynchronize(c->slot->done);
    for (chan_env*& x : c->envs)
      if (x == e) x = nullptr;
    e->in_flight = nullptr;
  }
  for (chan_batch* b : e->member_of) {
    erase_value(b->envs, e);
    stale_graphs(b, e);
  }
  e->member_of.clear();
  if (e->stream) (void)hipStreamSynchronize(e->stream);
  batch_free(e->self);
  if (e->dev_block) (void)hipFree(e->dev_block);
  if (e->host_status) (void)hipHostFree(e->host_status);
  delete e;
}

int chan_env_reset(chan_env* e, uint64_t seed) {
  if (!e) return CHAN_EINVAL;
  if (e->in_flight) return fail(CHAN_EBUSY, "env held by an unfinished call");
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
  if (e->in_flight) return fail(CHAN_EBUSY, "env held by an unfinished call");
  const Dims& d = e->d;
  const size_t n = (size_t)4 * d.nz * d.nkx * d.ny + 2 * (size_t)d.ny + 2 * (size_t)d.nz * d.nkx + 2;
  if (n_doubles != n) return CHAN_EINVAL;
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(host[i])) return CHAN_ENONFINITE;
  return upload_state(e, host);
}

int chan_env_get_state(const chan_env* e, double* host, size_t n_doubles) {
  if (!e || !host) return CHAN_EINVAL;
  if (e->in_flight) return fail(CHAN_EBUSY, "env held by an unfinished call");
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
  out->obs_doubles = (size_t)e->n_planes * __builtin_popcount(e->opts.obs_mask) * d.nz * d.nx;
  out->n_planes = e->n_planes;
  for (int k = 0; k < MAX_PLANES; ++k) {
    out->js_planes[k] = e->js_planes[k];
    out->y_plus_planes[k] = e->y_plus_planes[k];
  }
  out->footprint_bytes = e->dev_bytes;
  return CHAN_OK;
}

int chan_env_step(chan_env* e, const double* action, int32_t n_substeps, double* obs, double* tau_w,
                  double* drag) {
  if (!e) return CHAN_EINVAL;
  if (e->in_flight) return fail(CHAN_EBUSY, "env held by an unfinished call");
  return batch_step(e->self, 1, nullptr, &action, n_substeps, &obs, &tau_w, &drag, nullptr);
}

int chan_batch_create(int32_t n, chan_env* const* envs, chan_batch** out) {
  g_last_error.clear();
  if (!out) return CHAN_EINVAL;
  *out = nullptr;
  const int rc = batch_build(envs, n, out);
  if (rc == CHAN_OK)
    for (chan_env* e : (*out)->envs) e->member_of.push_back(*out);
  return rc;
}

int chan_batch_step(chan_batch* b, const double* const* actions, int32_t n_substeps, double* const* obs,
                    double* const* tau_w, double* const* drag, int32_t* results) {
  if (!b) return CHAN_EINVAL;
  return batch_step(b, (int32_t)b->envs.size(), nullptr, actions, n_substeps, obs, tau_w, drag, results);
}

int chan_batch_step_subset(chan_batch* b, int32_t n, const int32_t* idx, const double* const* actions,
                           int32_t n_substeps, double* const* obs, double* const* tau_w, double* const* drag,
                           int32_t* results) {
  if (!b || !idx) return CHAN_EINVAL;
  return batch_step(b, n, idx, actions, n_substeps, obs, tau_w, drag, results);
}

int chan_batch_launch(chan_batch* b, void* hip_stream, int32_t n, chan_env* const* envs,
                      const double* const* actions, int32_t n_substeps, double* const* obs, double* const* tau_w,
                      double* const* drag, chan_call** out) {
  g_last_error.clear();
  if (out) *out = nullptr;
  if (!b || !out) return CHAN_EINVAL;
  return batch_launch(b, (hipStream_t)hip_stream, n, envs, actions, n_substeps, obs, tau_w, drag, out);
}

int chan_call_query(const chan_call* c) {
  if (!c || !c->slot) return CHAN_EINVAL;
  const hipError_t err = hipEventQuery(c->slot->done);
  if (err == hipSuccess) return 0;
  if (err == hipErrorNotReady) return 1;
  return fail(CHAN_EDEVICE, "hipEventQuery", err);
}

int chan_call_finish(chan_call* c, int32_t* results) {
  if (!c || !c->slot) return CHAN_EINVAL;
  g_last_error.clear();
  return batch_finish(c, results);
}

int chan_batch_add(chan_batch* b, chan_env* env) {
  if (!b) return CHAN_EINVAL;
  g_last_error.clear();
  const int rc = batch_add(b, env);
  if (rc == CHAN_OK) env->member_of.push_back(b);
  return rc;
}

int chan_batch_remove(chan_batch* b, chan_env* env) {
  if (!b || !env) return CHAN_EINVAL;
  const int k = find_member(b, env);
  if (k < 0) return fail(CHAN_EINVAL, "batch: env not in the batch");
  if (env->in_flight) return fail(CHAN_EBUSY, "batch: env held by an unfinished call");
  b->envs.erase(b->envs.begin() + k);
  erase_value(env->member_of, b);
  stale_graphs(b, env);
  return CHAN_OK;
}

int chan_batch_capture(chan_batch* b, int32_t n, chan_env* const* envs, const double* const* actions,
                       int32_t n_substeps, double* const* obs, double* const* tau_w, double* const* drag,
                       chan_graph** out) {
  g_last_error.clear();
  if (out) *out = nullptr;
  if (!b || !out) return CHAN_EINVAL;
  return batch_capture(b, n, envs, actions, n_substeps, obs, tau_w, drag, out);
}

int chan_env_capture(chan_env* e, const double* action, int32_t n_substeps, double* obs, double* tau_w,
                     double* drag, chan_graph** out) {
  g_last_error.clear();
  if (out) *out = nullptr;
  if (!e || !out) return CHAN_EINVAL;
  return batch_capture(e->self, 1, &e, &action, n_substeps, &obs, &tau_w, &drag, out);
}

int chan_graph_launch(chan_graph* g, void* hip_stream, chan_call** out) {
  g_last_error.clear();
  if (out) *out = nullptr;
  if (!g || !out) return CHAN_EINVAL;
  return graph_launch(g, (hipStream_t)hip_stream, out);
}

void chan_graph_destroy(chan_graph* g) {
  if (g) graph_destroy(g);
}

void chan_batch_destroy(chan_batch* b) { batch_free(b); }

int32_t chan_batch_size(const chan_batch* b) { return b ? (int32_t)b->envs.size() : 0; }

int chan_batch_tuning(const chan_batch* b, int32_t max_shapes, int32_t* out) {
  if (!b || (max_shapes > 0 && !out)) return CHAN_EINVAL;
  const int n = (int)b->shapes.size();
  for (int k = 0; k < n && k < max_shapes; ++k) {
    const ShapeInfo& sh = b->shapes[k];
    int32_t* r = out + 7 * k;
    r[0] = sh.d.nx;
    r[1] = sh.d.ny;
    r[2] = sh.d.nz;
    r[3] = sh.tiles.PB;
    r[4] = sh.tiles.P;
    r[5] = sh.pm ? sh.col_cw : 0;
    r[6] = sh.tiles.fused;
  }
  return n;
}

int chan_batch_set_timing(chan_batch* b, int32_t enable) {
  if (!b) return CHAN_EINVAL;
  return batch_set_timing(b, enable);
}

int chan_batch_timing_read(chan_batch* b, int32_t nclass, int64_t* launches, double* ms) {
  if (!b) return CHAN_EINVAL;
  return batch_timing_read(b, nclass, launches, ms);
}

static const char* const kClassNames[KC_COUNT] = {
    "column_pass", "z_inverse_fft", "x_rows_fft_product", "z_forward_fft", "action_ingest", "outputs",
    "bookkeeping", "column_reconstruct", "column_solve_reconstruct"};

const char* chan_kernel_class_name(int32_t cls) {
  if (cls < 0 || cls >= KC_COUNT) return "";
  return kClassNames[cls];
}

int chan_env_set_timing(chan_env* e, int32_t enable) {
  if (!e) return CHAN_EINVAL;
  return batch_set_timing(e->self, enable);
}

int chan_env_timing_read(chan_env* e, int32_t nclass, int64_t* launches, double* ms) {
  if (!e) return CHAN_EINVAL;
  return batch_timing_read(e->self, nclass, launches, ms);
}

}  // extern "C"

// ---------------------------------------------------------------------------------------------
// chan_step_static: one env step of a caller-owned flow state without any allocation.  The
// operator tables, every work buffer and the launch arguments live in `scratch`, a file-scope
// device array (one copy per device, held until the process ends).  Host code never passes the
// array's name to a kernel or a copy: it uses the address from hipGetSymbolAddress, taken once
// per device on that device's first call and kept in static_slot[device].
// ---------------------------------------------------------------------------------------------
namespace {

constexpr size_t STATIC_SCRATCH_BYTES = (size_t)32 << 20;
constexpr size_t STATIC_ARGS_BYTES = 4096;   // front of the scratch: launch arguments, status words
constexpr size_t ARG_PRIME = 0, ARG_STEP = 1024, ARG_COL = 2048, ARG_PLANE = 3072, ARG_STATUS = 3840, ARG_INSTATUS = 3844;
static_assert(sizeof(StepChan) <= 1024 && sizeof(ColChan) <= 1024 && sizeof(PlaneChan) <= 768, "argument slots");
constexpr int MAX_STATIC_DEVICES = 64;

}  // namespace

static __device__ __align__(256) char scratch[STATIC_SCRATCH_BYTES];

namespace {

// What the scratch of one device holds: its address, and which configuration's tables.
struct StaticSlot {
  std::mutex lock;              // calls on one device are serialised
  char* ptr = nullptr;          // hipGetSymbolAddress(scratch) on this device
  bool have_tables = false;
  int nx = 0, ny = 0, nz = 0;
  PhysParams ph;
  TableLayout L;
  PlaneTiles tiles = {0, 0, 0};
};
StaticSlot static_slot[MAX_STATIC_DEVICES];

bool same_tables(const StaticSlot& s, const Dims& d, const PhysParams& p) {
  const PhysParams& q = s.ph;
  return s.have_tables && s.nx == d.nx && s.ny == d.ny && s.nz == d.nz && q.nu == p.nu && q.dt == p.dt &&
         q.ub == p.ub && q.forcing == p.forcing && q.px == p.px && q.lx == p.lx && q.lz == p.lz && q.open == p.open &&
         q.ys == p.ys;
}

// Launch arguments into the scratch (by value through the kernel arguments: no host copy).
__global__ void k_static_args(StepChan prime, StepChan step, ColChan col, PlaneChan plane, StepChan* d_prime,
                              StepChan* d_step, ColChan* d_col, PlaneChan* d_plane, int* in_status) {
  if (threadIdx.x == 0) {
    *d_prime = prime;
    *d_step = step;
    *d_col = col;
    *d_plane = plane;
    *in_status = 0;
  }
}

__global__ void k_static_zero(double* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0.0;
}

// The caller's state, exchange layout [q][p][n] (v, omega_y) | U | W | v_w,old [q][p] | t | step,
// into the device layout [p][q][n], with the canonical form chan_env_set_state gives it: zero
// (0, 0) pair of v and omega_y, zero Nyquist row, p = 0 column Hermitian (the q > 0 half kept).
// Any non-finite entry sets *in_status.
struct StaticIO {
  int nz, nkx, ny;
  gptr<double> flat;
  gptr<cplx> vS, oS, vw_old, vw_new;
  gptr<double> meanS;
  gptr<int> in_status;
  gptr<const int> status;
  double t_inc, n_inc;
};

__device__ __forceinline__ int canon_src_q(int p, int q, int nz) {
  // -1: the entry is zero; otherwise the source row (a negative value marks a conjugate)
  if (q == nz / 2 || (p == 0 && q == 0)) return -1;
  if (p == 0 && q > nz / 2) return -(nz - q) - 2;
  return q;
}

__global__ void k_state_in(StaticIO A) {
  const int nz = A.nz, nkx = A.nkx, NY = A.ny;
  const size_t nspec = (size_t)nz * nkx * NY;  // complex entries per field
  const size_t nvw = (size_t)nz * nkx;
  const size_t total = 2 * nspec + NY + nvw;
  bool bad = false;
  const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x, nthr = (size_t)gridDim.x * blockDim.x;
  for (size_t i = tid; i < total; i += nthr) {
    if (i < 2 * nspec) {
      const int f = i >= nspec;
      const size_t j = i - f * nspec;        // destination [p][q][n]
      const int n = (int)(j % NY);
      const int pq = (int)(j / NY), p = pq / nz, q = pq - p * nz;
      const gptr<const double> src = A.flat + (size_t)f * 2 * nspec;
      const double sr = src[2 * (((size_t)q * nkx + p) * NY + n)], si = src[2 * (((size_t)q * nkx + p) * NY + n) + 1];
      bad = bad || !isfinite(sr) || !isfinite(si);
      const int s = canon_src_q(p, q, nz);
      cplx v = make_double2(0.0, 0.0);
      if (s >= 0) {
        v = make_double2(sr, si);
      } else if (s < -1) {
        const int qs = -s - 2;
        const size_t o = 2 * (((size_t)qs * nkx + p) * NY + n);
        v = make_double2(src[o], -src[o + 1]);
      }
      (f ? A.oS : A.vS)[j] = v;
    } else if (i < 2 * nspec + NY) {
      const int k = (int)(i - 2 * nspec);    // U[k] and W[k]
      const double u = A.flat[4 * nspec + k], w = A.flat[4 * nspec + NY + k];
      bad = bad || !isfinite(u) || !isfinite(w);
      A.meanS[k] = u;
      A.meanS[NY + k] = w;
    } else {
      const size_t j = i - 2 * nspec - NY;   // destination [p][q]
      const int p = (int)(j / nz), q = (int)(j - (size_t)p * nz);
      const gptr<const double> src = A.flat + 4 * nspec + 2 * NY;
      const double sr = src[2 * ((size_t)q * nkx + p)], si = src[2 * ((size_t)q * nkx + p) + 1];
      bad = bad || !isfinite(sr) || !isfinite(si);
      const int s = canon_src_q(p, q, nz);
      cplx v = make_double2(0.0, 0.0);
      if (s >= 0) {
        v = make_double2(sr, si);
      } else if (s < -1) {
        const size_t o = 2 * ((size_t)(-s - 2) * nkx + p);
        v = make_double2(src[o], -src[o + 1]);
      }
      A.vw_old[j] = v;
      A.vw_new[j] = v;
    }
  }
  if (tid == 0) {
    const double t = A.flat[4 * nspec + 2 * NY + 2 * nvw], ns = A.flat[4 * nspec + 2 * NY + 2 * nvw + 1];
    bad = bad || !isfinite(t) || !isfinite(ns);
  }
  if (bad) *A.in_status = 1;
}

// The advanced state back into the caller's buffer, unless the input or the action was rejected
// (then the buffer is left as it was).
__global__ void k_state_out(StaticIO A) {
  if (*A.in_status != 0 || (*A.status & STATUS_BAD_ACTION)) return;
  const int nz = A.nz, nkx = A.nkx, NY = A.ny;
  const size_t nspec = (size_t)nz * nkx * NY;
  const size_t nvw = (size_t)nz * nkx;
  const size_t total = 2 * nspec + NY + nvw;
  const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x, nthr = (size_t)gridDim.x * blockDim.x;
  for (size_t i = tid; i < total; i += nthr) {
    if (i < 2 * nspec) {
      const int f = i >= nspec;
      const size_t j = i - f * nspec;        // destination [q][p][n]
      const int n = (int)(j % NY);
      const int qp = (int)(j / NY), q = qp / nkx, p = qp - q * nkx;
      const cplx v = (f ? A.oS : A.vS)[((size_t)p * nz + q) * NY + n];
      A.flat[(size_t)f * 2 * nspec + 2 * j] = v.x;
      A.flat[(size_t)f * 2 * nspec + 2 * j + 1] = v.y;
    } else if (i < 2 * nspec + NY) {
      const int k = (int)(i - 2 * nspec);
      A.flat[4 * nspec + k] = A.meanS[k];
      A.flat[4 * nspec + NY + k] = A.meanS[NY + k];
    } else {
      const size_t j = i - 2 * nspec - NY;   // destination [q][p]
      const int q = (int)(j / nkx), p = (int)(j - (size_t)q * nkx);
      const cplx v = A.vw_old[(size_t)p * nz + q];
      A.flat[4 * nspec + 2 * NY + 2 * j] = v.x;
      A.flat[4 * nspec + 2 * NY + 2 * j + 1] = v.y;
    }
  }
  if (tid == 0) {
    const size_t o = 4 * nspec + 2 * NY + 2 * nvw;
    A.flat[o] = A.flat[o] + A.t_inc;
    A.flat[o + 1] = A.flat[o + 1] + A.n_inc;
  }
}

// Column pass of the single channel e (the general kernel for N > 64 or when forced).
int static_column(chan_env* e, const ColChan& h, const ColStage& S, bool solve, bool recon, hipStream_t st) {
  if (uses_pm(e)) return launch_column_pm(e->d, nullptr, &h, 1, S, solve, recon, st, nullptr, 4);
  const int r = S.stage;
  int mode = WALL_OPP;
  double s = 0.0;
  if (e->opts.controller == CHAN_CTRL_EXTERNAL) {
    mode = WALL_RAMP;
    if (r >= 0) s = (e->opts.action_mode == CHAN_HOLD) ? 1.0 : (S.m + RK_C_END[r]) / (double)S.n_sub;
  }
  return launch_column_pass(e->d, e->s, e->ph, r, e->sc[r < 0 ? 0 : r], mode, s, e->js, e->opts.opp_alpha, r == 2,
                            recon, st, nullptr);
}

// A fixed plane-pass tiling (tilings change no result): three pairs of rows per x-row block
// where that is valid, pencil blocks of 16.
PlaneTiles static_tiles(const Dims& d) {
  std::vector<PlaneTiles> c;
  if (plane_tile_candidates(d, &c, 1) != 0 || c.empty()) return PlaneTiles{0, 0, 0};
  for (const PlaneTiles& t : c)
    if (t.P >= 3 && t.PB >= 16) return t;
  return c.back();
}

int static_step(chan_env* e, char* base, const PlaneTiles& tiles, double* state, const double* action,
                int32_t n_substeps, double* obs, double* tau_w, double* drag, hipStream_t st) {
  const Dims& d = e->d;
  StepChan* d_prime = (StepChan*)(base + ARG_PRIME);
  StepChan* d_step = (StepChan*)(base + ARG_STEP);
  ColChan* d_col = (ColChan*)(base + ARG_COL);
  PlaneChan* d_plane = (PlaneChan*)(base + ARG_PLANE);
  int* d_status = (int*)(base + ARG_STATUS);
  int* d_in = (int*)(base + ARG_INSTATUS);
  const bool ext = e->opts.controller == CHAN_CTRL_EXTERNAL;
  StepChan prime = make_step_chan_env(e, d_status, nullptr, 1, nullptr, nullptr, nullptr);
  prime.skip = 0;
  prime.zero_vw = 0;
  StepChan step = make_step_chan_env(e, d_status, action, n_substeps, obs, tau_w, drag);
  step.skip = 0;
  const ColChan h = make_col_chan(e);
  const PlaneChan pc = make_plane_chan(e);
  StaticIO io;
  std::memset(&io, 0, sizeof(io));
  io.nz = d.nz;
  io.nkx = d.nkx;
  io.ny = d.ny;
  io.flat = (decltype(io.flat))state;
  io.vS = (decltype(io.vS))e->s.vS;
  io.oS = (decltype(io.oS))e->s.oS;
  io.vw_old = (decltype(io.vw_old))e->s.vw_old;
  io.vw_new = (decltype(io.vw_new))e->s.vw_new;
  io.meanS = (decltype(io.meanS))e->s.meanS;
  io.in_status = (decltype(io.in_status))d_in;
  io.status = (decltype(io.status))e->s.status;
  io.t_inc = n_substeps * e->ph.dt;       // as chan_env_step advances its clock
  io.n_inc = (double)n_substeps;
  const size_t total = (size_t)2 * d.nz * d.nkx * d.ny + d.ny + (size_t)d.nz * d.nkx;
  const unsigned io_blocks = (unsigned)std::min<size_t>((total + 255) / 256, 1024);

  hipLaunchKernelGGL(k_static_args, dim3(1), dim3(64), 0, st, prime, step, h, pc, d_prime, d_step, d_col, d_plane,
                     d_in);
  // prime: the state, then the plane-pass input, opposition target and wall shear from it
  // (chan_env_set_state's sequence)
  if (launch_begin_step(d_prime, 1, st, nullptr)) return fail(CHAN_EDEVICE, "launch begin_step", hipGetLastError());
  hipLaunchKernelGGL(k_state_in, dim3(io_blocks), dim3(256), 0, st, io);
  if (static_column(e, h, ColStage{-1, 0, 1}, false, true, st))
    return fail(CHAN_EDEVICE, "launch column pass", hipGetLastError());
  // the env step (chan_env_step's sequence for one channel)
  if (launch_begin_step(d_step, 1, st, nullptr)) return fail(CHAN_EDEVICE, "launch begin_step", hipGetLastError());
  if (ext && action && launch_ingest(d_step, 1, d.nx, d.nz, d.nkx, st, nullptr))
    return fail(CHAN_EDEVICE, "launch ingest", hipGetLastError());
  for (int m = 0; m < n_substeps; ++m)
    for (int r = 0; r < 3; ++r) {
      const bool last = (m == n_substeps - 1) && (r == 2);
      if (launch_plane_pass(d, d_plane, 1, tiles, st, nullptr))
        return fail(CHAN_EDEVICE, "launch plane pass", hipGetLastError());
      if (static_column(e, h, ColStage{r, m, n_substeps}, true, !last, st))
        return fail(CHAN_EDEVICE, "launch column pass", hipGetLastError());
    }
  const ColStage S_end = {-1, 0, n_substeps};
  if (static_column(e, h, S_end, false, true, st)) return fail(CHAN_EDEVICE, "launch column pass", hipGetLastError());
  const bool pressure = obs != nullptr && (e->opts.obs_mask & CHAN_OBS_P);
  if (pressure) {
    if (launch_plane_pass(d, d_plane, 1, tiles, st, nullptr))
      return fail(CHAN_EDEVICE, "launch plane pass (pressure)", hipGetLastError());
    int rc = 0;
    if (uses_pm(e)) {
      rc = launch_pressure_pm(d, d_col, 1, S_end, st, nullptr);
    } else {
      const bool ramp = ext && e->opts.action_mode == CHAN_RAMP;
      rc = launch_pressure_generic(d, e->s, e->ph, e->n_planes, e->js_planes, ramp, n_substeps, st, nullptr);
    }
    if (rc) return fail(CHAN_EDEVICE, "launch pressure", hipGetLastError());
  }
  if (launch_finish_step(d_step, 1, st, nullptr)) return fail(CHAN_EDEVICE, "launch finish_step", hipGetLastError());
  const int nslots = pressure ? 1 + SLOTS_PER_PLANE * e->n_planes : SLOTS_PER_PLANE * e->n_planes - 3;
  if (launch_outputs(d_step, 1, d.nx, d.nz, d.nkx, nslots, st, nullptr))
    return fail(CHAN_EDEVICE, "launch outputs", hipGetLastError());
  if (pressure && launch_pressure_finish(d_step, 1, st, nullptr))
    return fail(CHAN_EDEVICE, "launch pressure finish", hipGetLastError());
  hipLaunchKernelGGL(k_state_out, dim3(io_blocks), dim3(256), 0, st, io);
  HIPCHECK(hipGetLastError());
  int words[2] = {0, 0};
  HIPCHECK(hipMemcpyAsync(words, d_status, sizeof(words), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
  if (words[1]) return fail(CHAN_ENONFINITE, "non-finite value in the state given (state unchanged)");
  if (words[0] & STATUS_BAD_ACTION) return fail(CHAN_ENONFINITE, "non-finite action (state unchanged)");
  if (words[0] & STATUS_NONFINITE) return fail(CHAN_ENONFINITE, "non-finite state after the step");
  return CHAN_OK;
}

}  // namespace

extern "C" int chan_step_static(const chan_grid_t* grid, const chan_opts_t* opts, void* hip_stream, double* state,
                                const double* action, int32_t n_substeps, double* obs, double* tau_w, double* drag) {
  g_last_error.clear();
  if (!state) return fail(CHAN_EINVAL, "state");
  if (n_substeps < 1) return fail(CHAN_EINVAL, "n_substeps < 1");
  chan_env e;
  int rc = setup_env(grid, opts, hip_stream, &e);
  if (rc != CHAN_OK) return rc;
  const Dims& d = e.d;
  const size_t tabd = table_doubles(d, e.ph.open);
  const Sizes z = buffer_sizes(d, tabd);
  if (STATIC_ARGS_BYTES + z.total > STATIC_SCRATCH_BYTES)
    return fail(CHAN_EINVAL, "grid too large for chan_step_static (its scratch holds 32 MiB; "
                             "chan_env_footprint_bytes must be at most 32 MiB - 4 KiB)");
  int dev = -1;
  HIPCHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_STATIC_DEVICES) return fail(CHAN_EDEVICE, "device index beyond the static slots");
  e.device = dev;
  StaticSlot& slot = static_slot[dev];
  std::lock_guard<std::mutex> guard(slot.lock);
  if (!slot.ptr) {
    void* p = nullptr;
    HIPCHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    slot.ptr = (char*)p;
  }
  char* base = slot.ptr + STATIC_ARGS_BYTES;
  hipStream_t st = e.stream;
  if (!same_tables(slot, d, e.ph)) {
    HostTables ht;
    rc = host_tables(d, e.ph, &ht);
    if (rc != CHAN_OK) return rc;
    slot.have_tables = false;
    carve_state(d, z, ht.L, base, &e.s);
    // clear every buffer (the Nyquist rows are never written by the kernels), then the tables
    hipLaunchKernelGGL(k_static_zero, dim3(1024), dim3(256), 0, st, (double*)base, z.total / sizeof(double));
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipMemcpyAsync(e.s.tab, ht.data.data(), ht.data.size() * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHECK(hipStreamSynchronize(st));
    slot.nx = d.nx;
    slot.ny = d.ny;
    slot.nz = d.nz;
    slot.ph = e.ph;
    slot.L = ht.L;
    slot.tiles = static_tiles(d);
    slot.have_tables = true;
  } else {
    carve_state(d, z, slot.L, base, &e.s);
  }
  return static_step(&e, slot.ptr, slot.tiles, state, action, n_substeps, obs, tau_w, drag, st);
}
