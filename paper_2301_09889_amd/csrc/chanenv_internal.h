// Internal declarations shared by the host driver and the HIP kernels.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "chanenv.h"

namespace chanenv {

typedef double2 cplx;

// Status bits written by the kernels (device word, read back after a step).
enum : int {
  STATUS_BAD_ACTION = 1,   // non-finite action: every state-changing kernel skips
  STATUS_NONFINITE = 2     // non-finite state produced by a stage
};

enum WallMode : int { WALL_RAMP = 0, WALL_OPP = 1 };

// Number of per-column tau operators: the three stage operators D^2 - (k^2 + 1/(b_r nu dt))
// and the velocity operator D^2 - k^2.
constexpr int NOPS = 4;

// Host-side geometry and the layout of the packed operator tables.
struct Dims {
  int nx, ny, nz, N, nkx, mx, mz, ncol;
  int ml;        // unknowns per parity, N/2 + 1
  int opsz;      // doubles per (column, operator, parity) record: w, u, f, F (ml each), 1/sum F, pad
};

// Offsets (in doubles) of each table inside the single device table buffer.
struct TableLayout {
  size_t cosk, rc, optab, vt, minv, up, inv_int_up, twz, twx, twnx, twnz, alpha, beta;
  // parity-major copies for the column kernel with N <= 64 (one lane per coefficient:
  // even n = 2l in lanes l < 32, odd n = 2i + 1 in lanes 32 + i, n = N as a 65th "tail" entry)
  size_t kfwd, ccos, rc_pm, intw_pm, op_pm, vt_pm, up_pm;
  // open channel only: phi_+ of every pair and stage (parity-major for N <= 64, natural order
  // above) and 1/(dphi_+/dxi)(+1)
  size_t pt_pm, ptinv, pt;
  // pressure: phi_+ of (D^2 - k^2/ys^2) per pair (parity-major for N <= 64, and natural
  // order for the general kernel) and the inverse of the 2x2 Neumann matrix (dphi_+-/dxi at +-1)
  size_t pk_pm, pkinv, pk;
  size_t total;
};

// Observation planes per env: the sensing plane and the extra ones.
constexpr int MAX_PLANES = 1 + CHAN_MAX_EXTRA_PLANES;

// Parity-major record of one tau operator: w, u, f, F (65 entries each: 64 lanes + tail),
// then 1/sum F for the even and the odd system.
constexpr int PM_ENTRIES = 65;
constexpr int PM_OPSZ = 4 * PM_ENTRIES + 4;

// Host precompute of every operator table, in FP64.
struct HostTables {
  std::vector<double> data;
  TableLayout L;
};

struct PhysParams {
  double nu, dt, ub;
  int forcing;
  double px;
  double lx, lz;
  // geometry: closed channel (walls at y = +-1) or open channel (wall at y = 0, free-slip
  // surface at y = 1); the Chebyshev variable is xi = y or xi = 2y - 1, d/dy = ys d/dxi
  int open;
  double ys;
  // the viscosity seen in the Chebyshev variable: nu ys^2
  double nu_xi() const { return nu * ys * ys; }
};

void precompute_tables(const Dims& d, const PhysParams& ph, HostTables* out);

// Host initial condition in the state exchange layout ([q][p][n] complex v, omega_y,
// U, W, zero old action, t = 0, step 0).
void initial_condition(const Dims& d, const PhysParams& ph, int profile, double amp,
                       uint64_t seed, std::vector<double>* flat);

// Device buffers of one env.
struct DeviceState {
  cplx *vS, *oS, *hist;         // [c][n] state, [2][c][n] previous-stage h_v, h_g
  double *meanS, *meanH;        // [2][n] U, W ; [2][n] previous-stage h_u, h_w
  cplx *F6, *Z6, *W3, *H3;      // plane-pass fields
  cplx *vw_old, *vw_new, *vw_opp, *tauw;  // [c]
  cplx *tmp2d;                  // [OUT_SLOTS][nz][nkx] small 2-D transform scratch
  double *tab;                  // operator tables (one allocation, see TableLayout)
  double *drag_acc;             // [1]
  int *status;                  // [1]
  // views into tab
  const double *cosk, *rc, *optab, *vt, *minv, *up, *inv_int_up, *alpha, *beta;
  const double *kfwd, *ccos, *rc_pm, *intw_pm, *op_pm, *vt_pm, *up_pm, *pt_pm, *ptinv, *pt, *pk_pm, *pkinv, *pk;
  cplx *pbuf;                   // [MAX_PLANES][nkx][nz] pressure spectra on the observation planes
  double *pscr;                 // [MAX_PLANES][3][nz][nx] u, v, w on the pressure planes
  const cplx *twz, *twx, *twnx, *twnz;
};

// Device memory pointers held in the per-channel argument structs.  In the device pass they are
// typed as global-address-space pointers: read from memory, an untyped pointer would make the
// compiler use flat memory instructions, whose completion shares the LDS counter (so every
// LDS wait would also wait for them).  In the host pass they are plain pointers (same size and
// layout); host code assigns them with a cast.
#if defined(__HIP_DEVICE_COMPILE__)
template <class T>
using gptr = __attribute__((address_space(1))) T*;
#else
template <class T>
using gptr = T*;
#endif

// ---- per-channel launch arguments (device-resident arrays, one entry per channel) ----
// A launch covers every channel of one grid shape (column and plane kernels) or of the whole
// batch (the per-env-step kernels); a single env is a batch of one, so a channel runs the
// same code alone and in a mix.

// N <= 64 column kernels: everything of one channel that does not change between launches.
struct ColChan {
  int nkx, nz, ncol;
  int ext;                      // 1: external action (ramped or held wall velocity); 0: opposition
  int hold;                     // external action held for the whole env step
  int forcing, js;
  int open;                     // free-slip top (open channel)
  // per RK stage: 1/(b nu' dt), a/b, g/(b nu'), z/(b nu') with nu' = nu ys^2, the viscosity
  // in the Chebyshev variable
  double lam0[3], ab[3], gb[3], zb[3];
  double nu_wall;               // nu ys: wall shear = nu_wall d/dxi
  double dt;                    // time step (the rate of a ramped wall velocity)
  int n_pplanes;                // pressure planes (0: no pressure observed)
  int pjs[MAX_PLANES];          // their nodes
  double ys, ysi;               // d/dy = ys d/dxi; ysi = 1/ys (both powers of two)
  double opp_alpha, ub2, px;
  size_t plane;                 // elements per field in F6 / H3 (ny nkx nz)
  gptr<cplx> vS, oS, hist;
  gptr<double> meanS, meanH;
  gptr<const cplx> H3;
  gptr<cplx> F6;
  gptr<const cplx> vw_old, vw_new;
  gptr<cplx> vw_opp, tauw;
  gptr<const double> kfwd, ccos, rc_pm, intw_pm, op_pm, vt_pm, up_pm, minv, inv_int_up, alpha, beta;
  gptr<const double> pt_pm, ptinv, pk_pm, pkinv;
  gptr<cplx> pbuf;
  gptr<double> drag_acc;
  gptr<int> status;
};

// The launch-wide part: RK stage (-1: reconstruction from the stored state, which ends an env
// step), time step m of n_sub in the env step.
struct ColStage {
  int stage, m, n_sub;
};

// Plane-pass kernels of one channel.
struct PlaneChan {
  int ny, nkx, nz;
  double scale;        // 1 / (M_x M_z)
  gptr<const cplx> F6;
  gptr<cplx> Z6;
  gptr<cplx> W3;
  gptr<cplx> H3;
  gptr<const cplx> twz;   // exp(-2 pi i k / M_z)
  gptr<const cplx> twx;   // exp(-2 pi i k / M_x)
  gptr<const int> status;
};

// Per-env-step kernels (begin, action ingest, end, outputs) of one channel; rebuilt for
// every step call (action and output pointers).
// Output transforms: slot 0 tau_w; for observation plane k (the sensing plane first, then up
// to CHAN_MAX_EXTRA_PLANES more) slot 1 + 7 k + f: component f of u, v, w, P into the
// observation, and 1 + 7 k + 4 + f: u, v, w into the pressure scratch.
constexpr int SLOTS_PER_PLANE = 7;
constexpr int OUT_SLOTS = 1 + SLOTS_PER_PLANE * MAX_PLANES;
struct StepChan {
  int nx, nz, nkx, ncol, n_sub;
  int skip;                     // not advanced this call (no valid state): marked like a
                                // rejected action, so every kernel leaves it untouched
  int zero_vw;                  // external action and none given: v_w,new := 0
  int copy_vw;                  // external action: v_w,old := v_w,new at the end
  double clip;
  gptr<const double> action;         // [nz][nx] device, or null
  gptr<double> drag_out;             // or null
  gptr<const cplx> out_src[OUT_SLOTS];  // spectra [p][q] (obs: the F6 plane at an observation node)
  gptr<double> out_dst[OUT_SLOTS];      // [nz][nx] device, or null
  gptr<cplx> vw_new, vw_old;
  gptr<cplx> tmp2d;                  // [OUT_SLOTS][nz][nkx]
  gptr<const cplx> twnx, twnz;
  gptr<double> drag_acc;
  gptr<int> status;
  gptr<int> status_out;         // batch-wide status array entry (read back once per call)
};

// Kernel classes for the optional event timing.
enum KernelClass : int {
  KC_COLUMN = 0, KC_ZINV = 1, KC_XROW = 2, KC_ZFWD = 3, KC_INGEST = 4, KC_OUTPUT = 5, KC_BOOK = 6,
  KC_RECON = 7, KC_FUSED = 8, KC_COUNT = 9
};

// Brackets kernel launches with HIP events when enabled (instrumentation only).
struct KernelTimer {
  bool on = false;
  std::vector<hipEvent_t> pool;     // created lazily, reused
  std::vector<int> cls;             // class of each recorded pair
  size_t used = 0;                  // pairs recorded since the last read
  // Event pair for the next launch of class c; hipExtLaunchKernel stamps them with that
  // kernel's own start and end (no marker commands of their own in the stream).
  hipError_t next(int c, hipEvent_t* start, hipEvent_t* stop);
};

// Launch, timed when tm is non-null.
template <typename... KArgs, typename... Args>
inline void timed_launch(KernelTimer* tm, int c, void (*kernel)(KArgs...), dim3 grid, dim3 block, size_t shm,
                         hipStream_t st, Args... args) {
  hipEvent_t a = nullptr, b = nullptr;
  if (tm && tm->next(c, &a, &b) != hipSuccess) a = b = nullptr;
  hipExtLaunchKernelGGL(kernel, grid, block, (std::uint32_t)shm, st, a, b, 0u, static_cast<KArgs>(args)...);
}

struct StageConsts {
  double lam0, ab, gb, zb;      // 1/(b nu dt), a/b, g/(b nu), z/(b nu)
};

// Kernel launchers (kernels.hip).  tm may be null.
// Per-env-step kernels over nch channels of any shapes (max_* size the LDS and the grid).
int launch_begin_step(const StepChan* d_step, int nch, hipStream_t st, KernelTimer* tm);
int launch_ingest(const StepChan* d_step, int nch, int max_nx, int max_nz, int max_nkx, hipStream_t st,
                  KernelTimer* tm);
int launch_finish_step(const StepChan* d_step, int nch, hipStream_t st, KernelTimer* tm);
// Pressure on the observation planes from the end-of-step state (H3 holds its non-linear term).
int launch_pressure_pm(const Dims& d, const ColChan* d_col, int nch, const ColStage& S, hipStream_t st,
                       KernelTimer* tm);
// The same with the general column kernel, for one channel.
int launch_pressure_generic(const Dims& d, const DeviceState& s, const PhysParams& ph, int n_planes,
                            const int* js_planes, bool ramp, int n_sub, hipStream_t st, KernelTimer* tm);
// p = P - (|u|^2/2 - its plane mean) on every pressure plane, after the output transforms.
int launch_pressure_finish(const StepChan* d_step, int nch, hipStream_t st, KernelTimer* tm);
int launch_outputs(const StepChan* d_step, int nch, int max_nx, int max_nz, int max_nkx, int nslots, hipStream_t st,
                   KernelTimer* tm);
// Plane pass over nch channels of one shape (M_x, M_z from nx, nz), with a tiling: PB pencils
// per z-kernel block, P pairs of padded z rows per x-row block, and fused = 1 for the z inverse
// and the x rows in one launch (k_zxrow, P = its pairs per block).  The tiling distributes
// independent transforms over blocks and does not change any result.
struct PlaneTiles {
  int PB, P, fused;
};
int launch_plane_pass(const Dims& d, const PlaneChan* d_plane, int nch, const PlaneTiles& t, hipStream_t st,
                      KernelTimer* tm);
// Every valid tiling for the shape (for the tuner); -1 if the shape has none.
int plane_tile_candidates(const Dims& d, std::vector<PlaneTiles>* out, int form = 0);
// N <= 64 column pass over nch channels of one shape: the solve of stage S.stage (if solve)
// and/or the reconstruction that follows it (if recon; S.stage -1: reconstruction only).
// d_col: the channels' arguments on the device; h_col (optional): the same on the host, used
// to pass a single channel's arguments by value.  batch_cw: columns per block when nch > 1
// (2 or 4; no result depends on it).
int launch_column_pm(const Dims& d, const ColChan* d_col, const ColChan* h_col, int nch, const ColStage& S,
                     bool solve, bool recon, hipStream_t st, KernelTimer* tm, int batch_cw);
// General column pass (any N, one channel per launch); stage -1 only reconstructs the
// plane-pass input from the state; with recon false the pass stops after the solve.
int launch_column_pass(const Dims& d, DeviceState& s, const PhysParams& ph, int stage,
                       const StageConsts& sc, int wall_mode, double s_ramp, int js,
                       double opp_alpha, bool accumulate_drag, bool recon, hipStream_t st,
                       KernelTimer* tm);

}  // namespace chanenv
