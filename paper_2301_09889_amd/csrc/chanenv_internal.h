// Internal declarations shared by the host driver and the HIP kernels.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

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
  size_t kfwd, kinv, rc_pm, intw_pm, op_pm, vt_pm, up_pm;
  size_t total;
};

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
  cplx *tmp2d;                  // [3][nz][nkx] small 2-D transform scratch
  double *tab;                  // operator tables (one allocation, see TableLayout)
  double *drag_acc;             // [1]
  int *status;                  // [1]
  // views into tab
  const double *cosk, *rc, *optab, *vt, *minv, *up, *inv_int_up, *alpha, *beta;
  const double *kfwd, *kinv, *rc_pm, *intw_pm, *op_pm, *vt_pm, *up_pm;
  const cplx *twz, *twx, *twnx, *twnz;
};

// Kernel classes for the optional event timing.
enum KernelClass : int {
  KC_COLUMN = 0, KC_ZINV = 1, KC_XROW = 2, KC_ZFWD = 3, KC_INGEST = 4, KC_OUTPUT = 5, KC_BOOK = 6,
  KC_RECON = 7, KC_COUNT = 8
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
int launch_begin_step(const Dims& d, DeviceState& s, bool zero_vw_new, hipStream_t st, KernelTimer* tm);
int launch_ingest(const Dims& d, DeviceState& s, const double* action, double clip, hipStream_t st,
                  KernelTimer* tm);
int launch_plane_pass(const Dims& d, DeviceState& s, hipStream_t st, KernelTimer* tm);
// Column pass; stage -1 only reconstructs the plane-pass input from the state.  With
// recon false the pass stops after the solve (the caller reconstructs separately).
int launch_column_pass_pm(const Dims& d, DeviceState& s, const PhysParams& ph, int stage,
                          const StageConsts& sc, int wall_mode, double s_ramp, int js,
                          double opp_alpha, bool accumulate_drag, bool recon, hipStream_t st,
                          KernelTimer* tm);
int launch_column_pass(const Dims& d, DeviceState& s, const PhysParams& ph, int stage,
                       const StageConsts& sc, int wall_mode, double s_ramp, int js,
                       double opp_alpha, bool accumulate_drag, bool recon, hipStream_t st,
                       KernelTimer* tm);
int launch_finish_step(const Dims& d, DeviceState& s, bool copy_vw, double* drag, int nsub,
                       hipStream_t st, KernelTimer* tm);
int launch_outputs(const Dims& d, DeviceState& s, int js, uint32_t obs_mask, double* obs,
                   double* tau_w, hipStream_t st, KernelTimer* tm);

}  // namespace chanenv
