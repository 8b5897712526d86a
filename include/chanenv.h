/*
 * chanenv.h -- C ABI of the MI355X channel-flow DNS environment.
 *
 * The library advances an incompressible channel flow with a Fourier (x, z) x
 * Chebyshev (y) pseudo-spectral method in velocity--vorticity form, RK3 for the
 * non-linear terms and Crank--Nicolson for the viscous terms (paper §3.1), with
 * wall-normal blowing/suction at the lower wall as the control (§3.2),
 * opposition control as the in-library controller (§4.1) and a wall-parallel
 * velocity plane as the observation (§3.2).  Every numerical stage runs in
 * FP64 HIP kernels on the device; the host only sequences launches.
 *
 * The calls map onto the request protocol of the paper's solver interface
 * (§3.3): STATE -> the observation output of chan_env_step (and
 * chan_env_get_state), CNTRL -> its action argument, EVOLVE -> its n_substeps
 * argument with the wall shear and drag outputs, TERMN -> chan_env_destroy
 * (chan_env_reset covers the restart of an episode).
 *
 * Units: lengths in h, velocities in the nominal friction velocity u_tau, so
 * nu = 1/Re_tau and t+ = t Re_tau.  Two geometries (§3.1):
 *   closed channel (default): walls at y = -1 and y = +1, h the half-height;
 *   open channel (CHAN_TOP_FREESLIP): a wall at y = 0 and a free-slip surface at
 *   y = h = 1 (u_y = w_y = v = 0 there).
 * The actuated wall is always the lower one.  The Chebyshev variable xi in
 * [-1, 1] is y (closed) or 2y - 1 (open); spectral state coefficients are those
 * of T_n(xi), and node j is xi_j = cos(pi j / N) in both.
 *
 * Layouts.  Wall planes are row-major [z][x] with x fastest, on the grid
 * x_i = i Lx/nx, z_k = k Lz/nz.  Spectral arrays are [q][p] with
 * p = 0 .. nx/2-1 and the signed spanwise index q stored at q mod nz.
 *
 * Errors.  Every int-returning call returns CHAN_OK (0) or a negative code;
 * no exception or abort crosses the ABI.  chan_strerror names a code.
 * Threading: one env per thread; calls on one env must not overlap.
 */
#ifndef CHANENV_H
#define CHANENV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  CHAN_OK = 0,
  CHAN_EINVAL = -1,      /* bad argument or unsupported option; nothing changed   */
  CHAN_ENOMEM = -2,      /* device or host allocation failed                      */
  CHAN_EDEVICE = -3,     /* a HIP runtime call failed                             */
  CHAN_ENONFINITE = -4,  /* non-finite action (state untouched) or state (poisoned) */
  CHAN_ESTATE = -5,      /* step or get_state before reset/set_state, or poisoned */
  CHAN_EBUSY = -6        /* the env is held by an unfinished asynchronous call (chan_batch_launch) */
};

/* Opaque environment handle, owned by the library. */
typedef struct chan_env chan_env;

enum { CHAN_TOP_WALL = 0, CHAN_TOP_FREESLIP = 1 };
enum { CHAN_CFR = 0, CHAN_CPG = 1 };
enum { CHAN_CTRL_EXTERNAL = 0, CHAN_CTRL_OPPOSITION = 1 };
enum { CHAN_RAMP = 0, CHAN_HOLD = 1 };
enum { CHAN_IC_LAMINAR = 0, CHAN_IC_REICHARDT = 1 };
enum { CHAN_OBS_U = 1, CHAN_OBS_V = 2, CHAN_OBS_W = 4, CHAN_OBS_P = 8 };
/* Observation planes: the sensing plane of chan_grid_t plus up to CHAN_MAX_EXTRA_PLANES more
 * (§3.2: the observed state is one or more wall-parallel planes). */
enum { CHAN_MAX_EXTRA_PLANES = 3 };

/* Grid and physical parameters (§3.1: N_x x N_y x N_z modes, Re_tau; §3.2:
 * sensing height).  Supported: nx, nz in {4, 8, 16, 32, 64, 128};
 * ny in {17, 33, 65, 97, 129}; re_tau > 0; dt_plus > 0; obs_y_plus > 0 and
 * below the node next to the top (wall or surface). */
typedef struct {
  int32_t nx, ny, nz;   /* Fourier modes in x, Chebyshev modes in y, Fourier modes in z */
  double lx, lz;        /* box lengths in h (minimal channel 2.67 x 0.8, larger 2 pi x pi) */
  double re_tau;        /* nominal friction Reynolds number; nu = 1/re_tau unless overridden */
  double dt_plus;       /* one substep = one full RK3/CN time step of dt = dt_plus/re_tau */
  double obs_y_plus;    /* sensing height above the lower wall in viscous units; rounded UP to a
                           Chebyshev node (§3.2); chan_env_query reports the node used */
} chan_grid_t;

/* Options; passing NULL to chan_env_create selects the defaults in brackets. */
typedef struct {
  int32_t top_bc;       /* [CHAN_TOP_WALL] closed channel | CHAN_TOP_FREESLIP open channel
                           (the paper's geometry) */
  int32_t forcing;      /* [CHAN_CFR] constant flow rate | CHAN_CPG constant pressure gradient */
  double ub_plus;       /* [<= 0: 15.66 (re_tau/180)^(1/7)] bulk velocity held by CFR */
  double px;            /* [0] pressure gradient for CPG */
  double nu_override;   /* [<= 0: unused] > 0 replaces nu = 1/re_tau */
  double dt_override;   /* [<= 0: unused] > 0 replaces dt = dt_plus/re_tau */
  int32_t controller;   /* [CHAN_CTRL_EXTERNAL] caller's actions | CHAN_CTRL_OPPOSITION */
  double opp_alpha;     /* [1.0] opposition gain alpha (§4.1) */
  int32_t action_mode;  /* [CHAN_RAMP] linear old->new over the env step (§3.2) | CHAN_HOLD */
  double clip;          /* [1.0] |action| bound in u_tau (§3.2); <= 0 disables clipping */
  uint32_t obs_mask;    /* [CHAN_OBS_U | CHAN_OBS_V] observed components (§3.2, §4.2); with
                           CHAN_OBS_P the static-pressure fluctuation p - <p>_plane (abstract:
                           velocity and pressure observable) */
  int32_t ic_profile;   /* [CHAN_IC_LAMINAR] mean profile of chan_env_reset | CHAN_IC_REICHARDT */
  double ic_amp;        /* [0.1] rms of the reset perturbation as a fraction of U_cl = 1.5 U_b */
  int32_t n_extra_planes;  /* [0] further observation planes, 0 .. CHAN_MAX_EXTRA_PLANES */
  double extra_obs_y_plus[CHAN_MAX_EXTRA_PLANES];  /* their heights above the lower wall in
                           viscous units, each rounded up to a node like obs_y_plus; observed
                           with the same obs_mask components */
} chan_opts_t;

/* Derived quantities, filled by chan_env_query. */
typedef struct {
  int32_t nx, ny, nz, js;      /* js: index of the sensing node, y_js = cos(pi js/(ny-1)) */
  double y_plus_node;          /* wall distance of node js / nu: the sensing height used */
  double nu, dt, ub;           /* viscosity, time step, bulk velocity */
  double t;                    /* simulated time since reset (units h/u_tau) */
  int64_t nstep;               /* time steps since reset */
  size_t state_doubles;        /* length of the get/set_state buffer */
  size_t obs_doubles;          /* (1 + n_extra_planes) * popcount(obs_mask) * nz * nx */
  size_t footprint_bytes;      /* device memory held by the env */
  int32_t n_planes;            /* observation planes: 1 + n_extra_planes */
  int32_t js_planes[1 + CHAN_MAX_EXTRA_PLANES];      /* node of each plane (js first) */
  double y_plus_planes[1 + CHAN_MAX_EXTRA_PLANES];   /* its wall distance / nu */
} chan_info_t;

/* Fill *opts with the defaults listed above. */
void chan_opts_default(chan_opts_t* opts);

/* Create an env: validate, precompute the operators in FP64 on the host (tau
 * factors, homogeneous solutions and 2x2 influence matrices per wavenumber
 * pair and stage, Chebyshev and FFT tables), allocate the device state.
 * hip_stream: the hipStream_t all work is queued on (NULL = default stream).
 * *out owns the device memory until chan_env_destroy.  The env has no flow
 * until chan_env_reset or chan_env_set_state.
 * Errors: CHAN_EINVAL (*out untouched), CHAN_ENOMEM, CHAN_EDEVICE. */
int chan_env_create(const chan_grid_t* grid, const chan_opts_t* opts, void* hip_stream,
                    struct chan_env** out);

/* Seeded initial condition (the paper's stored initial fields, §4.2, are
 * replaced by a synthetic one): the selected mean profile plus a random
 * divergence-free perturbation drawn from SplitMix64(seed), with v = dv/dy =
 * omega_y = 0 at the walls and rms velocity ic_amp * U_cl.  Also sets the old
 * action to zero, t = 0 and the step counter to 0, and clears a poisoned state.
 * Errors: CHAN_EDEVICE. */
int chan_env_reset(struct chan_env* env, uint64_t seed);

/* One environment step (§3.2, §3.3): ingest the action, advance n_substeps
 * time steps, and write the outputs.
 *   action  DEVICE pointer to nz*nx doubles [z][x], the wall-normal velocity at
 *           y = -1 requested by the agents.  Clipped to [-clip, clip], the
 *           plane mean and the Nyquist modes are removed (zero net mass flux,
 *           §4.1), and the wall velocity ramps linearly from the previous
 *           action to this one over the env step (CHAN_RAMP) or jumps to it
 *           (CHAN_HOLD).  NULL means an all-zero action.  Ignored under
 *           CHAN_CTRL_OPPOSITION, where v_w = -alpha (v(y_s) - <v(y_s)>) is
 *           evaluated at the start of every time step.
 *   n_substeps  number of RK3/CN time steps, >= 1.
 *   obs     DEVICE pointer, n_planes*popcount(obs_mask)*nz*nx doubles, layout
 *           [plane][component][z][x]: u, v, w, p (in that order, selected by
 *           obs_mask) at the sensing node, then at each extra observation plane, end
 *           of the step.  p: from lap P = div(u x omega), P = p + |u|^2/2, with
 *           dP/dy = H_y + nu lap v - dv/dt at both boundaries (dv/dt: the slope of a
 *           ramped external action at the lower wall, else 0), the plane mean removed.
 *           May be NULL.
 *   tau_w   DEVICE pointer, nz*nx doubles: nu du/dy at the lower wall, end of step.  May be NULL.
 *   drag    DEVICE pointer, 1 double: mean over the n_substeps time steps of the
 *           plane-averaged lower-wall shear stress, sampled after each step
 *           (the reward's input, §3.2).  May be NULL.
 * All device pointers must be valid on the env's stream; the call returns
 * after the stream has finished the step.
 * Errors: CHAN_ESTATE (no flow yet, or poisoned), CHAN_EINVAL (n_substeps < 1),
 * CHAN_ENONFINITE (non-finite action: nothing changed; or non-finite state
 * after the step: the env is poisoned until reset/set_state), CHAN_EDEVICE. */
int chan_env_step(struct chan_env* env, const double* action, int32_t n_substeps,
                  double* obs, double* tau_w, double* drag);

/* Copy the flow state to / from HOST memory, n_doubles = state_doubles:
 *   v-hat [q][p][n] (re, im) | omega_y-hat [q][p][n] (re, im) | U [n] | W [n] |
 *   v_w,old [q][p] (re, im) | t | step counter (as a double)
 * with n the Chebyshev index.  set_state zeroes the Nyquist row and the (0,0)
 * entries of v and omega_y, enforces the p = 0 Hermitian symmetry (the q > 0
 * half wins) and clears a poisoned state.
 * Errors: CHAN_EINVAL (wrong n_doubles or NULL), CHAN_ESTATE (get before any
 * flow), CHAN_ENONFINITE (set with a non-finite value; nothing changed),
 * CHAN_EDEVICE. */
int chan_env_get_state(const struct chan_env* env, double* host, size_t n_doubles);
int chan_env_set_state(struct chan_env* env, const double* host, size_t n_doubles);

/* Sizes, sensing node, constants and counters.  Errors: CHAN_EINVAL (NULL). */
int chan_env_query(const struct chan_env* env, chan_info_t* out);

/* Device bytes an env of this shape holds (for admission by HBM footprint);
 * 0 if the grid is invalid. */
size_t chan_env_footprint_bytes(const chan_grid_t* grid, const chan_opts_t* opts);

/* Free the env and its device memory.  NULL is a no-op.  An env held by an unfinished call
 * (chan_batch_launch) is first waited for and detached from the call, which then reports
 * CHAN_EINVAL for it when finished; the env leaves every batch that lists it (later positions
 * shift down by one). */
void chan_env_destroy(struct chan_env* env);

/* Kernel timing (instrumentation for benchmarks).  chan_env_set_timing(env, 1)
 * clears the counters and times every later kernel launch of the env's own steps
 * with a pair of HIP events that hipExtLaunchKernel stamps with the kernel's start
 * and end on the env's stream; (env, 0) stops recording.  Timed launches are
 * serialised by the runtime, so throughput runs leave timing off.
 * chan_env_timing_read synchronises the stream and fills, for the first nclass
 * kernel classes, the number of launches and the summed kernel time in ms since
 * timing was enabled; it returns the number of classes (>= 0) or a negative
 * code.  Classes (chan_kernel_class_name): 0 column_pass (the implicit solve of a
 * stage alone), 1 z_inverse_fft, 2 x_rows_fft_product, 3 z_forward_fft, 4 action_ingest,
 * 5 outputs, 6 bookkeeping, 7 column_reconstruct (velocity/vorticity reconstruction
 * and inverse Chebyshev transform after each stage, and from the stored state at
 * the end of every env step), 8 column_solve_reconstruct (both parts in one launch:
 * every stage but the last of an env step, whose solve counts under 0).  Errors:
 * CHAN_EINVAL, CHAN_EDEVICE. */
int chan_env_set_timing(struct chan_env* env, int32_t enable);
int chan_env_timing_read(struct chan_env* env, int32_t nclass, int64_t* launches, double* ms);
const char* chan_kernel_class_name(int32_t cls);

/* ---- Batches: many channels advanced together ----
 * Serving many RL workers means stepping many independent channels at once (they
 * may differ in grid, Re_tau, dt, controller and options).  A batch advances a
 * fixed set of existing
 * envs with one launch per kernel and grid shape instead of one per env, so that
 * small channels fill the GPU.  Each channel computes exactly what chan_env_step
 * would (the same kernels on the same per-channel data): results are bitwise the
 * same alone and in the batch.
 *
 * chan_batch_create: n envs (n >= 1), each listed once, all on the current device; the batch
 * refers to them and does not own them (destroy the batch first).  Its synchronous calls
 * (chan_batch_step, chan_batch_step_subset) run on the first env's stream.  Errors:
 * CHAN_EINVAL (empty, null, duplicate, other devices, more than 65535 / N_y channels of one
 * shape), CHAN_EBUSY (an env held by an unfinished call), CHAN_ENOMEM, CHAN_EDEVICE.
 *
 * chan_batch_step: one env step (n_substeps time steps) of every env, in the
 * order given at creation.  actions, obs, tau_w and drag are host arrays of n
 * device pointers with the meaning of chan_env_step's arguments (any entry may be
 * NULL; a NULL array means all NULL).  results, if non-NULL, receives n codes:
 * CHAN_OK; CHAN_ENONFINITE for a rejected action (that env untouched) or a
 * non-finite state (that env poisoned); CHAN_ESTATE for an env without a flow
 * state or poisoned, which is skipped (untouched, outputs not written) while the
 * others advance.  Returns CHAN_OK if every env succeeded, else the first failing
 * env's code; CHAN_ESTATE (nothing run) if no env has a valid state; CHAN_EINVAL
 * for n_substeps < 1; CHAN_EDEVICE.
 * Synchronises the stream before returning.  Calls on one batch, or on batches
 * sharing an env, must not overlap.
 *
 * chan_batch_step_subset: the same for the n envs idx[0..n) of the batch (indices
 * as at creation, each at most once), the others untouched; the per-env arrays are
 * indexed like idx.  This is how a request loop advances whichever channels have a
 * pending request.  Extra errors: CHAN_EINVAL for a bad, repeated or missing index.
 *
 * chan_batch_set_timing / chan_batch_timing_read: as for an env, for the batch's
 * launches.  chan_batch_size: number of envs (0 for NULL). */
typedef struct chan_batch chan_batch;
int chan_batch_create(int32_t n, struct chan_env* const* envs, struct chan_batch** out);
int chan_batch_step(struct chan_batch* batch, const double* const* actions, int32_t n_substeps,
                    double* const* obs, double* const* tau_w, double* const* drag, int32_t* results);
int chan_batch_step_subset(struct chan_batch* batch, int32_t n, const int32_t* idx,
                           const double* const* actions, int32_t n_substeps, double* const* obs,
                           double* const* tau_w, double* const* drag, int32_t* results);
void chan_batch_destroy(struct chan_batch* batch);
int32_t chan_batch_size(const struct chan_batch* batch);
int chan_batch_set_timing(struct chan_batch* batch, int32_t enable);
int chan_batch_timing_read(struct chan_batch* batch, int32_t nclass, int64_t* launches, double* ms);

/* The tuned launch shapes of the batch's grid shapes (instrumentation).  A batch times, when it is
 * created, every valid tiling of the plane pass for each grid shape on that shape's channels, and
 * for a shape with several channels on the parity-major column kernels (N_y <= 65) the columns per
 * block of the batched column launch (2 or 4); the fastest of each is kept.  No result depends on
 * either choice.  A shape that first arrives through chan_batch_add is tuned on that one channel's
 * plane pass and keeps 4 columns per block.  Writes up to max_shapes records of 7 int32
 * {nx, ny, nz, z pencils per block, x-row pairs per block, columns per block, plane fused}
 * (columns per block 0 for a shape on the general column kernel; plane fused 1 where the z
 * inverse and the x rows run as one launch, possible for padded lengths M_x, M_z of 48 or 96,
 * else 0) and returns the number of shapes; CHAN_EINVAL for NULL arguments.  The environment
 * variable CHANENV_PLANE_FORM, read when a shape is tuned, limits the plane-pass choice to
 * "split" (three launches) or "fused" forms (where the shape has one). */
int chan_batch_tuning(const struct chan_batch* batch, int32_t max_shapes, int32_t* out);

/* ---- Asynchronous batch calls and membership (a request loop over channels that come and go) ----
 * chan_batch_launch queues one env step of the batch's envs envs[0..n) (each at most once; the
 * per-env arrays indexed like envs, as for chan_batch_step) on hip_stream, any stream of the
 * batch's device, and returns at once with *out holding the call.  Outputs are written by the
 * stream; an env is held by the call until chan_call_finish, and meanwhile any other call
 * involving it (including its own chan_env_* calls) fails with CHAN_EBUSY.  Calls on different
 * streams with disjoint envs run concurrently on the device; each call stages its launch
 * arguments in buffers of its own.  Errors: CHAN_EINVAL (n_substeps < 1, an env not in the
 * batch or listed twice), CHAN_EBUSY, CHAN_ESTATE (no listed env has a flow state), CHAN_ENOMEM,
 * CHAN_EDEVICE; nothing is queued then, and *out (if given) is NULL.
 *
 * chan_call_query: 1 while the call's work is still queued or running, 0 once it has finished
 * (does not block); CHAN_EINVAL for a null call.
 *
 * chan_call_finish waits for the call, applies each env's outcome (clock, step counter, a
 * poisoned state), writes the per-env codes to results (if non-NULL; as for chan_batch_step)
 * and frees the call; returns CHAN_OK if every env succeeded, else the first failing env's
 * code.  chan_batch_destroy finishes the batch's unfinished calls itself (each env's outcome
 * applied as by chan_call_finish) and frees them: their handles are invalid afterwards.
 *
 * chan_batch_add: env joins the batch (its grid shape's plane-pass tiling is tuned on it if the
 * shape is new to the batch; later channels of the shape reuse it).  chan_batch_remove: env
 * leaves the batch (not destroyed); later positions shift down by one.  Errors: CHAN_EINVAL
 * (null, another device, already a member / not a member), CHAN_EBUSY (held by a call). */
typedef struct chan_call chan_call;
int chan_batch_launch(struct chan_batch* batch, void* hip_stream, int32_t n, struct chan_env* const* envs,
                      const double* const* actions, int32_t n_substeps, double* const* obs, double* const* tau_w,
                      double* const* drag, struct chan_call** out);
int chan_call_query(const struct chan_call* call);
int chan_call_finish(struct chan_call* call, int32_t* results);
int chan_batch_add(struct chan_batch* batch, struct chan_env* env);
int chan_batch_remove(struct chan_batch* batch, struct chan_env* env);

/* ---- Captured env steps (HIP graphs) ----
 * A worker repeats the same EVOLVE request every env step (§3.3): the same channels, the same
 * action and output buffers, the same number of time steps.  chan_batch_capture records one such
 * env step of the batch's envs envs[0..n) (arguments as for chan_batch_launch) as a HIP graph of
 * its kernel launches and status read-back; the launch arguments are staged once, in buffers the
 * graph owns.  Nothing runs at capture time.  chan_env_capture does the same for one env on its
 * own (its action, outputs and n_substeps as for chan_env_step).
 * chan_graph_launch replays the step on hip_stream (any stream of the batch's device) and returns
 * a call like chan_batch_launch: the envs are held by it, and chan_call_query / chan_call_finish
 * complete it (clock, step counter, per-env codes).  The replay reads the actions the buffers
 * hold when the stream reaches it, so a worker refills its action buffer on that stream and
 * replays again; its results are bitwise those of chan_batch_launch with the same arguments.
 * reset, set_state and get_state of the envs between replays are allowed (the replay steps the
 * state the env holds then).  A graph has one replay in flight at a time.
 * Errors of capture: CHAN_EINVAL (as for chan_batch_launch), CHAN_EBUSY, CHAN_ESTATE (an env
 * without a valid flow state: every env must have one), CHAN_ENOMEM, CHAN_EDEVICE.  Errors of
 * launch: CHAN_ESTATE (an env now without a valid flow state or poisoned; an env has left the
 * batch or been destroyed since the capture; the batch has been destroyed: capture again),
 * CHAN_EBUSY (an env held by another call, or the graph's previous replay unfinished),
 * CHAN_ENOMEM, CHAN_EDEVICE; nothing is queued then.  On every failure of capture or launch
 * *out (if given) is NULL.
 * chan_graph_destroy finishes the graph's replay in flight, if any (its call handle is invalid
 * afterwards), and frees the graph; NULL is a no-op.  Destroying the batch (or, for
 * chan_env_capture, the env) leaves its graphs to be destroyed by the caller. */
typedef struct chan_graph chan_graph;
int chan_batch_capture(struct chan_batch* batch, int32_t n, struct chan_env* const* envs,
                       const double* const* actions, int32_t n_substeps, double* const* obs, double* const* tau_w,
                       double* const* drag, struct chan_graph** out);
int chan_env_capture(struct chan_env* env, const double* action, int32_t n_substeps, double* obs, double* tau_w,
                     double* drag, struct chan_graph** out);
int chan_graph_launch(struct chan_graph* graph, void* hip_stream, struct chan_call** out);
void chan_graph_destroy(struct chan_graph* graph);

/* ---- No allocation ----
 * For callers that cannot allocate device memory (code inside a tight serving loop, harnesses
 * that forbid hipMalloc): one env step of a flow state the caller owns, with no env object and
 * no hipMalloc, hipHostMalloc, hipFree or other device-allocating call.  The operator tables,
 * every work buffer and the launch arguments live in a static device array of 32 MiB inside the
 * library (one per device, held until the process ends), so only grids whose
 * chan_env_footprint_bytes is at most 32 MiB - 4 KiB run here (16x65x16 and 32x65x32 do,
 * 64x65x64 does not).  It runs the kernels of chan_env_step on the canonical state that
 * chan_env_set_state would make, so its results equal chan_env_set_state + chan_env_step +
 * chan_env_get_state bitwise.
 *   grid, opts   as for chan_env_create (opts NULL: the defaults).
 *   hip_stream   the hipStream_t (on the current device) all work is queued on.
 *   state        DEVICE pointer to state_doubles doubles in the exchange layout of
 *                chan_env_get_state: read, advanced n_substeps time steps, written back (t and
 *                the step counter advance too).
 *   action, n_substeps, obs, tau_w, drag   as for chan_env_step (device pointers).
 * Returns after the stream has finished the step.  The first call on a device for a grid and
 * physical parameters (box, viscosity, time step, forcing, geometry) computes the operator
 * tables on the host, in ordinary heap memory, and copies them into the array; later calls
 * with the same ones reuse them.  Calls on one device share the array, which keeps the last
 * call's contents: overlapping calls would race, so the library serialises the calls made on
 * one device (each holds a per-device lock until its stream has finished), and other work must
 * not use the array.
 * Errors: CHAN_EINVAL (bad grid or options, n_substeps < 1, NULL state, or a footprint above the
 * array; nothing done), CHAN_ENONFINITE (a non-finite value in the state or the action: the
 * state is left unchanged; or a non-finite state after the step: written back), CHAN_EDEVICE. */
int chan_step_static(const chan_grid_t* grid, const chan_opts_t* opts, void* hip_stream, double* state,
                     const double* action, int32_t n_substeps, double* obs, double* tau_w, double* drag);

/* Static string naming an error code. */
const char* chan_strerror(int code);

/* Detail of the last failure on the calling thread (the HIP call and its error
 * string, or the argument that was rejected); "" if none.  Valid until the next
 * call into the library on this thread. */
const char* chan_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CHANENV_H */
