"""The channel-flow DNS step, written out plainly (oracle).

TEST INFRASTRUCTURE: see ``oracle/__init__.py``.

What is computed (paper §3.1, §3.2, §4.1, plus the published methods the
paper's solver is built on, named where used):

* Velocity--vorticity form (Kim, Moin & Moser 1987).  For every wavenumber
  pair (alpha, beta) != (0, 0) the state is the Chebyshev coefficients of the
  wall-normal velocity v and the wall-normal vorticity omega_y; the (0, 0)
  pair carries the mean profiles U(y), W(y) instead.
* Non-linear term in rotational form H = u x omega, evaluated pseudo-
  spectrally: products on the Gauss--Lobatto nodes in y and on the 3/2-padded
  grid in x and z.
* h_v = -k^2 H_2 - D(i alpha H_1 + i beta H_3),  h_g = i beta H_1 - i alpha H_3;
  the mean flow is driven by H_1, H_3 of the (0, 0) pair.
* Three-stage RK3 for the explicit part and Crank--Nicolson for the viscous
  part (§3.1), with the coefficients of Spalart, Moser & Rogers (1991).
* Per stage: a Chebyshev-tau Helmholtz solve for phi = (D^2 - k^2) v and for
  omega_y, a second solve for v, and a 2x2 influence-matrix correction that
  imposes dv/dy = 0 at both walls while v itself takes the blowing/suction
  value at the lower wall (§3.2: control by a wall-normal velocity).
* Constant flow rate: a pressure gradient chosen every stage so that the bulk
  velocity stays at U_b.
* Geometry: the closed channel (walls at y = -1 and y = +1, half-height h = 1)
  or the open channel of the paper's setup (§3.1: a wall at the bottom, a
  free-slip surface at height h = 1 on top).  Both are discretised on the
  Chebyshev variable xi in [-1, 1]; the physical wall-normal coordinate is
  y = xi (closed) or y = (1 + xi)/2 (open), so d/dy = s d/dxi with s = 1 or 2.
  At a free-slip surface du/dy = dw/dy = 0 and v = 0, hence (continuity)
  d^2v/dy^2 = 0 and d omega_y / dy = 0.
* Control boundary condition at the lower wall y = -1 (§3.2): clipped to
  [-clip, clip] u_tau, zero net mass flux (the (0, 0) mode of v_w is zero,
  §4.1), ramped linearly from the old action to the new one over the
  actuation interval.  Opposition control (§4.1 equation) as the in-library
  controller: v_w = -alpha (v(y_s) - <v(y_s)>).
* Observation: velocity components on the wall-parallel plane at the first
  Chebyshev node at or above y_s^+ (§3.2 "rounded up to the closest Chebyshev
  colocation node"), and on further planes chosen the same way (§3.2: one or
  more wall-parallel planes).  Wall-shear stress at the lower wall, and the drag as
  its plane mean averaged over the time steps between two actions (§3.2).

Where the paper is silent the code states the reading it takes where it is
used.
"""
from dataclasses import dataclass

import numpy as np

from . import chebyshev as cheb
from . import fourier as fr
from .tau import tau_solve

# Spalart, Moser & Rogers (1991) low-storage RK3/CN coefficients.
RK_GAMMA = (8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0)
RK_ZETA = (0.0, -17.0 / 60.0, -5.0 / 12.0)
RK_ALPHA = (4.0 / 15.0, 1.0 / 15.0, 1.0 / 6.0)
RK_BETA = (4.0 / 15.0, 1.0 / 15.0, 1.0 / 6.0)
RK_C_END = (8.0 / 15.0, 2.0 / 3.0, 1.0)  # stage-end times as fractions of dt

TOP_WALL, TOP_FREESLIP = 0, 1
CFR, CPG = 0, 1
CTRL_EXTERNAL, CTRL_OPPOSITION = 0, 1
RAMP, HOLD = 0, 1
IC_LAMINAR, IC_REICHARDT = 0, 1


class NonFinite(Exception):
    """A non-finite action or state."""


@dataclass
class Config:
    nx: int
    ny: int
    nz: int
    lx: float
    lz: float
    re_tau: float
    dt_plus: float
    obs_y_plus: float
    top_bc: int = TOP_WALL
    forcing: int = CFR
    ub_plus: float = 0.0
    px: float = 0.0
    nu_override: float = 0.0
    dt_override: float = 0.0
    controller: int = CTRL_EXTERNAL
    opp_alpha: float = 1.0
    action_mode: int = RAMP
    clip: float = 1.0
    obs_mask: int = 3
    ic_profile: int = IC_LAMINAR
    ic_amp: float = 0.1
    extra_obs_y_plus: tuple = ()


def default_bulk_velocity(re_tau):
    """U_b^+ = 15.66 (Re_tau/180)^(1/7).

    15.66 is the bulk velocity for which the relaminarisation bound
    1 - 3 U_b^+ / Re_tau equals the 73.9 % quoted for Re_tau = 180 (§3.2);
    the 1/7 power is Dean's correlation for other Re_tau (a reading)."""
    return 15.66 * (re_tau / 180.0) ** (1.0 / 7.0)


class Setup:
    """Grid, constants and matrices derived from a Config."""

    def __init__(self, cfg: Config):
        if cfg.nx < 4 or cfg.nz < 4 or cfg.nx % 4 or cfg.nz % 4:
            raise ValueError("nx, nz must be positive multiples of 4")
        if cfg.ny < 5 or cfg.ny % 2 == 0:
            raise ValueError("ny must be odd and >= 5")
        if cfg.top_bc not in (TOP_WALL, TOP_FREESLIP):
            raise ValueError("top_bc must be TOP_WALL or TOP_FREESLIP")
        self.cfg = cfg
        self.nx, self.ny, self.nz = cfg.nx, cfg.ny, cfg.nz
        self.N = cfg.ny - 1
        self.nkx = cfg.nx // 2
        self.mx, self.mz = 3 * cfg.nx // 2, 3 * cfg.nz // 2
        self.nu = cfg.nu_override if cfg.nu_override > 0 else 1.0 / cfg.re_tau
        self.dt = cfg.dt_override if cfg.dt_override > 0 else cfg.dt_plus / cfg.re_tau
        self.ub = cfg.ub_plus if cfg.ub_plus > 0 else default_bulk_velocity(cfg.re_tau)
        self.alpha, self.beta = fr.wavenumbers(cfg.nx, cfg.nz, cfg.lx, cfg.lz)
        self.k2 = self.alpha[None, :] ** 2 + self.beta[:, None] ** 2
        q = np.arange(cfg.nz)
        self.active = (self.k2 > 0) & (q[:, None] != cfg.nz // 2)
        N = self.N
        self.open = cfg.top_bc == TOP_FREESLIP
        # d/dy = s d/dxi: y = xi (closed channel) or y = (1 + xi)/2 (open channel)
        self.s = 2.0 if self.open else 1.0
        self.y = cheb.nodes(N)  # the Chebyshev variable xi at the nodes
        self.C = cheb.forward_matrix(N)
        self.B = cheb.inverse_matrix(N)
        # derivatives with respect to the physical y
        self.D = self.s * cheb.derivative_matrix(N)
        self.D2 = self.s ** 2 * cheb.second_derivative_matrix(N)
        self.top_val = cheb.value_row(N, +1)
        self.bot_val = cheb.value_row(N, -1)
        self.top_slope = self.s * cheb.slope_row(N, +1)
        self.bot_slope = self.s * cheb.slope_row(N, -1)
        self.top_curv = self.top_val @ self.D2  # d^2/dy^2 at the top
        self.bot_curv = self.bot_val @ self.D2
        # integral over xi; the bulk velocity is its half in both geometries
        # (closed: int_{-1}^{1} dy / 2; open: int_0^1 dy = int dxi / 2)
        self.intw = cheb.integral_weights(N)
        self.wall_dist = (1.0 + self.y) / self.s  # distance from the lower wall
        self.js = observation_node(self.wall_dist, 1.0 / self.nu, cfg.obs_y_plus)
        self.y_plus_node = self.wall_dist[self.js] / self.nu
        # observation planes: the sensing plane first, then the extra ones in order
        self.js_planes = [self.js] + [observation_node(self.wall_dist, 1.0 / self.nu, yp)
                                      for yp in cfg.extra_obs_y_plus]

    def helmholtz(self, lam, f, g_top, g_bot, top="dirichlet", bot="dirichlet"):
        """Solve (d^2/dy^2 - lam) X = f with, at each end, X = g ("dirichlet") or
        dX/dy = g ("neumann").  In xi this is (D_xi^2 - lam/s^2) X = f/s^2 with
        dX/dxi = g/s."""
        s2 = self.s ** 2
        gt = g_top / self.s if top == "neumann" else g_top
        gb = g_bot / self.s if bot == "neumann" else g_bot
        return tau_solve(self.N, np.asarray(lam) / s2, np.asarray(f) / s2, gt, gb,
                         bc=(top, bot))


def observation_node(d, inv_nu, y_plus):
    """Index j of the sensing plane: the first node at or above y_s^+
    measured from the lower wall, i.e. the smallest wall distance d_j
    (1 + xi_j closed, (1 + xi_j)/2 open) with d_j / nu >= y_s^+ (§3.2,
    "rounded up")."""
    ok = np.nonzero(d * inv_nu >= y_plus)[0]
    if len(ok) == 0:
        raise ValueError("observation height above the channel")
    return int(ok[-1])


@dataclass
class State:
    v: np.ndarray      # (N_z, N_x/2, N_y) complex Chebyshev coefficients of v
    om: np.ndarray     # (N_z, N_x/2, N_y) complex Chebyshev coefficients of omega_y
    ubar: np.ndarray   # (N_y,) Chebyshev coefficients of the mean streamwise velocity
    wbar: np.ndarray   # (N_y,) Chebyshev coefficients of the mean spanwise velocity
    vw_old: np.ndarray  # (N_z, N_x/2) complex wall velocity of the previous action
    t: float = 0.0
    nstep: int = 0

    def copy(self):
        return State(self.v.copy(), self.om.copy(), self.ubar.copy(), self.wbar.copy(),
                     self.vw_old.copy(), self.t, self.nstep)


def zero_state(S: Setup):
    z = np.zeros((S.nz, S.nkx, S.ny), dtype=complex)
    return State(z.copy(), z.copy(), np.zeros(S.ny), np.zeros(S.ny),
                 np.zeros((S.nz, S.nkx), dtype=complex))


def state_to_flat(S: Setup, st: State):
    """The library's state exchange format (host doubles):
    v [q][p][n] (re, im), omega_y [q][p][n] (re, im), U [n], W [n],
    v_w,old [q][p] (re, im), t, step counter."""
    parts = [np.ascontiguousarray(st.v).view(float).ravel(),
             np.ascontiguousarray(st.om).view(float).ravel(), st.ubar, st.wbar,
             np.ascontiguousarray(st.vw_old).view(float).ravel(),
             np.array([st.t, float(st.nstep)])]
    return np.concatenate([np.ascontiguousarray(p, dtype=float).ravel() for p in parts])


def state_from_flat(S: Setup, flat):
    flat = np.asarray(flat, dtype=float)
    nspec = S.nz * S.nkx * S.ny * 2
    o = 0
    v = flat[o:o + nspec].copy().view(complex).reshape(S.nz, S.nkx, S.ny); o += nspec
    om = flat[o:o + nspec].copy().view(complex).reshape(S.nz, S.nkx, S.ny); o += nspec
    ubar = flat[o:o + S.ny].copy(); o += S.ny
    wbar = flat[o:o + S.ny].copy(); o += S.ny
    nw = S.nz * S.nkx * 2
    vw = flat[o:o + nw].copy().view(complex).reshape(S.nz, S.nkx); o += nw
    t = float(flat[o]); nstep = int(flat[o + 1]); o += 2
    if o != flat.size:
        raise ValueError("state size mismatch")
    return State(v, om, ubar, wbar, vw, t, nstep)


def state_size(S: Setup):
    return 4 * S.nz * S.nkx * S.ny + 2 * S.ny + 2 * S.nz * S.nkx + 2


# ---------------------------------------------------------------------------
# Reconstruction of all velocity and vorticity components.
# ---------------------------------------------------------------------------

def reconstruct(S: Setup, st: State):
    """Chebyshev coefficients of (u, v, w, omega_x, omega_y, omega_z).

    From continuity i alpha u + D v + i beta w = 0 and the definition
    omega_y = i beta u - i alpha w (Kim, Moin & Moser 1987):
      u = (i alpha Dv - i beta omega_y) / k^2,  w = (i beta Dv + i alpha omega_y) / k^2,
      omega_x = Dw - i beta v,  omega_z = i alpha v - Du.
    The (0, 0) pair: u = U, w = W, v = omega_y = 0, omega_x = DW, omega_z = -DU."""
    act = S.active[..., None]
    ia = 1j * S.alpha[None, :, None]
    ib = 1j * S.beta[:, None, None]
    k2 = np.where(S.active, S.k2, 1.0)[..., None]
    v = np.where(act, st.v, 0.0)
    om = np.where(act, st.om, 0.0)
    Dv = v @ S.D.T
    u = np.where(act, (ia * Dv - ib * om) / k2, 0.0)
    w = np.where(act, (ib * Dv + ia * om) / k2, 0.0)
    ox = w @ S.D.T - ib * v
    oz = ia * v - u @ S.D.T
    u[0, 0] = st.ubar
    w[0, 0] = st.wbar
    ox[0, 0] = S.D @ st.wbar
    oz[0, 0] = -(S.D @ st.ubar)
    return u, v, w, ox, om, oz


def nonlinear(S: Setup, st: State):
    """Chebyshev coefficients of H = u x omega (rotational form; the kinetic
    energy goes into the pressure, which the v--omega form never needs).

    Each of the six fields goes to the Gauss--Lobatto nodes in y (no
    dealiasing in y) and to the 3/2-padded grid in x and z, the products are
    formed pointwise, and the three products come back through the forward
    FFT, truncation to the stored modes, the Hermitian fix and the forward
    DCT-I."""
    phys = []
    for f in reconstruct(S, st):
        fy = np.moveaxis(f @ S.B.T, -1, 0)         # (N_y, N_z, N_x/2) at the nodes
        phys.append(fr.to_padded_physical(fy, S.mx, S.mz))
    U, V, W, OX, OY, OZ = phys
    H1 = V * OZ - W * OY
    H2 = W * OX - U * OZ
    H3 = U * OY - V * OX
    out = []
    for Hp in (H1, H2, H3):
        hh = fr.from_padded_physical(Hp, S.nx, S.nz)  # (N_y, N_z, N_x/2)
        out.append(np.moveaxis(hh, 0, -1) @ S.C.T)
    return out


def explicit_terms(S: Setup, H):
    """h_v = -k^2 H_2 - D(i alpha H_1 + i beta H_3),  h_g = i beta H_1 - i alpha H_3,
    and the mean-flow terms h_u = H_1(0,0), h_w = H_3(0,0)."""
    H1, H2, H3 = H
    ia = 1j * S.alpha[None, :, None]
    ib = 1j * S.beta[:, None, None]
    act = S.active[..., None]
    hv = np.where(act, -S.k2[..., None] * H2 - (ia * H1 + ib * H3) @ S.D.T, 0.0)
    hg = np.where(act, ib * H1 - ia * H3, 0.0)
    return hv, hg, H1[0, 0].real.copy(), H3[0, 0].real.copy()


# ---------------------------------------------------------------------------
# One Runge--Kutta / Crank--Nicolson stage.
# ---------------------------------------------------------------------------

def stage(S: Setup, st: State, r: int, hist, vw):
    """Advance the state through RK3/CN stage r (0, 1, 2).

    u^r = u^{r-1} + dt [a_r L u^{r-1} + b_r L u^r + g_r N^{r-1} + z_r N^{r-2}]
    with L = nu (D^2 - k^2).  Dividing by -b_r nu dt gives, for X = phi or
    omega_y, the Helmholtz problem
      (D^2 - lam_r) X^r = -X^{r-1}/(b_r nu dt) - (a_r/b_r)(D^2 - k^2) X^{r-1}
                          - (g_r h^{r-1} + z_r h^{r-2}) / (b_r nu),
    lam_r = k^2 + 1/(b_r nu dt).  phi^{r-1} = (D^2 - k^2) v^{r-1} is formed
    from the stored v.  ``hist`` is the previous stage's (h_v, h_g, h_u, h_w)
    (None at stage 0, where z_0 = 0).  ``vw`` (N_z, N_x/2) is the lower-wall
    velocity at this stage's end time.  Returns (new state, this stage's h)."""
    a_r, b_r, g_r, z_r = RK_ALPHA[r], RK_BETA[r], RK_GAMMA[r], RK_ZETA[r]
    nu, dt, N = S.nu, S.dt, S.N
    lam0 = 1.0 / (b_r * nu * dt)
    H = nonlinear(S, st)
    hv, hg, hu, hw = explicit_terms(S, H)
    if hist is None:
        hv_p, hg_p, hu_p, hw_p = 0.0 * hv, 0.0 * hg, 0.0, 0.0
    else:
        hv_p, hg_p, hu_p, hw_p = hist

    def L(X, k2):
        return X @ S.D2.T - k2[..., None] * X

    act = S.active
    k2a = S.k2[act]
    lam = k2a + lam0
    v = st.v[act]
    om = st.om[act]
    phi0 = L(v, k2a)
    rhs_phi = (-phi0 * lam0 - (a_r / b_r) * L(phi0, k2a)
               - (g_r * hv[act] + z_r * hv_p[act]) / (b_r * nu))
    rhs_om = (-om * lam0 - (a_r / b_r) * L(om, k2a)
              - (g_r * hg[act] + z_r * hg_p[act]) / (b_r * nu))

    # Particular solutions: phi_p with phi_p(+-1) = 0, omega with omega(-1) = 0 and
    # omega(+1) = 0 (wall) or d omega/dy (+1) = 0 (free slip), then v_p from
    # (D^2 - k^2) v_p = phi_p, v_p(+1) = 0, v_p(-1) = v_w.
    phi_p = S.helmholtz(lam, rhs_phi, 0.0, 0.0)
    om_new = S.helmholtz(lam, rhs_om, 0.0, 0.0, top="neumann" if S.open else "dirichlet")
    v_p = S.helmholtz(k2a, phi_p, 0.0, vw[act])
    # Homogeneous solutions (influence matrix, Kim, Moin & Moser 1987):
    # phi_+- solve (D^2 - lam) phi = 0 with phi(+-1) = 1, phi(-+1) = 0, and
    # v_+- solve (D^2 - k^2) v = phi_+- with v(+-1) = 0.
    zero = np.zeros((k2a.size, S.ny))
    phi_t = S.helmholtz(lam, zero, 1.0, 0.0)
    phi_b = S.helmholtz(lam, zero, 0.0, 1.0)
    v_t = S.helmholtz(k2a, phi_t, 0.0, 0.0)
    v_b = S.helmholtz(k2a, phi_b, 0.0, 0.0)
    # 2x2 influence matrix: choose c so that Dv(-1) = 0 and, at the top, Dv(+1) = 0
    # (wall) or D^2 v(+1) = 0 (free slip).
    top = S.top_curv if S.open else S.top_slope
    M = np.empty((k2a.size, 2, 2))
    M[:, 0, 0] = v_t @ top
    M[:, 0, 1] = v_b @ top
    M[:, 1, 0] = v_t @ S.bot_slope
    M[:, 1, 1] = v_b @ S.bot_slope
    g = -np.stack([v_p @ top, v_p @ S.bot_slope], axis=-1)
    c = np.linalg.solve(M, np.stack([g.real, g.imag], axis=-1))
    c = c[..., 0] + 1j * c[..., 1]
    v_new = v_p + c[:, 0, None] * v_t + c[:, 1, None] * v_b

    out = st.copy()
    out.v = np.zeros_like(st.v)
    out.om = np.zeros_like(st.om)
    out.v[act] = v_new
    out.om[act] = om_new
    out.v = fr.hermitian_fix_qpy(out.v)
    out.om = fr.hermitian_fix_qpy(out.om)

    # Mean flow.  U^r = U* + P^r U_P where U_P carries the stage's share
    # (a_r + b_r) dt of a unit pressure gradient; constant flow rate picks P^r
    # so that int U^r dxi = 2 U_b, constant pressure gradient uses P^r = P_x.
    # U = W = 0 at the wall(s); dU/dy = dW/dy = 0 at a free-slip top.
    top_mean = "neumann" if S.open else "dirichlet"
    rhs_u = -st.ubar * lam0 - (a_r / b_r) * (S.D2 @ st.ubar) - (g_r * hu + z_r * hu_p) / (b_r * nu)
    rhs_w = -st.wbar * lam0 - (a_r / b_r) * (S.D2 @ st.wbar) - (g_r * hw + z_r * hw_p) / (b_r * nu)
    ustar = S.helmholtz(lam0, rhs_u, 0.0, 0.0, top=top_mean)
    forcing = np.zeros(S.ny)
    forcing[0] = -(a_r + b_r) / (b_r * nu)
    u_P = S.helmholtz(lam0, forcing, 0.0, 0.0, top=top_mean)
    if S.cfg.forcing == CFR:
        P = (2.0 * S.ub - S.intw @ ustar) / (S.intw @ u_P)
    else:
        P = S.cfg.px
    out.ubar = ustar + P * u_P
    out.wbar = S.helmholtz(lam0, rhs_w, 0.0, 0.0, top=top_mean)
    return out, (hv, hg, hu, hw)


def time_step(S: Setup, st: State, wall):
    """One full RK3/CN time step; ``wall(r)`` gives v_w at stage r's end time."""
    hist = None
    for r in range(3):
        st, hist = stage(S, st, r, hist, wall(r))
    st.t += S.dt
    st.nstep += 1
    return st


# ---------------------------------------------------------------------------
# Wall actuation, observation, wall shear and drag.
# ---------------------------------------------------------------------------

def ingest_action(S: Setup, action):
    """Action field a[z, x] on the N_z x N_x wall grid -> spectral wall velocity.

    Clip to [-clip, clip] (§3.2), forward FFT, drop the Nyquist modes and set
    the (0, 0) mode to zero (zero net mass flux, §4.1).  Reading: clip first,
    then remove the mean."""
    a = np.asarray(action, dtype=float)
    if a.shape != (S.nz, S.nx):
        raise ValueError("action must have shape (nz, nx)")
    if not np.all(np.isfinite(a)):
        raise NonFinite("non-finite action")
    if S.cfg.clip > 0:
        a = np.clip(a, -S.cfg.clip, S.cfg.clip)
    ah = fr.from_physical(a)
    ah[0, 0] = 0.0
    return ah


def values_at_node(S: Setup, coeffs, j):
    """sum_n a_n T_n(y_j) for every wavenumber pair."""
    return coeffs @ S.B[j]


def opposition_wall(S: Setup, st: State):
    """Opposition control, §4.1: v_w = -alpha (v(y_s) - <v(y_s)>).

    In Fourier space the plane mean is the (0, 0) mode, so v_w-hat =
    -alpha v-hat(y_s) with the (0, 0) mode set to zero.  Evaluated once per
    time step and held over its three stages (reading); not clipped."""
    vs = values_at_node(S, np.where(S.active[..., None], st.v, 0.0), S.js)
    vw = -S.cfg.opp_alpha * vs
    vw[0, 0] = 0.0
    vw[S.nz // 2, :] = 0.0
    return fr.hermitian_fix_qp(vw)


def mean_wall_shear(S: Setup, st: State):
    """nu dU/dy at the lower wall: the plane mean of tau_w (units rho u_tau^2)."""
    return S.nu * (S.bot_slope @ st.ubar)


def wall_shear_field(S: Setup, st: State):
    """tau_w(x, z) = nu du/dy at the lower wall on the N_z x N_x grid."""
    u = reconstruct(S, st)[0]
    th = S.nu * (u @ S.bot_slope)
    return fr.to_physical(th, S.nx, S.nz)


def pressure_coefficients(S: Setup, st: State, dvw_dt):
    """Chebyshev coefficients of the total pressure P = p + |u|^2/2 for every
    wavenumber pair except (0, 0), whose plane means the observable removes.

    Rotational form of the momentum equation: du/dt = -grad P + H + nu lap u
    with H = u x omega.  Its divergence gives lap P = div H, i.e. per pair
      (D^2 - k^2) P = i alpha H_1 + D H_2 + i beta H_3,
    and its wall-normal component at the two boundaries gives the Neumann
    conditions
      dP/dy = H_2 + nu (D^2 - k^2) v - dv/dt,
    where dv/dt is the rate of the lower wall's velocity (``dvw_dt``, (N_z,
    N_x/2)) and zero at the top.  H is the state's own non-linear term (the
    plane pass of the next stage).  Tau method with both conditions as
    boundary rows."""
    H1, H2, H3 = nonlinear(S, st)
    act = S.active
    ia = 1j * S.alpha[None, :]
    ib = 1j * S.beta[:, None]
    k2 = S.k2[act]
    rhs = (ia[..., None] * H1 + H2 @ S.D.T + ib[..., None] * H3)[act]
    v = st.v[act]
    lapv_top = S.nu * (v @ S.top_curv - k2 * (v @ S.top_val))
    lapv_bot = S.nu * (v @ S.bot_curv - k2 * (v @ S.bot_val))
    g_top = H2[act] @ S.top_val + lapv_top
    g_bot = H2[act] @ S.bot_val + lapv_bot - dvw_dt[act]
    P = np.zeros_like(st.v)
    P[act] = S.helmholtz(k2, rhs, g_top, g_bot, top="neumann", bot="neumann")
    return P


def observation(S: Setup, st: State, dvw_dt=None):
    """Selected components (bit 0 u, bit 1 v, bit 2 w, bit 3 p) on each
    observation plane (node j_s first, then the extra planes), each on the
    N_z x N_x grid, stacked plane by plane and in that order within a plane.

    p is the static-pressure fluctuation p - <p> (the plane mean removed):
    p = P - |u|^2/2 evaluated pointwise on the plane's grid, P from
    ``pressure_coefficients``.  ``dvw_dt`` is the lower wall's velocity rate
    (zero if None)."""
    fields = reconstruct(S, st)
    want_p = bool(S.cfg.obs_mask & 8)
    if want_p:
        P = pressure_coefficients(S, st, np.zeros_like(st.vw_old) if dvw_dt is None else dvw_dt)
    comps = []
    for j in S.js_planes:
        phys = [fr.to_physical(values_at_node(S, f, j), S.nx, S.nz) for f in fields[:3]]
        for bit, f in zip((1, 2, 4), phys):
            if S.cfg.obs_mask & bit:
                comps.append(f)
        if want_p:
            Pj = fr.to_physical(values_at_node(S, P, j), S.nx, S.nz)   # (0, 0) pair is zero
            b = 0.5 * (phys[0] ** 2 + phys[1] ** 2 + phys[2] ** 2)
            comps.append(Pj - (b - b.mean()))
    return np.stack(comps) if comps else np.zeros((0, S.nz, S.nx))


def flow_rate(S: Setup, st: State):
    return S.intw @ st.ubar


class Env:
    """The environment semantics behind the library's C ABI, on the CPU.

    create -> Env(cfg); reset(seed) -> initial condition; step(action, n)
    -> (observation, tau_w field, drag)."""

    def __init__(self, cfg: Config):
        self.S = Setup(cfg)
        self.state = None

    def set_state(self, st: State):
        self.state = st.copy()

    def reset(self, seed):
        from .ic import initial_state
        self.state = initial_state(self.S, seed)

    def step(self, action, n_substeps):
        S = self.S
        if self.state is None:
            raise RuntimeError("step before reset")
        if n_substeps < 1:
            raise ValueError("n_substeps must be >= 1")
        st = self.state
        ext = S.cfg.controller == CTRL_EXTERNAL
        if ext:
            vw_new = ingest_action(S, action) if action is not None else np.zeros_like(st.vw_old)
        vw_old = st.vw_old.copy()
        drags = []
        for m in range(n_substeps):
            if ext:
                if S.cfg.action_mode == HOLD:
                    def wall(r):
                        return vw_new
                else:
                    def wall(r, m=m):
                        s = (m + RK_C_END[r]) / n_substeps
                        return vw_old + s * (vw_new - vw_old)
            else:
                vw_opp = opposition_wall(S, st)

                def wall(r):
                    return vw_opp
            st = time_step(S, st, wall)
            drags.append(mean_wall_shear(S, st))
        if ext:
            st.vw_old = vw_new
        if not (np.all(np.isfinite(st.v)) and np.all(np.isfinite(st.om))
                and np.all(np.isfinite(st.ubar))):
            self.state = st
            raise NonFinite("non-finite state")
        self.state = st
        drag = 0.0
        for d in drags:
            drag += d
        drag /= n_substeps
        # rate of the lower wall's velocity at the end of the env step: the ramp's slope
        # (held actions and opposition control are constant over the last time step)
        dvw_dt = np.zeros_like(st.vw_old)
        if ext and S.cfg.action_mode == RAMP:
            dvw_dt = (vw_new - vw_old) / (n_substeps * S.dt)
        return observation(S, st, dvw_dt), wall_shear_field(S, st), drag
