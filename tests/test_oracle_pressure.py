"""Pins for the pressure observable of oracle/channel.py (static-pressure fluctuation on the
observation planes): the closed-form pressure of the unsteady-Stokes eigenmodes, zero
pressure fluctuation for the exact non-linear decaying mode, and the wall-normal momentum
balance dv/dt = -dP/dy + H_2 + nu lap v checked against the time stepper itself, with a
ramped wall velocity, at interior nodes."""
import numpy as np
import pytest

from oracle import channel as ch
from oracle.ic import initial_state
from tests.oracle_cases import minimal_channel, stokes_p, stokes_profile, tiny


def stokes_pressure(k, p, parity, y, amp):
    """Pressure of the v-mode amp * stokes_profile: from the x-momentum balance,
    p = sigma amp C sinh(k y)/k (even, C = cos p/cosh k) or sigma amp S cosh(k y)/k
    (odd, S = sin p/sinh k), sigma = -nu (k^2 + p^2) without the factor nu."""
    if parity == "even":
        return amp * np.cos(p) / np.cosh(k) * np.sinh(k * y) / k
    return amp * np.sin(p) / np.sinh(k) * np.cosh(k * y) / k


@pytest.mark.parametrize("parity,top", [("even", ch.TOP_WALL), ("odd", ch.TOP_WALL),
                                         ("odd", ch.TOP_FREESLIP)])
def test_stokes_mode_pressure(parity, top):
    """A small Stokes eigenmode in v (x-wavenumber alpha_1) and its pressure on three planes;
    in the open channel the odd mode's lower half.  The Bernoulli term is O(eps^2), 1e-10 of
    the pressure here."""
    cfg = tiny(nx=4, nz=4, ny=49, lx=2 * np.pi, forcing=ch.CPG, px=0.0, nu_override=0.01,
               dt_override=0.01, obs_mask=8, top_bc=top, obs_y_plus=1.0,
               extra_obs_y_plus=(0.2, 0.6, 0.95))
    S = ch.Setup(cfg)
    k = S.alpha[1]
    p = stokes_p(k, parity)
    eps = 1e-10
    yc = S.y if top == ch.TOP_WALL else (1 + S.y) / 2 - 1.0   # closed-channel coordinate
    st = ch.zero_state(S)
    st.v[0, 1] = S.C @ (eps / 2 * stokes_profile(k, p, parity, yc))
    sigma = -S.nu * (k * k + p * p)
    obs = ch.observation(S, st)
    x = np.arange(S.nx) * cfg.lx / S.nx
    for n, j in enumerate(S.js_planes):
        ref = 2 * sigma * stokes_pressure(k, p, parity, yc[j], eps / 2) * np.cos(k * x)
        ref = np.broadcast_to(ref, (S.nz, S.nx))
        assert np.abs(obs[n] - ref).max() < 1e-8 * np.abs(ref).max(), (n, j)
    assert np.abs(obs).max() > 0


@pytest.mark.parametrize("top", [ch.TOP_WALL, ch.TOP_FREESLIP], ids=["closed", "open"])
@pytest.mark.parametrize("direction", ["u(y,z)", "w(x,y)"])
def test_pressure_fluctuation_of_the_exact_decaying_modes_is_zero(direction, top):
    """u = A s(y) cos(beta z) x-hat, or w = A s(y) cos(alpha x) z-hat, with s = sin(pi (1+y))
    (closed) or sin(3 pi y/2) (open, zero slope at the surface): u x omega = grad(|u|^2/2)
    (H_2, H_3 or H_1, H_2 non-zero), so P = |u|^2/2 + const and the static pressure is uniform
    on every plane."""
    cfg = tiny(nx=8, nz=8, ny=49, lx=2.0, lz=1.3, forcing=ch.CPG, px=0.0, nu_override=0.01,
               dt_override=0.01, obs_mask=13, obs_y_plus=50.0, extra_obs_y_plus=(20.0, 90.0),
               top_bc=top)
    S = ch.Setup(cfg)
    st = ch.zero_state(S)
    shape = (np.sin(np.pi * (1 + S.y)) if top == ch.TOP_WALL
             else np.sin(1.5 * np.pi * (1 + S.y) / 2))
    prof = S.C @ (1.5 * shape)
    if direction == "u(y,z)":   # omega_y = du/dz
        st.om[1, 0] = 1j * S.beta[1] * prof / 2
        st.om[S.nz - 1, 0] = np.conj(st.om[1, 0])
    else:                       # omega_y = -dw/dx
        st.om[0, 1] = -1j * S.alpha[1] * prof / 2
    obs = ch.observation(S, st).reshape(3, 3, S.nz, S.nx)   # [plane][u, w, p]
    vel = obs[:, :2]
    pr = obs[:, 2]
    assert np.abs(vel).max() > 0.5
    assert np.abs(pr).max() < 1e-12 * np.abs(vel).max() ** 2


@pytest.mark.parametrize("top", [ch.TOP_WALL, ch.TOP_FREESLIP])
def test_wall_normal_momentum_balance(top):
    """Over one short time step of the stepper, (v(t + dt) - v(t))/dt equals the mean of
    -dP/dy + H_2 + nu (D^2 - k^2) v at t and t + dt at interior nodes, with the lower wall's
    velocity ramped during the step (which enters P through dP/dy at the wall).  A loose
    pin of the wall-rate reading; the Stokes modes pin the rest to 1e-8."""
    cfg = minimal_channel(top_bc=top, dt_override=2e-6, nu_override=1 / 180.0)
    S = ch.Setup(cfg)
    st0 = initial_state(S, 5)
    rng = np.random.default_rng(3)
    a = rng.standard_normal((S.nz, S.nx)) * 0.3
    vw_new = ch.ingest_action(S, a)
    vw_old = np.zeros_like(vw_new)
    rate = (vw_new - vw_old) / S.dt

    def wall(r):
        return vw_old + ch.RK_C_END[r] * (vw_new - vw_old)

    st1 = ch.time_step(S, st0.copy(), wall)

    def rhs(st, dvw):
        P = ch.pressure_coefficients(S, st, dvw)
        H1, H2, H3 = ch.nonlinear(S, st)
        lapv = st.v @ S.D2.T - S.k2[..., None] * st.v
        f = -(P @ S.D.T) + H2 + S.nu * lapv
        return np.where(S.active[..., None], f, 0.0) @ S.B.T     # at the nodes

    dvdt = (st1.v - st0.v) / S.dt @ S.B.T
    inner = slice(2, S.N - 1)
    scale = np.abs(dvdt[..., inner]).max()

    def misfit(rate_used):
        mid = 0.5 * (rhs(st0, rate_used) + rhs(st1, rate_used))
        return np.abs(dvdt[..., inner] - mid[..., inner]).max() / scale

    # measured 2.0 % (closed) and 1.1 % (open): the discrete scheme's own residual (at this
    # tiny dt the influence-matrix solutions have boundary layers far thinner than the grid)
    assert misfit(rate) < 0.05
    # without the wall-rate term, or with its sign flipped, the balance fails by O(1)
    assert misfit(0 * rate) > 0.3
    assert misfit(-rate) > 0.3
