"""Pins for the open channel (free-slip top, the geometry of §3.1) in oracle/channel.py.

The open channel of height h = 1 is the lower half of a closed channel of half-height 1
whose flow is mirror-symmetric about the centreline (u, w even and v odd in y): the
symmetry plane carries exactly the free-slip conditions.  The closed channel is pinned
independently (test_oracle_step.py), so evolving both from the same field is a check of
every open-channel term: the factor 2 of d/dy in the Chebyshev variable, the Neumann
conditions of omega_y and the mean flow, the d^2v/dy^2 = 0 row of the influence matrix,
the bulk velocity and the wall shear.  The closed forms below pin the same paths one at
a time."""
import numpy as np
import numpy.polynomial.chebyshev as npc
import pytest

from oracle import channel as ch
from oracle.ic import initial_state, volume_rms
from tests.oracle_cases import minimal_channel, rk_amplification, stokes_p, stokes_profile, tiny


def open_cfg(**kw):
    return tiny(top_bc=ch.TOP_FREESLIP, **kw)


def y_open(S):
    """Physical wall-normal coordinate of the open channel's nodes, 0 at the wall."""
    return (1.0 + S.y) / 2.0


@pytest.mark.parametrize("forcing", [ch.CPG, ch.CFR])
def test_open_laminar_profile_is_steady(forcing):
    """U = U_s (2y - y^2) on 0 <= y <= 1 (U = 0 at the wall, dU/dy = 0 at the surface) is
    an exact steady state: CPG with P_x = 2 nu U_s, CFR with U_b = 2 U_s / 3."""
    us = 15.0
    cfg = open_cfg(forcing=forcing, ub_plus=2 * us / 3, px=2 * (1 / 180.0) * us)
    S = ch.Setup(cfg)
    y = y_open(S)
    st = ch.zero_state(S)
    st.ubar = S.C @ (us * (2 * y - y * y))
    ref = st.ubar.copy()
    zero = np.zeros((S.nz, S.nkx), dtype=complex)
    for _ in range(100):
        st = ch.time_step(S, st, lambda r: zero)
    assert np.abs(st.ubar - ref).max() < 1e-12 * us
    # laminar wall shear nu dU/dy(0) = 2 nu U_s = 3 nu U_b
    assert np.isclose(ch.mean_wall_shear(S, st), 2 * S.nu * us, rtol=1e-12)


@pytest.mark.parametrize("m", [0, 1, 2])
def test_open_exact_decaying_mode(m):
    """u = A sin((m + 1/2) pi y) cos(beta z), v = w = 0 meets u = 0 at the wall and du/dy = 0
    at the surface and solves the Navier--Stokes equations exactly (u x omega is a
    gradient), decaying at sigma = -nu (beta^2 + ((m + 1/2) pi)^2)."""
    cfg = open_cfg(nx=4, nz=8, ny=49, lz=1.3, forcing=ch.CPG, px=0.0, nu_override=0.01,
                   dt_override=0.01)
    S = ch.Setup(cfg)
    st = ch.zero_state(S)
    A = 1.5
    kap = (m + 0.5) * np.pi
    prof = S.C @ (A * np.sin(kap * y_open(S)))
    beta = S.beta[1]
    st.om[1, 0] = 1j * beta * prof / 2
    st.om[S.nz - 1, 0] = np.conj(st.om[1, 0])
    ref0 = st.om.copy()
    G = rk_amplification(S.dt, -S.nu * (beta ** 2 + kap ** 2))
    zero = np.zeros((S.nz, S.nkx), dtype=complex)
    n = 40
    for _ in range(n):
        st = ch.time_step(S, st, lambda r: zero)
    assert np.abs(st.om - ref0 * G ** n).max() < 1e-12 * np.abs(ref0).max()
    assert np.abs(st.v).max() < 1e-12 * np.abs(ref0).max()
    assert abs(G ** n - 1.0) > 1e-2


def test_open_stokes_mode_decay():
    """The odd unsteady-Stokes eigenmode of the closed channel (sin/sinh pair) restricted to
    its lower half is an eigenmode of the open channel: v = dv/dy = 0 at the wall and
    v = d^2v/dy^2 = 0 at the surface.  Pins the influence-matrix row d^2v/dy^2(top) = 0."""
    cfg = open_cfg(nx=4, nz=4, ny=49, lx=2 * np.pi, forcing=ch.CPG, px=0.0, nu_override=0.01,
                   dt_override=0.01)
    S = ch.Setup(cfg)
    k = S.alpha[1]
    p = stokes_p(k, "odd")
    eps = 1e-8
    st = ch.zero_state(S)
    st.v[0, 1] = S.C @ (eps / 2 * stokes_profile(k, p, "odd", y_open(S) - 1.0))
    ref = st.v[0, 1].copy()
    G = rk_amplification(S.dt, -S.nu * (k * k + p * p))
    zero = np.zeros((S.nz, S.nkx), dtype=complex)
    n = 50
    for _ in range(n):
        st = ch.time_step(S, st, lambda r: zero)
    err = np.abs(st.v[0, 1] - ref * G ** n).max() / np.abs(ref).max()
    assert err < 1e-10
    assert abs(G ** n - 1.0) > 1e-2


def mirrored_pair(forcing=ch.CFR):
    """A mirror-symmetric closed-channel state and the open-channel state that is its lower
    half (same nu, dt, U_b; the open channel's nodes are the closed channel's points
    y_c = y_open - 1)."""
    common = dict(nx=8, nz=8, lx=2.0, lz=1.0, forcing=forcing, nu_override=0.05,
                  dt_override=0.00125, ub_plus=1.0, px=0.15)
    Sc = ch.Setup(ch.Config(ny=65, re_tau=180.0, dt_plus=0.05, obs_y_plus=15.0, **common))
    So = ch.Setup(ch.Config(ny=41, re_tau=180.0, dt_plus=0.05, obs_y_plus=15.0,
                            top_bc=ch.TOP_FREESLIP, **common))
    sc = initial_state(Sc, 7)
    n = np.arange(Sc.ny)
    sc.v[..., n % 2 == 0] = 0.0     # v odd in y
    sc.om[..., n % 2 == 1] = 0.0    # omega_y even
    sc.ubar[n % 2 == 1] = 0.0
    so = restrict(Sc, So, sc)
    return Sc, So, sc, so


def restrict(Sc, So, sc):
    """Open-channel coefficients of the closed state's lower half."""
    T = npc.chebvander(y_open(So) - 1.0, Sc.N)   # T_n(y_c) at the open nodes
    so = ch.zero_state(So)
    so.v = (sc.v @ T.T) @ So.C.T
    so.om = (sc.om @ T.T) @ So.C.T
    so.ubar = So.C @ (T @ sc.ubar)
    so.wbar = So.C @ (T @ sc.wbar)
    return so


def test_open_channel_is_the_half_of_a_mirrored_closed_channel():
    """Non-linear evolution: after 40 time steps the open channel equals the lower half of
    the mirror-symmetric closed channel field by field, and the wall shear agrees.

    The two are different discretisations of the same flow (65 Chebyshev nodes over the
    closed channel, 41 over the open one), so they agree to the spatial truncation error
    and to what Crank--Nicolson leaves of their different stiff modes; the latter shrinks
    fast with dt (measured differences of u relative to its change: 7e-6 at dt = 0.005,
    1e-6 at 0.0025, 9e-9 at 0.00125, the step used here)."""
    Sc, So, sc, so = mirrored_pair(ch.CFR)
    # the restriction is exact at t = 0 (polynomials of low degree)
    again = restrict(Sc, So, sc)
    assert np.abs(again.v - so.v).max() == 0
    zc = np.zeros((Sc.nz, Sc.nkx), dtype=complex)
    u0 = [f.copy() for f in ch.reconstruct(So, so)[:3]]
    tau0 = ch.wall_shear_field(So, so)
    for _ in range(40):
        sc = ch.time_step(Sc, sc, lambda r: zc)
        so = ch.time_step(So, so, lambda r: zc)
    # the closed flow stays mirror-symmetric
    n = np.arange(Sc.ny)
    assert np.abs(sc.v[..., n % 2 == 0]).max() < 1e-13 * np.abs(sc.v).max()
    ref = restrict(Sc, So, sc)
    uc = ch.reconstruct(So, ref)[:3]
    uo = ch.reconstruct(So, so)[:3]
    for a, b, a0 in zip(uc, uo, u0):
        change = np.abs(a - a0).max()
        assert change > 1e-2 * np.abs(a0).max()      # the flow has evolved
        assert np.abs(a - b).max() < 1e-7 * change
    assert np.abs(ref.ubar - so.ubar).max() < 1e-10 * np.abs(so.ubar).max()
    assert np.isclose(ch.mean_wall_shear(Sc, sc), ch.mean_wall_shear(So, so), rtol=1e-10)
    tc, to = ch.wall_shear_field(Sc, sc), ch.wall_shear_field(So, so)
    assert np.abs(tc - to).max() < 1e-4 * np.abs(tc - tau0).max()


def test_open_wall_and_surface_conditions_after_a_stage():
    """After any stage: v(0) = v_w, dv/dy(0) = 0, omega_y(0) = 0 at the wall; v = 0,
    d^2v/dy^2 = 0, d omega_y/dy = 0, dU/dy = dW/dy = 0 at the surface."""
    S = ch.Setup(minimal_channel(top_bc=ch.TOP_FREESLIP))
    st = initial_state(S, 2)
    rng = np.random.default_rng(0)
    vw = ch.ingest_action(S, rng.standard_normal((S.nz, S.nx)) * 0.3)
    out, _ = ch.stage(S, st, 0, None, vw)
    sv, so = np.abs(out.v).max(), np.abs(out.om).max()
    assert np.abs(out.v @ S.bot_val - np.where(S.active, vw, 0)).max() < 1e-12 * sv
    assert np.abs(out.v @ S.bot_slope).max() < 1e-9 * sv
    assert np.abs(out.v @ S.top_val).max() < 1e-12 * sv
    assert np.abs(out.v @ S.top_curv).max() < 1e-7 * sv
    assert np.abs(out.om @ S.bot_val).max() < 1e-12 * so
    assert np.abs(out.om @ S.top_slope).max() < 1e-9 * so
    assert abs(out.ubar @ S.top_slope) < 1e-9 * np.abs(out.ubar).max()
    assert abs(out.ubar @ S.bot_val) < 1e-12 * np.abs(out.ubar).max()


def test_open_initial_condition_and_sensing_node():
    """Seeded IC of the open channel: surface and wall conditions, bulk velocity, rms;
    the sensing node is the first node at or above y+ with y = (1 + xi)/2."""
    S = ch.Setup(minimal_channel(top_bc=ch.TOP_FREESLIP, ic_profile=ch.IC_REICHARDT))
    st = initial_state(S, 0)
    assert np.isclose(volume_rms(S, st), 0.1 * 1.5 * S.ub, rtol=1e-13)
    assert np.isclose(S.intw @ st.ubar, 2 * S.ub, rtol=1e-14)
    for f in (st.v, st.om):
        assert np.abs(f @ S.bot_val).max() < 1e-13
    assert np.abs(st.v @ S.top_val).max() < 1e-13
    assert np.abs(st.v @ S.bot_slope).max() < 1e-10
    # the curvature row's weights reach 4 N^2 (N^2 - 1)/3: compare with its rounding scale
    assert np.abs(st.v @ S.top_curv).max() < 1e-13 * np.abs(S.top_curv).sum() * np.abs(st.v).max()
    assert np.abs(st.om @ S.top_slope).max() < 1e-10
    d = (1 + S.y) / 2
    assert d[S.js] * 180 >= 15 > d[S.js + 1] * 180
    assert np.isclose(S.y_plus_node, d[S.js] * 180, rtol=1e-14)
    # half the closed channel's wall distance at the same node index
    Sc = ch.Setup(minimal_channel())
    assert S.js < Sc.js
