"""Pins for oracle/channel.py against closed forms, invariants and published values.

Each test names the fact it checks.  A plausible slip in the oracle (a dropped
term, a sign, a transposed index) changes at least one of these."""
import json
import os

import numpy as np
import numpy.polynomial.chebyshev as npc
import pytest

from oracle import channel as ch
from oracle import fourier as fr
from oracle.ic import SplitMix64, initial_state, volume_rms
from tests.oracle_cases import (minimal_channel, orr_sommerfeld_mode, rk_amplification,
                                stokes_p, stokes_profile, tiny)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def chebder_last(a, m=1):
    """Derivative along the last axis with numpy.polynomial (independent of the oracle)."""
    out = np.zeros_like(a)
    d = npc.chebder(np.moveaxis(a, -1, 0), m)
    out[..., :a.shape[-1] - m] = np.moveaxis(d, 0, -1)
    return out


def test_splitmix64_published_vectors():
    g = golden("splitmix64_seed1234567.json")
    r = SplitMix64(g["seed"])
    assert [r.next() for _ in range(5)] == [int(x) for x in g["outputs"]]


def test_observation_node_rounds_up():
    S = ch.Setup(minimal_channel())
    assert S.js == 55
    assert abs(S.y_plus_node - 180 * (1 - np.cos(9 * np.pi / 64))) < 1e-12
    assert abs(S.y_plus_node - 17.28) < 5e-3
    # the node below is under y+ = 15, the chosen one at or above it
    assert (1 + S.y[S.js + 1]) * 180 < 15 <= (1 + S.y[S.js]) * 180
    # a height exactly on a node selects that node
    yp = (1 + S.y[50]) * 180
    S2 = ch.Setup(minimal_channel(obs_y_plus=yp))
    assert S2.js == 50


def test_extra_observation_planes():
    """Each extra plane is rounded up to a node like the sensing plane; the observation is the
    sensing plane's block followed by one block per extra plane, each the components' values at
    that node (checked against numpy's Chebyshev series and FFT, not the oracle's helpers)."""
    cfg = minimal_channel(obs_mask=7, extra_obs_y_plus=(5.0, 40.0, 179.0))
    S = ch.Setup(cfg)
    d = 1 + S.y
    for j, yp in zip(S.js_planes[1:], cfg.extra_obs_y_plus):
        assert d[j] * 180 >= yp > d[j + 1] * 180
    st = initial_state(S, 4)
    obs = ch.observation(S, st)
    assert obs.shape == (12, S.nz, S.nx)
    one = ch.observation(ch.Setup(minimal_channel(obs_mask=7)), st)
    assert np.array_equal(obs[:3], one)
    u, v, w = ch.reconstruct(S, st)[:3]
    for k, j in enumerate(S.js_planes):
        for c, f in enumerate((u, v, w)):
            spec = npc.chebval(S.y[j], np.moveaxis(f, -1, 0))     # (nz, nkx) at node j
            phys = np.fft.irfft2(spec, s=(S.nz, S.nx)) * S.nx * S.nz  # Nyquist column zero
            assert np.abs(obs[3 * k + c] - phys).max() < 1e-12 * max(1.0, np.abs(phys).max())


def test_reconstruction_is_divergence_free():
    S = ch.Setup(minimal_channel())
    st = initial_state(S, 3)
    u, v, w, ox, oy, oz = ch.reconstruct(S, st)
    ia = 1j * S.alpha[None, :, None]
    ib = 1j * S.beta[:, None, None]
    div = ia * u + chebder_last(v) + ib * w
    scale = np.abs(u).max() * max(S.alpha.max(), np.abs(S.beta).max())
    assert np.abs(div).max() < 1e-13 * scale
    act = S.active[..., None]
    assert np.abs(np.where(act, ib * u - ia * w - oy, 0)).max() < 1e-13 * scale
    # omega_x, omega_z from their definitions with an independent derivative
    assert np.abs(ox - (chebder_last(w) - ib * v)).max() < 1e-11 * scale
    assert np.abs(oz - (ia * v - chebder_last(u))).max() < 1e-11 * scale


def test_initial_condition_invariants():
    S = ch.Setup(minimal_channel())
    st = initial_state(S, 0)
    assert np.isclose(volume_rms(S, st), 0.1 * 1.5 * S.ub, rtol=1e-13)
    assert np.isclose(S.intw @ st.ubar, 2 * S.ub, rtol=1e-14)
    for f in (st.v, st.om):
        assert np.abs(f @ S.top_val).max() < 1e-13 and np.abs(f @ S.bot_val).max() < 1e-13
    assert np.abs(st.v @ S.top_slope).max() < 1e-11 and np.abs(st.v @ S.bot_slope).max() < 1e-11
    # p = 0 column Hermitian, Nyquist row zero
    for q in range(1, S.nz // 2):
        assert np.all(st.v[S.nz - q, 0] == np.conj(st.v[q, 0]))
    assert np.all(st.v[S.nz // 2] == 0)
    # different seeds differ, same seed repeats
    assert not np.allclose(initial_state(S, 1).v, st.v)
    assert np.array_equal(initial_state(S, 0).v, st.v)


@pytest.mark.parametrize("forcing", [ch.CPG, ch.CFR])
def test_laminar_poiseuille_is_steady(forcing):
    """U = U_cl (1 - y^2) is an exact steady state: CPG with P_x = 2 nu U_cl,
    CFR with U_b = 2 U_cl / 3."""
    cfg = tiny(forcing=forcing, ub_plus=10.0, px=2 * (1 / 180.0) * 15.0)
    S = ch.Setup(cfg)
    st = ch.zero_state(S)
    ucl = 15.0
    st.ubar = np.zeros(S.ny)
    st.ubar[0] = ucl / 2
    st.ubar[2] = -ucl / 2
    ref = st.ubar.copy()
    zero = np.zeros((S.nz, S.nkx), dtype=complex)
    for _ in range(200):
        st = ch.time_step(S, st, lambda r: zero)
    assert np.abs(st.ubar - ref).max() < 1e-13 * ucl
    assert np.abs(st.v).max() == 0 and np.abs(st.om).max() == 0


def test_laminar_wall_shear_gives_paper_relaminarisation_bound():
    """Laminar CFR flow: tau_w = 3 nu U_b everywhere, so DR = 1 - 3 U_b^+/Re_tau
    equals the 73.9 % printed for Re_tau = 180 (§3.2)."""
    g = golden("paper_values.json")["relaminarisation_bound"]
    S = ch.Setup(minimal_channel())
    st = ch.zero_state(S)
    st.ubar = S.C @ (1.5 * S.ub * (1 - S.y ** 2))
    tau = ch.mean_wall_shear(S, st)
    assert np.isclose(tau, 3 * S.nu * S.ub, rtol=1e-13)
    assert round(1.0 - tau, 3) == g["value"]
    field = ch.wall_shear_field(S, st)
    assert np.allclose(field, tau, rtol=1e-13)


@pytest.mark.parametrize("m", [1, 2, 3])
def test_exact_nonlinear_decaying_mode(m):
    """u = A sin(m pi (1+y)/2) cos(beta z), v = w = 0 with no mean flow is an
    exact solution of the Navier--Stokes equations (u x omega is a gradient),
    decaying at sigma = -nu (beta^2 + (m pi / 2)^2); after n steps the
    amplitude is A G^n with G the RK3/CN factor of sigma."""
    cfg = tiny(nx=4, nz=8, ny=49, lz=1.3, forcing=ch.CPG, px=0.0, nu_override=0.01, dt_override=0.01)
    S = ch.Setup(cfg)
    st = ch.zero_state(S)
    A = 1.5
    prof = S.C @ (A * np.sin(m * np.pi * (1 + S.y) / 2))
    beta = S.beta[1]
    # u-hat(q = +-1) = A/2 prof ; omega_y = i beta u
    st.om[1, 0] = 1j * beta * prof / 2
    st.om[S.nz - 1, 0] = np.conj(st.om[1, 0])
    ref0 = st.om.copy()
    sigma = -S.nu * (beta ** 2 + (m * np.pi / 2) ** 2)
    G = rk_amplification(S.dt, sigma)
    zero = np.zeros((S.nz, S.nkx), dtype=complex)
    n = 40
    for _ in range(n):
        st = ch.time_step(S, st, lambda r: zero)
    assert np.abs(st.om - ref0 * G ** n).max() < 1e-12 * np.abs(ref0).max()
    assert np.abs(st.v).max() < 1e-12 * np.abs(ref0).max()
    assert np.abs(st.ubar).max() < 1e-12 and np.abs(st.wbar).max() < 1e-12
    # and G approaches exp(sigma dt) to third order... at least to O(dt^2)
    assert abs(G - np.exp(sigma * S.dt)) < (abs(sigma) * S.dt) ** 3


@pytest.mark.parametrize("parity", ["even", "odd"])
def test_stokes_mode_decay(parity):
    """Small 2-D unsteady-Stokes eigenmode of the channel: v = A cos py + B cosh ky
    (even) or the sin/sinh pair (odd), v = dv/dy = 0 at the walls, decaying at
    sigma = -nu (k^2 + p^2).  Exercises the phi--v split and the influence
    matrix; the self-interaction enters at O(eps^2)."""
    cfg = tiny(nx=4, nz=4, ny=49, lx=2 * np.pi, forcing=ch.CPG, px=0.0, nu_override=0.01,
               dt_override=0.01)
    S = ch.Setup(cfg)
    k = S.alpha[1]
    p = stokes_p(k, parity)
    eps = 1e-8
    st = ch.zero_state(S)
    st.v[0, 1] = S.C @ (eps / 2 * stokes_profile(k, p, parity, S.y))
    ref = st.v[0, 1].copy()
    sigma = -S.nu * (k * k + p * p)
    G = rk_amplification(S.dt, sigma)
    zero = np.zeros((S.nz, S.nkx), dtype=complex)
    n = 50
    for _ in range(n):
        st = ch.time_step(S, st, lambda r: zero)
    err = np.abs(st.v[0, 1] - ref * G ** n).max() / np.abs(ref).max()
    assert err < 1e-10
    assert abs(G ** n - 1.0) > 1e-2  # the test is not vacuous


def test_orr_sommerfeld_growth_rate():
    """Plane Poiseuille flow at Re = 10^4, alpha = 1: the least-stable 2-D mode
    grows at alpha c_i = 0.00373967 (Orszag 1971).  Pins the v--omega coupling
    with a mean shear, the non-linear term's linearisation and the time
    integrator together."""
    g = golden("paper_values.json")["orr_sommerfeld_re1e4_alpha1"]
    re = 1.0e4
    cfg = ch.Config(nx=4, ny=65, nz=4, lx=2 * np.pi, lz=1.0, re_tau=180.0, dt_plus=0.05,
                    obs_y_plus=15.0, forcing=ch.CPG, px=2.0 / re, nu_override=1.0 / re,
                    dt_override=0.01)
    S = ch.Setup(cfg)
    lam, phi = orr_sommerfeld_mode(S.N, re, 1.0)
    assert abs(lam.real - g["c_imag"]) < 1e-7     # the test's own eigen-solver
    st = ch.zero_state(S)
    st.ubar = S.C @ (1 - S.y ** 2)
    eps = 1e-6
    st.v[0, 1] = S.C @ (eps / 2 * phi)
    zero = np.zeros((S.nz, S.nkx), dtype=complex)
    amp = []
    n1, n2 = 100, 500
    for k in range(n2 + 1):
        if k in (n1, n2):
            amp.append(np.linalg.norm(st.v[0, 1]))
        if k < n2:
            st = ch.time_step(S, st, lambda r: zero)
    rate = np.log(amp[1] / amp[0]) / ((n2 - n1) * S.dt)
    # measured agreement is ~1e-7; the published value has 6 significant digits
    assert abs(rate - g["c_imag"]) < 1e-5 * g["c_imag"]


def test_wall_conditions_after_a_stage():
    """After any stage: v(-1) = v_w, v(+1) = 0, dv/dy(+-1) = 0 (influence
    matrix), omega_y(+-1) = 0, u = w = 0 at both walls."""
    S = ch.Setup(minimal_channel())
    st = initial_state(S, 2)
    rng = np.random.default_rng(0)
    act = rng.standard_normal((S.nz, S.nx)) * 0.3
    vw = ch.ingest_action(S, act)
    out, _ = ch.stage(S, st, 0, None, vw)
    scale = np.abs(out.v).max()
    assert np.abs(out.v @ S.bot_val - np.where(S.active, vw, 0)).max() < 1e-12 * scale
    assert np.abs(out.v @ S.top_val).max() < 1e-12 * scale
    assert np.abs(out.v @ S.top_slope).max() < 1e-9 * scale
    assert np.abs(out.v @ S.bot_slope).max() < 1e-9 * scale
    assert np.abs(out.om @ S.top_val).max() < 1e-12 * np.abs(out.om).max()
    assert np.abs(out.om @ S.bot_val).max() < 1e-12 * np.abs(out.om).max()
    u, v, w, _, _, _ = ch.reconstruct(S, out)
    for f in (u, w):
        assert np.abs(np.delete((f @ S.bot_val).ravel(), 0)).max() < 1e-9 * scale


def test_action_clip_and_zero_net_flux():
    S = ch.Setup(minimal_channel())
    rng = np.random.default_rng(1)
    a = rng.standard_normal((S.nz, S.nx)) * 2.0 + 0.7  # large, non-zero mean
    vw = ch.ingest_action(S, a)
    assert vw[0, 0] == 0
    phys = fr.to_physical(vw, S.nx, S.nz)
    assert abs(phys.mean()) < 1e-15
    clipped = np.clip(a, -1, 1)
    assert np.allclose(phys, clipped - clipped.mean() - _nyquist_part(clipped), atol=1e-13)
    with pytest.raises(ch.NonFinite):
        bad = a.copy()
        bad[3, 4] = np.nan
        ch.ingest_action(S, bad)


def _nyquist_part(f):
    """The Nyquist-mode content of a real grid field (dropped by the transform)."""
    F = np.fft.fft2(f)
    keep = np.zeros_like(F)
    nz, nx = f.shape
    keep[nz // 2, :] = F[nz // 2, :]
    keep[:, nx // 2] = F[:, nx // 2]
    return np.fft.ifft2(keep).real


def test_opposition_law_identity():
    """§4.1: v_w = -alpha (v(y_s) - <v(y_s)>) on the wall grid."""
    S = ch.Setup(minimal_channel(controller=ch.CTRL_OPPOSITION))
    st = initial_state(S, 4)
    vw = ch.opposition_wall(S, st)
    vs_phys = ch.observation(ch.Setup(minimal_channel(obs_mask=2)), st)[0]
    expect = -1.0 * (vs_phys - vs_phys.mean())
    assert np.allclose(fr.to_physical(vw, S.nx, S.nz), expect, atol=1e-14 * np.abs(expect).max())


def test_ramp_values_at_stage_ends():
    """§3.2: the wall velocity varies linearly from the old action to the new
    one over the actuation interval; with n substeps, stage r of step m ends
    at s = (m + c_r)/n."""
    S = ch.Setup(tiny())
    env = ch.Env(tiny())
    env.reset(0)
    rng = np.random.default_rng(2)
    a0 = rng.standard_normal((S.nz, S.nx)) * 0.2
    env.step(a0, 1)
    old = env.state.vw_old.copy()
    assert np.allclose(old, ch.ingest_action(S, a0))
    a1 = rng.standard_normal((S.nz, S.nx)) * 0.2
    new = ch.ingest_action(S, a1)
    st = env.state.copy()
    n = 2
    for m in range(n):
        hist = None
        for r in range(3):
            s = (m + ch.RK_C_END[r]) / n
            vw = old + s * (new - old)
            st, hist = ch.stage(S, st, r, hist, vw)
            assert np.allclose(st.v @ S.bot_val, np.where(S.active, vw, 0), atol=1e-13)
    env.step(a1, n)
    assert np.allclose(env.state.v, st.v, atol=1e-14 * np.abs(st.v).max())


def test_drag_is_mean_of_end_of_step_wall_shear():
    cfg = tiny()
    env = ch.Env(cfg)
    env.reset(5)
    st = env.state.copy()
    S = env.S
    zero = np.zeros((S.nz, S.nkx), dtype=complex)
    vals = []
    for _ in range(3):
        st = ch.time_step(S, st, lambda r: zero)
        vals.append(S.nu * (S.bot_slope @ st.ubar))
    obs, tw, drag = env.step(None, 3)
    assert np.isclose(drag, np.mean(vals), rtol=1e-14)
    assert np.isclose(tw.mean(), vals[-1], rtol=1e-12)
    assert obs.shape == (2, S.nz, S.nx)


def test_flow_rate_is_constant_and_state_stays_real():
    cfg = minimal_channel()
    env = ch.Env(cfg)
    env.reset(1)
    rng = np.random.default_rng(3)
    env.step(rng.standard_normal((16, 16)) * 0.1, 3)
    S, st = env.S, env.state
    assert abs(ch.flow_rate(S, st) - 2 * S.ub) < 1e-13 * 2 * S.ub
    for q in range(1, S.nz // 2):
        assert np.all(st.v[S.nz - q, 0] == np.conj(st.v[q, 0]))
    assert np.all(st.om[0, 0] == 0) and np.all(st.v[S.nz // 2] == 0)


def test_turbulent_drag_golden_is_consistent():
    """The stored oracle drag statistics (tests/golden/make_turbulent_drag.py) agree with
    themselves: window means are the means of their blocks, the ensemble mean is the mean of
    the seeds', and the drag of the controlled turbulent flow lies between the laminar value
    (3 U_b / Re_tau) and the uncontrolled turbulent level (about 1 in wall units)."""
    g = golden("turbulent_drag_minimal.json")
    a, b = g["window"]
    blk = g["block"]
    assert g["n_env_steps"] % blk == 0 and a % blk == 0 and b % blk == 0
    laminar = 3.0 * 15.66 / 180.0
    for s in g["seeds"]:
        bm = np.asarray(g["block_means"][str(s)])
        assert bm.size == g["n_env_steps"] // blk
        assert abs(bm[a // blk:b // blk].mean() - g["window_mean"][str(s)]) <= 1e-12
        assert laminar < g["window_mean"][str(s)] < 1.2
    ens = np.mean([g["window_mean"][str(s)] for s in g["seeds"]])
    assert abs(ens - g["ensemble_window_mean"]) <= 1e-12


def test_noise_floor_against_a_second_route(monkeypatch):
    """The oracle's intrinsic round-off: the same algorithm through a second numerical route
    (tau systems by an LU factorisation with the right-hand sides transformed separately, the
    Chebyshev transform matrices built column by column with scipy.fft.dct) differs by a few
    ulp after one time step and stays orders of magnitude below the parity bars (1e-12 after
    one step, 1e-9 after 100) after 100 steps."""
    import scipy.fft
    import scipy.linalg

    import oracle.tau as tau_mod

    cfg = tiny(controller=ch.CTRL_OPPOSITION)
    S1 = ch.Setup(cfg)
    st0 = initial_state(S1, 5)

    def run(S, n):
        st = st0.copy()
        for _ in range(n):
            vw = ch.opposition_wall(S, st)
            st = ch.time_step(S, st, lambda r: vw)
        return st

    ref1, ref100 = run(S1, 1), run(S1, 100)

    def lu_tau_solve(N, lam, f, g_top, g_bot, bc=("dirichlet", "dirichlet")):
        f = np.asarray(f)
        batch = f.shape[:-1]
        lam = np.broadcast_to(np.asarray(lam, dtype=float), batch)
        A = tau_mod.tau_matrix(N, lam, bc)
        rhs = np.zeros(batch + (N + 1,), dtype=complex)
        rhs[..., : N - 1] = f[..., : N - 1]
        rhs[..., N - 1] = np.broadcast_to(g_top, batch)
        rhs[..., N] = np.broadcast_to(g_bot, batch)
        out = np.empty(batch + (N + 1,), dtype=complex)
        for idx in np.ndindex(*batch):
            lu = scipy.linalg.lu_factor(A[idx])
            out[idx] = scipy.linalg.lu_solve(lu, rhs[idx].real) + 1j * scipy.linalg.lu_solve(lu, rhs[idx].imag)
        return out if np.iscomplexobj(f) or np.iscomplexobj(g_top) or np.iscomplexobj(g_bot) else out.real

    monkeypatch.setattr(ch, "tau_solve", lu_tau_solve)
    S2 = ch.Setup(cfg)
    N = S2.N
    eye = np.eye(N + 1)
    # forward: a = DCT-I(f) / N with the end coefficients halved; inverse from its definition
    C2 = scipy.fft.dct(eye, type=1, axis=0) / N
    C2[0] *= 0.5
    C2[N] *= 0.5
    S2.C = C2
    S2.B = np.cos(np.pi * np.outer(np.arange(N + 1), np.arange(N + 1)) / N)
    assert np.abs(S2.C - S1.C).max() < 1e-14 and np.abs(S2.B - S1.B).max() < 1e-14

    def rel(a, b):
        num = np.sqrt(np.sum(np.abs(a.v - b.v) ** 2) + np.sum(np.abs(a.om - b.om) ** 2) + np.sum((a.ubar - b.ubar) ** 2))
        den = np.sqrt(np.sum(np.abs(b.v) ** 2) + np.sum(np.abs(b.om) ** 2) + np.sum(b.ubar ** 2))
        return num / den

    d1, d100 = rel(run(S2, 1), ref1), rel(run(S2, 100), ref100)
    print(f"  second route: {d1:.2e} after one step, {d100:.2e} after 100")
    assert 0 < d1 < 1e-14
    assert d100 < 1e-12
