"""Broadband parity cases shared by the GPU tests and the script that measures the oracle's own
round-off floor on them (test infrastructure: input construction and comparison metrics).

Each case: a grid and options, a seeded broadband initial field (synth.broadband_field), and a
list of env steps (numbers of time steps) with seeded Gaussian actions; the comparison is made
after every env step (a checkpoint) with the metrics of ``compare``."""
import numpy as np

import synth
from oracle import channel as ch

TWO_PI = 2 * np.pi

CASES = {
    # minimal channel, opposition control: 1, 10 and 100 time steps
    "minimal_closed": dict(cfg=dict(nx=16, ny=65, nz=16, lx=2.67, lz=0.8, re_tau=180.0, dt_plus=0.05,
                                    obs_y_plus=15.0, controller=ch.CTRL_OPPOSITION, obs_mask=15),
                           seed=21, steps=[1, 9, 90], action_seed=500, sigma=0.3),
    "minimal_open": dict(cfg=dict(nx=16, ny=65, nz=16, lx=2.67, lz=0.8, re_tau=180.0, dt_plus=0.05,
                                  obs_y_plus=15.0, controller=ch.CTRL_OPPOSITION, obs_mask=15,
                                  top_bc=ch.TOP_FREESLIP),
                         seed=21, steps=[1, 9, 90], action_seed=500, sigma=0.3),
    # larger channel at full size, one time step with a ramped or held action (some clipped)
    "larger_ramp": dict(cfg=dict(nx=64, ny=65, nz=64, lx=TWO_PI, lz=np.pi, re_tau=180.0, dt_plus=0.05,
                                 obs_y_plus=15.0, action_mode=ch.RAMP, obs_mask=7),
                        seed=22, steps=[1], action_seed=500, sigma=0.5),
    "larger_hold": dict(cfg=dict(nx=64, ny=65, nz=64, lx=TWO_PI, lz=np.pi, re_tau=180.0, dt_plus=0.05,
                                 obs_y_plus=15.0, action_mode=ch.HOLD, obs_mask=7),
                        seed=22, steps=[1], action_seed=500, sigma=0.5),
    # the 192-point plane transforms (nx or nz = 128)
    "wide_128x33x128": dict(cfg=dict(nx=128, ny=33, nz=128, lx=TWO_PI, lz=np.pi, re_tau=180.0, dt_plus=0.05,
                                     obs_y_plus=15.0, obs_mask=7),
                            seed=23, steps=[1], action_seed=500, sigma=0.3),
    "wide_128x17x4": dict(cfg=dict(nx=128, ny=17, nz=4, lx=TWO_PI, lz=np.pi, re_tau=180.0, dt_plus=0.05,
                                   obs_y_plus=15.0, obs_mask=15),
                          seed=23, steps=[1, 2], action_seed=500, sigma=0.3),
    "wide_4x17x128": dict(cfg=dict(nx=4, ny=17, nz=128, lx=TWO_PI, lz=np.pi, re_tau=180.0, dt_plus=0.05,
                                   obs_y_plus=15.0, obs_mask=15),
                          seed=23, steps=[1, 2], action_seed=500, sigma=0.3),
    "wide_128x33x8": dict(cfg=dict(nx=128, ny=33, nz=8, lx=TWO_PI, lz=np.pi, re_tau=180.0, dt_plus=0.05,
                                   obs_y_plus=15.0, obs_mask=15),
                          seed=23, steps=[1, 2], action_seed=500, sigma=0.3),
    # N_y = 129 (the general column kernel at N = 128)
    "ny129_closed": dict(cfg=dict(nx=8, ny=129, nz=8, lx=2.67, lz=0.8, re_tau=180.0, dt_plus=0.05,
                                  obs_y_plus=15.0, obs_mask=15),
                         seed=24, steps=[1, 10], action_seed=500, sigma=0.3),
    "ny129_open": dict(cfg=dict(nx=8, ny=129, nz=8, lx=2.67, lz=0.8, re_tau=180.0, dt_plus=0.05,
                                obs_y_plus=15.0, obs_mask=15, top_bc=ch.TOP_FREESLIP),
                       seed=24, steps=[1, 10], action_seed=500, sigma=0.3),
    # full-size cases whose oracle run is stored (tests/golden/make_broadband_parity.py)
    "larger_100": dict(cfg=dict(nx=64, ny=65, nz=64, lx=TWO_PI, lz=np.pi, re_tau=180.0, dt_plus=0.05,
                                obs_y_plus=15.0, action_mode=ch.HOLD),
                       seed=11, steps=[10] * 10, action_seed=2000, sigma=0.1, stored=True),
    "re395": dict(cfg=dict(nx=128, ny=97, nz=128, lx=TWO_PI, lz=np.pi, re_tau=395.0, dt_plus=0.05,
                           obs_y_plus=15.0, action_mode=ch.RAMP),
                  seed=12, steps=[1], action_seed=3000, sigma=0.5, stored=True),
}

STATE_METRICS = ("v", "om", "U", "W", "v_pair", "om_pair")
OUTPUT_METRICS = ("obs", "tau_w", "drag")


def config(name):
    return ch.Config(**CASES[name]["cfg"])


def initial_state(S, seed):
    st = ch.zero_state(S)
    st.v, st.om, st.ubar, st.wbar, st.vw_old = synth.broadband_field(
        seed, S.nx, S.ny, S.nz, S.ub, top_freeslip=S.open)
    return st


def action(name, k, S):
    c = CASES[name]
    return synth.gaussian_action(c["action_seed"] + k, S.nz, S.nx, c["sigma"])


def checkpoints(name):
    """Cumulative time steps after each env step of the case."""
    return list(np.cumsum(CASES[name]["steps"]))


def bar(total_steps):
    """The stated parity bar for the state after n = total_steps time steps, 1e-12 after one step
    and 1e-9 after 100, interpolated between them as 1e-12 n^1.5 (a round-off difference that
    grows by a constant factor per step)."""
    return 1e-12 * float(max(1, total_steps)) ** 1.5


def output_bars(ny, total_steps):
    """The observation is a point evaluation (10x the state bar); tau_w and the drag are the
    wall slope sum_n n^2 a_n, a sum weighted towards the high degrees (N x the state bar)."""
    b = bar(total_steps)
    return {"obs": 10 * b, "tau_w": (ny - 1) * b, "drag": (ny - 1) * b}


def state_errors(a, b, pair_floor=1e-3):
    """Field-by-field comparison of state a against reference b: relative max-norm of v, om, U,
    W each against its own max-norm, and the worst pair (Chebyshev column) of v and om against
    its own coefficient norm (pairs below pair_floor x the field's largest pair norm against
    that floor instead)."""
    out = {}
    for name, x, y in (("v", a.v, b.v), ("om", a.om, b.om), ("U", a.ubar, b.ubar), ("W", a.wbar, b.wbar)):
        scale = np.abs(y).max()
        out[name] = float(np.abs(x - y).max() / scale) if scale > 0 else float(np.abs(x).max())
    for name, x, y in (("v", a.v, b.v), ("om", a.om, b.om)):
        cn = np.linalg.norm(y, axis=-1)
        den = np.maximum(cn, pair_floor * cn.max())
        out[name + "_pair"] = float((np.linalg.norm(x - y, axis=-1) / den).max())
    return out


def output_errors(got, ref):
    (obs_g, tau_g, drag_g), (obs_o, tau_o, drag_o) = got, ref
    obs_g, tau_g = np.asarray(obs_g, dtype=float), np.asarray(tau_g, dtype=float)
    e_obs = (np.linalg.norm((obs_g - obs_o).ravel()) / np.linalg.norm(obs_o.ravel())) if obs_o.size else 0.0
    return {"obs": float(e_obs),
            "tau_w": float(np.abs(tau_g - tau_o).max() / np.abs(tau_o).max()),
            "drag": float(abs(float(drag_g) - drag_o) / abs(drag_o))}


def tolerance(metric, total_steps, ny, floor):
    """max(stated bar, 3 x the oracle's own two-route floor for this metric and checkpoint)."""
    b = output_bars(ny, total_steps)[metric] if metric in OUTPUT_METRICS else bar(total_steps)
    return max(b, 3.0 * floor)
