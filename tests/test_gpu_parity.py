"""GPU parity: the HIP path (through the C ABI) against the oracle on identical
seeded inputs.  Tolerances: relative L2 over the spectral state <= 1e-12 after
one time step and <= 1e-9 after 100 (the stated bar); the oracle's own
round-off spread over 100 steps of the minimal channel is ~1e-14."""
import numpy as np
import pytest

from oracle import channel as ch
from oracle.ic import initial_state
from synth import gaussian_action
from tests.gpu_helpers import gpu_env, gpu_state, rel_field_diff, rel_state_diff, to_device
from tests.oracle_cases import larger_channel, minimal_channel

pytestmark = pytest.mark.gpu


def run_pair(cfg, seed, actions, n_sub, tol_state, check_each=True):
    """Same initial field (oracle's) into both sides, then the same env steps.

    Output tolerances follow from the state tolerance: the observation is a
    plain evaluation at a node (10x), while tau_w and the drag are wall
    derivatives, sum_n n^2 a_n, which weight the last coefficients by up to
    N^2 relative to the state norm."""
    tol_obs = 10 * tol_state
    tol_wall = (cfg.ny - 1) ** 2 * tol_state
    oenv = ch.Env(cfg)
    S = oenv.S
    st0 = initial_state(S, seed)
    oenv.set_state(st0)
    genv = gpu_env(cfg)
    genv.set_state(ch.state_to_flat(S, st0))
    worst = 0.0
    for k, act in enumerate(actions):
        obs_o, tau_o, drag_o = oenv.step(act, n_sub)
        obs_g, tau_g, drag_g = genv.step(to_device(act), n_sub)
        if check_each or k == len(actions) - 1:
            gs = gpu_state(S, genv)
            d = rel_state_diff(gs, oenv.state)
            worst = max(worst, d)
            print(f"  env step {k}: state rel diff {d:.3e}", flush=True)
            assert d <= tol_state, (k, d)
            assert rel_field_diff(obs_g.cpu().numpy(), obs_o) <= tol_obs
            assert rel_field_diff(tau_g.cpu().numpy(), tau_o) <= tol_wall
            assert abs(drag_g.item() - drag_o) <= tol_wall * abs(drag_o)
            assert gs.nstep == oenv.state.nstep
            assert abs(gs.t - oenv.state.t) <= 1e-15 * max(1.0, abs(gs.t))
    genv.close()
    return worst


def test_minimal_channel_opposition_one_step():
    cfg = minimal_channel(controller=ch.CTRL_OPPOSITION)
    run_pair(cfg, 0, [None], 1, 1e-12)


def test_minimal_channel_opposition_100_steps():
    """Minimal channel, opposition control at y+ = 15, seeded perturbation on the
    laminar profile, 10 env steps x 10 time steps (100 RK3 steps at dt+ = 0.05)."""
    cfg = minimal_channel(controller=ch.CTRL_OPPOSITION)
    run_pair(cfg, 0, [None] * 10, 10, 1e-9, check_each=False)


@pytest.mark.parametrize("shape,mode,forcing,mask", [
    ((8, 33, 4), ch.RAMP, ch.CFR, 3),
    ((4, 17, 8), ch.HOLD, ch.CPG, 7),
    ((32, 33, 16), ch.RAMP, ch.CFR, 5),
    ((16, 65, 32), ch.RAMP, ch.CPG, 2),
    ((8, 97, 8), ch.HOLD, ch.CFR, 1),
])
def test_external_actions_small_grids(shape, mode, forcing, mask):
    nx, ny, nz = shape
    cfg = ch.Config(nx=nx, ny=ny, nz=nz, lx=2.67, lz=0.8, re_tau=180.0, dt_plus=0.05,
                    obs_y_plus=15.0, action_mode=mode, forcing=forcing, px=0.02, obs_mask=mask,
                    ic_profile=ch.IC_REICHARDT)
    acts = [gaussian_action(1000 + k, nz, nx) * 4.0 for k in range(3)]  # some values clip
    acts[1][0, 0] = 5.0
    run_pair(cfg, 7, acts, 2, 1e-11)


def test_larger_channel_bench_configuration():
    """Larger channel at full size (64 x 65 x 64), Reichardt mean + seeded
    perturbation, one env step of 10 time steps with a seeded Gaussian action
    (sigma = 0.1 u_tau) held over the env step: the launch configuration the
    benchmark times."""
    cfg = larger_channel(action_mode=ch.HOLD)
    run_pair(cfg, 0, [gaussian_action(1000, 64, 64)], 10, 1e-11)


def test_larger_channel_one_step():
    cfg = larger_channel()
    run_pair(cfg, 1, [gaussian_action(1001, 64, 64)], 1, 1e-12)


def test_reset_matches_oracle_initial_condition():
    for cfg, seed in [(minimal_channel(), 3), (larger_channel(), 2)]:
        S = ch.Setup(cfg)
        genv = gpu_env(cfg)
        genv.reset(seed)
        gs = gpu_state(S, genv)
        ref = initial_state(S, seed)
        assert rel_state_diff(gs, ref) < 1e-13
        assert gs.t == 0 and gs.nstep == 0 and np.all(gs.vw_old == 0)
        genv.close()


def test_query_reports_sensing_node():
    genv = gpu_env(minimal_channel())
    info = genv.query()
    assert info.js == 55
    assert abs(info.y_plus_node - 17.2819272377802) < 1e-9
    assert abs(info.ub - 15.66) < 1e-12
    assert info.state_doubles == ch.state_size(ch.Setup(minimal_channel()))
    genv.close()


@pytest.mark.parametrize("top_bc", [ch.TOP_WALL, ch.TOP_FREESLIP], ids=["closed", "open"])
def test_extra_observation_planes(top_bc):
    """Three extra observation planes (y+ 5, 40, 150) with all three components: the
    observation is [plane][component] and matches the oracle plane by plane; query reports
    each plane's node."""
    cfg = minimal_channel(controller=ch.CTRL_OPPOSITION, obs_mask=7, top_bc=top_bc,
                          extra_obs_y_plus=(5.0, 40.0, 150.0))
    run_pair(cfg, 2, [None, None], 2, 1e-11)
    S = ch.Setup(cfg)
    genv = gpu_env(cfg)
    info = genv.query()
    assert info.n_planes == 4
    assert list(info.js_planes) == S.js_planes
    assert info.obs_doubles == 12 * cfg.nz * cfg.nx
    for k, j in enumerate(S.js_planes):
        assert abs(info.y_plus_planes[k] - S.wall_dist[j] / S.nu) < 1e-12 * info.y_plus_planes[k]
    genv.close()
