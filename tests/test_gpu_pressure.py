"""Pressure observable on the GPU (static-pressure fluctuation on the observation planes),
through the C ABI, against the oracle on the same seeded inputs: closed and open channel,
opposition control and ramped external actions (whose slope enters the wall condition),
several planes.  The state is held to the parity bar; the velocity planes to 10x it; the
pressure to its own bound, 10x looser than the velocity planes: the wall condition evaluates
d^2v/dy^2 at the walls, which weights the last Chebyshev coefficients by up to N^4/3."""
import numpy as np
import pytest

from oracle import channel as ch
from oracle.ic import initial_state
from synth import gaussian_action
from tests.gpu_helpers import gpu_env, gpu_state, rel_field_diff, rel_state_diff, to_device
from tests.oracle_cases import larger_channel, minimal_channel

pytestmark = pytest.mark.gpu

TOL_P = 1e-11   # measured 1e-14 - 8e-14


def run_pressure(cfg, seed, actions, n_sub, tol_state):
    oenv = ch.Env(cfg)
    S = oenv.S
    st0 = initial_state(S, seed)
    oenv.set_state(st0)
    genv = gpu_env(cfg)
    genv.set_state(ch.state_to_flat(S, st0))
    ncomp = bin(cfg.obs_mask).count("1")
    for k, act in enumerate(actions):
        obs_o, _, _ = oenv.step(act, n_sub)
        obs_g, _, _ = genv.step(to_device(act), n_sub)
        obs_g = obs_g.cpu().numpy()
        d = rel_state_diff(gpu_state(S, genv), oenv.state)
        po = obs_o.reshape(-1, ncomp, S.nz, S.nx)
        pg = obs_g.reshape(-1, ncomp, S.nz, S.nx)
        dv = rel_field_diff(pg[:, :-1], po[:, :-1])
        dp = rel_field_diff(pg[:, -1], po[:, -1])
        print(f"  env step {k}: state {d:.2e} velocity planes {dv:.2e} pressure planes {dp:.2e} "
              f"(|p| max {np.abs(po[:, -1]).max():.3e})", flush=True)
        assert d <= tol_state
        assert dv <= 10 * tol_state
        assert dp <= TOL_P
        assert np.abs(po[:, -1]).max() > 0
    genv.close()


def test_pressure_minimal_channel_opposition():
    cfg = minimal_channel(controller=ch.CTRL_OPPOSITION, obs_mask=15, extra_obs_y_plus=(5.0, 40.0))
    run_pressure(cfg, 0, [None, None], 3, 1e-11)


@pytest.mark.parametrize("top_bc", [ch.TOP_WALL, ch.TOP_FREESLIP], ids=["closed", "open"])
def test_pressure_ramped_actions(top_bc):
    cfg = minimal_channel(top_bc=top_bc, obs_mask=11, ic_profile=ch.IC_REICHARDT,
                          extra_obs_y_plus=(2.0, 100.0))
    acts = [gaussian_action(3000 + k, cfg.nz, cfg.nx) * 3.0 for k in range(2)]
    run_pressure(cfg, 4, acts, 2, 1e-11)


def test_pressure_larger_channel_one_step():
    cfg = larger_channel(obs_mask=15)
    run_pressure(cfg, 1, [gaussian_action(1001, 64, 64)], 1, 1e-12)


def test_pressure_general_kernel(monkeypatch):
    """The general column kernel's pressure step: N_y = 97 (open channel, ramped actions), and
    forced at N_y = 65 (CHANENV_GENERIC_COLUMN=1, read at creation) with opposition control."""
    cfg = ch.Config(nx=8, ny=97, nz=8, lx=2.67, lz=0.8, re_tau=180.0, dt_plus=0.05, obs_y_plus=15.0,
                    obs_mask=15, top_bc=ch.TOP_FREESLIP, extra_obs_y_plus=(3.0, 60.0))
    acts = [gaussian_action(4000 + k, cfg.nz, cfg.nx) * 3.0 for k in range(2)]
    run_pressure(cfg, 6, acts, 2, 1e-11)
    monkeypatch.setenv("CHANENV_GENERIC_COLUMN", "1")
    run_pressure(minimal_channel(controller=ch.CTRL_OPPOSITION, obs_mask=15), 0, [None], 2, 1e-11)
