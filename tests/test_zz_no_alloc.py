"""chan_step_static, the entry point that allocates nothing, against chan_env_step.

Both run the same kernels on the same canonical state, so their results must agree bitwise:
the advanced state, the observation, tau_w and the drag.  Calls in a row change the grid (the
second call smaller than the first, then larger again), which makes the library rebuild the
tables in its static scratch.  Also: a grid whose footprint exceeds the scratch is refused with
CHAN_EINVAL, and a non-finite action or state gives CHAN_ENONFINITE with the caller's state
left as it was."""
import numpy as np
import pytest

import synth
from oracle import channel as ch
from tests.gpu_helpers import grid_opts, gpu_env, to_device

pytestmark = pytest.mark.gpu


def broadband_flat(cfg, seed):
    S = ch.Setup(cfg)
    st = ch.zero_state(S)
    st.v, st.om, st.ubar, st.wbar, st.vw_old = synth.broadband_field(seed, S.nx, S.ny, S.nz, S.ub,
                                                                     top_freeslip=S.open)
    st.t, st.nstep = 0.125, 7
    return S, ch.state_to_flat(S, st)


def step_static(cfg, flat_dev, action, n):
    import torch
    import paper_2301_09889_amd.binding as b
    grid, opts = grid_opts(cfg)
    S = ch.Setup(cfg)
    nobs = bin(cfg.obs_mask).count("1") * (1 + len(cfg.extra_obs_y_plus))
    obs = torch.full((nobs, cfg.nz, cfg.nx), -7.0, dtype=torch.float64, device="cuda")
    tau = torch.full((cfg.nz, cfg.nx), -7.0, dtype=torch.float64, device="cuda")
    drag = torch.full((1,), -7.0, dtype=torch.float64, device="cuda")
    a = to_device(action)
    rc = b.chan_step_static(grid, opts, torch.cuda.current_stream().cuda_stream, flat_dev.data_ptr(),
                            a.data_ptr() if a is not None else 0, n, obs.data_ptr(), tau.data_ptr(), drag.data_ptr())
    torch.cuda.synchronize()
    return rc, obs, tau, drag, S


def compare_with_env(cfg, seed, action, n):
    import torch
    S, flat = broadband_flat(cfg, seed)
    genv = gpu_env(cfg)
    genv.set_state(flat)
    obs_e, tau_e, drag_e = genv.step(to_device(action), n)
    ref = genv.get_state()
    obs_e, tau_e, drag_e = obs_e.cpu().numpy(), tau_e.cpu().numpy(), drag_e.cpu().numpy()
    genv.close()
    dev = torch.tensor(flat, dtype=torch.float64, device="cuda")
    rc, obs, tau, drag, _ = step_static(cfg, dev, action, n)
    assert rc == 0, rc
    got = dev.cpu().numpy()
    print(f"  {cfg.nx}x{cfg.ny}x{cfg.nz}: state max diff {np.abs(got - ref).max():.1e}, "
          f"drag {drag.item():.12f} vs {drag_e[0]:.12f}", flush=True)
    assert np.array_equal(got, ref)
    assert np.array_equal(obs.cpu().numpy(), obs_e)
    assert np.array_equal(tau.cpu().numpy(), tau_e)
    assert np.array_equal(drag.cpu().numpy(), drag_e)


def minimal(**kw):
    base = dict(nx=16, ny=65, nz=16, lx=2.67, lz=0.8, re_tau=180.0, dt_plus=0.05, obs_y_plus=15.0)
    base.update(kw)
    return ch.Config(**base)


def test_static_step_equals_env_step_in_a_row():
    """Minimal channel with opposition control, then a smaller grid with a ramped external
    action, pressure and extra planes, then a larger one (32x65x32, held action), then the
    general column kernel (N = 96), then the minimal channel again."""
    cfgs = [
        (minimal(controller=ch.CTRL_OPPOSITION), None, 3),
        (ch.Config(nx=8, ny=33, nz=8, lx=2.0, lz=1.0, re_tau=180.0, dt_plus=0.05, obs_y_plus=15.0,
                   obs_mask=15, extra_obs_y_plus=(40.0,)), synth.gaussian_action(5, 8, 8, 0.5), 2),
        (minimal(nx=32, nz=32, action_mode=ch.HOLD, obs_mask=7), synth.gaussian_action(6, 32, 32), 2),
        (ch.Config(nx=8, ny=97, nz=8, lx=2.0, lz=1.0, re_tau=180.0, dt_plus=0.05, obs_y_plus=15.0,
                   top_bc=ch.TOP_FREESLIP, obs_mask=11), synth.gaussian_action(7, 8, 8, 0.2), 2),
        (minimal(controller=ch.CTRL_OPPOSITION), None, 3),
    ]
    for k, (cfg, act, n) in enumerate(cfgs):
        compare_with_env(cfg, 40 + k, act, n)


def test_static_step_refuses_and_rejects():
    import torch
    import paper_2301_09889_amd.binding as b
    # footprint beyond the scratch
    big = minimal(nx=64, nz=64, lx=2 * np.pi, lz=np.pi)
    S, flat = broadband_flat(big, 1)
    dev = torch.tensor(flat, dtype=torch.float64, device="cuda")
    rc, *_ = step_static(big, dev, None, 1)
    assert rc == b.CHAN_EINVAL
    assert "too large" in b.chan_last_error()
    assert np.array_equal(dev.cpu().numpy(), flat)
    # non-finite action: state unchanged
    cfg = minimal()
    S, flat = broadband_flat(cfg, 2)
    dev = torch.tensor(flat, dtype=torch.float64, device="cuda")
    bad = synth.gaussian_action(1, 16, 16)
    bad[3, 4] = np.nan
    rc, *_ = step_static(cfg, dev, bad, 2)
    assert rc == b.CHAN_ENONFINITE
    assert np.array_equal(dev.cpu().numpy(), flat)
    # non-finite state: unchanged, and the next good call still works
    flat_bad = flat.copy()
    flat_bad[11] = np.inf
    dev = torch.tensor(flat_bad, dtype=torch.float64, device="cuda")
    rc, *_ = step_static(cfg, dev, None, 1)
    assert rc == b.CHAN_ENONFINITE
    assert np.array_equal(dev.cpu().numpy(), flat_bad)
    compare_with_env(cfg, 3, synth.gaussian_action(2, 16, 16), 2)
