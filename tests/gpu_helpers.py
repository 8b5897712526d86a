"""Helpers for the GPU tests: build a library env from an oracle Config and compare states."""
import numpy as np

from oracle import channel as ch


def grid_opts(cfg):
    import paper_2301_09889_amd.binding as b
    grid = b.ChanGrid(cfg.nx, cfg.ny, cfg.nz, cfg.lx, cfg.lz, cfg.re_tau, cfg.dt_plus, cfg.obs_y_plus)
    opts = b.make_opts(top_bc=cfg.top_bc, forcing=cfg.forcing, ub_plus=cfg.ub_plus, px=cfg.px,
                       nu_override=cfg.nu_override, dt_override=cfg.dt_override,
                       controller=cfg.controller, opp_alpha=cfg.opp_alpha,
                       action_mode=cfg.action_mode, clip=cfg.clip, obs_mask=cfg.obs_mask,
                       ic_profile=cfg.ic_profile, ic_amp=cfg.ic_amp,
                       extra_obs_y_plus=cfg.extra_obs_y_plus)
    return grid, opts


def gpu_env(cfg):
    import paper_2301_09889_amd.binding as b
    grid, opts = grid_opts(cfg)
    return b.ChanEnv(grid, opts)


def to_device(a):
    import torch
    if a is None:
        return None
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def state_norm(st):
    return np.sqrt(np.sum(np.abs(st.v) ** 2) + np.sum(np.abs(st.om) ** 2)
                   + np.sum(st.ubar ** 2) + np.sum(st.wbar ** 2))


def rel_state_diff(a, b):
    """Relative L2 difference over the whole spectral state (v, omega_y, U, W)."""
    d = np.sqrt(np.sum(np.abs(a.v - b.v) ** 2) + np.sum(np.abs(a.om - b.om) ** 2)
                + np.sum((a.ubar - b.ubar) ** 2) + np.sum((a.wbar - b.wbar) ** 2))
    return d / state_norm(b)


def rel_field_diff(a, b):
    a = np.asarray(a, dtype=float)
    b = np.asarray(b, dtype=float)
    return np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300)


def gpu_state(S, genv):
    return ch.state_from_flat(S, genv.get_state())


def field_errors(a, b, pair_floor=1e-3):
    """Element-wise comparison of two states field by field.

    Returns a dict: for v, om, U, W the relative max-norm error max|a - b| / max|b| of that
    field alone; for v and om also 'v_pair', 'om_pair': the worst pair (one Chebyshev column)
    measured against that pair's own coefficient norm, with pairs whose norm is below
    pair_floor x the field's largest pair norm measured against that floor instead."""
    out = {}
    for name, x, y in (("v", a.v, b.v), ("om", a.om, b.om), ("U", a.ubar, b.ubar), ("W", a.wbar, b.wbar)):
        scale = np.abs(y).max()
        out[name] = float(np.abs(x - y).max() / scale) if scale > 0 else float(np.abs(x).max())
    for name, x, y in (("v", a.v, b.v), ("om", a.om, b.om)):
        cn = np.linalg.norm(y, axis=-1)
        den = np.maximum(cn, pair_floor * cn.max())
        out[name + "_pair"] = float((np.linalg.norm(x - y, axis=-1) / den).max())
    return out


def assert_fields(a, b, tol, what=""):
    e = field_errors(a, b)
    print(f"  {what} " + " ".join(f"{k} {v:.1e}" for k, v in e.items()), flush=True)
    bad = {k: v for k, v in e.items() if not v <= tol}
    assert not bad, (what, bad, tol)
    return e
