"""The plane pass in its two forms, through the C ABI: the z inverse and the x rows as one
launch (k_zxrow, padded lengths M_z, M_x of 48 and 96) against the three-launch form.

The forms differ only in which block computes what and where the padded z rows live (LDS
instead of HBM); every transform, product and packing is the same arithmetic, so the state and
the outputs must agree bit for bit, for square and non-square padded planes, for a batch whose
node count is not a multiple of the eight-node groups the fused launch deals out, and for a
rejected action.  One fused channel is also compared with the oracle."""
import numpy as np
import pytest

from oracle import channel as ch
from oracle.ic import initial_state
from synth import gaussian_action
from tests.gpu_helpers import gpu_state, grid_opts, rel_field_diff, rel_state_diff, to_device
from tests.test_gpu_batch import outputs

pytestmark = pytest.mark.gpu


def cfg_of(nx, ny, nz):
    return ch.Config(nx=nx, ny=ny, nz=nz, lx=2 * np.pi if nx >= 64 else 2.67, lz=np.pi if nz >= 64 else 0.8,
                     re_tau=180.0, dt_plus=0.05, obs_y_plus=15.0, controller=ch.CTRL_EXTERNAL,
                     action_mode=ch.RAMP, ic_profile=ch.IC_REICHARDT, obs_mask=7)


def envs_in_form(cfg, seeds, form, monkeypatch):
    """Envs of one grid and a batch of them, every plane-pass tiling (the env's own and the
    batch's) tuned with only the given form allowed."""
    import paper_2301_09889_amd.binding as b
    monkeypatch.setenv("CHANENV_PLANE_FORM", form)
    envs = []
    for s in seeds:
        e = b.ChanEnv(*grid_opts(cfg))
        e.reset(s)
        envs.append(e)
    batch = b.ChanBatch(envs)
    monkeypatch.delenv("CHANENV_PLANE_FORM")
    return envs, batch


def assert_same(ea, eb, what):
    sa, sb = ea.get_state(), eb.get_state()
    nd = int(np.count_nonzero(sa != sb))
    oa, ob = outputs(ea), outputs(eb)
    dmax = float(np.max(np.abs(sa - sb))) if nd else 0.0
    print(f"  {what}: state entries differing {nd}, largest difference {dmax:.2e}", flush=True)
    assert nd == 0, what
    assert np.array_equal(oa[0], ob[0]) and np.array_equal(oa[1], ob[1]) and oa[2] == ob[2], what


@pytest.mark.parametrize("shape", [(32, 65, 32), (64, 65, 64), (64, 33, 32), (32, 33, 64)])
def test_fused_plane_pass_equals_split(shape, monkeypatch):
    """One channel per grid: M_z x M_x = 48x48, 96x96, 48x96 and 96x48.  Three env steps of two
    time steps through each form's batch, then two through each env's own step."""
    import paper_2301_09889_amd.binding as b
    cfg = cfg_of(*shape)
    (es,), bs = envs_in_form(cfg, [3], "split", monkeypatch)
    (ef,), bf = envs_in_form(cfg, [3], "fused", monkeypatch)
    ts, tf = b.chan_batch_tuning(bs.handle), b.chan_batch_tuning(bf.handle)
    print(f"  {shape} split tiling {ts[0]}, fused tiling {tf[0]}", flush=True)
    assert ts[0]["plane_fused"] == 0 and tf[0]["plane_fused"] == 1
    for k in range(3):
        a = to_device(gaussian_action(500 + k, cfg.nz, cfg.nx))
        assert bs.step([a], 2) == [0] and bf.step([a], 2) == [0]
        assert_same(es, ef, f"{shape} batch step {k}")
    for k in range(2):
        a = to_device(gaussian_action(600 + k, cfg.nz, cfg.nx))
        es.step(a, 2)
        ef.step(a, 2)
        assert_same(es, ef, f"{shape} env step {k}")
    for x in (bs, bf):
        x.close()
    es.close()
    ef.close()


def test_fused_plane_pass_batch_and_rejected_action(monkeypatch):
    """Three 32x33x32 channels in one batch (99 nodes: the last group of eight is partly empty),
    then a non-finite action for the second channel: reported, that channel untouched, the others
    stepped, in both forms alike."""
    import paper_2301_09889_amd.binding as b
    cfg = cfg_of(32, 33, 32)
    seeds = [1, 2, 3]
    envs_s, bs = envs_in_form(cfg, seeds, "split", monkeypatch)
    envs_f, bf = envs_in_form(cfg, seeds, "fused", monkeypatch)
    assert b.chan_batch_tuning(bf.handle)[0]["plane_fused"] == 1
    for k in range(2):
        acts = [to_device(gaussian_action(700 + 10 * i + k, cfg.nz, cfg.nx)) for i in range(3)]
        assert bs.step(acts, 2) == [0, 0, 0] and bf.step(acts, 2) == [0, 0, 0]
        for i in range(3):
            assert_same(envs_s[i], envs_f[i], f"batch of three, step {k}, channel {i}")
    before = [e.get_state() for e in envs_f]
    acts = [to_device(gaussian_action(800 + i, cfg.nz, cfg.nx)) for i in range(3)]
    acts[1][4, 5] = float("nan")
    assert bs.step(acts, 2) == [0, b.CHAN_ENONFINITE, 0]
    assert bf.step(acts, 2) == [0, b.CHAN_ENONFINITE, 0]
    assert np.array_equal(envs_f[1].get_state(), before[1])
    assert not np.array_equal(envs_f[0].get_state(), before[0])
    for i in range(3):
        assert np.array_equal(envs_s[i].get_state(), envs_f[i].get_state()), i
    for x in [bs, bf] + envs_s + envs_f:
        x.close()


def test_fused_plane_pass_matches_oracle(monkeypatch):
    """The 32x65x32 channel with the fused plane pass from an oracle initial state: one env step
    of two time steps against the oracle, state and outputs."""
    cfg = cfg_of(32, 65, 32)
    oenv = ch.Env(cfg)
    st0 = initial_state(oenv.S, 11)
    oenv.set_state(st0)
    (e,), bf = envs_in_form(cfg, [0], "fused", monkeypatch)
    e.set_state(ch.state_to_flat(oenv.S, st0))
    a = gaussian_action(900, cfg.nz, cfg.nx)
    obs_o, tau_o, drag_o = oenv.step(a, 2)
    assert bf.step([to_device(a)], 2) == [0]
    d = rel_state_diff(gpu_state(oenv.S, e), oenv.state)
    do = rel_field_diff(e.obs.cpu().numpy(), obs_o)
    dt = rel_field_diff(e.tau_w.cpu().numpy(), tau_o)
    print(f"  fused plane pass vs oracle: state {d:.2e} obs {do:.2e} tau_w {dt:.2e}", flush=True)
    assert d <= 1e-12 and do <= 1e-11 and dt <= 64 ** 2 * 1e-12
    assert abs(e.drag.item() - drag_o) <= 64 ** 2 * 1e-12 * abs(drag_o)
    bf.close()
    e.close()
