"""Captured env steps (HIP graphs) on the GPU, through the C ABI.

Every replay of a captured step gives bitwise the outputs and state of the same step run directly,
with the program's own eager work, synchronisations and action refills between the replays
(replays are checked one by one, not only at the end); a replayed channel matches the oracle;
reset between replays is honoured; and the error paths (no flow state, a replay already in
flight, an env held, a non-finite action, an env that left the batch, a destroyed batch) refuse
or report without stepping anything they should not."""
import numpy as np
import pytest

from oracle import channel as ch
from oracle.ic import initial_state
from synth import gaussian_action
from tests.gpu_helpers import gpu_state, grid_opts, rel_field_diff, rel_state_diff, to_device
from tests.test_gpu_batch import MIX, actions_for, make_envs, outputs

pytestmark = pytest.mark.gpu


def cfg_of(nx, ny, nz, ctrl=ch.CTRL_EXTERNAL, mode=ch.RAMP):
    return ch.Config(nx=nx, ny=ny, nz=nz, lx=2.67 if nx <= 32 else 2 * np.pi, lz=0.8 if nx <= 32 else np.pi,
                     re_tau=180.0, dt_plus=0.05, obs_y_plus=15.0, controller=ctrl, action_mode=mode,
                     ic_profile=ch.IC_REICHARDT, obs_mask=7)


def env_of(cfg, seed):
    import paper_2301_09889_amd.binding as b
    e = b.ChanEnv(*grid_opts(cfg))
    e.reset(seed)
    return e


def eager_noise():
    """Work of the program's own between replays: a library reduction and a synchronisation."""
    import torch
    x = torch.randn(1 << 20, dtype=torch.float64, device="cuda")
    s = float(x.sum().item())
    torch.cuda.synchronize()
    return s


@pytest.mark.parametrize("shape", [(16, 65, 16), (64, 65, 64), (8, 97, 8)])
def test_env_graph_replays_equal_direct_steps(shape):
    """One channel (the minimal channel, the larger channel's single-channel launches, and the
    general column kernel at N_y = 97): four replays of one captured env step of two time steps,
    each against the same step run directly."""
    import torch
    cfg = cfg_of(*shape)
    direct, graphed = env_of(cfg, 5), env_of(cfg, 5)
    abuf = torch.zeros((cfg.nz, cfg.nx), dtype=torch.float64, device="cuda")
    g = graphed.capture(abuf, 2)
    for k in range(4):
        a = to_device(gaussian_action(300 + k, cfg.nz, cfg.nx))
        direct.step(a, 2)
        abuf.copy_(a)
        codes = g.launch().finish()
        assert codes == [0], (k, codes)
        od, og = outputs(direct), outputs(graphed)
        assert np.array_equal(od[0], og[0]) and np.array_equal(od[1], og[1]) and od[2] == og[2], (shape, k)
        sd, sg = direct.get_state(), graphed.get_state()
        nd = int(np.count_nonzero(sd != sg))
        print(f"  {shape} replay {k}: state entries differing {nd}", flush=True)
        assert nd == 0, (shape, k)
        qd, qg = direct.query(), graphed.query()
        assert (qd.nstep, qd.t) == (qg.nstep, qg.t)
        eager_noise()
    g.close()
    direct.close()
    graphed.close()


def test_batch_graph_replays_equal_direct_launches():
    """The seven-channel mix (two parity-major shapes, the general kernel, opposition, ramped and
    held actions): three replays of one captured batch step against chan_batch_launch."""
    import paper_2301_09889_amd.binding as b
    import torch
    direct, graphed = make_envs(MIX), make_envs(MIX)
    bd, bg = b.ChanBatch(direct), b.ChanBatch(graphed)
    abufs = [torch.zeros((s[2], s[0]), dtype=torch.float64, device="cuda") if s[4] == ch.CTRL_EXTERNAL else None
             for s in MIX]
    g = bg.capture(graphed, abufs, 2, [e.obs for e in graphed], [e.tau_w for e in graphed],
                   [e.drag for e in graphed])
    for k in range(3):
        acts = actions_for(MIX, k)
        c = bd.launch(direct, acts, 2, [e.obs for e in direct], [e.tau_w for e in direct], [e.drag for e in direct])
        assert c.finish() == [0] * len(MIX)
        for buf, a in zip(abufs, acts):
            if buf is not None:
                buf.copy_(a)
        assert g.launch().finish() == [0] * len(MIX)
        for i, (ed, eg) in enumerate(zip(direct, graphed)):
            nd = int(np.count_nonzero(ed.get_state() != eg.get_state()))
            od, og = outputs(ed), outputs(eg)
            assert nd == 0 and np.array_equal(od[0], og[0]) and np.array_equal(od[1], og[1]) and od[2] == og[2], \
                (k, i, nd)
        print(f"  batch replay {k}: all {len(MIX)} channels bitwise equal", flush=True)
        eager_noise()
    g.close()
    bd.close()
    bg.close()
    for e in direct + graphed:
        e.close()


def test_graph_replay_matches_oracle():
    """The 32x65x32 channel from an oracle initial state: two replays of one captured env step of
    two time steps against the oracle, state and outputs."""
    import torch
    cfg = cfg_of(32, 65, 32)
    oenv = ch.Env(cfg)
    st0 = initial_state(oenv.S, 11)
    oenv.set_state(st0)
    e = env_of(cfg, 0)
    e.set_state(ch.state_to_flat(oenv.S, st0))
    abuf = torch.zeros((cfg.nz, cfg.nx), dtype=torch.float64, device="cuda")
    g = e.capture(abuf, 2)
    for k in range(2):
        a = gaussian_action(700 + k, cfg.nz, cfg.nx)
        obs_o, tau_o, drag_o = oenv.step(a, 2)
        abuf.copy_(to_device(a))
        assert g.launch().finish() == [0]
        d = rel_state_diff(gpu_state(oenv.S, e), oenv.state)
        do = rel_field_diff(e.obs.cpu().numpy(), obs_o)
        dt = rel_field_diff(e.tau_w.cpu().numpy(), tau_o)
        print(f"  replay {k} vs oracle: state {d:.2e} obs {do:.2e} tau_w {dt:.2e}", flush=True)
        assert d <= 1e-12 and do <= 1e-11 and dt <= 64 ** 2 * 1e-12, (k, d, do, dt)
        assert abs(e.drag.item() - drag_o) <= 64 ** 2 * 1e-12 * abs(drag_o)
    g.close()
    e.close()


def test_graph_after_reset_and_set_state():
    """reset and set_state between replays: the replay steps the state the env holds then."""
    import torch
    cfg = cfg_of(16, 65, 16)
    direct, graphed = env_of(cfg, 1), env_of(cfg, 1)
    abuf = torch.zeros((cfg.nz, cfg.nx), dtype=torch.float64, device="cuda")
    g = graphed.capture(abuf, 3)
    a = to_device(gaussian_action(41, cfg.nz, cfg.nx))
    abuf.copy_(a)
    assert g.launch().finish() == [0]
    direct.step(a, 3)
    for e in (direct, graphed):
        e.reset(9)
    direct.step(a, 3)
    assert g.launch().finish() == [0]
    assert np.array_equal(direct.get_state(), graphed.get_state())
    flat = direct.get_state()
    graphed.set_state(flat)
    direct.step(a, 3)
    assert g.launch().finish() == [0]
    assert np.array_equal(direct.get_state(), graphed.get_state())
    assert np.array_equal(outputs(direct)[0], outputs(graphed)[0])
    g.close()
    direct.close()
    graphed.close()


def test_graph_errors():
    import paper_2301_09889_amd.binding as b
    import torch
    cfg = cfg_of(16, 65, 16)
    fresh = b.ChanEnv(*grid_opts(cfg))            # no flow state yet
    abuf = torch.zeros((cfg.nz, cfg.nx), dtype=torch.float64, device="cuda")
    with pytest.raises(b.ChanError) as ei:
        fresh.capture(abuf, 1)
    assert ei.value.code == b.CHAN_ESTATE
    with pytest.raises(b.ChanError) as ei:
        env_of(cfg, 0).capture(abuf, 0)
    assert ei.value.code == b.CHAN_EINVAL

    e = env_of(cfg, 2)
    abuf.copy_(to_device(gaussian_action(5, cfg.nz, cfg.nx)))
    g = e.capture(abuf, 2)
    c = g.launch()
    with pytest.raises(b.ChanError) as ei:       # one replay in flight per graph
        g.launch()
    assert ei.value.code == b.CHAN_EBUSY
    with pytest.raises(b.ChanError) as ei:       # the env is held by the replay
        e.step(None, 1)
    assert ei.value.code == b.CHAN_EBUSY
    assert c.finish() == [0]

    # a non-finite action: reported, the state untouched; a finite refill steps normally
    before = e.get_state()
    abuf[2, 3] = float("nan")
    assert g.launch().finish() == [b.CHAN_ENONFINITE]
    assert np.array_equal(e.get_state(), before)
    abuf.copy_(to_device(gaussian_action(6, cfg.nz, cfg.nx)))
    assert g.launch().finish() == [0]
    assert not np.array_equal(e.get_state(), before)

    # closing a graph with a replay in flight finishes the replay (outcome applied)
    n0 = e.query().nstep
    c = g.launch()
    g.close()
    assert c.finish() == [b.CHAN_EINVAL]         # handle abandoned: the library finished it
    assert e.query().nstep == n0 + 2
    e.step(None, 1)

    # batch graphs: an env that left the batch, then a destroyed batch
    envs = [env_of(cfg, 3), env_of(cfg, 4)]
    bt = b.ChanBatch(envs)
    gb = bt.capture(envs, None, 1, None, None, None)
    assert gb.launch().finish() == [0, 0]
    bt.remove(envs[1])
    with pytest.raises(b.ChanError) as ei:
        gb.launch()
    assert ei.value.code == b.CHAN_ESTATE
    gb.close()
    gb2 = bt.capture([envs[0]], None, 1, None, None, None)
    assert gb2.launch().finish() == [0]
    bt.close()
    with pytest.raises(b.ChanError) as ei:
        gb2.launch()
    assert ei.value.code == b.CHAN_ESTATE
    gb2.close()

    # an env destroyed after its own capture: the graph refuses, closing it is safe
    g3 = envs[0].capture(None, 1)
    envs[0].close()
    with pytest.raises(b.ChanError) as ei:
        g3.launch()
    assert ei.value.code == b.CHAN_ESTATE
    g3.close()
    for x in (fresh, e, envs[1]):
        x.close()
