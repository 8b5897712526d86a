"""Batched channels on the GPU (through the C ABI): a channel advanced in a mixed batch gives
bitwise the result it gives alone, one batch member matches the oracle, and a rejected action
stays with its own channel."""
import numpy as np
import pytest

from oracle import channel as ch
from oracle.ic import initial_state
from synth import gaussian_action
from tests.gpu_helpers import grid_opts, gpu_state, rel_field_diff, rel_state_diff, to_device

pytestmark = pytest.mark.gpu

# (nx, ny, nz, re_tau, controller, action_mode, ic_profile, seed): two shapes on the
# parity-major kernels, one N_y = 97 channel on the general column kernel, Re_tau 100 / 180,
# opposition, ramped and held external actions.
MIX = [
    (16, 65, 16, 180.0, ch.CTRL_OPPOSITION, ch.RAMP, ch.IC_LAMINAR, 0),
    (32, 65, 32, 180.0, ch.CTRL_EXTERNAL, ch.RAMP, ch.IC_REICHARDT, 1),
    (16, 65, 16, 100.0, ch.CTRL_EXTERNAL, ch.HOLD, ch.IC_LAMINAR, 2),
    (32, 65, 32, 100.0, ch.CTRL_OPPOSITION, ch.RAMP, ch.IC_REICHARDT, 3),
    (16, 65, 16, 180.0, ch.CTRL_EXTERNAL, ch.RAMP, ch.IC_REICHARDT, 4),
    (8, 33, 8, 180.0, ch.CTRL_EXTERNAL, ch.RAMP, ch.IC_LAMINAR, 5),
    (8, 97, 8, 180.0, ch.CTRL_OPPOSITION, ch.RAMP, ch.IC_LAMINAR, 6),
]


def mix_cfg(spec):
    nx, ny, nz, re, ctrl, mode, ic, _ = spec
    return ch.Config(nx=nx, ny=ny, nz=nz, lx=2.67, lz=0.8, re_tau=re, dt_plus=0.05, obs_y_plus=15.0,
                     controller=ctrl, action_mode=mode, ic_profile=ic, obs_mask=7)


def make_envs(specs):
    import paper_2301_09889_amd.binding as b
    envs = []
    for spec in specs:
        grid, opts = grid_opts(mix_cfg(spec))
        e = b.ChanEnv(grid, opts)
        e.reset(spec[-1])
        envs.append(e)
    return envs


def actions_for(specs, k):
    return [to_device(gaussian_action(1000 + 10 * i + k, s[2], s[0])) if s[4] == ch.CTRL_EXTERNAL else None
            for i, s in enumerate(specs)]


def outputs(e):
    return e.obs.cpu().numpy().copy(), e.tau_w.cpu().numpy().copy(), e.drag.item()


def test_batch_matches_alone_bitwise():
    import paper_2301_09889_amd.binding as b
    alone, mixed = make_envs(MIX), make_envs(MIX)
    batch = b.ChanBatch(mixed)
    assert b.chan_batch_size(batch.handle) == len(MIX)
    for k in range(3):
        acts = actions_for(MIX, k)
        for e, a in zip(alone, acts):
            e.step(a, 2)
        codes = batch.step(acts, 2)
        assert codes == [0] * len(MIX)
        for i, (ea, em) in enumerate(zip(alone, mixed)):
            sa, sm = ea.get_state(), em.get_state()
            nd = int(np.count_nonzero(sa != sm))
            print(f"  env step {k}, channel {i} {MIX[i][:3]}: state entries differing {nd}", flush=True)
            assert nd == 0, (k, i)
            oa, om = outputs(ea), outputs(em)
            assert np.array_equal(oa[0], om[0]) and np.array_equal(oa[1], om[1]) and oa[2] == om[2], (k, i)
    batch.close()
    for e in alone + mixed:
        e.close()


def test_batch_member_matches_oracle():
    """The 32x65x32 externally actuated channel of the mix against the oracle, one env step of
    two time steps, inside the full mixed batch."""
    import paper_2301_09889_amd.binding as b
    envs = make_envs(MIX)
    i = 1
    cfg = mix_cfg(MIX[i])
    oenv = ch.Env(cfg)
    st0 = initial_state(oenv.S, MIX[i][-1])
    oenv.set_state(st0)
    envs[i].set_state(ch.state_to_flat(oenv.S, st0))
    batch = b.ChanBatch(envs)
    acts = actions_for(MIX, 0)
    obs_o, tau_o, drag_o = oenv.step(acts[i].cpu().numpy(), 2)
    assert batch.step(acts, 2) == [0] * len(MIX)
    d = rel_state_diff(gpu_state(oenv.S, envs[i]), oenv.state)
    print(f"  batch member vs oracle: state rel diff {d:.3e}", flush=True)
    assert d <= 1e-12
    assert rel_field_diff(envs[i].obs.cpu().numpy(), obs_o) <= 1e-11
    assert rel_field_diff(envs[i].tau_w.cpu().numpy(), tau_o) <= 64 ** 2 * 1e-12
    batch.close()
    for e in envs:
        e.close()


def test_rejected_action_stays_with_its_channel():
    import paper_2301_09889_amd.binding as b
    specs = MIX[:3]
    alone, mixed = make_envs(specs), make_envs(specs)
    batch = b.ChanBatch(mixed)
    acts = actions_for(specs, 0)
    bad = acts[1].clone()
    bad[3, 5] = float("nan")
    before = mixed[1].get_state()
    codes = batch.step([acts[0], bad, acts[2]], 2)
    assert codes == [0, b.CHAN_ENONFINITE, 0]
    assert np.array_equal(mixed[1].get_state(), before)
    for i in (0, 2):
        alone[i].step(acts[i], 2)
        assert np.array_equal(alone[i].get_state(), mixed[i].get_state()), i
    # the rejected channel continues normally afterwards
    assert batch.step(acts, 2) == [0, 0, 0]
    batch.close()
    for e in alone + mixed:
        e.close()


def test_batch_create_errors():
    import paper_2301_09889_amd.binding as b
    envs = make_envs(MIX[:2])
    with pytest.raises(b.ChanError) as ei:
        b.chan_batch_create([envs[0].handle, envs[0].handle])
    assert ei.value.code == b.CHAN_EINVAL
    with pytest.raises(b.ChanError) as ei:
        b.chan_batch_create([])
    assert ei.value.code == b.CHAN_EINVAL
    for e in envs:
        e.close()


def test_invalid_channel_is_skipped():
    """A channel without a flow state is skipped (CHAN_ESTATE, untouched) while the others
    advance; a batch with no valid channel fails without running."""
    import paper_2301_09889_amd.binding as b
    specs = MIX[:3]
    alone, mixed = make_envs(specs), make_envs(specs)
    grid, opts = grid_opts(mix_cfg(specs[1]))
    fresh = b.ChanEnv(grid, opts)           # never reset: no flow state
    mixed[1].close()
    mixed[1] = fresh
    batch = b.ChanBatch(mixed)
    acts = actions_for(specs, 0)
    fresh.obs.fill_(7.0)
    codes = batch.step(acts, 2)
    assert codes == [0, b.CHAN_ESTATE, 0]
    assert float(fresh.obs.min()) == 7.0 and float(fresh.obs.max()) == 7.0
    for i in (0, 2):
        alone[i].step(acts[i], 2)
        assert np.array_equal(alone[i].get_state(), mixed[i].get_state()), i
    batch.close()
    only = b.ChanBatch([fresh])
    with pytest.raises(b.ChanError) as ei:
        only.step([acts[1]], 2)
    assert ei.value.code == b.CHAN_ESTATE
    only.close()
    for e in alone + mixed:
        e.close()


def test_subsets_match_alone_bitwise():
    """Different subsets of a mixed batch advanced over several calls (what a request loop
    does): every channel ends bitwise where its twin, advanced alone by the same calls, ends;
    channels outside a call's subset are untouched by it."""
    import paper_2301_09889_amd.binding as b
    alone, mixed = make_envs(MIX), make_envs(MIX)
    batch = b.ChanBatch(mixed)
    plan = [[0, 1, 2, 3, 4, 5, 6], [1, 3, 5], [6, 0], [2], [4, 5, 6, 1]]
    for k, idx in enumerate(plan):
        acts = actions_for(MIX, k)
        before = {i: mixed[i].get_state() for i in range(len(MIX)) if i not in idx}
        codes = batch.step_subset(idx, [acts[i] for i in idx], 2)
        assert codes == [0] * len(idx), (k, codes)
        for i in idx:
            alone[i].step(acts[i], 2)
        for i in range(len(MIX)):
            if i in idx:
                assert np.array_equal(alone[i].get_state(), mixed[i].get_state()), (k, i)
                oa, om = outputs(alone[i]), outputs(mixed[i])
                assert np.array_equal(oa[0], om[0]) and np.array_equal(oa[1], om[1]) and oa[2] == om[2], (k, i)
            else:
                assert np.array_equal(before[i], mixed[i].get_state()), (k, i)
    with pytest.raises(b.ChanError) as ei:
        batch.step_subset([1, 1], None, 2)
    assert ei.value.code == b.CHAN_EINVAL
    batch.close()
    for e in alone + mixed:
        e.close()


def test_large_batch_matches_alone_bitwise():
    """17 channels of 32x65x32 (8432 columns per column launch) stepped as one batch end
    bitwise where each ends alone."""
    import paper_2301_09889_amd.binding as b
    specs = [(32, 65, 32, 180.0, ch.CTRL_EXTERNAL, ch.RAMP, ch.IC_REICHARDT, 20 + i) for i in range(17)]
    alone, mixed = make_envs(specs), make_envs(specs)
    batch = b.ChanBatch(mixed)
    for k in range(2):
        acts = actions_for(specs, k)
        for e, a in zip(alone, acts):
            e.step(a, 2)
        assert batch.step(acts, 2) == [0] * len(specs)
    for i, (ea, em) in enumerate(zip(alone, mixed)):
        assert np.array_equal(ea.get_state(), em.get_state()), i
        oa, om = outputs(ea), outputs(em)
        assert np.array_equal(oa[0], om[0]) and np.array_equal(oa[1], om[1]) and oa[2] == om[2], i
    batch.close()
    for e in alone + mixed:
        e.close()


def test_bench_batch_members_match_oracle():
    """The benchmark's 256-channel uneven batch (bench.py --workload batched), one env step of
    10 time steps in that launch configuration; sampled members (both shapes, both Re_tau,
    opposition and external actions) against the oracle from the same state."""
    import torch
    import paper_2301_09889_amd.binding as b
    import bench
    specs = bench.batched_specs(256, "uneven")
    envs, acts = [], []
    for sp in specs:
        grid = b.ChanGrid(sp["nx"], sp["ny"], sp["nz"], sp["lx"], sp["lz"], sp["re_tau"], sp["dt_plus"],
                          sp["obs_y_plus"])
        e = b.ChanEnv(grid, b.make_opts(controller=0 if sp["external"] else 1))
        e.reset(sp["seed"])
        envs.append(e)
        acts.append(torch.tensor(gaussian_action(1000 + sp["seed"], sp["nz"], sp["nx"]), dtype=torch.float64,
                                 device="cuda") if sp["external"] else None)
    sample = [0, 1, 3, 254]
    start = {i: envs[i].get_state() for i in sample}
    batch = b.ChanBatch(envs)
    assert batch.step(acts, 10) == [0] * len(specs)
    for i in sample:
        sp = specs[i]
        cfg = ch.Config(nx=sp["nx"], ny=sp["ny"], nz=sp["nz"], lx=sp["lx"], lz=sp["lz"], re_tau=sp["re_tau"],
                        dt_plus=sp["dt_plus"], obs_y_plus=sp["obs_y_plus"],
                        controller=ch.CTRL_EXTERNAL if sp["external"] else ch.CTRL_OPPOSITION)
        oenv = ch.Env(cfg)
        oenv.set_state(ch.state_from_flat(oenv.S, start[i]))
        obs_o, tau_o, drag_o = oenv.step(acts[i].cpu().numpy() if acts[i] is not None else None, 10)
        d = rel_state_diff(gpu_state(oenv.S, envs[i]), oenv.state)
        print(f"  member {i} {sp['nx']}x65x{sp['nz']} Re_tau {sp['re_tau']:.0f} "
              f"{'external' if sp['external'] else 'opposition'}: state rel diff {d:.3e}", flush=True)
        assert d <= 1e-11, i
        assert rel_field_diff(envs[i].obs.cpu().numpy(), obs_o) <= 1e-10
        assert rel_field_diff(envs[i].tau_w.cpu().numpy(), tau_o) <= 64 ** 2 * 1e-11
    batch.close()
    for e in envs:
        e.close()


def test_batch_tuning_reported():
    """The tuned launch shapes of the mix: one record per grid shape in first-seen order; the
    parity-major shapes with several channels get 2 or 4 columns per block, the general kernel 0;
    the mix's bitwise equality with the channels alone (above) holds whichever was picked."""
    import paper_2301_09889_amd.binding as b
    envs = make_envs(MIX)
    batch = b.ChanBatch(envs)
    t = b.chan_batch_tuning(batch.handle)
    print("  tuning:", t, flush=True)
    assert [(r["nx"], r["ny"], r["nz"]) for r in t] == [(16, 65, 16), (32, 65, 32), (8, 33, 8), (8, 97, 8)]
    assert t[0]["columns_per_block"] in (2, 4) and t[1]["columns_per_block"] in (2, 4)
    assert t[2]["columns_per_block"] == 4 and t[3]["columns_per_block"] == 0
    assert all(r["z_pencils_per_block"] > 0 and r["x_pairs_per_block"] > 0 for r in t)
    # the fused plane form exists for M_z, M_x in {48, 96} only (here the 32x65x32 channels)
    assert t[1]["plane_fused"] in (0, 1) and all(r["plane_fused"] == 0 for k, r in enumerate(t) if k != 1)
    batch.close()
    for e in envs:
        e.close()
