"""Turbulent mean-drag statistics on the GPU against the oracle.

Minimal channel 16x65x16 at Re_tau 180 under opposition control (sensing at y+ 15,
alpha = 1), seeds 0-11, 5000 env steps of 10 time steps (t+ 2500).  The oracle's drag
histories (block means of 50 env steps, t+ 25) were written by tests/golden/make_turbulent_drag.py,
which calls only oracle/; the GPU advances the twelve channels in one batch.

Both runs start from the same seeded fields and differ only by rounding, which the turbulent
flow amplifies.  How long a seed stays predictable was measured on the oracle alone
(tests/golden/make_turbulent_horizon.py -> turbulent_horizon.json: the same run with v perturbed
by a relative 1e-15, compared block by block): eleven seeds stay within 1e-6 of themselves over
the whole initial transient (t+ 0-500, which the paper's appendix puts at about t+ 500); seed 9
goes through a burst at t+ ~14-17 in which the drag jumps from 0.34 to 0.50, rounding grows
about fifty-fold per env step and the oracle diverges from itself within its first block.
What is compared:
* every block mean of the transient up to the seed's own horizon, per seed, to 1e-5 (the two
  codes integrate the same trajectory; measured ~1e-7), with at least ten seeds predictable
  over the whole transient;
* the mean drag of the seeds predictable over the transient (eleven) over the first turbulent
  window t+ 500-1000 to 1 %: these are still the same turbulent trajectories there (per-seed
  agreement ~1e-3), so the 1 % agreement is a parity statement, not a sampling outcome (the
  twelve-seed figure, with seed 9 an independent sample by then, is printed);
* the twelve-seed mean drag over t+ 500-2500 within three sampling errors of the difference.
  Past the decorrelation (t+ ~1250) this compares two samples of the same turbulence: the
  per-seed window means spread by ~7 %, so the sampling error of the difference of two
  twelve-seed means is ~2.5 %, and a 1 % agreement over this window is not resolved by twelve
  oracle seeds (about 100 per side would be needed, some 300 hours of the single-core oracle).
  Whether it happens to fall within 1 % is printed, not asserted.
"""
import json
import os

import numpy as np
import pytest

from oracle import channel as ch
from tests.gpu_helpers import grid_opts

pytestmark = pytest.mark.gpu

GOLDEN12 = os.path.join(os.path.dirname(__file__), "golden", "turbulent_drag_minimal_12seeds.json")
HORIZON = os.path.join(os.path.dirname(__file__), "golden", "turbulent_horizon.json")


def config():
    return ch.Config(nx=16, ny=65, nz=16, lx=2.67, lz=0.8, re_tau=180.0, dt_plus=0.05, obs_y_plus=15.0,
                     controller=ch.CTRL_OPPOSITION, opp_alpha=1.0)


def gpu_histories(seeds, n_env, n_sub):
    """Drag after every env step of each seed, all channels advanced in one batch."""
    import torch
    import paper_2301_09889_amd.binding as b
    grid, opts = grid_opts(config())
    envs = []
    for s in seeds:
        e = b.ChanEnv(grid, opts)
        e.reset(s)
        envs.append(e)
    batch = b.ChanBatch(envs)
    hist = torch.zeros((len(seeds), n_env), dtype=torch.float64, device="cuda")
    for k in range(n_env):
        codes = batch.step([None] * len(seeds), n_sub)
        assert codes == [0] * len(seeds), (k, codes)
        for i, e in enumerate(envs):
            hist[i, k] = e.drag[0]
        if k % 1000 == 999:
            print(f"  env step {k + 1} of {n_env}", flush=True)
    out = hist.cpu().numpy()
    batch.close()
    for e in envs:
        e.close()
    return out


@pytest.fixture(scope="module")
def runs():
    with open(GOLDEN12) as fh:
        ref = json.load(fh)
    g = gpu_histories(ref["seeds"], ref["n_env_steps"], ref["n_substeps"])
    return ref, g


def test_drag_histories_track_the_oracle(runs):
    ref, g = runs
    with open(HORIZON) as fh:
        hz = json.load(fh)
    assert hz["block"] == ref["block"] and hz["seeds"] == ref["seeds"]
    blk = ref["block"]
    gb = g.reshape(len(ref["seeds"]), -1, blk).mean(axis=2)
    n_transient = ref["window"][0] // blk
    whole = 0
    for i, s in enumerate(ref["seeds"]):
        ob = np.asarray(ref["block_means"][str(s)])
        r = np.abs(gb[i] - ob) / np.abs(ob)
        h = min(int(hz["horizon_blocks"][str(s)]), n_transient)
        within = np.nonzero(r > 1e-3)[0]
        tracked = (within[0] if within.size else r.size) * blk
        worst = f"{r[:h].max():.1e}" if h else "-"
        print(f"  seed {s}: oracle horizon {h} of {n_transient} transient blocks, max rel diff there {worst}; "
              f"blocks within 1e-3 up to env step {tracked}", flush=True)
        if h:
            assert r[:h].max() <= 1e-5, s
        whole += h == n_transient
    assert whole >= 10, whole


def _window(ref, g, a, b):
    blk = ref["block"]
    wg = np.array([g[i, a:b].mean() for i in range(len(ref["seeds"]))])
    wo = np.array([np.mean(ref["block_means"][str(s)][a // blk:b // blk]) for s in ref["seeds"]])
    return wg, wo


def test_mean_drag_first_turbulent_window_within_one_percent(runs):
    ref, g = runs
    with open(HORIZON) as fh:
        hz = json.load(fh)
    n_transient = ref["window"][0] // ref["block"]
    wg, wo = _window(ref, g, 1000, 2000)        # t+ 500-1000
    keep = np.array([int(hz["horizon_blocks"][str(s)]) >= n_transient for s in ref["seeds"]])
    rel = abs(wg[keep].mean() - wo[keep].mean()) / wo[keep].mean()
    rel_all = abs(wg.mean() - wo.mean()) / wo.mean()
    print(f"  mean drag, t+ 500-1000, the {keep.sum()} seeds predictable over the transient: GPU "
          f"{wg[keep].mean():.5f} oracle {wo[keep].mean():.5f} rel diff {rel:.1e}, per seed max "
          f"{np.max(np.abs(wg[keep] - wo[keep]) / wo[keep]):.1e}; all twelve: rel diff {rel_all:.1e}", flush=True)
    assert keep.sum() >= 10
    assert rel <= 0.01


def test_mean_drag_long_window_within_sampling_error(runs):
    ref, g = runs
    a, b = ref["window"]                         # t+ 500-2500
    wg, wo = _window(ref, g, a, b)
    assert abs(wo.mean() - ref["ensemble_window_mean"]) <= 1e-12
    n = len(ref["seeds"])
    rel = abs(wg.mean() - wo.mean()) / wo.mean()
    sig = np.sqrt(wg.var(ddof=1) / n + wo.var(ddof=1) / n) / wo.mean()
    print(f"  twelve-seed mean drag, t+ 500-2500: GPU {wg.mean():.5f} oracle {wo.mean():.5f} rel diff {rel:.4f} "
          f"(sampling error of the difference {sig:.4f}; within 1 %: {rel <= 0.01})", flush=True)
    assert rel <= 3 * sig
