"""Writes turbulent_horizon.json: how long each seed of the turbulent drag workload stays
predictable under rounding, measured on the oracle alone.  Calls only oracle/.

Workload: the minimal channel of make_turbulent_drag.py (16x65x16, Re_tau 180, opposition
control at y+ 15), seeds 0-11.  For each seed the oracle is run again over the initial
transient (1000 env steps of 10 time steps, t+ 500) from the seeded field with v perturbed by
a relative 1e-15 (seeded normal factors, one per coefficient), and its block means (50 env
steps) are compared with the unperturbed run stored in turbulent_drag_minimal_12seeds.json.
Two codes that differ only by rounding cannot be expected to agree beyond the first block
where this self-divergence passes 1e-6; that block index is the seed's horizon (20 = the whole
transient stays below).

Run one process per seed, then combine:
    python tests/golden/make_turbulent_horizon.py --seed K --work DIR      (K = 0..11)
    python tests/golden/make_turbulent_horizon.py --combine --work DIR
Each seed takes about 35 minutes on one core.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import channel as ch  # noqa: E402

SEEDS = list(range(12))
N_ENV = 1000
N_SUB = 10
BLOCK = 50
REL_PERTURBATION = 1e-15
DIVERGED = 1e-6
GOLDEN12 = os.path.join(HERE, "turbulent_drag_minimal_12seeds.json")
OUT = os.path.join(HERE, "turbulent_horizon.json")


def config():
    return ch.Config(nx=16, ny=65, nz=16, lx=2.67, lz=0.8, re_tau=180.0, dt_plus=0.05, obs_y_plus=15.0,
                     controller=ch.CTRL_OPPOSITION, opp_alpha=1.0)


def run_seed(seed, work):
    os.makedirs(work, exist_ok=True)
    env = ch.Env(config())
    env.reset(seed)
    st = env.state.copy()
    rng = np.random.Generator(np.random.PCG64(9000 + seed))
    st.v = st.v * (1.0 + REL_PERTURBATION * rng.standard_normal(st.v.shape))
    env.set_state(st)
    drags = []
    t0 = time.time()
    for k in range(N_ENV):
        drags.append(env.step(None, N_SUB)[2])
        if k % 100 == 99:
            print(f"seed {seed}: {k + 1} env steps, {time.time() - t0:.0f} s", flush=True)
    blocks = np.asarray(drags).reshape(-1, BLOCK).mean(axis=1)
    np.save(os.path.join(work, f"horizon_seed{seed}.npy"), blocks)


def combine(work):
    with open(GOLDEN12) as fh:
        ref = json.load(fh)
    assert ref["block"] == BLOCK and ref["n_substeps"] == N_SUB
    out = {"seeds": SEEDS, "block": BLOCK, "n_env_steps": N_ENV, "rel_perturbation": REL_PERTURBATION,
           "diverged": DIVERGED, "self_divergence": {}, "horizon_blocks": {}}
    for s in SEEDS:
        pert = np.load(os.path.join(work, f"horizon_seed{s}.npy"))
        base = np.asarray(ref["block_means"][str(s)][:len(pert)])
        rel = np.abs(pert - base) / np.abs(base)
        over = np.nonzero(rel > DIVERGED)[0]
        out["self_divergence"][str(s)] = [float(r) for r in rel]
        out["horizon_blocks"][str(s)] = int(over[0]) if over.size else len(rel)
        print(f"seed {s}: horizon {out['horizon_blocks'][str(s)]} blocks; max self-divergence "
              f"in the first five blocks {rel[:5].max():.1e}")
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", OUT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--seed", type=int)
    ap.add_argument("--combine", action="store_true")
    ap.add_argument("--work", default="turbulent_horizon_work")
    a = ap.parse_args()
    if a.combine:
        combine(a.work)
    else:
        run_seed(a.seed, a.work)


if __name__ == "__main__":
    main()
