"""Writes turbulent_drag_minimal.json: the oracle's drag history of the minimal channel under
opposition control, for the GPU-vs-oracle mean-drag statistics test.  Calls only oracle/.

Workload: minimal channel 2.67 x 2 x 0.8 (h), 16x65x16, Re_tau 180, dt+ 0.05, constant flow
rate, opposition control sensing at y+ 15 (alpha = 1), seeded initial field (seeds 0-5, the
paper's six initial conditions), 5000 env steps of 10 time steps (t+ 2500).  The statistic is
the mean over t+ 500 - 2500 of the drag (plane-mean wall shear averaged over each env step),
per seed and over the six seeds.

Run one process per seed, then combine:
    python tests/golden/make_turbulent_drag.py --seed K --work DIR      (K = 0..5)
    python tests/golden/make_turbulent_drag.py --combine --work DIR
The six seeds 0-5 give turbulent_drag_minimal.json; with --nseeds 12 (seeds 0-11, run the
same way) the combination goes to turbulent_drag_minimal_12seeds.json.
Each seed takes about three hours on one core; partial histories are saved in DIR every 100
env steps and a restarted run continues from them.
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

SEEDS = list(range(6))
N_ENV = 5000          # env steps of N_SUB time steps
N_SUB = 10
WINDOW = (1000, 5000)  # env steps averaged: t+ 500 .. 2500
BLOCK = 50             # env steps per stored block mean (t+ 25)
OUT = os.path.join(HERE, "turbulent_drag_minimal.json")


def config():
    return ch.Config(nx=16, ny=65, nz=16, lx=2.67, lz=0.8, re_tau=180.0, dt_plus=0.05, obs_y_plus=15.0,
                     controller=ch.CTRL_OPPOSITION, opp_alpha=1.0)


def run_seed(seed, work):
    """Advance the oracle for one seed, saving the drag history (and the state, to resume)."""
    os.makedirs(work, exist_ok=True)
    path = os.path.join(work, f"seed{seed}.npz")
    env = ch.Env(config())
    drags = []
    if os.path.exists(path):
        z = np.load(path)
        drags = list(z["drag"])
        env.set_state(ch.state_from_flat(env.S, z["state"]))
    else:
        env.reset(seed)
    t0 = time.time()
    while len(drags) < N_ENV:
        _, _, d = env.step(None, N_SUB)
        drags.append(float(d))
        if len(drags) % 100 == 0 or len(drags) == N_ENV:
            tmp = path + ".tmp.npz"
            np.savez(tmp, drag=np.array(drags), state=ch.state_to_flat(env.S, env.state))
            os.replace(tmp, path)
            print(f"seed {seed}: {len(drags)} env steps, {time.time() - t0:.0f} s", flush=True)


def combine(work, seeds=SEEDS, out_path=OUT):
    series = {}
    for s in seeds:
        z = np.load(os.path.join(work, f"seed{s}.npz"))
        d = z["drag"]
        if d.size < N_ENV:
            raise SystemExit(f"seed {s}: only {d.size} of {N_ENV} env steps")
        series[s] = d[:N_ENV]
    a, b = WINDOW
    out = {
        "what": "oracle drag history, minimal channel 16x65x16, Re_tau 180, dt+ 0.05, CFR, opposition control "
                "at y+ 15 (alpha 1), seeded initial fields; env step = 10 time steps",
        "written_by": "tests/golden/make_turbulent_drag.py (oracle only)",
        "seeds": list(seeds), "n_env_steps": N_ENV, "n_substeps": N_SUB, "window": [a, b], "block": BLOCK,
        "window_mean": {str(s): float(series[s][a:b].mean()) for s in seeds},
        "block_means": {str(s): [float(x) for x in series[s].reshape(-1, BLOCK).mean(axis=1)] for s in seeds},
    }
    out["ensemble_window_mean"] = float(np.mean([out["window_mean"][str(s)] for s in seeds]))
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"wrote {out_path}: ensemble window mean {out['ensemble_window_mean']:.6f}")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--seed", type=int)
    ap.add_argument("--combine", action="store_true")
    ap.add_argument("--work", required=True)
    ap.add_argument("--nseeds", type=int, default=len(SEEDS), help="combine seeds 0 .. nseeds-1")
    args = ap.parse_args()
    os.makedirs(args.work, exist_ok=True)
    if args.combine:
        if args.nseeds == len(SEEDS):
            combine(args.work)
        else:
            combine(args.work, list(range(args.nseeds)),
                    os.path.join(HERE, f"turbulent_drag_minimal_{args.nseeds}seeds.json"))
    else:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            run_seed(args.seed, args.work)


if __name__ == "__main__":
    main()
