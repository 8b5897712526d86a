"""Drag reduction by opposition control in the larger channel (§4.1: opposition control as the
classical baseline, sensing plane at y+ 10 and 15).

Every case runs as one channel per seed, all advanced together in one batch:
* uncontrolled: zero wall velocity (external controller, no action);
* opposition control with the sensing plane at each requested y+ (alpha = 1, zero net flux).
All channels: 64x65x64 modes, 2 pi x 2 x pi (h), Re_tau 180, dt+ 0.05, constant flow rate,
Reichardt mean profile with the seeded perturbation; or the minimal box (16x65x16,
2.67 x 2 x 0.8); closed channel, or with --top freeslip the open channel of §3.1 (a wall and a
free-slip surface at height h, the box 2 pi x 1 x pi or 2.67 x 1 x 0.8).  The drag (plane-mean
wall shear in wall units) is averaged over a window after the initial transient;
DR = 1 - D_controlled / D_uncontrolled with the means over the seeds.

    python -m paper_2301_09889_amd.drag_reduction [--env-steps 6000] [--seeds 0 1 2] [--y-plus 10 15]
        [--grid larger|minimal] [--top wall|freeslip]
"""
import argparse
import json
import time

import numpy as np

from . import binding as b

LARGER = dict(nx=64, ny=65, nz=64, lx=2 * np.pi, lz=np.pi, re_tau=180.0, dt_plus=0.05)
MINIMAL = dict(nx=16, ny=65, nz=16, lx=2.67, lz=0.8, re_tau=180.0, dt_plus=0.05)


def run(y_plus=(10.0, 15.0), seeds=(0, 1, 2), n_env=6000, n_sub=10, window_start=1000, grid=LARGER,
        progress=None, top_bc=b.CHAN_TOP_WALL, drop_failed=False):
    """Drag histories and drag reduction.  Returns a dict with, per case, the per-seed window
    means, their mean, and DR against the uncontrolled case.  A channel whose step fails (a
    non-finite state: opposition control with alpha = 1 diverges from some initial fields)
    raises, or with ``drop_failed`` is left out of its case's mean and listed under "failed"
    (the batch advances the other channels)."""
    import torch
    cases = [("uncontrolled", 15.0, b.CHAN_CTRL_EXTERNAL)] + \
            [(f"opposition y+{yp:g}", float(yp), b.CHAN_CTRL_OPPOSITION) for yp in y_plus]
    envs, labels = [], []
    for name, yp, ctrl in cases:
        for s in seeds:
            g = b.ChanGrid(grid["nx"], grid["ny"], grid["nz"], grid["lx"], grid["lz"], grid["re_tau"],
                           grid["dt_plus"], yp)
            e = b.ChanEnv(g, b.make_opts(controller=ctrl, ic_profile=1, top_bc=top_bc))
            e.reset(s)
            envs.append(e)
            labels.append((name, s))
    batch = b.ChanBatch(envs)
    hist = torch.zeros((len(envs), n_env), dtype=torch.float64, device=envs[0].obs.device)
    t0 = time.perf_counter()
    failed = {}
    try:
        for k in range(n_env):
            codes = batch.step(None, n_sub)
            bad = [i for i, c in enumerate(codes) if c != 0 and labels[i] not in failed]
            if bad and not drop_failed:
                raise RuntimeError(f"env step {k}: channels {[labels[i] for i in bad]} failed")
            for i in bad:
                failed[labels[i]] = k
            for i, e in enumerate(envs):
                hist[i, k] = e.drag[0]
            if progress and (k + 1) % 1000 == 0:
                progress(k + 1, time.perf_counter() - t0)
        h = hist.cpu().numpy()
    finally:
        batch.close()
        for e in envs:
            e.close()
    out = {"grid": [grid["nx"], grid["ny"], grid["nz"]], "top_bc": top_bc,
           "window_env_steps": [window_start, n_env], "t_plus_per_env_step": n_sub * grid["dt_plus"],
           "seeds": list(seeds), "cases": {}}
    for name, _, _ in cases:
        w = [float(h[i, window_start:].mean()) for i, lab in enumerate(labels) if lab[0] == name and lab not in failed]
        out["cases"][name] = {"window_mean_per_seed": w, "mean": float(np.mean(w)),
                              "std_error": float(np.std(w, ddof=1) / np.sqrt(len(w))) if len(w) > 1 else None}
    out["failed"] = [{"case": nm, "seed": sd, "env_step": k} for (nm, sd), k in failed.items()]
    ref = out["cases"]["uncontrolled"]["mean"]
    for c in out["cases"].values():
        c["drag_reduction"] = 1.0 - c["mean"] / ref
    out["elapsed_s"] = time.perf_counter() - t0
    out["histories"] = {f"{nm} seed {s}": h[i].tolist() for i, (nm, s) in enumerate(labels) if (nm, s) not in failed}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--env-steps", type=int, default=6000)
    ap.add_argument("--window-start", type=int, default=1000)
    ap.add_argument("--seeds", type=int, nargs="+", default=[0, 1, 2])
    ap.add_argument("--y-plus", type=float, nargs="+", default=[10.0, 15.0])
    ap.add_argument("--grid", choices=["larger", "minimal"], default="larger")
    ap.add_argument("--top", choices=["wall", "freeslip"], default="wall")
    ap.add_argument("--histories", help="write the drag histories (JSON) to this file")
    ap.add_argument("--drop-failed", action="store_true", help="leave diverged channels out instead of stopping")
    args = ap.parse_args()
    res = run(args.y_plus, args.seeds, args.env_steps, window_start=args.window_start,
              grid=LARGER if args.grid == "larger" else MINIMAL,
              top_bc=b.CHAN_TOP_FREESLIP if args.top == "freeslip" else b.CHAN_TOP_WALL,
              progress=lambda k, t: print(f"env step {k} ({t:.0f} s)", flush=True), drop_failed=args.drop_failed)
    hist = res.pop("histories")
    if args.histories:
        with open(args.histories, "w") as fh:
            json.dump(hist, fh)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
