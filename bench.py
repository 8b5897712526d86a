#!/usr/bin/env python
"""Benchmark of the channel-flow DNS environment step on one MI355X.

Workload (the larger channel of §3.1, closed-channel reading): 2 pi h x 2h x pi h,
64 x 65 x 64 modes, Re_tau = 180, dt+ = 0.05, Reichardt mean profile plus a seeded
perturbation, one env step = a seeded Gaussian wall-velocity action (sigma = 0.1
u_tau, plane mean removed) held for 10 RK3/CN time steps, then the observation
plane (u, v at y+ = 15 -> node y+ 17.3), the wall-shear field and the drag.  All
actions are on the device before the timed region starts.

Prints one JSON line: env-steps/s (whole job), grid-point-substeps/s, p50/p99 env
step latency, the roofline entry of the dominant kernel measured with HIP events
inside the timed region, and the oracle timed on the host as the CPU baseline.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "DNS env-steps/sec & grid-pt-substeps/s vs plain; p50/p99 step latency"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6

LARGER = dict(nx=64, ny=65, nz=64, lx=2 * np.pi, lz=np.pi, re_tau=180.0, dt_plus=0.05, obs_y_plus=15.0)
MINIMAL = dict(nx=16, ny=65, nz=16, lx=2.67, lz=0.8, re_tau=180.0, dt_plus=0.05, obs_y_plus=15.0)
RE395 = dict(nx=128, ny=97, nz=128, lx=2 * np.pi, lz=np.pi, re_tau=395.0, dt_plus=0.05, obs_y_plus=15.0)


# HBM bytes per launch on the larger channel, from two rocprofv3 --pmc runs of
# "bench.py --steps 3 --warmup 1 --no-cpu-baseline --copy-probe" (FETCH_SIZE, then WRITE_SIZE,
# KiB per dispatch; profiles/hbm_traffic_larger_channel.md).  FETCH_SIZE is scaled by 2.0 and
# WRITE_SIZE by 1.0: what the two counters read for the 256 MiB device copy of --copy-probe
# (131084 and 262144 KiB).  Each figure holds for the kernel source with the listed SHA-256
# (plane_pass.hip includes small_dft.inc, unchanged since) and is reported as null for any
# other source.  The plane figures are the three-launch form the tuner keeps for one channel.
TRAFFIC = {
    "column_solve_reconstruct": (3.8932e+07, "column_pass.hip", "d9c39fcd5336c91daa763a605300bc19ab60214ffbb05590762bcbdc319b2779"),
    "x_rows_fft_product": (2.8902e+07, "plane_pass.hip", "8a08bd7f959abeedfc6fc9893ee51a5a8ae72b7da0de4e745d7d1def2938cc33"),
    "z_inverse_fft": (3.2047e+07, "plane_pass.hip", "8a08bd7f959abeedfc6fc9893ee51a5a8ae72b7da0de4e745d7d1def2938cc33"),
    "z_forward_fft": (1.6087e+07, "plane_pass.hip", "8a08bd7f959abeedfc6fc9893ee51a5a8ae72b7da0de4e745d7d1def2938cc33"),
    "column_pass": (2.4452e+07, "column_pass.hip", "d9c39fcd5336c91daa763a605300bc19ab60214ffbb05590762bcbdc319b2779"),
    "column_reconstruct": (1.7564e+07, "column_pass.hip", "d9c39fcd5336c91daa763a605300bc19ab60214ffbb05590762bcbdc319b2779"),
}


def measured_traffic(kclass, workload):
    """Profiled HBM bytes per launch of a kernel class on the larger channel, or None (other
    workload, or the kernel source changed since the counters were taken)."""
    if workload != "larger" or kclass not in TRAFFIC:
        return None
    nbytes, src, sha = TRAFFIC[kclass]
    path = os.path.join(ROOT, "paper_2301_09889_amd", "csrc", src)
    try:
        with open(path, "rb") as fh:
            ok = hashlib.sha256(fh.read()).hexdigest() == sha
    except OSError:
        ok = False
    return nbytes if ok else None


def resolved_points(g):
    """K = (N_x/2)(N_z - 1) N_y: complex spectral unknowns of one field."""
    return (g["nx"] // 2) * (g["nz"] - 1) * g["ny"]


def algorithmic_bytes_per_launch(kclass, g, n_sub=10):
    """Minimum HBM bytes one launch of a kernel class must move, from the
    two-layout pass model: 16 K bytes per complex field pass.  The column solve
    reads H (3 fields), v and omega_y (2) and, from the second stage on, the
    previous stage's h_v, h_g (2); it writes v, omega_y (2) and h_v, h_g (2, first
    two stages): 9 2/3 passes per launch on average over the three stages.  The
    column reconstruction reads v, omega_y (2) and writes the six node fields for
    the plane pass (6); run in the same launch as the solve it reads nothing more
    (15 2/3 passes for both).  Precomputed operator tables are not counted.  The general
    column kernel (N_y > 65) runs solve and reconstruction in one launch of the column_pass
    class except at the last stage of an env step: the mean over the 3 n_sub launches."""
    K = resolved_points(g)
    if kclass == "column_pass" and g["ny"] > 65:
        solve, both = 3 + 2 + 2.0 / 3.0 * 2 + 2 + 2.0 / 3.0 * 2, 3 + 2 + 2.0 / 3.0 * 2 + 2 + 2.0 / 3.0 * 2 + 6
        n = 3 * n_sub
        return ((n - 1) * both + solve) / n * 16.0 * K
    if kclass == "column_pass":
        return (3 + 2 + 2.0 / 3.0 * 2 + 2 + 2.0 / 3.0 * 2) * 16.0 * K
    if kclass == "column_reconstruct":
        return (2 + 6) * 16.0 * K
    if kclass == "column_solve_reconstruct":     # both parts in one launch: no state reload
        return (3 + 2 + 2.0 / 3.0 * 2 + 2 + 2.0 / 3.0 * 2 + 6) * 16.0 * K
    nkx, ny, mz = g["nx"] // 2, g["ny"], 3 * g["nz"] // 2
    padded = 16.0 * ny * mz * nkx          # one field on the z-padded intermediate
    if kclass == "z_inverse_fft":
        return 6 * 16.0 * K + 6 * padded
    if kclass == "x_rows_fft_product":
        return 6 * padded + 3 * padded
    if kclass == "z_forward_fft":
        return 3 * padded + 3 * 16.0 * K
    return None


def path_bytes_per_substep(g):
    """Algorithmic bytes of one RK3/CN time step over the whole path: 74 complex-field passes
    of 16 K bytes (13 per stage in the column pass, 9 per stage in the plane pass, 8 of
    history per step)."""
    return 74 * 16.0 * resolved_points(g)


def path_flops_per_substep(g):
    """Algorithmic FP64 flops of one time step: per stage the 9 padded 2D FFTs at every node
    (2.5 M log2 M each), the 9 Chebyshev transforms of every column (as real FFTs of 2N),
    the products and ~120 flops per unknown for the solves."""
    nx, ny, nz = g["nx"], g["ny"], g["nz"]
    mx, mz = 3 * nx // 2, 3 * nz // 2
    n = ny - 1
    m = mx * mz
    fft = 9 * ny * 2.5 * m * np.log2(m)
    dct = 9 * (nx // 2) * (nz - 1) * 2 * 2.5 * 2 * n * np.log2(2 * n)
    return 3 * (fft + dct + 9 * m * ny + 120 * resolved_points(g))


def copy_bandwidth_gbs(torch, nbytes=256 * 1024 * 1024, reps=10):
    """Achievable device copy bandwidth (read + write bytes per second) of a plain copy."""
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    return 2.0 * nbytes * reps / (e0.elapsed_time(e1) / 1e3) / 1e9


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _oracle_sample(job):
    """One oracle process of the CPU baseline: warm-up time step, then budget_substeps time
    steps of one env step of the workload on one BLAS thread; returns their wall seconds."""
    g, opts_kw, seed, budget_substeps = job
    from threadpoolctl import threadpool_limits

    from oracle import channel as ch
    from synth import gaussian_action
    env = ch.Env(ch.Config(**g, **opts_kw))
    env.reset(seed)
    act = gaussian_action(1000 + seed, g["nz"], g["nx"])
    with threadpool_limits(limits=1):
        env.step(act, 1)  # warm caches and matrices
        t0 = time.perf_counter()
        env.step(act, budget_substeps)
        return time.perf_counter() - t0


def host_cores():
    """Cores this process may run on, capped at 16 (the host share of one GPU)."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


def cpu_baseline(g, opts_kw, n_sub_env, seed, budget_substeps):
    """The oracle (test infrastructure) on a bounded sample of the same workload: one process
    per available core (each on its own seed, one BLAS thread, all at once; throughputs
    summed), and the single-core figure of the first of them run alone.  Runs before any GPU
    work (the processes are forked)."""
    import multiprocessing as mp
    single = _oracle_sample((g, opts_kw, seed, budget_substeps))
    n = host_cores()
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(n) as pool:
        times = pool.map(_oracle_sample, [(g, opts_kw, seed + k, budget_substeps) for k in range(n)])
    wall = time.perf_counter() - t0
    per_env_step = [t / budget_substeps * n_sub_env for t in times]
    total = float(sum(1.0 / t for t in per_env_step))
    return {"value": total, "unit": "env-steps/s", "cores": n, "kind": "oracle",
            "host_cpu": host_cpu_model(), "host_cores_available": len(os.sched_getaffinity(0)),
            "single_core_value": 1.0 / (single / budget_substeps * n_sub_env),
            "sample": f"{n} oracle processes at once, one per core and one BLAS thread each, seeds {seed}.."
                      f"{seed + n - 1}, each {budget_substeps} time steps of one env step of the same workload "
                      f"(slowest {max(times):.1f} s, {wall:.1f} s wall with start-up), scaled to {n_sub_env} time "
                      f"steps per env step and summed; single_core_value: the first alone ({single:.1f} s)"}


def batched_specs(n, mix="uneven"):
    """Uneven mix: 16x65x16 and 32x65x32 minimal-box channels alternating, Re_tau 180 / 100 in
    pairs, seed = channel index; opposition control on the 16x65x16 channels at Re_tau 180,
    Gaussian wall actions on the others (opposition control with alpha = 1 from the seeded
    initial fields diverges for some seeds at Re_tau 100 and on 32x65x32, in the oracle too)."""
    specs = []
    for i in range(n):
        m = 16 if (i % 2 == 0 or mix == "minimal") else 32
        re = 180.0 if (i // 2) % 2 == 0 else 100.0
        specs.append(dict(nx=m, ny=65, nz=m, lx=2.67, lz=0.8, re_tau=re, dt_plus=0.05, obs_y_plus=15.0,
                          external=not (m == 16 and re == 180.0), seed=i))
    return specs


def run_batched(args, torch, b, gaussian_action):
    """Many channels advanced together (one launch per kernel and grid shape), against the same
    channels advanced one per launch."""
    specs = batched_specs(args.channels, args.mix)
    torch.cuda.set_device(0)
    envs, acts = [], []
    for sp in specs:
        grid = b.ChanGrid(sp["nx"], sp["ny"], sp["nz"], sp["lx"], sp["lz"], sp["re_tau"], sp["dt_plus"],
                          sp["obs_y_plus"])
        e = b.ChanEnv(grid, b.make_opts(controller=0 if sp["external"] else 1))
        e.reset(sp["seed"])
        envs.append(e)
        acts.append(torch.tensor(gaussian_action(1000 + sp["seed"], sp["nz"], sp["nx"]), dtype=torch.float64,
                                 device="cuda") if sp["external"] else None)
    batch = b.ChanBatch(envs)
    tuning = b.chan_batch_tuning(batch.handle)
    for _ in range(args.warmup):
        batch.step(acts, args.substeps)
    torch.cuda.synchronize()
    lat, codes = [], []
    done = 0                                  # env steps completed (a diverged channel stops)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        codes = batch.step(acts, args.substeps)
        lat.append(time.perf_counter() - s0)
        done += sum(1 for c in codes if c == 0)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    active = sum(1 for c in codes if c == 0)
    value = done / elapsed
    b.chan_batch_set_timing(batch.handle, 1)
    batch.step(acts, args.substeps)
    kt = b.chan_batch_timing_read(batch.handle)
    b.chan_batch_set_timing(batch.handle, 0)
    # host time to enqueue one batch step (asynchronous launch, returns once every launch is
    # queued) against the whole step: what capturing the launches in a graph could save at most
    enq, whole = [], []
    for _ in range(5):
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        call = batch.launch(envs, acts, args.substeps, [e.obs for e in envs], [e.tau_w for e in envs],
                            [e.drag for e in envs], stream=torch.cuda.current_stream())
        s1 = time.perf_counter()
        call.finish()
        whole.append(time.perf_counter() - s0)
        enq.append(s1 - s0)
    # the same batch step captured once as a HIP graph and replayed (same buffers each time)
    graph_value = None
    try:
        gr = batch.capture(envs, acts, args.substeps, [e.obs for e in envs], [e.tau_w for e in envs],
                           [e.drag for e in envs])
        gr.launch().finish()
        torch.cuda.synchronize()
        n_rep, gdone = max(5, args.steps // 4), 0
        t2 = time.perf_counter()
        for _ in range(n_rep):
            gdone += sum(1 for c in gr.launch().finish() if c == 0)
        torch.cuda.synchronize()
        graph_value = gdone / (time.perf_counter() - t2)
        gr.close()
    except b.ChanError as err:                # a diverged channel has no valid state to capture
        print(f"graph replay skipped: {err}", file=sys.stderr, flush=True)
    # the plain form: the same kind of channels, one channel per launch
    sub = list(range(min(16, len(envs))))
    for i in sub:
        envs[i].step(acts[i], args.substeps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    reps = 3
    for _ in range(reps):
        for i in sub:
            envs[i].step(acts[i], args.substeps)
    torch.cuda.synchronize()
    plain = len(sub) * reps / (time.perf_counter() - t1)
    # and one captured graph per channel, replayed one channel at a time
    plain_graph = None
    try:
        graphs = [envs[i].capture(acts[i], args.substeps) for i in sub]
        for gi in graphs:
            gi.launch().finish()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(reps):
            for gi in graphs:
                gi.launch().finish()
        torch.cuda.synchronize()
        plain_graph = len(sub) * reps / (time.perf_counter() - t1)
        for gi in graphs:
            gi.close()
    except b.ChanError as err:
        print(f"plain graph replay skipped: {err}", file=sys.stderr, flush=True)
    batch.close()
    path_bytes = sum(path_bytes_per_substep(sp) for k, sp in enumerate(specs) if codes[k] == 0)
    sub_s = elapsed / (args.steps * args.substeps)
    copy_gbs = copy_bandwidth_gbs(torch)
    lat_ms = np.array(lat) * 1e3
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "env-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"batched: {len(specs)} minimal-box channels (2.67 x 2 x 0.8 h), "
                               + ("16x65x16 and 32x65x32 alternating" if args.mix == "uneven" else "all 16x65x16")
                               + ", Re_tau 180/100, opposition control (16x65x16 at Re_tau 180) or Gaussian wall "
                               "actions sigma 0.1 u_tau, 10 time steps per env step, one batch step advances "
                               "every channel",
                   "channels": len(specs), "active_channels": active, "substeps_per_env_step": args.substeps},
        "grid_pt_substeps_per_s": sum(sp["nx"] * sp["ny"] * sp["nz"] for k, sp in enumerate(specs) if codes[k] == 0)
        * args.steps * args.substeps / elapsed,
        "env_steps_completed": done,
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99))},
        "plain_one_channel_per_launch": {"value": plain, "unit": "env-steps/s",
                                         "sample": f"channels 0-{len(sub) - 1} of the mix, each stepped alone",
                                         "graph_replay_value": plain_graph},
        "tuning": tuning,
        "graph_replay": {"value": graph_value, "unit": "env-steps/s",
                         "note": "the batch step captured once as a HIP graph (chan_batch_capture) and replayed"},
        "host_enqueue_ms": {"enqueue_p50": 1e3 * float(np.median(enq)), "step_p50": 1e3 * float(np.median(whole)),
                            "note": "host time to queue one batch step's launches vs the whole step (5 steps)"},
        "batched_over_plain": value / plain,
        "roofline": None,
        "path_roofline": {"alg_bytes_per_substep": path_bytes, "achieved_GBs": path_bytes / sub_s / 1e9,
                          "frac_hbm_peak": path_bytes / sub_s / 1e9 / HBM_PEAK_GBS,
                          "frac_copy": path_bytes / sub_s / 1e9 / copy_gbs},
        "copy_bandwidth_GBs": copy_gbs,
        "kernels_ms_per_env_step": {k: round(v[1], 3) for k, v in kt.items() if v[0] > 0},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def run_served(args, torch, b, gaussian_action):
    """Request loop: Poisson arrivals from many workers, one channel each on mixed grids, served
    with continuous batching (paper_2301_09889_amd.serve)."""
    from paper_2301_09889_amd.serve import ChannelServer, run_open_loop
    torch.cuda.set_device(0)
    free, _ = torch.cuda.mem_get_info()
    server = ChannelServer(hbm_budget=free // 2)
    sizes = (16, 32, 64)
    lx = {16: 2.67, 32: 2.67, 64: 2 * np.pi}
    lz = {16: 0.8, 32: 0.8, 64: np.pi}
    ids, grid_of = [], []
    t_setup = time.perf_counter()
    for w in range(args.workers):
        m = sizes[w % 3]
        grid = b.ChanGrid(m, 65, m, lx[m], lz[m], 180.0, 0.05, 15.0)
        cid = server.admit(grid, b.make_opts(controller=0, ic_profile=1), w)
        if cid is not None:
            ids.append(cid)
            grid_of.append(m)
    t_setup = time.perf_counter() - t_setup
    rng = np.random.default_rng(args.seed)
    acts = {}

    def make_action(cid, k):
        key = (cid, k % 4)
        if key not in acts:
            m = grid_of[cid]
            acts[key] = torch.tensor(gaussian_action(1000 + 7 * cid + k % 4, m, m), dtype=torch.float64, device="cuda")
        return acts[key]

    # warm-up: every channel once (also builds the batch and tunes the tilings)
    for cid in ids:
        server.submit(cid, make_action(cid, 0), args.substeps)
    while server.has_pending():
        server.step_once()
    torch.cuda.synchronize()
    # closed loop: every channel always has a request pending (saturation); each channel's next
    # request is submitted as soon as its last one is polled done
    t0 = time.perf_counter()
    n_done = 0
    left = {cid: 2 for cid in ids}
    for cid in ids:
        server.submit(cid, make_action(cid, 1), args.substeps)
    while server.has_pending():
        server.launch()
        for r in server.poll():
            n_done += 1 if r.code == 0 else 0
            if left[r.channel] > 0:
                left[r.channel] -= 1
                server.submit(r.channel, make_action(r.channel, 1), args.substeps)
    sat = n_done / (time.perf_counter() - t0)
    sweep = []
    for rate in [float(x) for x in args.rates.split(",")]:
        gaps = rng.exponential(1.0 / rate, size=args.requests)
        arrivals = list(zip(np.cumsum(gaps), rng.integers(0, len(ids), size=args.requests)))
        done, wall = run_open_loop(server, [(float(t), int(c)) for t, c in arrivals], make_action, args.substeps)
        lat = np.array([(r.t_done - r.t_arrival) * 1e3 for r in done if r.code == 0])
        sweep.append({"offered_per_s": rate, "served_per_s": len(lat) / wall, "p50_ms": float(np.percentile(lat, 50)),
                      "p99_ms": float(np.percentile(lat, 99)), "requests": len(done)})
    server.close()
    out = {
        "metric": METRIC,
        "value": sat,
        "unit": "env-steps/s",
        "n_gpus": 1,
        "steps": 3,
        "warmup": 1,
        "ms_per_step": 1e3 * len(ids) / sat,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"served: {args.workers} workers, one channel each, grids 16x65x16 / 32x65x32 / "
                               f"64x65x64 in thirds (minimal box for 16 and 32, 2pi x 2 x pi for 64), Re_tau 180, "
                               f"Gaussian wall actions, {args.substeps} time steps per request, admission by HBM "
                               f"footprint against half the free HBM",
                   "admitted": len(ids), "rejected": server.rejected_channels, "hbm_budget_bytes": server.budget,
                   "hbm_admitted_bytes": server.used, "setup_s": t_setup},
        "saturation": {"value": sat, "note": "closed loop: every channel always has one request pending"},
        "sweep": sweep,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def run_scale(args, torch, b, gaussian_action):
    """Batched and served at scale: 8 channels of 128x97x128 at Re_tau 395 and 64 minimal
    channels in one request loop (continuous batching, admission by HBM footprint), every
    channel advancing 2000 time steps in requests of args.substeps with Gaussian zero-net-flux
    actions; closed loop (each channel submits its next request as soon as the last is done)."""
    from paper_2301_09889_amd.serve import ChannelServer
    torch.cuda.set_device(0)
    free, _ = torch.cuda.mem_get_info()
    server = ChannelServer(hbm_budget=free // 2)
    mix = [(RE395, 8), (MINIMAL, 64)]
    ids, kind = [], []
    for gi, (g, count) in enumerate(mix):
        for i in range(count):
            grid = b.ChanGrid(g["nx"], g["ny"], g["nz"], g["lx"], g["lz"], g["re_tau"], g["dt_plus"],
                              g["obs_y_plus"])
            cid = server.admit(grid, b.make_opts(controller=0, ic_profile=1), 100 * gi + i)
            if cid is not None:
                ids.append(cid)
                kind.append(gi)
    acts = {}

    def make_action(cid, k):
        key = (cid, k % 4)
        if key not in acts:
            g = mix[kind[cid]][0]
            acts[key] = torch.tensor(gaussian_action(5000 + 7 * cid + k % 4, g["nz"], g["nx"]),
                                     dtype=torch.float64, device="cuda")
        return acts[key]

    for cid in ids:  # warm-up: builds the batch and tunes the plane-pass tilings
        server.submit(cid, make_action(cid, 0), args.substeps)
    while server.has_pending():
        server.step_once()
    torch.cuda.synchronize()
    n_req = max(1, 2000 // args.substeps)
    left = {cid: n_req - 1 for cid in ids}
    lat = {0: [], 1: []}
    failed = 0
    t0 = time.perf_counter()
    for cid in ids:
        server.submit(cid, make_action(cid, 1), args.substeps)
    while server.has_pending():
        server.launch()
        for r in server.poll():
            if r.code != 0:
                failed += 1
                continue
            lat[kind[r.channel]].append((r.t_done - r.t_arrival) * 1e3)
            if left[r.channel] > 0:
                left[r.channel] -= 1
                server.submit(r.channel, make_action(r.channel, n_req - left[r.channel]), args.substeps)
    wall = time.perf_counter() - t0
    server.close()
    done = sum(len(v) for v in lat.values())
    pct = {name: {"p50_ms": float(np.percentile(lat[gi], 50)), "p99_ms": float(np.percentile(lat[gi], 99)),
                  "requests": len(lat[gi])}
           for gi, name in enumerate(["128x97x128", "16x65x16"]) if lat[gi]}
    out = {
        "metric": METRIC,
        "value": done / wall,
        "unit": "env-steps/s",
        "n_gpus": 1,
        "steps": n_req,
        "warmup": 1,
        "ms_per_step": 1e3 * wall / n_req,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"batched and served at scale: 8 channels 128x97x128 (2pi x 2 x pi h, Re_tau 395) "
                               f"and 64 minimal channels 16x65x16 (Re_tau 180) in one request loop, Gaussian "
                               f"wall actions, {n_req} requests of {args.substeps} time steps per channel, "
                               f"closed loop", "admitted": len(ids), "rejected": server.rejected_channels},
        "grid_pt_substeps_per_s": sum(mix[k][0]["nx"] * mix[k][0]["ny"] * mix[k][0]["nz"] for k in kind)
                                  * n_req * args.substeps / wall,
        "latency_ms": pct,
        "failed_requests": failed,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100, help="timed env steps")
    ap.add_argument("--warmup", type=int, default=5, help="untimed env steps")
    ap.add_argument("--substeps", type=int, default=10, help="RK3 time steps per env step")
    ap.add_argument("--workload", choices=["larger", "minimal", "re395", "batched", "served", "scale"], default="larger")
    ap.add_argument("--workers", type=int, default=512, help="workers (one channel each) of the served workload")
    ap.add_argument("--rates", default="200,1000,4000", help="offered request rates (1/s) of the served sweep")
    ap.add_argument("--requests", type=int, default=600, help="requests per rate of the served sweep")
    ap.add_argument("--channels", type=int, default=256, help="channels of the batched workload")
    ap.add_argument("--mix", choices=["uneven", "minimal"], default="uneven",
                    help="batched workload: 16x65x16 / 32x65x32 alternating, or 16x65x16 only")
    ap.add_argument("--top", choices=["wall", "freeslip"], default="wall",
                    help="larger/minimal workloads: closed channel (wall) or open channel (free-slip top)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-substeps", type=int, default=8, help="time steps in the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the benchmark, run a plain 256 MiB device copy (for scaling the HBM "
                         "byte counters of a profiler run)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the channel step runs on a single MI355X; "
              "multi-GPU sharding is a design note only (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2301_09889_amd.binding as b
    from synth import gaussian_action

    if args.workload == "batched":
        run_batched(args, torch, b, gaussian_action)
        return
    if args.workload == "served":
        run_served(args, torch, b, gaussian_action)
        return
    if args.workload == "scale":
        run_scale(args, torch, b, gaussian_action)
        return
    g = {"larger": LARGER, "minimal": MINIMAL, "re395": RE395}[args.workload]
    if args.workload == "re395":
        opts_kw = dict(ic_profile=1, action_mode=1)
        workload = ("channel at Re_tau 395, 2pi x 2 x pi (h), 128x97x128 modes (general column kernel), "
                    "dt+ 0.05, seeded Gaussian wall action sigma 0.1 u_tau held for 10 time steps, obs u,v at y+ 15")
    elif args.workload == "larger":
        opts_kw = dict(ic_profile=1, action_mode=1)    # Reichardt mean; action held over the env step
        workload = ("larger channel 2pi x 2 x pi (h), 64x65x64 modes, Re_tau 180, dt+ 0.05, seeded Gaussian "
                    "wall action sigma 0.1 u_tau held for 10 time steps, obs u,v at y+ 15")
    else:
        opts_kw = dict(controller=1)                   # opposition control at y+ = 15
        workload = ("minimal channel 2.67 x 2 x 0.8 (h), 16x65x16 modes, Re_tau 180, dt+ 0.05, opposition "
                    "control sensing at y+ 15")
    if args.top == "freeslip":
        opts_kw["top_bc"] = 1
        workload = "open " + workload.replace(" x 2 x ", " x 1 x ")
    # the oracle's CPU figure first, before any GPU work (its processes are forked)
    cpu = None
    if not args.no_cpu_baseline and args.workload != "re395":  # one oracle time step takes minutes there
        cpu = cpu_baseline(g, opts_kw, args.substeps, args.seed, args.cpu_substeps)
        print(f"cpu baseline: {cpu['value']:.3f} env-steps/s on {cpu['cores']} cores", file=sys.stderr, flush=True)
    torch.cuda.set_device(0)
    grid = b.ChanGrid(g["nx"], g["ny"], g["nz"], g["lx"], g["lz"], g["re_tau"], g["dt_plus"], g["obs_y_plus"])
    opts = b.make_opts(**opts_kw)
    env = b.ChanEnv(grid, opts)
    env.reset(args.seed)
    n_act = args.warmup + 2 * args.steps
    acts = torch.stack([torch.tensor(gaussian_action(1000 + args.seed + k, g["nz"], g["nx"]),
                                     dtype=torch.float64) for k in range(n_act)]).cuda()
    use_action = args.workload in ("larger", "re395")
    for k in range(args.warmup):
        env.step(acts[k] if use_action else None, args.substeps)
    torch.cuda.synchronize()

    # timed region: throughput and per-step latency (timing instrumentation off)
    lat = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        s0 = time.perf_counter()
        env.step(acts[args.warmup + k] if use_action else None, args.substeps)
        lat.append(time.perf_counter() - s0)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    # same number of env steps with every kernel bracketed by HIP events on the env's stream
    b.chan_env_set_timing(env.handle, 1)
    t1 = time.perf_counter()
    for k in range(args.steps):
        env.step(acts[args.warmup + args.steps + k] if use_action else None, args.substeps)
    torch.cuda.synchronize()
    elapsed_timed = time.perf_counter() - t1
    kt = b.chan_env_timing_read(env.handle)
    b.chan_env_set_timing(env.handle, 0)
    # host time to enqueue one env step (asynchronous launch through a batch of one) against
    # the whole step: what capturing the launches in a graph could save at most
    one = b.ChanBatch([env])
    enq, whole = [], []
    for k in range(5):
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        call = one.launch([env], [acts[k]] if use_action else None, args.substeps, [env.obs], [env.tau_w], [env.drag],
                          stream=torch.cuda.current_stream())
        s1 = time.perf_counter()
        call.finish()
        whole.append(time.perf_counter() - s0)
        enq.append(s1 - s0)
    one.close()
    # the same env step captured once as a HIP graph (chan_env_capture) and replayed, the action
    # copied into the captured buffer on the stream before each replay
    abuf = torch.zeros_like(acts[0])
    gr = env.capture(abuf if use_action else None, args.substeps)
    for k in range(2):
        abuf.copy_(acts[k])
        gr.launch().finish()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for k in range(args.steps):
        abuf.copy_(acts[args.warmup + k])
        gr.launch().finish()
    torch.cuda.synchronize()
    elapsed_graph = time.perf_counter() - t2
    gr.close()
    env.close()

    dom = max((k for k in kt if kt[k][0] > 0), key=lambda k: kt[k][1])
    n_launch, ms = kt[dom]
    avg_s = ms / 1e3 / n_launch
    alg = algorithmic_bytes_per_launch(dom, g, args.substeps)
    achieved = alg / avg_s / 1e9 if alg else None
    roof = {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
            "traffic": measured_traffic(dom, args.workload) if args.top == "wall" else None,
            "avg_launch_us": avg_s * 1e6, "launches": n_launch,
            "algorithmic_bytes_per_launch": alg}
    kernels = {k: {"launches": v[0], "total_ms": round(v[1], 4), "avg_us": round(1e3 * v[1] / v[0], 3)}
               for k, v in kt.items() if v[0] > 0}

    value = args.steps / elapsed
    pts = g["nx"] * g["ny"] * g["nz"]
    lat_ms = np.array(lat) * 1e3
    copy_gbs = copy_bandwidth_gbs(torch)
    sub_s = elapsed / (args.steps * args.substeps)
    path_gbs = path_bytes_per_substep(g) / sub_s / 1e9
    path = {"alg_bytes_per_substep": path_bytes_per_substep(g), "achieved_GBs": path_gbs,
            "frac_hbm_peak": path_gbs / HBM_PEAK_GBS, "frac_copy": path_gbs / copy_gbs,
            "alg_flops_per_substep": path_flops_per_substep(g),
            "achieved_TFs_fp64": path_flops_per_substep(g) / sub_s / 1e12,
            "frac_fp64_peak": path_flops_per_substep(g) / sub_s / 1e12 / FP64_PEAK_TFS}
    roof["frac_copy"] = (achieved / copy_gbs) if achieved else None
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "env-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": workload, "grid": [g["nx"], g["ny"], g["nz"]], "substeps_per_env_step": args.substeps,
                   "seed": args.seed},
        "grid_pt_substeps_per_s": value * args.substeps * pts,
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99))},
        "roofline": roof,
        "path_roofline": path,
        "copy_bandwidth_GBs": copy_gbs,
        "kernels": kernels,
        "timing_pass_ms_per_step": 1e3 * elapsed_timed / args.steps,
        "host_enqueue_ms": {"enqueue_p50": 1e3 * float(np.median(enq)), "step_p50": 1e3 * float(np.median(whole)),
                            "note": "host time to queue one env step's launches vs the whole step (5 steps)"},
        "graph_replay": {"value": args.steps / elapsed_graph, "unit": "env-steps/s",
                         "ms_per_step": 1e3 * elapsed_graph / args.steps,
                         "note": "the same env steps captured once as a HIP graph (chan_env_capture) and replayed"},
    }
    if args.copy_probe:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes_each_way"] = src.numel() * 8
    out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
