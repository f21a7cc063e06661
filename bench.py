"""Benchmark of the hot path on one MI355X.

Headline: FP64 cell-updates/s of the 2D nonlinear shallow-water step
(f-wave Roe solver, MC limiter, transverse corrections, dry threshold, CFL
reduction with device-side time-step control) on the 1024 x 1024 synthetic
ocean basin, as absolute rate and as a fraction of the HBM roofline.  One
"step" is one time-step attempt of the whole grid: the marching step kernel
plus the device-side CFL control.

Prints ONE JSON line.  Secondary figures (adjoint step, flagging pass, the
4096^2 grid that does not fit in the last-level cache) go under "extra".

usage: python bench.py [--gpus 1] [--steps 2000] [--warmup 20] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
BYTES_PER_CELL_STEP = 56       # read h, hu, hv, B; write h, hu, hv (8 B each)
METRIC = "cell-updates/s FP64 2D SWE step (% HBM roofline); batched/served scen/s + p99 vs plain"


def kernel_source_hash() -> str:
    """sha256 of the kernels' sources and the header, comments and blank
    lines left out (a change to the text of a comment leaves the profiles
    of the code valid)."""
    import re
    h = hashlib.sha256()
    for f in ("paper_1605_05320_amd/csrc/swe_device.h", "paper_1605_05320_amd/csrc/swe_kernels.hip",
              "include/swe.h"):
        with open(os.path.join(ROOT, f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        h.update("\n".join(ln.rstrip() for ln in text.splitlines() if ln.strip()).encode())
    return h.hexdigest()[:16]


COPY_PROBE_BYTES = 64 * 1024 * 1024 * 8    # the --copy-probe copy: 512 MiB read and written
STEP_KERNEL = "k_march2d<swe::NL"


def _counter_rows(d: str, counter: str):
    import csv
    import glob
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    rows = []
    for f in files:
        with open(f) as fh:
            rows += [r for r in csv.DictReader(fh) if r["Counter_Name"] == counter]
    return rows


def traffic_from(fetch_dir: str, write_dir: str, n: int):
    """HBM bytes per step-kernel launch from FETCH_SIZE and WRITE_SIZE (KiB per
    dispatch), each scaled by what the same counter reads for the 512 MiB
    device copy of --copy-probe."""
    out = {"kernel": "k_march2d<NL> (order 2, transverse)", "kernel_source_sha": kernel_source_hash(),
           "workload": f"{n}x{n} synthetic basin, seed 2", "copy_probe_bytes": COPY_PROBE_BYTES}
    for kind, d in (("fetch", fetch_dir), ("write", write_dir)):
        rows = _counter_rows(d, kind.upper() + "_SIZE")
        step = [float(r["Counter_Value"]) for r in rows if STEP_KERNEL in r["Kernel_Name"]]
        copies = [r for r in rows if "copyBuffer" in r["Kernel_Name"] or "copy" in r["Kernel_Name"].lower()]
        probe = max(copies, key=lambda r: int(r["Grid_Size"]))
        probe_kib = float(probe["Counter_Value"])
        scale = COPY_PROBE_BYTES / 1024.0 / probe_kib
        out[f"{kind}_kib_per_launch"] = sum(step) / len(step)
        out[f"{kind}_launches"] = len(step)
        out[f"{kind}_copy_probe_kib"] = probe_kib
        out[f"{kind}_scale"] = scale
        out[f"{kind}_bytes_per_launch"] = sum(step) / len(step) * 1024.0 * scale
    out["hbm_bytes_per_launch"] = out["fetch_bytes_per_launch"] + out["write_bytes_per_launch"]
    out["algorithmic_bytes_per_launch"] = BYTES_PER_CELL_STEP * n * n
    out["traffic_over_algorithmic"] = out["hbm_bytes_per_launch"] / out["algorithmic_bytes_per_launch"]
    path = os.path.join(ROOT, "profiles", "step_nl_1024_traffic.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out, indent=1))


# VALU issue peak: 256 CUs x 4 SIMDs x 2.4 GHz, one wave64 instruction per SIMD
# every 4 cycles (16 lanes wide); for FP64 FMAs that is the published 78.6
# TFLOP/s (x 64 lanes x 2 flops).
VALU_PEAK_G = 256 * 4 * 2.4 / 4


def valu_from(sq_dir: str, n: int):
    """VALU wave-instructions per step-kernel launch from an SQ_INSTS_VALU
    counter run of 'bench.py --busy-only 10 --n 1024' (the step with waves on
    every edge)."""
    rows = _counter_rows(sq_dir, "SQ_INSTS_VALU")
    step = [float(r["Counter_Value"]) for r in rows if STEP_KERNEL in r["Kernel_Name"]]
    out = {"kernel": "k_march2d<NL> (order 2, transverse)", "kernel_source_sha": kernel_source_hash(),
           "workload": f"{n}x{n} synthetic basin, seed 2, a centimetre of noise on every wet cell",
           "launches": len(step), "valu_instr_per_launch": sum(step) / len(step)}
    path = os.path.join(ROOT, "profiles", "step_nl_1024_valu.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out, indent=1))


def load_valu():
    """VALU instructions per launch of the busy 1024^2 step from the committed
    counter summary, if it was taken on the current kernel source; else None."""
    try:
        with open(os.path.join(ROOT, "profiles", "step_nl_1024_valu.json")) as f:
            d = json.load(f)
    except OSError:
        return None
    return d.get("valu_instr_per_launch") if d.get("kernel_source_sha") == kernel_source_hash() else None


def load_traffic(kind: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "step_nl_1024_traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except OSError:
        return None
    if d.get("kernel_source_sha") != kernel_source_hash():
        return None
    return d.get(kind)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip the secondary measurements")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--graph", type=int, default=100,
                    help="attempts per captured HIP graph (0: plain stream launches)")
    ap.add_argument("--serve-requests", type=int, default=64,
                    help="requests in the serving trace (grids --serve-nmin..--serve-nmax a side)")
    ap.add_argument("--serve-nmin", type=int, default=256)
    ap.add_argument("--serve-nmax", type=int, default=1024)
    ap.add_argument("--serve-full", action="store_true",
                    help="the full serving workload: 256 requests, grids 256^2..2048^2")
    ap.add_argument("--serve-only", action="store_true", help="run the serving leg only (no headline)")
    ap.add_argument("--valu-from", metavar="SQ_DIR",
                    help="no GPU: read a rocprofv3 --pmc SQ_INSTS_VALU output of 'bench.py --busy-only 10' "
                         "and write profiles/step_nl_1024_valu.json")
    ap.add_argument("--adj-only", type=int, default=0, metavar="K",
                    help="run the 1024^2 adjoint step K times and exit (profiler runs)")
    ap.add_argument("--flag-only", type=int, default=0, metavar="K",
                    help="run the --flag-n flag pass (34-snapshot window) K times and exit (profiler runs)")
    ap.add_argument("--flag-n", type=int, default=512, help="grid side of the --flag-only pass")
    ap.add_argument("--run1d-only", type=int, default=0, metavar="K",
                    help="run the 1D shelf problem (2000 cells, 3 h, 60 snapshots) K times and exit")
    ap.add_argument("--run1d-per-step", type=int, default=0, choices=(0, 1),
                    help="with --run1d-only: 1 launches every step (launch_per_step)")
    ap.add_argument("--run2d-only", type=int, default=0, metavar="K",
                    help="run the 512^2 adjoint-flagged problem (64 snapshots, flags every step) K times and exit")
    ap.add_argument("--level-only", action="store_true",
                    help="run the batched-level leg (3000 patches, 100 steps, tuner, baselines) and exit")
    ap.add_argument("--busy-only", type=int, default=0, metavar="K",
                    help="launch the --n step with waves on every edge K times and exit (counter runs)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one device copy of known size (HBM counter calibration)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="no GPU: read two rocprofv3 --pmc outputs (FETCH_SIZE, WRITE_SIZE) of "
                         "'bench.py --graph 0 --copy-probe' and write the step kernel's HBM traffic "
                         "to profiles/step_nl_1024_traffic.json")
    args = ap.parse_args()
    if args.traffic_from:
        traffic_from(*args.traffic_from, n=args.n)
        return
    if args.valu_from:
        valu_from(args.valu_from, n=args.n)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "the grid and scenario decompositions across GPUs are described, not run.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1605_05320_amd import inputs as I
    from paper_1605_05320_amd import swe as S

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    S.lib()
    dev = torch.device("cuda")
    f64 = dict(dtype=torch.float64, device=dev)
    if args.serve_full:
        args.serve_requests, args.serve_nmin, args.serve_nmax = 256, 256, 2048
    if args.serve_only:
        print(json.dumps({"serve": serve_bench(S, torch, I, np, args.serve_requests, args.serve_nmin,
                                               args.serve_nmax)}), flush=True)
        return
    if args.adj_only > 0:
        step = adj_step_1024(S, torch, I, f64)
        for _ in range(args.adj_only):
            step()
        torch.cuda.synchronize()
        print(json.dumps({"adj_launches": args.adj_only}), flush=True)
        return
    if args.flag_only > 0:
        flag, _, _ = flag_pass(S, torch, I, np, f64, n=args.flag_n)
        for _ in range(args.flag_only):
            flag()
        if args.copy_probe:
            src = torch.ones(64 * 1024 * 1024, **f64)
            torch.empty_like(src).copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"flag_launches": args.flag_only}), flush=True)
        return
    if args.run1d_only > 0:
        times = [round(run1d_shelf(S, torch, I, np, f64, launch_per_step=args.run1d_per_step), 4)
                 for _ in range(args.run1d_only)]
        print(json.dumps({"run1d_s": times, "launch_per_step": args.run1d_per_step}), flush=True)
        return
    if args.run2d_only > 0:
        print(json.dumps({"run2d_512_s": [round(run2d_512(S, torch, I, f64), 4) for _ in range(args.run2d_only)]}),
              flush=True)
        return
    if args.level_only:
        print(json.dumps({"level": level_bench(S, torch, I, np, f64)}), flush=True)
        return
    if args.busy_only > 0:
        g, p, B, qa, qb, dt = busy_state(S, torch, I, np, f64, args.n)
        for _ in range(args.busy_only):
            S.swe_step(g, p, B, qa, qb, dt)
        torch.cuda.synchronize()
        print(json.dumps({"busy_launches": args.busy_only, "n": args.n}), flush=True)
        return

    n = args.n
    b = I.basin(n, args.seed)
    grid = S.Grid(n, n, b.grid.dx, b.grid.dy)
    prm = S.Params()
    B = torch.tensor(b.B, **f64)
    eta0 = torch.tensor(b.eta0, **f64)
    qa = [torch.empty(n, n, **f64) for _ in range(3)]
    qb = [torch.empty(n, n, **f64) for _ in range(3)]
    S.swe_init(grid, prm, B, eta0, qa)
    spd = torch.zeros(1, dtype=torch.int64, device=dev)
    S.swe_max_speed(grid, prm, B, qa, 0, spd)
    dt0 = prm.cfl_desired / float(spd.view(torch.float64).item())
    ctl = S.new_ctl()
    S.swe_ctl_set(ctl, 0.0, dt0, 1.0e30, 0)     # open-ended segment: every attempt runs

    stream = torch.cuda.current_stream()
    S.swe_advance(grid, prm, B, qa, qb, ctl, args.warmup)
    torch.cuda.synchronize()
    run = lambda k: S.swe_advance(grid, prm, B, qa, qb, ctl, k)
    chunk = args.graph if args.graph > 0 and args.steps % args.graph == 0 else 0
    if chunk:
        # the attempts of one chunk captured once as a HIP graph and replayed
        # (kernel arguments fixed; dt, the state buffer and the Courant number
        # travel through the device-side control block)
        gs = torch.cuda.Stream()
        gs.wait_stream(stream)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.stream(gs):
            with torch.cuda.graph(graph, stream=gs):
                S.swe_advance(grid, prm, B, qa, qb, ctl, chunk, stream=gs)
        stream.wait_stream(gs)
        torch.cuda.synchronize()
        run = lambda k: [graph.replay() for _ in range(k // chunk)]
        run(chunk)                      # one warm replay
        torch.cuda.synchronize()
    c0 = S.read_ctl(ctl)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    e0.record(stream)
    run(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms = e0.elapsed_time(e1)
    c1 = S.read_ctl(ctl)
    accepted = c1.n_accepted - c0.n_accepted
    rejected = c1.n_rejected - c0.n_rejected
    cells = n * n
    value = cells * accepted / (ms * 1e-3)
    ms_per_step = ms / args.steps

    # dominant kernel: the marching step.  Under device-side control every
    # attempt is exactly one launch of it, so its average launch duration is
    # the timed region over the attempts (HIP events on the launch stream).
    k_us = ms_per_step * 1e3
    algo_bytes = BYTES_PER_CELL_STEP * cells
    achieved = algo_bytes / (k_us * 1e-6) / 1e9
    traffic = load_traffic("hbm_bytes_per_launch")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "k_march2d<NL>", "kernel_avg_us": round(k_us, 3),
                "algorithmic_bytes_per_launch": algo_bytes}

    extra = {"accepted_steps": accepted, "rejected_steps": rejected, "t_sim_s": round(c1.t, 3),
             "wall_s": round(t_wall, 4), "graph_chunk": chunk}
    if not args.no_extra:
        extra.update(secondary(S, torch, I, np, f64))
        # the VALU-issue roofline of the same kernel on the step with waves on
        # every edge: counted instructions per launch over the live duration
        vi = load_valu()
        if vi is not None and n == 1024:
            us = extra["step_busy_1024_us"]
            ach = vi / (us * 1e-6) / 1e9
            roofline["valu"] = {"bound": "alu", "achieved": round(ach, 1), "peak": VALU_PEAK_G,
                                "unit": "G VALU wave-instr/s", "frac": round(ach / VALU_PEAK_G, 4),
                                "case": "1024x1024, waves on every edge", "kernel_avg_us": round(us, 3),
                                "valu_instr_per_launch": vi}
        extra["serve"] = serve_bench(S, torch, I, np, args.serve_requests, args.serve_nmin, args.serve_nmax)

    if args.copy_probe:
        # one copy of known size, for scaling the HBM counters
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device=dev)   # 512 MiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        extra["copy_probe_bytes"] = src.numel() * 8

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(b, n, args.cpu_seconds)

    out = {
        "metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"2D nonlinear shallow water, {n}x{n} synthetic ocean basin "
                               f"(seed {args.seed}: 4000 m plain, tanh shelf, 20 seamounts, dry land), "
                               "1 m elliptical Gaussian source, f-wave Roe + MC limiter + transverse, "
                               "dry tol 1e-3 m, CFL 0.9 with device-side dt control",
                   "nx": n, "ny": n, "dx_m": b.grid.dx},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)


def _time_events(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    z.record()
    torch.cuda.synchronize()
    return a.elapsed_time(z) * 1e-3 / reps


def busy_state(S, torch, I, np, f64, n):
    """The n x n basin (seed 2) with a centimetre of seeded noise on the
    surface of every wet cell, so that every edge carries waves, and a step
    at half the desired Courant number."""
    b = I.basin(n, 2)
    g = S.Grid(n, n, b.grid.dx, b.grid.dy)
    p = S.Params()
    B = torch.tensor(b.B, **f64)
    noise = np.random.default_rng(7).uniform(-0.01, 0.01, b.B.shape)
    qa = [torch.empty(n, n, **f64) for _ in range(3)]
    qb = [torch.empty(n, n, **f64) for _ in range(3)]
    S.swe_init(g, p, B, torch.tensor(b.eta0 + noise, **f64), qa)
    spd = torch.zeros(1, dtype=torch.int64, device=B.device)
    S.swe_max_speed(g, p, B, qa, 0, spd)
    dt = 0.5 * p.cfl_desired / float(spd.view(torch.float64).item())
    return g, p, B, qa, qb, dt


FLAG_BYTES_PER_CELL_W34 = 32 + 24 * 34 + 1 + 1 + 1 + 16   # q, B, 34 snapshots, flag, accumulators


def flag_pass(S, torch, I, np, f64, n=512):
    """The flag pass at n^2 with a 34-snapshot window (the widest window of
    the adjoint-flagging workload: snapshots 30..63 of 64), with the running
    flag and max-inner-product accumulators; returns the call and its
    algorithmic bytes."""
    b = I.basin(n, 3)
    g = S.Grid(n, n, b.grid.dx, b.grid.dy)
    p = S.Params()
    B = torch.tensor(b.B, **f64)
    K = 64
    frames = torch.randn(K + 1, 3, n, n, **f64) * 1e-3
    q = [torch.tensor(np.maximum(0.0, -b.B) + 0.0, **f64), torch.zeros(n, n, **f64), torch.zeros(n, n, **f64)]
    fl = torch.empty(n, n, dtype=torch.int8, device=B.device)
    acc = torch.zeros(n, n, dtype=torch.int8, device=B.device)
    macc = torch.zeros(n, n, **f64)
    ctx = dict(g=g, p=p, B=B, q=q, K=K, fl=fl, acc=acc, macc=macc)
    return (lambda: S.adj_flag(g, p, B, q, frames, K, 30, 63, 1e-4, fl, None, acc, macc)), \
        n * n * FLAG_BYTES_PER_CELL_W34, ctx


def adj_step_1024(S, torch, I, f64):
    """One adjoint step at 1024^2 (basin seed 3) from the Gaussian target of
    radius 20 km, as a call."""
    n = 1024
    b = I.basin(n, 3)
    g = S.Grid(n, n, b.grid.dx, b.grid.dy)
    p = S.Params()
    B = torch.tensor(b.B, **f64)
    q = [torch.zeros(n, n, **f64) for _ in range(3)]
    r = [torch.empty(n, n, **f64) for _ in range(3)]
    S.adj_target(g, p, B, b.target[0], b.target[1], 20e3, S.GAUSS, q)
    return lambda: S.adj_step(g, p, B, q, r, 1.0)


def secondary(S, torch, I, np, f64):
    out = {}
    # measured device copy bandwidth (512 MiB read + 512 MiB written), the
    # practical ceiling beside the published 8 TB/s
    src = torch.ones(64 * 1024 * 1024, **f64)
    dst = torch.empty_like(src)
    t = min(_time_events(torch, lambda: dst.copy_(src), 10) for _ in range(3))
    out["copy_512MiB_GBs"] = 2 * src.numel() * 8 / t / 1e9
    del src, dst
    torch.cuda.empty_cache()
    # adjoint step at 1024^2 (linearized, f-wave, transverse)
    n = 1024
    # (best of five runs of 40 calls: launched one by one from Python, a
    # 28 us kernel is exposed to host hiccups)
    adj = adj_step_1024(S, torch, I, f64)
    t = min(_time_events(torch, adj, 40) for _ in range(5))
    out["adj_step_1024_cell_updates_per_s"] = n * n / t
    out["adj_step_1024_us"] = t * 1e6
    flag, fbytes, ctx = flag_pass(S, torch, I, np, f64)
    t = min(_time_events(torch, flag, 25) for _ in range(4))
    n = 512
    g, p, B, q, K, fl, acc, macc = (ctx[k] for k in ("g", "p", "B", "q", "K", "fl", "acc", "macc"))
    out["flag_512_w34_us"] = t * 1e6
    out["flag_512_w34_GBs"] = fbytes / t / 1e9
    # the same window at 1024^2: 34 snapshots of 25 MB, 855 MB in all, more
    # than the 256 MB last-level cache holds, so every pass streams from HBM
    flag1, fbytes1, _ = flag_pass(S, torch, I, np, f64, n=1024)
    t = min(_time_events(torch, flag1, 10) for _ in range(3))
    out["flag_1024_w34_us"] = t * 1e6
    out["flag_1024_w34_GBs"] = fbytes1 / t / 1e9
    del flag1
    torch.cuda.empty_cache()
    # the same pass with the snapshots on a 256^2 adjoint grid (bilinear
    # interpolation at every cell and snapshot)
    nc = n // 2
    bc = I.basin(nc, 3)
    gcs = S.Grid(nc, nc, bc.grid.dx, bc.grid.dy)
    Bc = torch.tensor(bc.B, **f64)
    framesc = torch.randn(K + 1, 3, nc, nc, **f64) * 1e-3
    t = _time_events(torch, lambda: S.adj_flag_interp(g, p, B, q, gcs, Bc, framesc, K, 30, 63, 1e-4, fl, None,
                                                      acc, macc), 100)
    out["flag_interp_512_from_256_w34_us"] = t * 1e6
    out["flag_interp_512_from_256_w34_cells_per_s"] = n * n / t
    # the 4096^2 grid (~0.9 GB working set, beyond the 256 MB last-level cache),
    # from the initial state (the sea mostly at rest)
    n = 4096
    b = I.basin(n, 2)
    g = S.Grid(n, n, b.grid.dx, b.grid.dy)
    B = torch.tensor(b.B, **f64)
    e = torch.tensor(b.eta0, **f64)
    qa = [torch.empty(n, n, **f64) for _ in range(3)]
    qb = [torch.empty(n, n, **f64) for _ in range(3)]
    S.swe_init(g, p, B, e, qa)
    spd = torch.zeros(1, dtype=torch.int64, device=B.device)
    S.swe_max_speed(g, p, B, qa, 0, spd)
    dt = 0.5 * p.cfl_desired / float(spd.view(torch.float64).item())
    t = min(_time_events(torch, lambda: S.swe_step(g, p, B, qa, qb, dt), 40) for _ in range(3))
    out["step_4096_cell_updates_per_s"] = n * n / t
    out["step_4096_us"] = t * 1e6
    out["step_4096_algorithmic_GBs"] = BYTES_PER_CELL_STEP * n * n / t / 1e9
    del qa, qb, B, e
    torch.cuda.empty_cache()
    # the step with waves on every edge (noise on the surface of every wet
    # cell), so that no row of sea at rest is skipped
    for n, reps in ((1024, 100), (4096, 20)):
        g, p, B, qa, qb, dt = busy_state(S, torch, I, np, f64, n)
        t = min(_time_events(torch, lambda: S.swe_step(g, p, B, qa, qb, dt), reps) for _ in range(3))
        out[f"step_busy_{n}_cell_updates_per_s"] = n * n / t
        out[f"step_busy_{n}_us"] = t * 1e6
        del qa, qb, B
        torch.cuda.empty_cache()
    out.update(run_bench(S, torch, I, np, f64))
    out.update(level_bench(S, torch, I, np, f64))
    return out


def _box_fraction(bnd, K, nx, ny):
    """Mean over the snapshots of the fraction of the grid inside each one's box."""
    b = bnd.view(K + 1, 4).cpu().tolist()
    a = [(r[1] - r[0] + 1) * (r[3] - r[2] + 1) if r[1] >= r[0] else 0 for r in b]
    return round(sum(a) / (len(a) * nx * ny), 4)


def run1d_shelf(S, torch, I, np, f64, launch_per_step=0):
    """One swe_run of the 1D shelf (2000 cells on [-400 km, 0], 3 h, 60
    snapshots, tol 1e-3, flags every step); returns its wall time in s."""
    n, K, tf, tol = 2000, 60, 10800.0, 1e-3
    s1 = I.shelf1d(n, seed=0)
    g = S.Grid(n, 1, s1.dx, 1.0, s1.x_lo)
    B = torch.tensor(s1.B.reshape(1, n), **f64)
    E = torch.tensor(s1.eta0.reshape(1, n), **f64)
    frames = torch.zeros(K + 1, 2, 1, n, **f64)
    q = [torch.zeros(1, n, **f64) for _ in range(2)]
    acc = torch.zeros(1, n, dtype=torch.int8, device=B.device)
    macc = torch.zeros(1, n, **f64)
    pb = S.make_problem(g, S.Params(model=S.LINEAR), B, E, s1.target, 0.0, 0.0, tf, K, tol, frames, q, None, acc,
                        macc, launch_per_step=launch_per_step)
    ws = torch.empty(S.swe_run_workspace_bytes(pb) // 8 + 64, **f64)
    torch.cuda.synchronize()
    t = time.perf_counter()
    S.swe_run(pb, ws)
    torch.cuda.synchronize()
    return time.perf_counter() - t


def run2d_512(S, torch, I, f64):
    """One swe_run of the adjoint-flagging workload of run_bench (512^2 basin,
    64 snapshots, window [3600 s, 7200 s], tol 1e-4, flags every step);
    returns its wall time."""
    n, K = 512, 64
    b = I.basin(n, 3)
    g = S.Grid(n, n, b.grid.dx, b.grid.dy)
    prm = S.Params()
    B = torch.tensor(b.B, **f64)
    E = torch.tensor(b.eta0, **f64)
    frames = torch.zeros(K + 1, 3, n, n, **f64)
    q = [torch.zeros(n, n, **f64) for _ in range(3)]
    acc = torch.zeros(n, n, dtype=torch.int8, device=B.device)
    macc = torch.zeros(n, n, **f64)
    pb = S.make_problem(g, prm, B, E, b.target, 0.0, 3600.0, 7200.0, K, 1e-4, frames, q, None, acc, macc)
    ws = torch.empty(S.swe_run_workspace_bytes(pb) // 8 + 64, **f64)
    torch.cuda.synchronize()
    t = time.perf_counter()
    S.swe_run(pb, ws)
    torch.cuda.synchronize()
    return time.perf_counter() - t


def run_bench(S, torch, I, np, f64):
    """The two-phase driver on the adjoint-flagging workload (512^2 basin,
    64 snapshots, window [3600 s, 7200 s], tol 1e-4, flags every step) and on
    the 1D shelf (2000 cells, 60 snapshots, 3 h, tol 1e-3)."""
    out = {}
    for tag, n, ny, K, ts, tf, tol, model in (("run2d_512", 512, 512, 64, 3600.0, 7200.0, 1e-4, S.NONLINEAR),
                                              ("run1d_2000", 2000, 1, 60, 0.0, 10800.0, 1e-3, S.LINEAR)):
        if ny > 1:
            b = I.basin(n, 3)
            g = S.Grid(n, n, b.grid.dx, b.grid.dy)
            Bn, En, target = b.B, b.eta0, b.target
        else:
            s1 = I.shelf1d(n, seed=0)
            g = S.Grid(n, 1, s1.dx, 1.0, s1.x_lo)
            Bn, En, target = s1.B.reshape(1, n), s1.eta0.reshape(1, n), s1.target
        ncomp = 3 if ny > 1 else 2
        prm = S.Params(model=model)
        B = torch.tensor(Bn, **f64)
        E = torch.tensor(En, **f64)
        frames = torch.zeros(K + 1, ncomp, ny, n, **f64)
        q = [torch.zeros(ny, n, **f64) for _ in range(ncomp)]
        acc = torch.zeros(ny, n, dtype=torch.int8, device=B.device)
        macc = torch.zeros(ny, n, **f64)
        # warm-up, recording the adjoint flags and the surface flags (|eta| >
        # surface_tol) at t0 and the K output times for comparison
        flags_at = torch.zeros(K + 1, ny, n, dtype=torch.int8, device=B.device)
        sflags = torch.zeros(K + 1, ny, n, dtype=torch.int8, device=B.device)
        stol = 0.05 if ny > 1 else 0.02
        pw = S.make_problem(g, prm, B, E, target, 0.0, ts, tf, K, tol, frames, q, flags_at, acc, macc,
                            surface_tol=stol, surface_flags_at=sflags)
        ws = torch.empty(S.swe_run_workspace_bytes(pw) // 8 + 64, **f64)
        S.swe_run(pw, ws)
        adj_counts = flags_at.view(K + 1, -1).sum(dim=1, dtype=torch.int64).cpu().tolist()
        srf_counts = sflags.view(K + 1, -1).sum(dim=1, dtype=torch.int64).cpu().tolist()
        if ny > 1:
            out["regrid_512"] = regrid_bench(S, torch, np, g, B, q, flags_at[K], f64)
        pb = S.make_problem(g, prm, B, E, target, 0.0, ts, tf, K, tol, frames, q, None, acc, macc)
        acc.zero_(); macc.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = S.swe_run(pb, ws)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        cells = n * ny
        if ny == 1:
            # the same run with one launch per step and per flag pass
            pl = S.make_problem(g, prm, B, E, target, 0.0, ts, tf, K, tol, frames, q, None, acc, macc,
                                launch_per_step=1)
            wl = torch.empty(S.swe_run_workspace_bytes(pl) // 8 + 64, **f64)
            acc.zero_(); macc.zero_()
            torch.cuda.synchronize()
            t = time.perf_counter()
            S.swe_run(pl, wl)
            torch.cuda.synchronize()
            out[tag + "_launch_per_step_s"] = round(time.perf_counter() - t, 4)
            del wl
        if ny > 1:
            # the same run reading every snapshot in full in every flag pass
            pf = S.make_problem(g, prm, B, E, target, 0.0, ts, tf, K, tol, frames, q, None, acc, macc,
                                full_frames=1)
            acc.zero_(); macc.zero_()
            torch.cuda.synchronize()
            t = time.perf_counter()
            S.swe_run(pf, ws)
            torch.cuda.synchronize()
            out[tag + "_full_frames_s"] = round(time.perf_counter() - t, 4)
            # single flag passes over this run's snapshots: the window of the
            # first output times (snapshots 32..64, spread over the basin) and of
            # the last ones (0..2, near the target), with and without the boxes
            bnd = torch.empty(4 * (K + 1), dtype=torch.int32, device=B.device)
            S.adj_frame_bounds(g, frames, K, bnd)
            fl = torch.empty(ny, n, dtype=torch.int8, device=B.device)
            for lo, hi in ((32, 64), (0, 2)):
                for use in (False, True):
                    tt = _time_events(torch, lambda: S.adj_flag(g, prm, B, q, frames, K, lo, hi, tol, fl,
                                                                bounds=bnd if use else None), 20)
                    out[f"flag_512_snapshots_{lo}_{hi}_{'boxes' if use else 'full'}_us"] = round(tt * 1e6, 2)
            out[tag + "_snapshot_box_fraction"] = _box_fraction(bnd, K, n, ny)
            # the paper's own target, the indicator of a disk (Sec. 6): its
            # snapshots are exactly zero outside the adjoint's numerical domain
            # of dependence, so the boxes are tighter than a Gaussian's
            for full in (0, 1):
                pd = S.make_problem(g, prm, B, E, target, 0.0, ts, tf, K, tol, frames, q, None, acc, macc,
                                    shape=S.DISK, full_frames=full)
                acc.zero_(); macc.zero_()
                torch.cuda.synchronize()
                t = time.perf_counter()
                S.swe_run(pd, ws)
                torch.cuda.synchronize()
                out[tag + ("_disk_full_frames_s" if full else "_disk_s")] = round(time.perf_counter() - t, 4)
            S.adj_frame_bounds(g, frames, K, bnd)
            out[tag + "_disk_snapshot_box_fraction"] = _box_fraction(bnd, K, n, ny)
            for use in (False, True):
                tt = _time_events(torch, lambda: S.adj_flag(g, prm, B, q, frames, K, 32, 64, tol, fl,
                                                            bounds=bnd if use else None), 20)
                out[f"flag_512_disk_snapshots_32_64_{'boxes' if use else 'full'}_us"] = round(tt * 1e6, 2)
        out[tag] = {"s": round(el, 4), "adjoint_steps": r.n_adj_steps, "forward_steps": r.n_fwd_steps,
                    "flag_passes": r.n_flag_calls, "flagged_cells": int(acc.sum().item()),
                    "cell_updates_per_s": cells * (r.n_adj_steps + r.n_fwd_steps) / el,
                    "flagged_per_output": {"adjoint_tol": tol, "surface_tol_m": stol,
                                           "adjoint": adj_counts, "surface": srf_counts,
                                           "adjoint_mean": sum(adj_counts) / len(adj_counts),
                                           "surface_mean": sum(srf_counts) / len(srf_counts)}}
    # the 512^2 adjoint-flagging run with the adjoint on a 256^2 grid
    n, nc, K, ts, tf, tol = 512, 256, 64, 3600.0, 7200.0, 1e-4
    b, bc = I.basin(n, 3), I.basin(nc, 3)
    g = S.Grid(n, n, b.grid.dx, b.grid.dy)
    gc = S.Grid(nc, nc, bc.grid.dx, bc.grid.dy)
    prm = S.Params()
    B, E, Bc = torch.tensor(b.B, **f64), torch.tensor(b.eta0, **f64), torch.tensor(bc.B, **f64)
    frames = torch.zeros(K + 1, 3, nc, nc, **f64)
    q = [torch.zeros(n, n, **f64) for _ in range(3)]
    acc = torch.zeros(n, n, dtype=torch.int8, device=B.device)
    macc = torch.zeros(n, n, **f64)
    pb = S.make_problem(g, prm, B, E, b.target, 0.0, ts, tf, K, tol, frames, q, None, acc, macc,
                        adj_grid=gc, adj_B=Bc)
    ws = torch.empty(S.swe_run_workspace_bytes(pb) // 8 + 64, **f64)
    S.swe_run(pb, ws)
    acc.zero_(); macc.zero_()
    torch.cuda.synchronize()
    t = time.perf_counter()
    r = S.swe_run(pb, ws)
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    out["run2d_512_adjoint256"] = {"s": round(el, 4), "adjoint_steps": r.n_adj_steps, "adjoint_cells": nc * nc,
                                   "forward_steps": r.n_fwd_steps, "flag_passes": r.n_flag_calls,
                                   "flagged_cells": int(acc.sum().item())}
    return out


def regrid_bench(S, torch, np, g, B, q, flags, f64, ratio=2, n_steps=20):
    """One regrid of the adaptive loop on the 512^2 run's final adjoint flags:
    host clustering, injection of the coarse state into the 2x refined
    patches, and steps of the refined level."""
    fl = flags.cpu().numpy()
    t_cluster = float("inf")
    for _ in range(5):              # host call: best of five
        t = time.perf_counter()
        boxes = S.cluster(fl, 0.7, 4, 32)
        t_cluster = min(t_cluster, time.perf_counter() - t)
    if not boxes:
        return {"boxes": 0}
    nxp = [nx * ratio for (_, _, nx, _) in boxes]
    nyp = [ny * ratio for (_, _, _, ny) in boxes]
    tab, ncell = S.patch_table(nxp, nyp, [g.dx / ratio] * len(boxes))
    lvl = S.Level(tab, S.SCHED_PACKED)
    # a few small patches fill a fraction of the chip: the autotuner picks
    # the row chunks (short ones give more, shorter marches)
    chunks = (1, 2, 4, 8, 16)
    cands = [lvl] + [S.Level(tab, S.SCHED_PACKED, chunk_rows=r) for r in chunks]
    box_t = torch.tensor(np.array(boxes, np.int32), device=B.device)
    Bp = torch.empty(ncell, **f64)
    qa = [torch.empty(ncell, **f64) for _ in range(3)]
    qb = [torch.empty(ncell, **f64) for _ in range(3)]
    t_prolong = _time_events(torch, lambda: S.prolong(g, B, q, box_t, lvl.patches_t, len(boxes), ratio, Bp, qa), 20)
    spd = torch.zeros(1, dtype=torch.int64, device=B.device)
    S.swe_max_speed(S.Grid(int(g.nx), int(g.ny), g.dx / ratio, g.dy / ratio), S.Params(), B, q, 0, spd)
    dt0 = S.Params().cfl_desired / float(spd.view(torch.float64).item())
    init = [x.clone() for x in qa]

    def timed(level, persistent=0):
        for c_ in range(3):
            qa[c_].copy_(init[c_])
        ctl = S.new_ctl()
        S.swe_ctl_set(ctl, 0.0, dt0, 1.0e300, 0)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        S.level_advance(level, S.Params(), Bp, qa, qb, ctl, n_steps, persistent)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1), S.read_ctl(ctl)

    wa = [torch.empty(ncell, **f64) for _ in range(3)]
    wb = [torch.empty(ncell, **f64) for _ in range(3)]
    ref = [torch.empty(ncell, **f64) for _ in range(3)]
    mism = torch.zeros(1, dtype=torch.int32, device=B.device)
    entries, best = S.level_tune(cands, S.Params(), Bp, init, wa, wb, ref, S.new_ctl(), mism, dt0, 10, ncell)
    lb, pb_, _ = entries[best]
    ms_whole, _ = timed(lvl)
    ms, c = timed(cands[lb], pb_)
    area = sum(nx * ny for (_, _, nx, ny) in boxes)
    names = ["whole"] + [f"{r}-row-chunks" for r in chunks]
    return {"flagged_cells": int(fl.sum()), "boxes": len(boxes), "box_efficiency": round(int(fl.sum()) / area, 3),
            "cluster_ms": round(t_cluster * 1e3, 3), "refined_cells": ncell, "prolong_us": round(t_prolong * 1e6, 2),
            "level_steps": n_steps, "level_accepted": c.n_accepted,
            "level_us_per_step_whole_patches": round(ms_whole * 1e3 / n_steps, 2),
            "level_candidates_us_per_step": {f"{names[l]}/{'persistent' if pm else 'launch-per-step'}": round(u, 2)
                                             for l, pm, u in entries if u >= 0},
            "level_us_per_step": round(ms * 1e3 / n_steps, 2),
            "level_schedule": f"{names[lb]}/{'persistent' if pb_ else 'launch-per-step'}",
            "level_cell_updates_per_s": ncell * c.n_accepted / (ms * 1e-3)}


def level_bench(S, torch, I, np, f64, n_patches=3000, n_steps=100, seed=4):
    """Batched AMR level: 3000 patches of 8..64 cells a side, 100 steps with a
    level-wide dt; the autotuned schedule against one launch per patch per step."""
    ps = I.patches(n_patches, seed=seed)
    tab, ncell = S.patch_table(ps.nx, ps.ny, ps.dx)
    dev = B0 = None
    B = torch.tensor(np.concatenate([b.ravel() for b in ps.B]), **f64)
    eta = torch.tensor(np.concatenate([e.ravel() for e in ps.eta0]), **f64)
    prm = S.Params()
    init = [torch.empty(ncell, **f64) for _ in range(3)]
    # initial state and level speed, patch by patch through the library
    spd = torch.zeros(1, dtype=torch.int64, device=B.device)
    for k in range(n_patches):
        o, n = tab[k].offset, tab[k].nx * tab[k].ny
        g = S.Grid(tab[k].nx, tab[k].ny, tab[k].dx, tab[k].dy)
        q = [x[o:o + n] for x in init]
        S.swe_init(g, prm, B[o:o + n], eta[o:o + n], q)
        S.swe_max_speed(g, prm, B[o:o + n], q, 0, spd)
    dt0 = prm.cfl_desired / float(spd.view(torch.float64).item())
    chunks = (8, 12, 16, 24, 32)
    levels = [S.Level(tab, S.SCHED_STRIP), S.Level(tab, S.SCHED_PACKED)] + \
        [S.Level(tab, S.SCHED_PACKED, chunk_rows=r) for r in chunks]
    wa = [torch.empty(ncell, **f64) for _ in range(3)]
    wb = [torch.empty(ncell, **f64) for _ in range(3)]
    ref = [torch.empty(ncell, **f64) for _ in range(3)]
    ctl = S.new_ctl()
    mism = torch.zeros(1, dtype=torch.int32, device=B.device)
    entries, best = S.level_tune(levels, prm, B, init, wa, wb, ref, ctl, mism, dt0, 10, ncell)
    lnames = ["strip", "packed"] + [f"packed-{r}-row-chunks" for r in chunks]
    names = {(l, pm): f"{lnames[l]}/{'persistent' if pm else 'launch-per-step'}"
             for l in range(len(levels)) for pm in (0, 1)}
    lv, pers, _ = entries[best]
    # timed run of the chosen schedule
    for c in range(3):
        wa[c].copy_(init[c])
    S.swe_ctl_set(ctl, 0.0, dt0, 1.0e300, 0)
    torch.cuda.synchronize()
    t = _time_events(torch, lambda: None, 1)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    S.level_advance(levels[lv], prm, B, wa, wb, ctl, n_steps, pers)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    c = S.read_ctl(ctl)
    best_rate = ncell * c.n_accepted / (ms * 1e-3)
    # the same attempts captured once as one HIP graph and replayed from the
    # same state (launch-per-step schedules; the persistent kernel is one
    # launch already): the whole advance is a single launch from the host
    graph_ms = graph_same = None
    if not pers:
        eager = [x.clone() for x in (wb if c.s.cur else wa)]
        gs = torch.cuda.Stream()
        gs.wait_stream(torch.cuda.current_stream())
        lgraph = torch.cuda.CUDAGraph()
        with torch.cuda.stream(gs):
            with torch.cuda.graph(lgraph, stream=gs):
                S.level_advance(levels[lv], prm, B, wa, wb, ctl, n_steps, 0, stream=gs)
        torch.cuda.current_stream().wait_stream(gs)
        for k in range(3):
            wa[k].copy_(init[k])
        S.swe_ctl_set(ctl, 0.0, dt0, 1.0e300, 0)
        torch.cuda.synchronize()
        e0.record()
        lgraph.replay()
        e1.record()
        torch.cuda.synchronize()
        graph_ms = e0.elapsed_time(e1) / n_steps
        cg = S.read_ctl(ctl)
        got = wb if cg.s.cur else wa
        graph_same = bool(cg.s.n_accepted == c.s.n_accepted and
                          all(torch.equal(x, y) for x, y in zip(got, eager)))
    # the fastest persistent schedule, its single cooperative launch of the
    # 100 attempts captured in a HIP graph and replayed from the same state
    pers_entries = [(u, l) for l, pm, u in entries if pm == 1 and u >= 0]
    pgraph_ms = pgraph_same = pname = None
    if pers_entries:
        _, lp = min(pers_entries)
        pname = names[(lp, 1)]
        ref_state = [x.clone() for x in (wb if c.s.cur else wa)]
        gs = torch.cuda.Stream()
        gs.wait_stream(torch.cuda.current_stream())
        pgraph = torch.cuda.CUDAGraph()
        with torch.cuda.stream(gs):
            with torch.cuda.graph(pgraph, stream=gs):
                S.level_advance(levels[lp], prm, B, wa, wb, ctl, n_steps, 1, stream=gs)
        torch.cuda.current_stream().wait_stream(gs)
        for k in range(3):
            wa[k].copy_(init[k])
        S.swe_ctl_set(ctl, 0.0, dt0, 1.0e300, 0)
        torch.cuda.synchronize()
        e0.record()
        pgraph.replay()
        e1.record()
        torch.cuda.synchronize()
        pgraph_ms = e0.elapsed_time(e1) / n_steps
        cp = S.read_ctl(ctl)
        got = wb if cp.s.cur else wa
        pgraph_same = bool(cp.s.n_accepted == c.s.n_accepted and int(levels[lp].sync_t[2].item()) == 0 and
                           all(torch.equal(x, y) for x, y in zip(got, ref_state)))
    # baseline: one launch per patch per step (fixed dt; no level reduction
    # round-trip charged to it)
    views = []
    for k in range(n_patches):
        o, n = tab[k].offset, tab[k].nx * tab[k].ny
        views.append((S.Grid(tab[k].nx, tab[k].ny, tab[k].dx, tab[k].dy), B[o:o + n],
                      [x[o:o + n] for x in wa], [x[o:o + n] for x in wb]))
    def per_patch_step(stream=None):
        for g, bb, qa_, qb_ in views:
            S.swe_step(g, prm, bb, qa_, qb_, 0.5 * dt0, stream=stream)
    per_patch_eager = _time_events(torch, per_patch_step, 2)
    # the fair baseline: the 3000 launches of one step captured once in a HIP
    # graph and replayed (no host cost per launch)
    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(cs):
        with torch.cuda.graph(graph, stream=cs):
            per_patch_step(stream=cs)
    torch.cuda.current_stream().wait_stream(cs)
    torch.cuda.synchronize()
    per_patch = _time_events(torch, graph.replay, 5)
    # the same level with waves on every edge (a centimetre of seeded noise on
    # the surface of every wet cell): a refined level sits where the waves are,
    # while the patches above are mostly sea at rest (the zero-flux fast path)
    noise = torch.tensor(np.random.default_rng(seed + 11).uniform(-0.01, 0.01, ncell), **f64)
    eta_b = eta + noise
    spd.zero_()
    for k in range(n_patches):
        o, n = tab[k].offset, tab[k].nx * tab[k].ny
        g = S.Grid(tab[k].nx, tab[k].ny, tab[k].dx, tab[k].dy)
        q = [x[o:o + n] for x in wa]
        S.swe_init(g, prm, B[o:o + n], eta_b[o:o + n], q)
        S.swe_max_speed(g, prm, B[o:o + n], q, 0, spd)
    dtb = prm.cfl_desired / float(spd.view(torch.float64).item())
    S.swe_ctl_set(ctl, 0.0, dtb, 1.0e300, 0)
    torch.cuda.synchronize()
    e0.record()
    S.level_advance(levels[lv], prm, B, wa, wb, ctl, n_steps, pers)
    e1.record()
    torch.cuda.synchronize()
    busy_ms = e0.elapsed_time(e1)
    cb = S.read_ctl(ctl)
    return {"level_patches": n_patches, "level_cells": ncell,
            "level_busy_ms_per_step": busy_ms / n_steps,
            "level_busy_cell_updates_per_s": ncell * cb.n_accepted / (busy_ms * 1e-3),
            "level_candidates_us_per_step": {names[(l, p)]: round(u, 2) for l, p, u in entries if u >= 0},
            "level_schedule": names[(lv, pers)],
            "level_lane_occupancy": {lnames[k]: round(levels[k].lane_occupancy, 3) for k in range(len(levels))},
            "level_steps": n_steps, "level_accepted": c.n_accepted,
            "level_cell_updates_per_s": best_rate,
            "level_ms_per_step": ms / n_steps,
            "level_graph_ms_per_step": graph_ms, "level_graph_result_identical": graph_same,
            "level_persistent_graph_schedule": pname, "level_persistent_graph_ms_per_step": pgraph_ms,
            "level_persistent_graph_result_identical": pgraph_same,
            "level_baseline_launch_per_patch_ms_per_step": per_patch * 1e3,
            "level_baseline_launch_per_patch_eager_ms_per_step": per_patch_eager * 1e3,
            "level_baseline_cell_updates_per_s": ncell / per_patch,
            "level_speedup_vs_launch_per_patch": per_patch * 1e3 / (ms / n_steps)}


def serve_bench(S, torch, I, np, n_req, nmin, nmax, K=32, ts=3600.0, tf=7200.0, tol=1e-4, flag_every=4,
                max_active=8, load=1.5, seed=17):
    """Serving: scenarios (basin seed 1000 + k, grid n ~ U{nmin..nmax} a side,
    32 adjoint snapshots, forward to 2 h with flagging) through swe_serve.

    1. sequential plain solves (one scenario at a time, all queued at t = 0)
       give the service rate mu;
    2. offline capacity of the served loop (max_active in flight);
    3. a Poisson trace at lambda = load * mu, replayed in real time through
       the sequential solver and through the served loop: p50/p99 latency
       (arrival to results on the host) and scenarios/s.
    Each served result is compared bit for bit with its sequential one."""
    trace = I.arrivals(n_req, 1.0, nmin, nmax, seed=seed)
    reqs = []
    for k, a in enumerate(trace):
        if k % 32 == 0:
            print(f"serve: building request {k} of {n_req}", file=sys.stderr, flush=True)
        b = I.basin(a.n, a.seed)
        g = S.Grid(a.n, a.n, b.grid.dx, b.grid.dy)
        reqs.append(S.Request(g, S.Params(), b.B, b.eta0, b.target, 0.0, ts, tf, K, tol,
                              flag_every=flag_every))
    foot = [S.serve_footprint(r) for r in reqs]
    free, _ = torch.cuda.mem_get_info()
    arena_bytes = int(min(0.8 * free, max(foot) * max_active * 1.25, 200 * 2**30))
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device="cuda")
    S.serve(reqs[:1], arena, 1)                         # warm-up (code objects, first launches)

    def progress(k, count=[0]):
        count[0] += 1
        if count[0] % 16 == 0:
            print(f"serve: {count[0] % n_req or n_req} of {n_req} done", file=sys.stderr, flush=True)

    def run(active, realtime):
        t = time.perf_counter()
        _, st = S.serve(reqs, arena, active, realtime=realtime, on_done=progress, check=False)
        el = time.perf_counter() - t
        print(f"serve: {n_req} requests, {active} in flight, {'realtime' if realtime else 'offline'}: "
              f"{el:.1f} s", file=sys.stderr, flush=True)
        return el, st

    el_seq, st_seq = run(1, False)
    ref = [(r.flag_acc.copy(), r.maxip_acc.copy(), [q.copy() for q in r.q]) for r in reqs]
    mu = n_req / el_seq
    el_cap, st_cap = run(max_active, False)

    def same():
        return all(np.array_equal(r.flag_acc, f) and np.array_equal(r.maxip_acc, m)
                   and all(np.array_equal(x, y) for x, y in zip(r.q, qs))
                   for r, (f, m, qs) in zip(reqs, ref))

    ok_cap = same()
    lam = load * mu
    for r, a in zip(reqs, trace):
        r.c.arrival = a.arrival / lam                   # rate-1 exponential gaps scaled to lambda
    el_rt_seq, st_rt_seq = run(1, True)
    el_rt, st_rt = run(max_active, True)
    ok_rt = same()

    def lat(st):
        x = np.array([s["latency"] for s in st])
        return {"p50_s": round(float(np.percentile(x, 50)), 4), "p99_s": round(float(np.percentile(x, 99)), 4),
                "mean_s": round(float(x.mean()), 4)}

    span = lambda st: max(s["finished"] for s in st) - min(r.c.arrival for r in reqs)
    cells = [a.n * a.n for a in trace]
    steps = [s["n_adj_steps"] + s["n_fwd_steps"] for s in st_seq]
    return {
        "trace": ("full: 256 requests, sides 256..2048" if (n_req, nmin, nmax) == (256, 256, 2048) else
                  f"reduced: {n_req} requests, sides {nmin}..{nmax} (the full trace of 256 requests, sides "
                  "256..2048, runs with --serve-full: about 5 minutes)"),
        "requests": n_req, "grid_side": [nmin, nmax], "snapshots": K, "t_final_s": tf, "window_start_s": ts,
        "tol": tol, "flag_every": flag_every, "max_active": max_active,
        "arena_GiB": round(arena_bytes / 2**30, 2), "footprint_GiB_max": round(max(foot) / 2**30, 3),
        "cell_updates_total": int(sum(c * s for c, s in zip(cells, steps))),
        "sequential_scen_per_s": round(mu, 3),
        "served_offline_scen_per_s": round(n_req / el_cap, 3),
        "served_offline_speedup": round(el_seq / el_cap, 3),
        "served_offline_cell_updates_per_s": sum(c * s for c, s in zip(cells, steps)) / el_cap,
        "poisson_rate_per_s": round(lam, 3), "load_vs_sequential": load,
        "sequential_realtime": dict(lat(st_rt_seq), scen_per_s=round(n_req / span(st_rt_seq), 3)),
        "served_realtime": dict(lat(st_rt), scen_per_s=round(n_req / span(st_rt), 3)),
        "p99_speedup": round(lat(st_rt_seq)["p99_s"] / max(lat(st_rt)["p99_s"], 1e-9), 3),
        "results_identical_to_sequential": bool(ok_cap and ok_rt),
        # requests whose run ended with an error (the same ones in every pass):
        # index, grid side and status
        "failed": [[k, trace[k].n, s["status"]] for k, s in enumerate(st_seq) if s["status"] != 0],
        "failed_same_in_every_pass": all([s["status"] for s in x] == [s["status"] for s in st_seq]
                                         for x in (st_cap, st_rt_seq, st_rt)),
    }


def cpu_baseline(b, n, budget_s):
    """The CPU oracle (plain C, fp64, OpenMP over rows) on the same input:
    a bounded number of steps of the same 1024^2 grid."""
    import numpy as np
    from oracle import oracle as O
    g = O.Grid(n, n, b.grid.dx, b.grid.dy)
    p = O.Params()
    h, hu, hv = O.init_state(g, p, O.NONLINEAR, b.B, b.eta0)
    dt = O.dt0(g, p, O.NONLINEAR, b.B, h, hu, hv)
    t = time.perf_counter()
    h, hu, hv, cfl, _ = O.swe_step(g, p, b.B, h, hu, hv, dt)
    t1 = time.perf_counter() - t
    m = int(max(2, min(200, budget_s / max(t1, 1e-6))))
    t = time.perf_counter()
    for _ in range(m):
        dt = dt * p.cfl_desired / cfl
        h, hu, hv, cfl, _ = O.swe_step(g, p, b.B, h, hu, hv, dt)
    el = time.perf_counter() - t
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    del np
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": n * n * m / el, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "cpu_model": model,
            "sample": f"{m} steps of the {n}x{n} basin after 1 warm-up step ({el:.1f} s), "
                      f"OpenMP over rows on {threads} threads of {model}"}


if __name__ == "__main__":
    main()
