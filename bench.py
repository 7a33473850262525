#!/usr/bin/env python3
"""Throughput of the WENO5 / SSP-RK3 Teukolsky hot path on one MI355X.

Workload: the gravitational solve s = -2, m = 2, a/M = 0.999 on an 8192 (r_*)
x 256 (theta) grid, x in [-200, 400], seeded Gaussian pulse times the
spin-weighted harmonic, dt = 0.5 x the device stability bound, waveform sampled
at r_* = 30 every 10 steps.  One benchmark step is one SSP-RK(3,3) time step
(three fused stage kernels over the whole grid, plus the waveform sample when
due).  Inputs are resident in HBM before the timed region.

Reported: point-updates/s (one point-update = one RHS evaluation with its RK
combination at one grid point, all four planes; three per point per step), the
HBM roofline of the fused stage kernel (algorithmic bytes: 64 B per point in
stage 1, 96 B in stages 2 and 3, i.e. 256 B per point-step), and the FP64 CPU
oracle timed on a bounded sample of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
BYTES_PER_POINT_STEP = 256.0   # 64 + 96 + 96 (fields only; coefficients rebuilt on chip)
KERNEL_SRC = os.path.join(ROOT, "paper_2010_04760_amd", "csrc", "teuk_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stage_kernel_c2_traffic.json")


def kernel_sha() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def measured_traffic(weights: str):
    """HBM bytes per stage launch from the committed rocprofv3 counter runs, or
    None if they were taken on a different kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    rec = json.load(open(TRAFFIC_FILE))
    if rec.get("kernel_sha") != kernel_sha() or weights not in rec.get("bytes_per_launch", {}):
        return None
    return float(rec["bytes_per_launch"][weights])


def cpu_baseline(wl, u0, target_s: float):
    """The FP64 oracle on the host cores, on the same grid and initial data."""
    from oracle import solver as S
    threads = min(os.cpu_count() or 1, 16)
    S.set_threads(threads)
    prob = S.Problem(wl.s, wl.m, wl.a, wl.nr, wl.nth, wl.x_min, wl.x_max)
    o = S.TeukOracle(prob)
    dt = o.dt_bound(0.5)
    t0 = time.perf_counter()
    u1, _ = o.evolve(u0, dt, 1)
    t1 = time.perf_counter() - t0
    n = max(1, int(target_s / max(t1, 1e-3)))
    t0 = time.perf_counter()
    o.evolve(u1, dt, n)
    el = time.perf_counter() - t0
    return {"value": 3.0 * wl.points * n / el, "unit": "point-updates/s", "cores": S.num_threads(),
            "kind": "oracle",
            "sample": f"{wl.nr}x{wl.nth} grid of the same workload, {n} SSP-RK3 steps "
                      f"({3 * wl.points * n:.3g} point-updates, {el:.1f} s) on {S.num_threads()} OpenMP threads"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000, help="timed SSP-RK3 steps (workload length: 20000)")
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--weights", default="fp64", choices=["fp64", "fp32", "fp16", "bf16"])
    ap.add_argument("--workgroups", type=int, default=0, help="stage-kernel workgroups (0: all the GPU holds at once)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one MI355X only: this build has no multi-GPU path "
              "(a single solve would shard into radial slabs; see the design notes).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2010_04760_amd as T
    import workloads as W

    wl = W.C2
    u0 = W.gaussian_pulse(wl)
    total = args.warmup + args.steps
    cfg = T.make_config(s=wl.s, m=wl.m, a=wl.a, nr=wl.nr, ntheta=wl.nth, x_min=wl.x_min, x_max=wl.x_max,
                        M=wl.M, dt=0.0, cfl=0.5, weight_prec=args.weights, x_extract=wl.x_e,
                        extract_every=wl.every, max_samples=total // wl.every + 1, workgroups=args.workgroups)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    sv = T.Solver(cfg, stream=stream)
    sv.set_initial(u0)
    print(f"# warmup {args.warmup} steps", file=sys.stderr, flush=True)
    sv.step(args.warmup)
    torch.cuda.synchronize()

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    print(f"# timing {args.steps} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(stream)
    sv.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    gpu_s = ev0.elapsed_time(ev1) / 1e3
    sv.check_finite()
    info = sv.info()
    sv.close()

    npts = wl.points
    pu = 3.0 * npts * args.steps
    value = pu / gpu_s
    # Stage kernels: 3 launches per step; the sample kernel (one per 10 steps)
    # is included in the time and is < 0.5 % of it.
    launches = 3 * args.steps
    t_launch = gpu_s / launches
    bytes_launch = BYTES_PER_POINT_STEP * npts / 3.0
    achieved = bytes_launch / t_launch / 1e9
    traffic = measured_traffic(args.weights)

    out = {
        "metric": "WENO5 RHS point-updates/s, %HBM peak; mixed vs FP64 speedup at equal error",
        "value": value,
        "unit": "point-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": gpu_s / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.weights == "fp64" else f"f64 (weights {args.weights})",
        "data": "synthetic",
        "config": {"workload": wl.name, "nr": wl.nr, "ntheta": wl.nth, "s": wl.s, "m": wl.m, "a": wl.a,
                   "weights": args.weights, "dt": info.dt, "workgroups": info.workgroups,
                   "extract_every": wl.every, "seed": wl.seed},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "kernel": "stage_kernel (fused SSP-RK3 stage)",
                     "algorithmic_bytes_per_launch": bytes_launch,
                     "avg_launch_us": t_launch * 1e6},
        "wall_s": wall,
    }
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl, u0, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
