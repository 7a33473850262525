#!/usr/bin/env python3
"""Throughput of the WENO5 / SSP-RK3 Teukolsky hot path on one MI355X.

Default workload (C2): the gravitational solve s = -2, m = 2, a/M = 0.999 on an
8192 (r_*) x 256 (theta) grid, x in [-200, 400], seeded Gaussian pulse times
the spin-weighted harmonic, dt = 0.5 x the device stability bound, waveform
sampled at r_* = 30 every 10 steps.  One benchmark step is one SSP-RK(3,3)
time step (three fused stage kernels over the whole grid, plus the waveform
sample when due).  Inputs are resident in HBM before the timed region.

Reported: point-updates/s (one point-update = one RHS evaluation with its RK
combination at one grid point, all four planes; three per point per step), the
HBM roofline of the fused stage kernel (algorithmic bytes: 64 B per point in
stage 1, 96 B in stages 2 and 3, i.e. 256 B per point-step), the same workload
with FP32 / FP16 / BF16 WENO weights (speed and waveform error against FP64),
and the FP64 CPU oracle timed on a bounded sample of the workload on the host
cores.

Other workloads (one JSON line each):
  --workload C3   s = 0, m = 0 extremal Kerr on 16384 x 128, 200000 steps, with
                  FP64 / FP32 / FP16 / BF16 weights: speed, waveform error and
                  late-time tail index against FP64.
  --workload C3H  the horizon experiment of Sec. 4 in the hyperboloidal chart
                  (s = -2, l = 2, a = M, 16384 x 64) per weight precision, with the
                  charge proxy d_rho Phi on the horizon against FP64, and a coarser
                  FP64 run to tau = 2000 for the horizon power laws.
  --workload C4   64 independent solves of uneven size advanced together
                  through the group extension (FP32 weights, 2000 steps).
  --workload C5   Poisson arrivals of such solves served by continuous
                  batching (admission by HBM footprint); p50/p99 latency.
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
METRIC = "WENO5 RHS point-updates/s, %HBM peak; mixed vs FP64 speedup at equal error"


def kernel_sha() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def measured_traffic(weights: str, key: str = "bytes_per_launch"):
    """HBM bytes per launch from the committed rocprofv3 counter runs (per
    stage launch, or with key "bytes_per_blocked_step" per blocked step), or
    None if they were taken on a different kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    rec = json.load(open(TRAFFIC_FILE))
    if rec.get("kernel_sha") != kernel_sha() or weights not in rec.get(key, {}):
        return None
    return float(rec[key][weights])


def log(msg: str):
    print("# " + msg, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(S, o, u0, dt, points, target_s, threads):
    """Point-updates/s of the oracle on `threads` OpenMP threads, timed over
    whole steps until target_s seconds have passed."""
    S.set_threads(threads)
    u, _ = o.evolve(u0, dt, 1)                 # first call: thread start-up, page faults
    n, el, chunk = 0, 0.0, 1
    while el < target_s:
        t0 = time.perf_counter()
        u, _ = o.evolve(u, dt, chunk)
        dt_chunk = time.perf_counter() - t0
        n, el = n + chunk, el + dt_chunk
        chunk = max(1, min(64, int(0.25 * target_s / max(dt_chunk / chunk, 1e-4))))
    return 3.0 * points * n / el, n, el, S.num_threads()


def cpu_baseline(wl, u0, target_s: float):
    """The FP64 oracle on the host, on the same grid and initial data: one
    thread, and every core the process may use (at most 16, the host share of
    one GPU).  `value` is the all-cores rate."""
    from oracle import solver as S
    prob = S.Problem(wl.s, wl.m, wl.a, wl.nr, wl.nth, wl.x_min, wl.x_max)
    o = S.TeukOracle(prob)
    dt = o.dt_bound(0.5)
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    many = max(1, min(avail, 16))
    r1, n1, e1, t1 = _oracle_rate(S, o, u0, dt, wl.points, 0.4 * target_s, 1)
    rn, nn, en, tn = _oracle_rate(S, o, u0, dt, wl.points, 0.6 * target_s, many)
    grid = f"{wl.nr}x{wl.nth} grid ({wl.name.split(':')[0]})"
    return {"value": rn, "unit": "point-updates/s", "cores": tn, "kind": "oracle",
            "sample": f"{grid}, {nn} SSP-RK3 steps ({3 * wl.points * nn:.3g} point-updates, {en:.1f} s) "
                      f"on {tn} OpenMP threads; single thread: {n1} steps in {e1:.1f} s",
            "single_thread": {"value": r1, "unit": "point-updates/s", "cores": t1},
            "speedup_all_cores_vs_one": rn / r1,
            "cpu": {"model": cpu_model(), "nproc": os.cpu_count(), "affinity": avail}}


def roofline(points_per_launch: float, t_launch: float, traffic):
    bytes_launch = BYTES_PER_POINT_STEP * points_per_launch / 3.0
    achieved = bytes_launch / t_launch / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": "stage_kernel (fused SSP-RK3 stage)",
            "algorithmic_bytes_per_launch": bytes_launch, "avg_launch_us": t_launch * 1e6}


# SSP-RK(10,4) step: eight stages read u and write u (64 B per point), the
# fifth reads u^(4) and u^n and writes two outputs (128 B), the last reads
# u^(9) and q and writes (96 B): 736 B per point-step.
RK104_BYTES_PER_POINT_STEP = 8 * 64 + 128 + 96

# FP64 operations (FMA counted twice) and VALU instructions per point-stage of
# the double-double stage kernel, counted in its gfx950 ISA (stages 2 and 3;
# one lane per point): it is bound by FP64 instruction issue.
DD_OPS = {"dd_weights": (4701, 4311), "fp64_weights": (2807, 2697)}
FP64_VECTOR_TFLOPS = 78.6                 # MI355X FP64 vector peak (FMA = 2 flops)
VALU_ISSUE_PER_S = 256 * 4 * 16 * 2.4e9   # lane-instructions/s: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz


def dd_roofline(points_per_launch: float, t_launch: float, variant: str):
    flops, instrs = DD_OPS[variant]
    achieved = flops * points_per_launch / t_launch / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP64_VECTOR_TFLOPS, "traffic": None, "avg_launch_us": t_launch * 1e6,
            "valu_issue_frac": instrs * points_per_launch / t_launch / VALU_ISSUE_PER_S}


def solver_config(T, wl, weights, total_steps, workgroups=0, every=None, state="fp64", integrator="rk3",
                  theta_order=2):
    every = wl.every if every is None else every
    return T.make_config(s=wl.s, m=wl.m, a=wl.a, nr=wl.nr, ntheta=wl.nth, x_min=wl.x_min, x_max=wl.x_max,
                         M=wl.M, dt=0.0, cfl=0.5, weight_prec=weights, x_extract=wl.x_e, extract_every=every,
                         max_samples=total_steps // every + 1 if every > 0 else 0, workgroups=workgroups,
                         state=state, integrator=integrator, theta_order=theta_order)


def copy_probe(mib, torch):
    """A plain device copy of `mib` MiB, three times: a kernel of known traffic
    that calibrates the rocprofv3 FETCH_SIZE / WRITE_SIZE counters of the run."""
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copy probe: {n * 8} bytes read and written per copy")
    del src, dst


# ----------------------------------------------------------------------------- C2: one solve
def bench_single(args, torch, T, W):
    c1 = args.workload == "C1"
    wl = W.C1 if c1 else W.C2
    steps = (wl.steps if c1 else 20000) if args.steps is None else args.steps
    warmup = 100 if args.warmup is None else args.warmup
    weights = args.weights or "fp64"
    u0 = W.gaussian_pulse(wl)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)

    def make(wp, total, state="fp64", integrator="rk3", every=None, theta_order=2):
        """A solver of the workload with the initial data set (host work: tables,
        bound, upload)."""
        sv = T.Solver(solver_config(T, wl, wp, total, args.workgroups, state=state, integrator=integrator,
                                    every=every, theta_order=theta_order), stream=stream)
        sv.set_initial(u0)
        return sv

    def warm(sv, nwarm, label=""):
        """Queue the warmup steps on the stream (behind whatever it holds)."""
        log(f"{label}: warmup {nwarm} steps")
        sv.step(nwarm)

    def capture(sv, graph, label=""):
        """Capture the solver's graph at the sampling phase its warmup leaves."""
        if graph:
            log(f"{label}: graph capture of {graph} steps")
            sv.set_graph(graph)

    def time_steps(sv, nsteps, label="", before=None, after=None):
        """Synchronize, then time exactly `nsteps` steps of a warmed solver
        with HIP events on the solver's stream, and synchronize.  `before`
        runs after the timed launches are queued and before the closing
        synchronization (the next run's plain warmup launches, so that the
        GPU does not idle between runs); `after` runs after it (host work that
        would slow timed launches still being fed to the GPU on a
        launch-bound grid: graph captures, cooperative launches).  Returns
        (seconds, wall seconds)."""
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        log(f"{label}: timing {nsteps} steps")
        w0 = time.perf_counter()
        ev0.record(stream)
        sv.step(nsteps)
        ev1.record(stream)
        if before is not None:
            before()
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        if after is not None:
            after()
        return ev0.elapsed_time(ev1) / 1e3, wall

    def finish(sv):
        """Guard, counters and waveform of a timed solver; releases it."""
        sv.check_finite()
        info = sv.info()
        _, wave = sv.waveform()
        sv.close()
        return info, wave

    def run(wp, state="fp64", nsteps=None, nwarm=None, integrator="rk3", every=None, graph=0, theta_order=2):
        """make + time_steps + finish: (seconds, wall seconds, info, waveform samples)."""
        nsteps = steps if nsteps is None else nsteps
        nwarm = warmup if nwarm is None else nwarm
        sv = make(wp, nwarm + nsteps, state, integrator, every, theta_order)
        label = f"{state}/{wp}/{integrator}"
        warm(sv, nwarm, label)
        capture(sv, graph, label)
        sec, wall = time_steps(sv, nsteps, label)
        info, wave = finish(sv)
        return sec, wall, info, wave

    # Launch shapes from the project's autotuner (it times stage-kernel
    # workgroup budgets on a scratch solver of this grid; solvers created
    # afterwards with workgroups = 0 use the winner).
    tuned = {}
    if not args.no_tune and args.workgroups == 0:
        for integ in ("rk3", "rk3_blocked") if (weights == "fp64" and not args.no_blocked) else ("rk3",):
            cfg = solver_config(T, wl, weights, 1, 0, every=0, integrator=integ)
            log(f"autotuner: {integ}")
            ti = T.teuk_tune(cfg, 0)
            tuned[integ] = {"workgroups": ti.workgroups, "segs_per_strip": ti.segs, "candidates": ti.candidates,
                            "us_per_step": ti.us_per_step, "default_workgroups": ti.default_workgroups,
                            "default_segs_per_strip": ti.default_segs, "us_per_step_default": ti.us_per_step_default}
        if not args.no_theta4:
            log("autotuner: rk3, fourth-order theta differences")
            ti = T.teuk_tune(solver_config(T, wl, weights, 1, 0, every=0, theta_order=4), 0)
            tuned["rk3_theta4"] = {"workgroups": ti.workgroups, "segs_per_strip": ti.segs,
                                   "us_per_step": ti.us_per_step, "us_per_step_default": ti.us_per_step_default}

    # Every timed solver of the headline and of the legs compared with it is
    # created here, before any timing.  The GPU's clock drops within about
    # 10 ms of idling and takes tens of milliseconds of load to recover
    # (measured: 20 steps after 5 warmup steps take 96.5-99 us each when the
    # GPU idled < 3 ms before the warmup, 105-113 us after 10 ms - 1 s), and
    # creating a solver of this grid idles it for longer than that.  So the
    # timed runs follow each other with the GPU kept busy: each run's warmup
    # steps are queued behind the run before it -- the headline's behind the
    # last reduced-precision run -- and short runs time the kernels at the
    # clock of a long solve.
    # Headline launch mode: graph replay where launches bound the step (C1,
    # 11 us per step), one launch per stage where kernels do (C2: replaying a
    # 10-step graph measured 0.5 % slower than launching); the graph leg
    # reports the other mode.
    graph = args.graph if args.graph >= 0 else (50 if c1 else 0)
    other = 0 if graph else (50 if c1 else 10)   # the other launch mode (a multiple of the 10-step cadence)
    # The legs compared with the headline time at least 500 C2 steps (about
    # 50 ms), whatever K is: over 20 steps their times scatter by 10-15 %.
    lsteps = steps if c1 else max(steps, 500)
    n4, w4 = max(lsteps // 6, 1), warmup // 6
    hs = make(weights, warmup + steps)
    # (name, solver, timed steps, warmup steps, graph chunk, label), timed in this order
    chain = [("headline", hs, steps, warmup, graph, f"fp64/{weights}/rk3 (headline)")]
    if weights == "fp64" and not args.no_blocked:
        # in the headline's launch mode (C1: one launch per step, replayed from a graph)
        chain.append(("blocked", make("fp64", warmup + lsteps, integrator="rk3_blocked"), lsteps, warmup, graph,
                      "fp64/fp64/rk3_blocked"))
    if not args.no_graph_leg:
        chain.append(("graph", make(weights, warmup + lsteps), lsteps, warmup, other,
                      f"fp64/{weights}/rk3 (other launch mode)"))
    if not args.no_theta4:
        chain.append(("theta4", make(weights, warmup + lsteps, theta_order=4), lsteps, warmup, graph,
                      f"fp64/{weights}/rk3 theta order 4"))
    if weights == "fp64" and not args.no_pipelined:
        chain.append(("pipelined", make("fp64", warmup + lsteps, integrator="rk3_pipelined"), lsteps, warmup, 0,
                      "fp64/fp64/rk3_pipelined"))
    if not c1 and weights == "fp64" and not args.no_rk104:
        chain.append(("rk104", make("fp64", n4 + w4, integrator="rk104", every=5), n4, w4, 0,
                      "fp64/fp64/rk104"))

    def link(i):
        """(before, after) callables that warm up chain[i] behind the run before
        it: plain warmup launches before that run's closing synchronization,
        a cooperative (pipelined) warmup and the graph capture after it."""
        if i >= len(chain):
            return None, None
        name, sv, _, nw, g, label = chain[i]
        if name == "pipelined":
            return None, lambda: warm(sv, nw, label)
        return (lambda: warm(sv, nw, label)), (lambda: capture(sv, g, label))

    # Reduced-precision weights over the workload's full length (the waveform
    # at x_e needs the pulse to have passed it), before the headline timing:
    # speed and waveform error (relative L2 over every sample) against FP64.
    # The headline's warmup follows the last of these runs directly (its
    # solver is finished afterwards).
    mixed = None
    tail = None
    if weights == "fp64" and not args.no_mixed:
        full = wl.steps if args.mixed_steps <= 0 else args.mixed_steps
        sec64f, _, _, wave64f = run("fp64", nsteps=full, nwarm=0)
        mixed = {"steps": full, "fp64": {"value": 3.0 * wl.points * full / sec64f, "seconds": sec64f}}
        for wp in ("fp32", "fp16"):
            sec_w, _, _, wave_w = run(wp, nsteps=full, nwarm=0)
            mixed[wp] = (sec_w, wave_w)
        sv_t = make("bf16", full)
        b0, a0 = link(0)
        tail = (sv_t, time_steps(sv_t, full, "fp64/bf16/rk3", before=b0, after=a0)[0])
    else:
        b0, a0 = link(0)
        for f in (b0, a0):
            if f is not None:
                f()

    # the chain: headline, then the legs compared with it
    timed = {}
    for i, (name, sv, nst, _, _, label) in enumerate(chain):
        b, a = link(i + 1)
        timed[name] = time_steps(sv, nst, label, before=b, after=a)
    gpu_s, wall = timed["headline"]
    if tail is not None:
        sv_t, sec_t = tail
        mixed["bf16"] = (sec_t, finish(sv_t)[1])
        for wp in ("fp32", "fp16", "bf16"):
            sec_w, wave_w = mixed[wp]
            mixed[wp] = {"value": 3.0 * wl.points * full / sec_w, "seconds": sec_w,
                         "speedup_vs_fp64": sec64f / sec_w,
                         "waveform_rel_l2_vs_fp64": float(np.linalg.norm(wave_w - wave64f) / np.linalg.norm(wave64f))}
        mixed["waveform"] = (f"{wave64f.shape[0]} samples x {wl.nth} rows at r* = {wl.x_e}, t = 0 .. "
                             f"{full} steps; the FP64 run is the parity-tested path")
    info, wave = finish(hs)
    results = {name: timed[name] + finish(sv) for name, sv, *_ in chain[1:]}
    do_graph_leg, do_theta4 = "graph" in results, "theta4" in results
    do_pipe, do_blocked, do_rk104 = "pipelined" in results, "blocked" in results, "rk104" in results

    pu = 3.0 * wl.points * steps
    # 3 stage launches per step; the sample kernel (one per 10 steps) is
    # included in the time and is < 0.5 % of it.
    out = {
        "metric": METRIC, "value": pu / gpu_s, "unit": "point-updates/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": gpu_s / steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if weights == "fp64" else f"f64 (weights {weights})",
        "data": "synthetic",
        "config": {"workload": wl.name, "nr": wl.nr, "ntheta": wl.nth, "s": wl.s, "m": wl.m, "a": wl.a,
                   "weights": weights, "dt": info.dt, "workgroups": info.workgroups,
                   "extract_every": wl.every, "seed": wl.seed, "graph_chunk_steps": graph,
                   "launch_shape": "autotuned" if "rk3" in tuned else ("given" if args.workgroups else "default")},
        "roofline": roofline(wl.points, gpu_s / (3 * steps), measured_traffic(weights) if not c1 else None),
        "wall_s": wall,
    }
    if tuned:
        out["autotuner"] = tuned
    if mixed is not None:
        out["mixed_precision"] = mixed
    t_step = gpu_s / steps                   # headline seconds per step
    lpu = 3.0 * wl.points * lsteps           # point-updates of a leg

    def same_prefix(a, b):
        # the runs start from the same state with the same dt: their common
        # samples must agree
        m = min(a.shape[0], b.shape[0])
        return a[:m], b[:m]

    if do_graph_leg:
        sec_o, _, _, wave_o = results["graph"]
        wo, wh = same_prefix(wave_o, wave)
        out["graph"] = {"chunk_steps": other, "steps": lsteps, "ms_per_step": sec_o / lsteps * 1e3,
                        "value": lpu / sec_o, "speedup_vs_headline": t_step / (sec_o / lsteps),
                        "waveform_identical": bool(np.array_equal(wo, wh))}
    if do_theta4:
        # the same workload with fourth-order theta differences (two rows
        # ahead and behind; the same HBM traffic per point, a smaller dt)
        sec4, _, info4, _ = results["theta4"]
        out["theta4"] = {"steps": lsteps, "dt": info4.dt, "ms_per_step": sec4 / lsteps * 1e3, "value": lpu / sec4,
                         "speed_vs_second_order": t_step / (sec4 / lsteps),
                         "simulated_time_per_s_vs_second_order": (info4.dt * lsteps / sec4) / (info.dt / t_step),
                         "hbm_frac": roofline(wl.points, sec4 / (3 * lsteps), None)["frac"]}
    if do_pipe:
        # the same steps in one cooperative launch per waveform interval (tiles
        # wait for their neighbours' previous stage only)
        secp, _, infop, wavep = results["pipelined"]
        wp_, wh = same_prefix(wavep, wave)
        out["pipelined"] = {"steps": lsteps, "ms_per_step": secp / lsteps * 1e3, "value": lpu / secp,
                            "speedup_vs_headline": t_step / (secp / lsteps), "workgroups": infop.workgroups,
                            "waveform_identical": bool(np.array_equal(wp_, wh)),
                            "launches": "one per waveform interval (every %d steps)" % wl.every}
    if do_blocked:
        # Temporal blocking: the same SSP-RK(3,3) step as one launch per step
        # (u(1), u(2) in LDS; 64 B of HBM traffic per point-step; "traffic" is
        # the measured bytes per step).
        secb, _, infob, waveb = results["blocked"]
        wb, wh = same_prefix(waveb, wave)
        out["blocked"] = {
            "steps": lsteps, "ms_per_step": secb / lsteps * 1e3, "value": lpu / secb, "unit": "point-updates/s",
            "speedup_vs_three_launch": t_step / (secb / lsteps), "tiles": infob.workgroups,
            "waveform_rel_diff_vs_three_launch": float(np.max(np.abs(wb - wh)) / max(np.max(np.abs(wh)), 1e-300)),
            "hbm": {"bytes_per_point_step": 64, "achieved_GBs": 64.0 * wl.points * lsteps / secb / 1e9,
                    "frac": 64.0 * wl.points * lsteps / secb / 1e9 / HBM_PEAK_GBS,
                    "traffic": None if c1 else measured_traffic("fp64", "bytes_per_blocked_step")},
        }
    if c1:
        if not args.no_cpu_baseline:
            log("cpu baseline (oracle)")
            out["cpu_baseline"] = cpu_baseline(wl, u0, args.cpu_seconds)
        return out
    if do_rk104:
        # SSP-RK(10,4) (Sec. 3.2) over the same simulated time: its default step
        # is 6x the SSP-RK(3,3) step (SSP coefficients 6 and 1), ten stages per
        # step.  Waveforms compared at common sample times (every 5th step of
        # SSP-RK(10,4) = every 30th of SSP-RK(3,3)).
        sec4, _, info4, wave4 = results["rk104"]
        ref = wave[::3][: wave4.shape[0]]
        m = min(ref.shape[0], wave4.shape[0])
        stages = 10 * n4
        t_stage = sec4 / stages
        out["rk104"] = {
            "steps": n4, "warmup": w4, "dt": info4.dt, "ms_per_step": sec4 / n4 * 1e3,
            "value": wl.points * stages / sec4, "unit": "point-updates/s",
            "simulated_time_per_s_vs_rk3": (n4 * info4.dt / sec4) / (info.dt / t_step),
            "waveform_rel_l2_vs_rk3": float(np.linalg.norm(wave4[:m] - ref[:m]) / np.linalg.norm(ref[:m])),
            "hbm": {"bytes_per_point_step": RK104_BYTES_PER_POINT_STEP,
                    "achieved_GBs": RK104_BYTES_PER_POINT_STEP * wl.points * n4 / sec4 / 1e9,
                    "frac": RK104_BYTES_PER_POINT_STEP * wl.points * n4 / sec4 / 1e9 / HBM_PEAK_GBS,
                    "avg_launch_us": t_stage * 1e6},
        }
    if weights == "fp64" and args.quad_steps > 0:
        # The paper's own experiment (Sec. 3.1.3): a high-precision state with
        # weights in that precision, against the same state with weights in
        # double.  Here the high precision is double-double (106 bits).
        qs, qw = args.quad_steps, 10
        pq = 3.0 * wl.points * qs
        sec64, _, _, wave64 = run("fp64", nsteps=qs, nwarm=qw)
        sec_dd, _, _, wave_dd = run("dd", state="dd", nsteps=qs, nwarm=qw)
        sec_mx, _, _, wave_mx = run("fp64", state="dd", nsteps=qs, nwarm=qw)
        vdd = wave_dd[..., 0] + wave_dd[..., 1]
        dmx = (wave_mx[..., 0] - wave_dd[..., 0]) + (wave_mx[..., 1] - wave_dd[..., 1])
        out["quad_baseline"] = {
            "state": "double-double", "steps": qs, "warmup": qw,
            "dd_weights": {"value": pq / sec_dd, "ms_per_step": sec_dd / qs * 1e3},
            "fp64_weights": {"value": pq / sec_mx, "ms_per_step": sec_mx / qs * 1e3},
            "speedup_fp64_weights_vs_dd_weights": sec_dd / sec_mx,
            "waveform_rel_l2_fp64_weights_vs_dd_weights": float(np.linalg.norm(dmx) / np.linalg.norm(vdd)),
            "waveform_rel_l2_fp64_state_vs_dd": float(np.linalg.norm(wave64 - wave_dd[..., 0] - wave_dd[..., 1])
                                                      / np.linalg.norm(vdd)),
            "cost_vs_fp64_state": {"dd_weights": sec_dd / sec64, "fp64_weights": sec_mx / sec64},
            "roofline": {wv: dd_roofline(wl.points, sec / (3 * qs), wv)
                         for wv, sec in (("dd_weights", sec_dd), ("fp64_weights", sec_mx))},
        }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(wl, u0, args.cpu_seconds)
    return out


# ----------------------------------------------------------------------------- C3: precision sweep
def local_index(t, y):
    """p(t) = t (dy/dt) / y by centred differences of a sampled series."""
    return t[1:-1] * (y[2:] - y[:-2]) / (t[2:] - t[:-2]) / y[1:-1]


def bench_sweep(args, torch, T, W):
    wl = W.C3
    steps = wl.steps if args.steps is None else args.steps
    u0 = W.gaussian_pulse(wl)
    stream = torch.cuda.current_stream()
    k_star = wl.nth // 4                      # fixed polar node for the tail (theta ~ pi/4)
    runs = {}
    for wp in ("fp64", "fp32", "fp16", "bf16"):
        sv = T.Solver(solver_config(T, wl, wp, steps), stream=stream)
        sv.set_initial(u0)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        log(f"C3 {wp}: {steps} steps")
        ev0.record(stream)
        sv.step(steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        sec = ev0.elapsed_time(ev1) / 1e3
        sv.check_finite()
        t, w = sv.waveform()
        dt = sv.info().dt
        sv.close()
        runs[wp] = (sec, t, w, dt)
        log(f"C3 {wp}: {sec:.2f} s")
    pu = 3.0 * wl.points * steps
    sec64, t, w64, dt = runs["fp64"]
    lo, hi = 200.0, min(800.0, t[-1])
    win = (t >= lo) & (t <= hi)
    late = (t >= 0.75 * hi) & (t <= hi)

    def tail(w):
        y = w[:, k_star, 0]
        p = local_index(t, y)
        tm = t[1:-1]
        sel = (tm >= 0.75 * hi) & (tm <= hi)
        return float(np.mean(p[sel])), float(p[np.searchsorted(tm, hi) - 1])

    p64 = tail(w64)
    per = {}
    for wp, (sec, _, w, _) in runs.items():
        pm, pe = tail(w)
        err = float(np.linalg.norm(w[win] - w64[win]) / np.linalg.norm(w64[win]))
        err_late = float(np.linalg.norm(w[late] - w64[late]) / np.linalg.norm(w64[late]))
        per[wp] = {"value": pu / sec, "seconds": sec, "speedup_vs_fp64": sec64 / sec,
                   "waveform_rel_l2_vs_fp64": err, "late_rel_l2_vs_fp64": err_late,
                   "tail_index_mean": pm, "tail_index_end": pe, "tail_index_diff_vs_fp64": pm - p64[0]}
    return {
        "metric": METRIC, "value": pu / sec64, "unit": "point-updates/s", "n_gpus": 1, "steps": steps,
        "warmup": 0, "ms_per_step": sec64 / steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": wl.name, "nr": wl.nr, "ntheta": wl.nth, "s": wl.s, "m": wl.m, "a": wl.a,
                   "dt": dt, "x_extract": wl.x_e, "theta_star": float((k_star + 0.5) * np.pi / wl.nth),
                   "window": [lo, hi], "reference": "FP64 GPU run (the oracle checks it at this size for "
                                                    "a few steps; the full run is beyond the host)"},
        "roofline": roofline(wl.points, sec64 / (3 * steps), None),
        "per_dtype": per,
    }


# ----------------------------------------------------------------------------- C3-H: horizon chart
def horizon_series(T, torch, wl, weights, steps, every, stream, scheme="weno5"):
    """Run the hyperboloidal-chart workload; returns (seconds, dt, tau, Phi_H, dPhi_H, theta)."""
    cfg = T.make_config(s=wl.s, m=wl.m, a=wl.a, nr=wl.nr, ntheta=wl.nth, x_min=wl.x_min, x_max=wl.x_max,
                        M=wl.M, dt=0.0, cfl=0.5, weight_prec=weights, x_extract=wl.x_e, extract_every=every,
                        max_samples=steps // every + 1, chart="H", S=wl.S, scheme=scheme)
    import workloads as W
    sv = T.Solver(cfg, stream=stream)
    sv.set_initial(W.gaussian_pulse(wl))
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    done = 0
    while done < steps:                     # in chunks, so that progress is visible
        k = min(steps - done, 50000)
        sv.step(k)
        done += k
        torch.cuda.synchronize()
        log(f"  {scheme}/{weights}: {done}/{steps} steps")
    ev1.record(stream)
    torch.cuda.synchronize()
    sec = ev0.elapsed_time(ev1) / 1e3
    sv.check_finite()
    tau, ph, dph = sv.horizon()
    dt = sv.info().dt
    sv.close()
    theta = (np.arange(wl.nth) + 0.5) * np.pi / wl.nth
    return sec, dt, tau, ph, dph, theta


def charge(dph, theta):
    """Aretakis-charge proxy: the sin(theta)-weighted theta integral of d_rho Phi on the horizon."""
    w = np.sin(theta) * (np.pi / len(theta))
    return dph @ w


def bench_horizon(args, torch, T, W):
    wl = W.C3H
    steps = wl.steps if args.steps is None else args.steps
    stream = torch.cuda.current_stream()
    k_star = wl.nth // 4
    runs = {}
    for wp in ("fp64", "fp32", "fp16", "bf16"):
        log(f"C3-H {wp}: {steps} steps")
        runs[wp] = horizon_series(T, torch, wl, wp, steps, wl.every, stream)
    sec64, dt, tau, ph64, dph64, theta = runs["fp64"]
    q64 = charge(dph64, theta)
    pu = 3.0 * wl.points * steps
    late = tau >= 0.5 * tau[-1]
    per = {}
    for wp, (sec, _, _, ph, dph, _) in runs.items():
        q = charge(dph, theta)
        per[wp] = {"value": pu / sec, "seconds": sec, "speedup_vs_fp64": sec64 / sec,
                   "phi_h_rel_l2_vs_fp64": float(np.linalg.norm(ph - ph64) / np.linalg.norm(ph64)),
                   "charge_rel_drift_vs_fp64": float(np.max(np.abs(q[late] - q64[late])) / np.max(np.abs(q64[late]))),
                   "charge_change_late": float(abs(q[-1] / q[late][0] - 1.0))}
    out = {
        "metric": METRIC, "value": pu / sec64, "unit": "point-updates/s", "n_gpus": 1, "steps": steps,
        "warmup": 0, "ms_per_step": sec64 / steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": wl.name, "nr": wl.nr, "ntheta": wl.nth, "s": wl.s, "m": wl.m, "a": wl.a,
                   "S": wl.S, "dt": dt, "tau_end": float(tau[-1]), "theta_star": float(theta[k_star])},
        # the chart-H kernel streams ten coefficients per point: 80 B more per point-stage
        "roofline": {"bound": "hbm", "algorithmic_bytes_per_point_stage": 85.33 + 80.0,
                     "achieved": (85.33 + 80.0) * wl.points / (sec64 / (3 * steps)) / 1e9,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (85.33 + 80.0) * wl.points / (sec64 / (3 * steps)) / 1e9 / HBM_PEAK_GBS,
                     "traffic": None},
        "per_dtype": per,
    }
    if not args.no_physics:
        # The horizon laws of Sec. 4 (Phi_H ~ 1/tau, d_rho Phi_H -> constant) on two
        # coarser grids run to tau = 2000 in FP64.  The inner edge on the horizon
        # closes with end-value ghosts, which leaves a floor in Phi_H of first
        # order in the radial step; the two-grid Richardson value 2 Phi_H(fine) -
        # Phi_H(coarse) removes it.
        series = {}
        for nrp in (args.physics_nr, 2 * args.physics_nr):
            pw = wl.with_(nr=nrp, nth=32)
            cfg = T.make_config(s=pw.s, m=pw.m, a=pw.a, nr=pw.nr, ntheta=pw.nth, x_min=pw.x_min,
                                x_max=pw.x_max, chart="H", S=pw.S)
            probe = T.Solver(cfg, stream=stream)
            dtp = probe.info().dt
            probe.close()
            nsteps = int(np.ceil(args.tau_end / dtp))
            every = max(1, nsteps // 4000)
            log(f"C3-H horizon laws: {pw.nr}x{pw.nth}, {nsteps} steps to tau = {args.tau_end}")
            secp, _, taup, php, dphp, thp = horizon_series(T, torch, pw, "fp64", nsteps, every, stream)
            series[nrp] = (taup, php[:, pw.nth // 4].real, dphp[:, pw.nth // 4].real, secp, nsteps)
        (tc, yc, dc, _, _), (tf, yf, df, secf, nf) = series[args.physics_nr], series[2 * args.physics_nr]
        probe_t = np.linspace(25.0, args.tau_end, 400)
        re = 2 * np.interp(probe_t, tf, yf) - np.interp(probe_t, tc, yc)
        pre = local_index(probe_t, re)
        early = (probe_t[1:-1] >= 50.0) & (probe_t[1:-1] <= 110.0)
        late = tf[1:-1] >= 0.5 * tf[-1]
        out["horizon_laws"] = {
            "grids": [f"{args.physics_nr}x32", f"{2 * args.physics_nr}x32"], "tau_end": float(tf[-1]),
            "phi_h_local_index_richardson_tau_50_110": float(np.mean(pre[early])), "expected_phi_h": -1.0,
            "dphi_h_local_index_fine_late": float(np.mean(local_index(tf, df)[late])), "expected_dphi_h": 0.0,
            "phi_h_floor_coarse": float(yc[-1]), "phi_h_floor_fine": float(yf[-1]),
            "dphi_h_end_fine": float(df[-1]), "seconds_fine": secf, "steps_fine": nf,
        }
    if not args.no_schemes:
        # The paper's scheme comparison (Sec. 4, Fig. 2): Phi and d_rho Phi on the
        # horizon from WENO5, WENO3 and FD6 + KO8 (sigma 0.01) on one grid.
        pw = wl.with_(nr=args.physics_nr, nth=32)
        cfg = T.make_config(s=pw.s, m=pw.m, a=pw.a, nr=pw.nr, ntheta=pw.nth, x_min=pw.x_min, x_max=pw.x_max,
                            chart="H", S=pw.S)
        probe = T.Solver(cfg, stream=stream)
        dtp = probe.info().dt
        probe.close()
        nsteps = int(np.ceil(args.scheme_tau / dtp))
        every = max(1, nsteps // 2000)
        sch = {}
        for scheme in ("weno5", "weno3", "fd6ko8"):
            log(f"C3-H scheme {scheme}: {pw.nr}x{pw.nth}, {nsteps} steps to tau = {args.scheme_tau}")
            secs, _, ts, phs, dphs, _ = horizon_series(T, torch, pw, "fp64", nsteps, every, stream, scheme=scheme)
            sch[scheme] = (ts, phs[:, pw.nth // 4].real, dphs[:, pw.nth // 4].real, secs)
        t5, y5, d5, _ = sch["weno5"]
        res = {}
        for scheme, (ts, ys, ds, secs) in sch.items():
            li = local_index(ts, ys)
            early = (ts[1:-1] >= 50.0) & (ts[1:-1] <= 110.0)
            late = ts[1:-1] >= 0.5 * ts[-1]
            res[scheme] = {
                "ms_per_step": secs / nsteps * 1e3,
                "phi_h_local_index_tau_50_110": float(np.mean(li[early])),
                "dphi_h_local_index_late": float(np.mean(local_index(ts, ds)[late])),
                "dphi_h_end": float(ds[-1]),
                "phi_h_rel_l2_vs_weno5": float(np.linalg.norm(ys - y5) / np.linalg.norm(y5)),
                "dphi_h_rel_l2_vs_weno5": float(np.linalg.norm(ds - d5) / np.linalg.norm(d5)),
            }
        out["schemes"] = {"grid": f"{pw.nr}x{pw.nth}", "tau_end": float(t5[-1]), "steps": nsteps,
                          "ko_sigma": 0.01, "per_scheme": res}
    return out


# ----------------------------------------------------------------------------- C4: batched solves
def bench_batched(args, torch, T, W):
    mix = W.batch_workloads()
    steps = 2000 if args.steps is None else args.steps
    warmup = 20 if args.warmup is None else args.warmup
    weights = args.weights or "fp32"
    stream = torch.cuda.current_stream()
    members = []
    log(f"C4: creating {len(mix)} solves")
    for w in mix:
        sv = T.Solver(solver_config(T, w, weights, warmup + steps), stream=stream)
        sv.set_initial(W.gaussian_pulse(w))
        members.append(sv)
    points = sum(w.points for w in mix)

    # the same solves advanced one after another with teuk_step (context for
    # the batching gain; a few steps each)
    alone_steps = max(1, min(20, steps))
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    for sv in members:
        sv.step(2)
    ev0.record(stream)
    for sv in members:
        sv.step(alone_steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    alone_s = ev0.elapsed_time(ev1) / 1e3
    for sv, w in zip(members, mix):     # restart from the initial data
        sv.set_initial(W.gaussian_pulse(w))

    g = T.Group(len(mix), workgroups=args.workgroups, rows_per_tile=args.rows_per_tile, stream=stream)
    for sv in members:
        g.add(sv)
    tuned = None
    if not args.no_tune and args.rows_per_tile == 0:
        # tile height x cache-block size, timed on clones of the members
        log("C4: group autotuner")
        ti = g.tune(0)
        tuned = {"rows_per_tile": ti.rows_per_tile, "block_mib": ti.block_mib, "candidates": ti.candidates,
                 "us_per_step": ti.us_per_step, "default_rows_per_tile": ti.default_rows_per_tile,
                 "default_block_mib": ti.default_block_mib, "us_per_step_default": ti.us_per_step_default}
    graph = max(args.graph, 0)
    ginfo = g.info()
    log(f"C4: warmup {warmup} steps")
    g.step(warmup)
    g.set_graph(graph)                   # captured here (untimed)
    torch.cuda.synchronize()
    log(f"C4: timing {steps} steps{' (graph chunk ' + str(graph) + ')' if graph else ''}")
    w0 = time.perf_counter()
    ev0.record(stream)
    g.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    gpu_s = ev0.elapsed_time(ev1) / 1e3
    blocked = None
    if not args.no_blocked:
        # the same solves with the temporally blocked step (one launch per
        # step and member, each member a cache block of its own), from the
        # initial data for as many steps; compared with the group above at
        # equal steps on three members
        log(f"C4: the same solves with the blocked step, warmup {warmup} + {steps} steps")
        bmembers = []
        for w in mix:
            sv = T.Solver(solver_config(T, w, weights, warmup + steps, integrator="rk3_blocked"), stream=stream)
            sv.set_initial(W.gaussian_pulse(w))
            bmembers.append(sv)
        bg = T.Group(len(mix), stream=stream)
        for sv in bmembers:
            bg.add(sv)
        bg.step(warmup)
        torch.cuda.synchronize()
        ev0.record(stream)
        bg.step(steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        b_s = ev0.elapsed_time(ev1) / 1e3
        diff = 0.0
        for i in (0, len(mix) // 2, len(mix) - 1):
            ref = members[i].state()
            diff = max(diff, float(np.max(np.abs(bmembers[i].state() - ref))) / float(np.max(np.abs(ref))))
        for sv in bmembers:
            sv.check_finite()
        bg.close()
        for sv in bmembers:
            sv.close()
        blocked = {"steps": steps, "ms_per_step": b_s / steps * 1e3, "value": 3.0 * points * steps / b_s,
                   "speedup_vs_headline": gpu_s / b_s, "state_rel_diff_vs_three_launch": diff,
                   "compared": "members 0, 32, 63 after warmup + steps steps"}
    other = None
    if not args.no_graph_leg:
        # the same number of steps in the other launch mode
        og = 0 if graph else 10
        g.set_graph(og)
        torch.cuda.synchronize()
        log(f"C4: timing {steps} steps, graph chunk {og}")
        ev0.record(stream)
        g.step(steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        other = {"chunk_steps": og, "ms_per_step": ev0.elapsed_time(ev1) / steps,
                 "speedup_vs_headline": gpu_s / (ev0.elapsed_time(ev1) / 1e3)}
    for sv in members:
        sv.check_finite()
    g.close()
    for sv in members:
        sv.close()
    pu = 3.0 * points * steps
    # one stage = one launch per weight precision present (one here)
    out = {
        "metric": METRIC, "value": pu / gpu_s, "unit": "point-updates/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": gpu_s / steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": f"f64 (weights {weights})", "data": "synthetic",
        "config": {"workload": f"C4: {len(mix)} solves, Nr~U{{2048..16384}}, Ntheta~U{{64..256}}, "
                               f"{points} points, {steps} steps",
                   "solves": len(mix), "points": points, "weights": weights, "seeds": "1000..1063",
                   "workgroups_per_stage": int(ginfo.workgroups), "tiles_per_stage": int(ginfo.tiles),
                   "rows_per_tile": tuned["rows_per_tile"] if tuned else (args.rows_per_tile or 8),
                   "block_mib": tuned["block_mib"] if tuned else 256, "graph_chunk_steps": graph},
        "roofline": roofline(points, gpu_s / (3 * steps), None),
        "alone_sequential": {"value": 3.0 * points * alone_steps / alone_s, "steps": alone_steps},
        "batching_speedup": (pu / gpu_s) / (3.0 * points * alone_steps / alone_s),
        "wall_s": wall,
    }
    if tuned:
        out["autotuner"] = tuned
    if blocked:
        out["blocked_members"] = blocked
    if other:
        out["graph"] = other
    if not args.no_cpu_baseline:
        # the oracle on the member nearest the mean size
        mean = points / len(mix)
        w = min(mix, key=lambda x: abs(x.points - mean))
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(w, W.gaussian_pulse(w), args.cpu_seconds)
    return out


# ----------------------------------------------------------------------------- C5: serving
def bench_serving(args, torch, T, W):
    from paper_2010_04760_amd import serving
    nreq = args.requests
    load = args.load
    reqs = serving.poisson_requests(nreq, seed=args.serve_seed)
    work = sum(r.work for r in reqs)
    cap_rate = args.capacity_rate
    if cap_rate <= 0:
        # calibrate the offered load against the batched throughput of the mix
        log("C5: measuring batched throughput for the load calibration")
        cap_rate = serving.measure_capacity(reqs[:16], steps=200)
    rate = load * cap_rate / (work / nreq)          # requests per second
    arrivals = serving.arrival_times(nreq, rate, seed=args.serve_seed)
    budget = int(args.hbm_budget_gb * (1 << 30)) if args.hbm_budget_gb > 0 else None
    log(f"C5: {nreq} requests, offered load {load:.2f} x {cap_rate:.3g} pu/s = {rate:.3g} req/s")
    srv = serving.Server(max_members=nreq, hbm_budget=budget, chunk_steps=args.chunk_steps,
                         workgroups=args.workgroups, rows_per_tile=args.rows_per_tile,
                         graph_chunk=max(args.graph, 0))
    res = srv.run(reqs, arrivals, progress=log)
    lat = np.array([r.latency for r in res.done])
    queued = np.array([r.queued for r in res.done])
    pu = 3.0 * sum(r.req.points * r.req.steps for r in res.done)
    return {
        "metric": METRIC, "value": pu / res.makespan, "unit": "point-updates/s", "n_gpus": 1,
        "steps": int(sum(r.req.steps for r in res.done)), "warmup": 0,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": f"f64 (weights {reqs[0].weights})", "data": "synthetic",
        "config": {"workload": f"C5: {nreq} Poisson requests, steps~U{{5000..50000}}, offered load {load}",
                   "requests": nreq, "offered_load": load, "capacity_rate": cap_rate, "arrival_rate": rate,
                   "hbm_budget_bytes": res.budget, "chunk_steps": args.chunk_steps,
                   "graph_chunk_steps": max(args.graph, 0)},
        "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                      "max": float(lat.max()), "mean": float(lat.mean())},
        "queue_s": {"p50": float(np.percentile(queued, 50)), "p99": float(np.percentile(queued, 99))},
        "max_resident": res.max_resident, "makespan_s": res.makespan,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="C2", choices=["C1", "C2", "C3", "C3H", "C4", "C5"])
    ap.add_argument("--steps", type=int, default=None,
                    help="timed SSP-RK3 steps (C2: 20000, C3: 200000, C4: 2000)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps first (C2: 100, C4: 20)")
    ap.add_argument("--weights", default=None, choices=["fp64", "fp32", "fp16", "bf16"],
                    help="WENO weight precision (C2: fp64, C4/C5: fp32)")
    ap.add_argument("--workgroups", type=int, default=0,
                    help="stage-kernel workgroups (C2, 0: all the GPU holds at once; C4/C5, 0: one per tile)")
    ap.add_argument("--rows-per-tile", type=int, default=0, help="C4/C5: theta rows per group tile (0: 8)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="C1/C2: skip the launch-shape autotuner")
    ap.add_argument("--graph", type=int, default=-1,
                    help="C1/C2/C4/C5: steps per captured HIP graph of the headline run (0: one launch per "
                         "stage; default: 50 for C1, 0 for C2, C4 and C5)")
    ap.add_argument("--no-graph-leg", action="store_true",
                    help="C1/C2/C4: skip the run in the other launch mode (graph vs launch by launch)")
    ap.add_argument("--no-mixed", action="store_true", help="skip the FP32/FP16/BF16-weight runs")
    ap.add_argument("--mixed-steps", type=int, default=0,
                    help="C1/C2: steps of each weight-precision run (0: the workload's full length, which the "
                         "waveform comparison needs; fewer for profiling)")
    ap.add_argument("--no-rk104", action="store_true", help="C2: skip the SSP-RK(10,4) run")
    ap.add_argument("--no-blocked", action="store_true", help="C2, C4: skip the temporally blocked run")
    ap.add_argument("--no-pipelined", action="store_true", help="C1/C2: skip the pipelined-step run")
    ap.add_argument("--no-theta4", action="store_true",
                    help="C1/C2: skip the run with fourth-order theta differences")
    ap.add_argument("--quad-steps", type=int, default=1000,
                    help="C2: steps of the double-double state runs (0: skip them)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="seconds of oracle time for the CPU baseline (40 %% on one thread, 60 %% on all cores)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="before the solve, run a plain device copy of MIB MiB three times (a known-size "
                         "kernel that calibrates rocprofv3 FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--requests", type=int, default=32, help="C5: number of requests")
    ap.add_argument("--load", type=float, default=0.9, help="C5: offered load / batched capacity")
    ap.add_argument("--capacity-rate", type=float, default=0.0,
                    help="C5: batched point-updates/s used for the load (0: measure)")
    ap.add_argument("--chunk-steps", type=int, default=250, help="C5: steps between admission checks")
    ap.add_argument("--hbm-budget-gb", type=float, default=0.0, help="C5: admission budget (0: free HBM)")
    ap.add_argument("--serve-seed", type=int, default=5)
    ap.add_argument("--no-physics", action="store_true", help="C3H: skip the coarse run to tau = 2000")
    ap.add_argument("--physics-nr", type=int, default=4096,
                    help="C3H: radial points of the coarser horizon-law run (the finer has twice as many)")
    ap.add_argument("--tau-end", type=float, default=2000.0, help="C3H: end time of the coarse run")
    ap.add_argument("--no-schemes", action="store_true", help="C3H: skip the WENO5/WENO3/FD6 comparison")
    ap.add_argument("--scheme-tau", type=float, default=500.0, help="C3H: end time of the scheme comparison")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one MI355X only: the library has no multi-GPU path (a single solve would "
              "shard into radial slabs exchanging a three-cell halo per stage, and batched solves would be "
              "dealt out whole per GPU).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2010_04760_amd as T
    import workloads as W

    torch.cuda.set_device(0)
    if args.copy_probe > 0:
        copy_probe(args.copy_probe, torch)
    fn = {"C1": bench_single, "C2": bench_single, "C3": bench_sweep, "C3H": bench_horizon, "C4": bench_batched,
          "C5": bench_serving}[args.workload]
    out = fn(args, torch, T, W)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
