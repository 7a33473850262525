"""Continuous batching of independent Teukolsky solves on one GPU.

Requests (one solve each: background, mode, grid, initial pulse, step count)
arrive over time.  The server keeps the admitted solves resident in HBM as one
group (the C ABI's group extension: one stage launch per SSP-RK stage for each
cache block of members), admits waiting requests first-come first-served while their
footprint (teuk_footprint_bytes) fits the HBM budget, steps the group in
chunks so that arrivals can join between chunks, and on completion copies the
request's waveform out and frees its memory.  Every solve's arithmetic is the
single-solve arithmetic, so a served result equals the same request run alone
bit for bit.

All device work goes through the library; this module only schedules.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np
import torch

from . import _binding as T


@dataclass
class Request:
    rid: int
    wl: object                      # a workloads.Workload (grid, physics, pulse seed, steps)
    u0: Optional[np.ndarray] = None  # initial state; default: the workload's seeded Gaussian pulse
    weights: str = "fp32"

    @property
    def steps(self) -> int:
        return int(self.wl.steps)

    @property
    def points(self) -> int:
        return int(self.wl.nr * self.wl.nth)

    @property
    def work(self) -> float:
        """Point-updates the request needs (3 per point per step)."""
        return 3.0 * self.points * self.steps

    def config(self) -> T.teuk_config:
        w = self.wl
        every = w.every
        return T.make_config(s=w.s, m=w.m, a=w.a, nr=w.nr, ntheta=w.nth, x_min=w.x_min, x_max=w.x_max, M=w.M,
                             dt=0.0, cfl=0.5, weight_prec=self.weights, x_extract=w.x_e, extract_every=every,
                             max_samples=self.steps // every + 1)


@dataclass
class Done:
    req: Request
    arrival: float
    admitted: float
    finished: float
    times: np.ndarray
    waveform: np.ndarray
    state: Optional[np.ndarray] = None

    @property
    def latency(self) -> float:
        """Time to waveform: arrival to the waveform being on the host."""
        return self.finished - self.arrival

    @property
    def queued(self) -> float:
        return self.admitted - self.arrival


@dataclass
class Result:
    done: List[Done] = field(default_factory=list)
    rejected: List[Request] = field(default_factory=list)
    makespan: float = 0.0
    max_resident: int = 0
    budget: int = 0


def _initial(req: Request) -> np.ndarray:
    if req.u0 is not None:
        return req.u0
    import workloads
    return workloads.gaussian_pulse(req.wl)


def poisson_requests(n: int, seed: int = 5, weights: str = "fp32") -> List[Request]:
    import workloads
    return [Request(i, w, weights=weights) for i, w in enumerate(workloads.serving_requests(n, seed))]


def arrival_times(n: int, rate: float, seed: int = 5) -> np.ndarray:
    import workloads
    return workloads.poisson_arrivals(n, rate, seed)


def measure_capacity(reqs: List[Request], steps: int = 200, workgroups: int = 0, rows_per_tile: int = 0) -> float:
    """Batched point-updates/s of these requests advanced together."""
    stream = torch.cuda.current_stream()
    solvers = []
    for r in reqs:
        sv = T.Solver(r.config(), stream=stream)
        sv.set_initial(_initial(r))
        solvers.append(sv)
    with T.Group(len(solvers), workgroups=workgroups, rows_per_tile=rows_per_tile, stream=stream) as g:
        for sv in solvers:
            g.add(sv)
        g.step(5)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        g.step(steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        sec = ev0.elapsed_time(ev1) / 1e3
    for sv in solvers:
        sv.close()
    return 3.0 * sum(r.points for r in reqs) * steps / sec


class Server:
    """Continuous-batching server on the current device and stream.

    max_members: most solves resident at once; hbm_budget: bytes of solver
    footprint allowed at once (default: 90 % of the free HBM when run starts);
    chunk_steps: steps between admission checks (a chunk ends early when a
    resident request finishes); graph_chunk: steps per captured HIP graph of
    the group (0: one launch per stage; it must be a multiple of every
    request's waveform cadence)."""

    def __init__(self, max_members: int = 256, hbm_budget: Optional[int] = None, chunk_steps: int = 250,
                 workgroups: int = 0, rows_per_tile: int = 0, keep_state: bool = False, graph_chunk: int = 0):
        self.graph_chunk = int(graph_chunk)
        self.max_members = max_members
        self.hbm_budget = hbm_budget
        self.chunk_steps = max(1, int(chunk_steps))
        self.workgroups = workgroups
        self.rows_per_tile = rows_per_tile
        self.keep_state = keep_state

    def run(self, requests: List[Request], arrivals, progress: Optional[Callable[[str], None]] = None) -> Result:
        stream = torch.cuda.current_stream()
        budget = self.hbm_budget
        if budget is None:
            free, _ = torch.cuda.mem_get_info()
            budget = int(0.9 * free)
        res = Result(budget=budget)
        order = np.argsort(np.asarray(arrivals, dtype=np.float64), kind="stable")
        pending = deque((float(arrivals[i]), requests[i]) for i in order)
        waiting: deque = deque()
        resident = []          # [solver, request, arrival, admitted, remaining, footprint]
        used = 0
        group = T.Group(self.max_members, workgroups=self.workgroups, rows_per_tile=self.rows_per_tile,
                        stream=stream)
        if self.graph_chunk:
            group.set_graph(self.graph_chunk)
        t0 = time.perf_counter()
        try:
            while pending or waiting or resident:
                now = time.perf_counter() - t0
                while pending and pending[0][0] <= now:
                    waiting.append(pending.popleft())
                # admission: first come first served while the footprint fits
                while waiting and len(resident) < self.max_members:
                    arr, req = waiting[0]
                    cfg = req.config()
                    fp = T.teuk_footprint_bytes(cfg)
                    if fp == 0 or fp > budget:
                        waiting.popleft()
                        res.rejected.append(req)
                        continue
                    if used + fp > budget:
                        break
                    waiting.popleft()
                    sv = T.Solver(cfg, stream=stream)
                    sv.set_initial(_initial(req))
                    group.add(sv)
                    used += fp
                    resident.append([sv, req, arr, time.perf_counter() - t0, req.steps, fp])
                    res.max_resident = max(res.max_resident, len(resident))
                    if progress:
                        progress(f"admit request {req.rid} ({req.wl.nr}x{req.wl.nth}, {req.steps} steps), "
                                 f"{len(resident)} resident")
                if not resident:
                    if pending:
                        time.sleep(max(0.0, pending[0][0] - (time.perf_counter() - t0)))
                    continue
                k = min(self.chunk_steps, min(r[4] for r in resident))
                group.step(k)
                stream.synchronize()
                for r in resident:
                    r[4] -= k
                for r in [r for r in resident if r[4] == 0]:
                    sv, req, arr, adm, _, fp = r
                    times, wave = sv.waveform()
                    state = sv.state() if self.keep_state else None
                    fin = time.perf_counter() - t0
                    group.remove(sv)
                    sv.close()
                    used -= fp
                    resident.remove(r)
                    res.done.append(Done(req, arr, adm, fin, times, wave, state))
                    if progress:
                        progress(f"done request {req.rid}: latency {fin - arr:.3f} s, {len(resident)} resident")
        finally:
            for r in resident:
                r[0].close()
            group.close()
        res.makespan = time.perf_counter() - t0
        return res
