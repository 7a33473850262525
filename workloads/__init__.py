"""Seeded synthetic inputs for the Teukolsky workloads.

This module only draws inputs: grid sizes, background and field parameters and
the initial data.  It holds none of the solver's arithmetic, and both the
product path and the oracle take their inputs from it.

Initial data (paper Sec. 4 uses a Gaussian radial wave packet times a
spherical-harmonic angular profile, starting from real data):

    Phi(0, x, theta) = A exp(-((x - x_c)/w)^2) Theta_{s,m}(theta),   Im Phi = 0,
    pi(0) = 0,

with A, x_c, w drawn from numpy's PCG64 generator seeded per workload, and
Theta_{s,m} the lowest-l spin-weighted harmonic of spin s and azimuthal number
m, up to normalisation (or the l = 2, m = 0 Legendre profile where the paper's
(l, m) = (2, 0) choice is asked for).  Grids: x_j = x_min + j (x_max - x_min)/(nr-1),
theta_k = (k + 1/2) pi / nth.
"""
from __future__ import annotations

from dataclasses import dataclass, replace
from typing import List

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    s: int
    m: int
    a: float
    nr: int
    nth: int
    x_min: float
    x_max: float
    steps: int
    seed: int
    angular: str = "lowest"          # "lowest" or "P2"
    x_e: float = 30.0                # waveform extraction radius (x = r_*)
    every: int = 10                  # steps between waveform samples
    M: float = 1.0
    amp_range: tuple = (0.5, 2.0)
    xc_range: tuple = (5.0, 15.0)
    w_range: tuple = (1.0, 4.0)
    chart: str = "T"                 # "T": x = r_*; "H": x = rho (hyperboloidal, parameter S)
    S: float = 20.0

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)

    @property
    def points(self) -> int:
        return self.nr * self.nth


# The five workloads (sizes and parameters as in the benchmark definition).
C1 = Workload("C1: s=0 m=0 a=0.5 512x32, 1000 steps", s=0, m=0, a=0.5, nr=512, nth=32,
              x_min=-64.0, x_max=64.0, steps=1000, seed=1, angular="P2", x_e=30.0, every=10)
C2 = Workload("C2: s=-2 m=2 a=0.999 8192x256, 20000 steps", s=-2, m=2, a=0.999, nr=8192, nth=256,
              x_min=-200.0, x_max=400.0, steps=20000, seed=2, angular="lowest", x_e=30.0, every=10)
C3 = Workload("C3: s=0 m=0 a=1 16384x128, 200000 steps", s=0, m=0, a=1.0, nr=16384, nth=128,
              x_min=-400.0, x_max=800.0, steps=200000, seed=3, angular="P2", x_e=30.0, every=100)


# The horizon experiment of Sec. 4 in the hyperboloidal chart: s = -2, the
# (l, m) = (2, 0) profile, extremal Kerr, a Gaussian packet centred at rho = 1.0
# of width 0.22, S = 20, 16384 (rho) x 64 (theta).  The grid starts on the
# horizon rho_H = 20/21 (r = M), where the pi-row speed vanishes, so that its
# inner edge takes no incoming data, and stops short of null infinity
# (rho = S); the waveform is read at rho = 19.5 (r = 780).
C3H = Workload("C3-H: s=-2 m=0 a=1 hyperboloidal 16384x64", s=-2, m=0, a=1.0, nr=16384, nth=64,
               x_min=20.0 / 21.0, x_max=19.99, steps=200000, seed=3, angular="P2", x_e=19.5, every=100,
               amp_range=(1.0, 1.0), xc_range=(1.0, 1.0), w_range=(0.22, 0.22), chart="H", S=20.0)


def grid_x(wl: Workload) -> np.ndarray:
    return wl.x_min + (wl.x_max - wl.x_min) / (wl.nr - 1) * np.arange(wl.nr)


def grid_theta(nth: int) -> np.ndarray:
    return (np.arange(nth) + 0.5) * (np.pi / nth)


def angular_profile(s: int, m: int, theta: np.ndarray, kind: str = "lowest") -> np.ndarray:
    """Unnormalised lowest-l spin-weighted harmonic _sY_lm(theta), l = max(|s|,|m|).

    kind="P2" gives the l = 2, m = 0 profile (3 cos^2 - 1)/2 for s = 0 and
    sin^2 for s = -2 (both are l = 2).
    """
    c, sn = np.cos(theta), np.sin(theta)
    if kind == "P2":
        if m != 0:
            raise ValueError("P2 profile is m = 0")
        if s == 0:
            return 0.5 * (3.0 * c * c - 1.0)
        if s == -2:
            return sn * sn
        raise ValueError("P2 profile defined for s in {0, -2}")
    if s == 0:
        return np.ones_like(theta) if m == 0 else sn ** abs(m)
    if s == -2:
        table = {0: sn * sn, 1: sn * (1 + c), 2: (1 + c) ** 2, 3: sn * (1 + c) ** 2,
                 4: sn * sn * (1 + c) ** 2}
        if m not in table:
            raise ValueError("s=-2 profiles defined for m in 0..4")
        return table[m]
    raise ValueError("profiles defined for s in {0, -2}")


def pulse_params(wl: Workload, seed: int | None = None) -> dict:
    rng = np.random.default_rng(wl.seed if seed is None else seed)
    A = rng.uniform(*wl.amp_range)
    xc = rng.uniform(*wl.xc_range)
    w = rng.uniform(*wl.w_range)
    return {"A": float(A), "x_c": float(xc), "w": float(w)}


def gaussian_pulse(wl: Workload, seed: int | None = None) -> np.ndarray:
    """Initial state u0 of shape [4][nth][nr] (Phi_R, Phi_I, pi_R, pi_I), float64."""
    p = pulse_params(wl, seed)
    x = grid_x(wl)
    th = grid_theta(wl.nth)
    radial = p["A"] * np.exp(-(((x - p["x_c"]) / p["w"]) ** 2))
    u = np.zeros((4, wl.nth, wl.nr))
    u[0] = angular_profile(wl.s, wl.m, th, wl.angular)[:, None] * radial[None, :]
    return u


def random_state(nr: int, nth: int, seed: int, smooth: bool = False) -> np.ndarray:
    """A seeded random state [4][nth][nr] for operator-level tests (brute force)."""
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((4, nth, nr))
    if smooth:
        x = np.linspace(0, 1, nr)
        u = u * 0.1 + np.sin(2 * np.pi * x)[None, None, :]
    return u


def separable_state(nr: int, nth: int, seed: int) -> np.ndarray:
    """A seeded state [4][nth][nr] whose plane p is the outer product of a
    random theta profile and a random radial profile (standard normal, plus
    one on both): rough in both directions, yet drawn from only 4 (nr + nth)
    numbers, so that grids of billions of points are cheap to build."""
    rng = np.random.default_rng(seed)
    a = 1.0 + rng.standard_normal((4, nth))
    b = 1.0 + rng.standard_normal((4, nr))
    u = np.empty((4, nth, nr))
    for p in range(4):
        np.multiply(a[p][:, None], b[p][None, :], out=u[p])
    return u


def batch_workloads(n: int = 64, seed0: int = 1000, steps: int = 2000) -> List[Workload]:
    """The batched mix: uneven grids and (s, m, a) per solve, seeded per solve.

    N_r ~ U{2048..16384} rounded down to a multiple of 64, N_theta ~ U{64..256},
    s in {0, -2}, m in 0..4, a ~ U[0.5, 1.0], x in [-200, 400].
    """
    out = []
    for i in range(n):
        rng = np.random.default_rng(seed0 + i)
        nr = int(rng.integers(2048, 16385)) // 64 * 64
        nth = int(rng.integers(64, 257))
        s = int(rng.choice([0, -2]))
        m = int(rng.integers(0, 5))
        a = float(rng.uniform(0.5, 1.0))
        out.append(Workload(f"batch[{i}]", s=s, m=m, a=a, nr=nr, nth=nth, x_min=-200.0, x_max=400.0,
                            steps=steps, seed=seed0 + i, angular="lowest", x_e=30.0, every=10))
    return out


def serving_requests(n: int = 32, seed: int = 5, seed0: int = 2000) -> List[Workload]:
    """Requests of the served workload: solves drawn as in `batch_workloads`
    (per-request seeds seed0 + i), with a step count ~ U{5000..50000} per
    request drawn from `seed`."""
    rng = np.random.default_rng(seed)
    steps = rng.integers(5000, 50001, size=n)
    base = batch_workloads(n, seed0=seed0)
    return [replace(w, name=f"request[{i}]", steps=int(steps[i])) for i, w in enumerate(base)]


def poisson_arrivals(n: int, rate: float, seed: int = 5) -> np.ndarray:
    """Arrival times (seconds from the start) of a Poisson process of the given
    rate: cumulative sums of exponential gaps drawn from `seed`."""
    rng = np.random.default_rng(seed + 7919)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))
