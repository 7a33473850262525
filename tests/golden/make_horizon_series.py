"""Write tests/golden/horizon_series.txt: horizon samples of the FP64 oracle.

The run is the horizon experiment of paper Sec. 4 in the hyperboloidal chart
(s = -2, the (l, m) = (2, 0) profile sin^2(theta), extremal Kerr a = M, S = 20,
a real Gaussian packet of width 0.22 centred at rho = 1.0, pi(0) = 0), on
radial grids of 512, 1024, 2048 and 4096 points that start on the horizon
rho_H = 20/21 and stop at rho = 19.99, with 8 polar rows, SSP-RK(3,3) at
dt = 0.5 x the oracle's stability bound, to tau = 500.  Every sample is Phi
and d_rho Phi on the horizon at theta* = theta_2 (the oracle's 4-point
Lagrange sampler), taken every round(1/dt) steps, i.e. about once per unit of
tau.

Only the oracle and the seeded input generator are used.  It takes about
16 minutes on 8 cores (the 4096-point grid takes most of it):

    python tests/golden/make_horizon_series.py
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import solver as S  # noqa: E402
import workloads as W  # noqa: E402

GRIDS = (512, 1024, 2048, 4096)
NTH = 8
K_STAR = NTH // 4          # theta_2 = 5 pi / 16
TAU_END = 500.0
OUT = os.path.join(HERE, "horizon_series.txt")


def problem(nr: int) -> tuple:
    wl = W.C3H.with_(nr=nr, nth=NTH)
    p = S.Problem(wl.s, wl.m, wl.a, nr, NTH, wl.x_min, wl.x_max, chart="H", S=wl.S)
    return wl, p


def series(nr: int, tau_end: float = TAU_END, max_samples: int | None = None):
    """(dt, every, t[], Phi_H[], dPhi_H[]) of one grid, real parts at theta*."""
    wl, p = problem(nr)
    o = S.TeukOracle(p)
    dt = o.dt_bound(0.5)
    every = max(1, int(round(1.0 / dt)))
    nsamp = int(np.ceil(tau_end / (every * dt)))
    if max_samples is not None:
        nsamp = min(nsamp, max_samples)
    u = W.gaussian_pulse(wl)
    t, ph, dph = [0.0], [], []
    a, b = o.horizon(u)
    ph.append(a[K_STAR].real)
    dph.append(b[K_STAR].real)
    for k in range(1, nsamp + 1):
        u, _ = o.evolve(u, dt, every)
        a, b = o.horizon(u)
        t.append(k * every * dt)
        ph.append(a[K_STAR].real)
        dph.append(b[K_STAR].real)
    return dt, every, np.array(t), np.array(ph), np.array(dph)


def main():
    S.set_threads(os.cpu_count() or 1)
    lines = ["# Horizon samples of the FP64 oracle (chart H, paper Sec. 4 horizon experiment).",
             "# Written by tests/golden/make_horizon_series.py, which calls only oracle/ and workloads/.",
             f"# s=-2 m=0 a=1 S=20, rho in [20/21, 19.99], nth={NTH}, theta*=theta_{K_STAR}, "
             "Gaussian A=1 x_c=1.0 w=0.22 times sin^2(theta), pi(0)=0, SSP-RK(3,3), dt = 0.5 x bound.",
             "# Per grid: a line 'grid <nr> dt <dt> every <steps>' then rows 'tau Phi_H d_rho Phi_H' (real parts)."]
    for nr in GRIDS:
        t0 = time.time()
        dt, every, t, ph, dph = series(nr)
        print(f"grid {nr}: {len(t)} samples, {time.time() - t0:.0f} s", flush=True)
        lines.append(f"grid {nr} dt {dt!r} every {every}")
        lines += [f"{a:.17g} {b:.17g} {c:.17g}" for a, b, c in zip(t, ph, dph)]
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
