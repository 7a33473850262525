"""Full-solver pins of the oracle (WENO5 + SSP-RK3 on the chart-T system) against
black-hole physics with known answers:

* Schwarzschild quasinormal ringing: the fitted fundamental frequency of the
  l = 2 mode for s = 0 and s = -2 (values in tests/golden/schwarzschild_qnm.txt).
* Price's late-time tail at fixed radius: local power index p = t Phi_t / Phi
  (the paper's local index, Sec. 4) tends to -(2l+3) for data with pi(0) = 0.
"""
import os

import numpy as np
import pytest
from scipy.optimize import least_squares

from oracle import solver as S
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "schwarzschild_qnm.txt")


def golden_qnm(s, l):
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        ss, ll, wr, wi = line.split()
        if int(ss) == s and int(ll) == l:
            return float(wr), float(wi)
    raise KeyError((s, l))


def _ringdown(s, m, kind, nth, dx=0.25, T=200.0, x_e=30.0):
    x_min, x_max = -120.0, 200.0
    nr = int(round((x_max - x_min) / dx)) + 1
    prob = S.Problem(s, m, 0.0, nr, nth, x_min, x_max)
    o = S.TeukOracle(prob)
    Y = W.angular_profile(s, m, prob.theta(), kind)
    u = np.zeros((4, nth, nr))
    u[0] = Y[:, None] * np.exp(-(((prob.x() - 10.0) / 2.0) ** 2))[None, :]
    dt = o.dt_bound()
    n = int(np.ceil(T / dt))
    dt = T / n
    every = max(1, int(round(0.5 / dt)))
    _, wave = o.evolve(u, dt, n, x_e, every)
    t = np.arange(wave.shape[0]) * every * dt
    return t, wave[:, int(np.argmax(np.abs(Y))), 0]


def _fit(t, y, t0, t1):
    sel = (t >= t0) & (t <= t1)
    tt, yy = t[sel], y[sel]
    res = lambda p: p[0] * np.exp(p[3] * (tt - t0)) * np.cos(p[2] * (tt - t0) + p[1]) - yy
    best = min((least_squares(res, [yy[0], 0.0, w0, -0.09]) for w0 in (0.3, 0.4, 0.5)),
               key=lambda r: r.cost)
    return abs(best.x[2]), best.x[3]


@pytest.mark.slow
def test_qnm_scalar_l2():
    # theta error is second order: Richardson-extrapolate nth = 16, 24.
    want = golden_qnm(0, 2)
    om = {}
    for nth in (16, 24):
        t, y = _ringdown(0, 0, "P2", nth)
        om[nth] = np.array(_fit(t, y, 70.0, 130.0))
    ext = om[24] + (om[24] - om[16]) * 16**2 / (24**2 - 16**2)
    assert ext[0] == pytest.approx(want[0], rel=2e-3), (om, ext)
    assert ext[1] == pytest.approx(want[1], rel=1.2e-2), (om, ext)
    # and the unextrapolated value is already within 0.5 % / 1.5 %
    assert om[24][0] == pytest.approx(want[0], rel=5e-3)
    assert om[24][1] == pytest.approx(want[1], rel=1.5e-2)


@pytest.mark.slow
def test_qnm_gravitational_l2():
    want = golden_qnm(-2, 2)
    t, y = _ringdown(-2, 2, "lowest", 16)
    wr, wi = _fit(t, y, 80.0, 140.0)
    assert wr == pytest.approx(want[0], rel=4e-3)
    assert wi == pytest.approx(want[1], rel=6e-3)


def _tail(dx=1.0):
    x_min, x_max = -700.0, 800.0
    nr = int(round((x_max - x_min) / dx)) + 1
    prob = S.Problem(0, 0, 0.0, nr, 2, x_min, x_max)
    o = S.TeukOracle(prob)
    x = prob.x()
    g = np.exp(-(((x - 10.0) / 2.0) ** 2))
    u = np.zeros((4, 2, nr))
    u[0] = g[None, :]
    T = 1300.0
    dt = o.dt_bound()
    n = int(np.ceil(T / dt))
    dt = T / n
    every = max(1, int(round(1.0 / dt)))
    _, wave = o.evolve(u, dt, n, 30.0, every)
    t = np.arange(wave.shape[0]) * every * dt
    phi = wave[:, 0, 0]
    p = t * np.gradient(phi, t) / phi
    return t, p


@pytest.mark.slow
def test_price_tail_generic_data():
    t, p = _tail()
    at = lambda tq: p[np.argmin(np.abs(t - tq))]
    assert -3.04 < at(1200.0) < -2.95
    assert abs(at(1200.0) + 3) < abs(at(600.0) + 3)       # approaching -3
