"""Why the GPU parity test holds each plane to 5e-12 and the whole state to 1e-12.

Two correct FP64 evaluations of the same scheme that differ only in rounding
(here: the oracle as built, and the same C source built with FMA contraction)
agree on the whole state to ~1e-15, but on the first steps from pi(0) = 0 the
pi_R plane, which is still small, differs by ~1e-12 of its own size: the
centred theta second difference divides one-ulp differences of Phi by
dtheta^2 (256 rows: dtheta^2 = 1.5e-4).  The check runs the C2 background and
theta grid on a shortened radial range at the C2 spacing.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from oracle import solver as S
import workloads as W

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "teuk_oracle.c")


@pytest.fixture(scope="module")
def fma_oracle(tmp_path_factory):
    out = tmp_path_factory.mktemp("fma") / "liboracle_fma.so"
    r = subprocess.run(["gcc", "-O2", "-ffp-contract=fast", "-mfma", "-fopenmp", "-fPIC", "-shared", SRC,
                        "-o", str(out), "-lm"], capture_output=True)
    if r.returncode != 0:
        pytest.skip("gcc cannot build an FMA variant here")
    L = ctypes.CDLL(str(out))
    L.oracle_teuk_evolve.argtypes = [ctypes.POINTER(S._OracleTeuk), S._dp, ctypes.c_double, ctypes.c_long,
                                     ctypes.c_long, ctypes.c_long, S._dp, ctypes.c_long]
    return L


def test_rounding_spread_between_two_correct_builds(fma_oracle):
    wl = W.C2
    dx = (wl.x_max - wl.x_min) / (wl.nr - 1)
    nr = 1093
    x_min = -20.0
    prob = S.Problem(wl.s, wl.m, wl.a, nr, wl.nth, x_min, x_min + dx * (nr - 1))
    o = S.TeukOracle(prob)
    dt = o.dt_bound(0.5)
    u0 = W.gaussian_pulse(wl.with_(nr=nr, x_min=prob.x_min, x_max=prob.x_max))
    ua, _ = o.evolve(u0, dt, 3)
    ub = np.ascontiguousarray(u0.copy())
    fma_oracle.oracle_teuk_evolve(ctypes.byref(o._s), S.ptr(ub), dt, 3, 0, 0, None, 0)
    state = np.max(np.abs(ua - ub)) / np.max(np.abs(ua))
    per_plane = [np.max(np.abs(ua[p] - ub[p])) / np.max(np.abs(ua[p])) for p in (0, 2, 3)]
    assert state < 1e-14
    assert per_plane[1] > 1e-13          # the amplification is real ...
    assert max(per_plane) < 5e-12        # ... and bounded by the per-plane bar
