"""GPU: extreme grid shapes and launch shapes of the fused stage kernel against
the FP64 oracle, through the C ABI (same bar as the parity tests: whole-state
max-norm relative error <= 1e-12, each plane <= 5e-12).

* a tall grid (2048 theta rows on two radial strips): the default launch cuts
  every strip into about 2000 theta segments of one or two rows, so a wave's
  march is shorter than its three-row load pipeline;
* one row per segment, asked for explicitly (workgroups = strips x rows);
* a wide grid (2^19 radial points, 4 theta rows): 8323 strips, more
  workgroups than the GPU holds at once, one segment per strip;
* the same shapes stepped by SSP-RK(10,4) and by the temporally blocked step
  (tall grid: one tile row per workgroup; wide grid: 4600 tiles)."""
import numpy as np
import pytest

import paper_2010_04760_amd as T
import workloads as W
from oracle import solver as S

pytestmark = pytest.mark.gpu

TOL = 1e-12
TOL_PLANE = 5e-12


def say(*a):
    print(*a, flush=True)


def errors(g, o):
    big = max(float(np.max(np.abs(o))), 1e-300)
    se = float(np.max(np.abs(g - o))) / big
    pe = []
    for p in range(o.shape[0]):
        ref = float(np.max(np.abs(o[p])))
        pe.append(float(np.max(np.abs(g[p] - o[p]))) / (ref if ref > 0 else big))
    return se, pe


def cfg_for(prob, dt, **kw):
    return T.make_config(s=prob.s, m=prob.m, a=prob.a, nr=prob.nr, ntheta=prob.nth, x_min=prob.x_min,
                         x_max=prob.x_max, M=prob.M, dt=dt, weno_eps=prob.eps, **kw)


def check(prob, nsteps, integrator="rk3", cfl=0.4, **kw):
    o = S.TeukOracle(prob)
    dt = cfl * o.dt_bound(1.0)
    u0 = W.random_state(prob.nr, prob.nth, seed=prob.nr % 1000 + prob.nth, smooth=True)
    oint = "rk3" if integrator == "rk3_blocked" else integrator
    ref, _ = o.evolve(u0, dt, nsteps, integrator=oint)
    with T.Solver(cfg_for(prob, dt, integrator=integrator, **kw)) as sv:
        sv.set_initial(u0)
        sv.step(nsteps)
        got = sv.state()
        wg = sv.info().workgroups
    se, pe = errors(got, ref)
    say("   ", integrator, "workgroups", wg, "error", se, max(pe))
    assert se <= TOL and max(pe) <= TOL_PLANE, (integrator, se, pe)
    return wg


def test_tall_grid_short_segments():
    say("case tall grid 70 x 2048")
    prob = S.Problem(-2, 2, 0.999, 70, 2048, -30.0, 50.0)
    wg = check(prob, 3)
    assert wg >= 2 * 1000                      # segments of one or two rows
    check(prob, 2, integrator="rk104", cfl=1.5)
    check(prob, 3, integrator="rk3_blocked", workgroups=2048)   # one tile row per workgroup


def test_one_row_per_segment():
    say("case one row per segment 130 x 64")
    prob = S.Problem(0, 1, 0.7, 130, 64, -30.0, 50.0)
    wg = check(prob, 3, workgroups=3 * 64)
    assert wg == 3 * 64


def test_wide_grid_more_strips_than_slots():
    say("case wide grid 2^19 x 4")
    prob = S.Problem(-2, 1, 0.9, 1 << 19, 4, -30.0, 50.0)
    wg = check(prob, 3)
    assert wg == -(-(1 << 19) // 63)            # one segment per strip
    check(prob, 3, integrator="rk3_blocked")
