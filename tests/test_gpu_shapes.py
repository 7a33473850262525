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
  (tall grid: one tile row per workgroup; wide grid: 4600 tiles);
* the largest theta count the ABI accepts (65536 rows), against the oracle on
  the whole grid;
* the largest radial count (2^24 points), and a plane of 4.4 GB (2^22 x 130
  points, 17.4 GB per state, 52 GB on the device) whose row offsets pass 2^32
  bytes, by the three-launch and the blocked step.  There the oracle runs on
  radial windows of the grid with every theta row (its tables for 2^24 radial
  points alone take minutes to build): the points farther than the steps'
  domain of dependence (three stages of three cells per step) from a window
  edge that is not a grid edge see the same data as in the whole grid."""
import dataclasses

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


def test_largest_theta_count():
    say("case largest theta count 64 x 65536")
    prob = S.Problem(-2, 2, 0.999, 64, 65536, -30.0, 50.0)
    check(prob, 3)
    check(prob, 2, integrator="rk3_blocked")


@dataclasses.dataclass
class _Window(S.Problem):
    """Radial nodes ja .. ja + nr - 1 of a larger grid that starts at x_min
    with spacing full_dx: the very floating-point nodes and spacing of that
    grid (a spacing recomputed from two nodes near x = 200 would be off by
    ulp(200) / (79 dx), 5e-12 of it on the 2^24-point grid)."""
    ja: int = 0
    full_dx: float = 0.0

    @property
    def dx(self):
        return self.full_dx

    def x(self):
        return self.x_min + self.full_dx * np.arange(self.ja, self.ja + self.nr)


def _window(prob, ja, nw):
    """The sub-problem of radial nodes ja .. ja + nw - 1 of prob, every row."""
    w = _Window(prob.s, prob.m, prob.a, nw, prob.nth, prob.x_min, prob.x_max, M=prob.M, eps=prob.eps,
                ja=ja, full_dx=prob.dx)
    assert np.array_equal(w.x(), prob.x()[ja:ja + nw])
    return w


def check_windows(prob, u0, integrator, nsteps=1, nw=80):
    """GPU on the whole grid against the oracle on radial windows (grid start,
    middle, an unaligned spot near the end, grid end) with every theta row."""
    nr = prob.nr
    halo = 9 * nsteps                           # domain of dependence of nsteps SSP-RK(3,3) steps
    wins = [0, nr // 2 - 37, nr - 1 - nw - 61, nr - nw]
    subs = [_window(prob, ja, nw) for ja in wins]
    dt = 0.4 * min(S.TeukOracle(p).dt_bound(1.0) for p in subs)
    with T.Solver(cfg_for(prob, dt, integrator=integrator)) as sv:
        sv.set_initial(u0)
        sv.step(nsteps)
        say("   stepped; extracting")
        got = sv.state()
    for ja, p in zip(wins, subs):
        ref, _ = S.TeukOracle(p).evolve(np.ascontiguousarray(u0[:, :, ja:ja + nw]), dt, nsteps)
        lo = 0 if ja == 0 else halo
        hi = nw if ja + nw == nr else nw - halo
        se, pe = errors(got[:, :, ja + lo:ja + hi], ref[:, :, lo:hi])
        say("   ", integrator, "window", ja, "error", se, max(pe))
        assert se <= TOL and max(pe) <= TOL_PLANE, (integrator, ja, se, pe)


@pytest.mark.parametrize("integrator", ["rk3", "rk3_blocked"])
def test_largest_radial_count(integrator):
    say("case largest radial count 2^24 x 2", integrator)
    prob = S.Problem(0, 1, 0.8, 1 << 24, 2, -400.0, 800.0)
    check_windows(prob, W.separable_state(prob.nr, prob.nth, seed=24), integrator, nsteps=2)


@pytest.mark.parametrize("integrator", ["rk3", "rk3_blocked"])
def test_plane_beyond_4gib(integrator):
    say("case plane beyond 4 GiB 2^22 x 130", integrator)
    prob = S.Problem(-2, 2, 0.9, 1 << 22, 130, -400.0, 800.0)
    u0 = W.separable_state(prob.nr, prob.nth, seed=22)
    say("   state built", u0.nbytes / 2**30, "GiB")
    check_windows(prob, u0, integrator)
    del u0
