"""GPU: temporal blocking (one launch per SSP-RK(3,3) step, the stages of a
tile fused in LDS) against the three-launch step and the FP64 oracle.

The blocked step runs the same arithmetic per point and stage as the
three-launch step; the compiler may fuse multiply-adds differently in the two
kernels, so they agree to rounding (measured: a few ulp after three steps),
held here to 1e-13 of the state's scale per plane and to the oracle bar
(whole-state <= 1e-12, planes <= 5e-12).  Cases: ragged
radial sizes around the 114-point tile (smaller than one tile, one tile, a
tile plus one point, the 127 points one workgroup spans, two tiles and one
more point, several tiles), theta sizes from 2 rows, tile counts from one
tile per strip to one row per tile, both pole parities, a = M, the waveform
samples, the C2 grid at full size, and the configurations not offered.

FP32 weights: the blocked step and the three-launch step both form the
weights in FP32 from the same FP64 differences, so a difference of one FP64
ulp in a difference (from a different fused multiply-add) can move a weight
by one FP32 ulp in one kernel and not the other.  Each is held to the
reduced-precision bar against the FP64 oracle (1e-6 of the state's scale
after 200 steps of a Gaussian pulse), and the two to 1e-9 of each other after
three steps of rough data (measured far below: the weights multiply the
candidate differences, which are small against the flux)."""
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


def cfg_for(prob, dt, integrator, **kw):
    return T.make_config(s=prob.s, m=prob.m, a=prob.a, nr=prob.nr, ntheta=prob.nth, x_min=prob.x_min,
                         x_max=prob.x_max, dt=dt, weno_eps=prob.eps, integrator=integrator, **kw)


def run(prob, dt, u0, n, integrator, **kw):
    with T.Solver(cfg_for(prob, dt, integrator, **kw)) as sv:
        sv.set_initial(u0)
        sv.step(n)
        st = sv.state()
        inf = sv.info()
        w = sv.waveform() if kw.get("extract_every") else None
    return st, inf, w


def oracle_errors(g, o):
    big = max(float(np.max(np.abs(o))), 1e-300)
    se = float(np.max(np.abs(g - o))) / big
    pe = [float(np.max(np.abs(g[p] - o[p]))) / max(float(np.max(np.abs(o[p]))), big * 1e-300) for p in range(4)]
    return se, pe


TILE = 114     # output points per tile

GRIDS = [(7, 2, 0, 0, 0.5), (63, 3, -2, 2, 0.999), (114, 5, 0, 1, 1.0), (115, 4, -2, 1, 0.7), (127, 9, 0, 2, 0.9),
         (229, 6, -2, 3, 0.999), (300, 17, -2, 0, 0.3), (200, 33, 1, -1, 0.6), (513, 8, 0, 0, 0.5)]


@pytest.mark.parametrize("grid", GRIDS)
def test_equals_three_launch_step_and_oracle(grid):
    nr, nth, s, m, a = grid
    say("case blocked", grid)
    prob = S.Problem(s, m, a, nr, nth, -30.0, 50.0)
    o = S.TeukOracle(prob)
    dt = 0.4 * o.dt_bound(1.0)
    u0 = W.random_state(nr, nth, seed=nr * 3 + nth, smooth=True)
    ref3, _, _ = run(prob, dt, u0, 3, "rk3")
    oref, _ = o.evolve(u0, dt, 3)
    strips = -(-nr // TILE)
    for wg in (0, strips, 2 * strips, strips * nth):
        got, inf, _ = run(prob, dt, u0, 3, "rk3_blocked", workgroups=wg)
        d = float(np.max(np.abs(got - ref3)))
        say("  workgroups", wg, "->", inf.workgroups, "max |blocked - three-launch|", d)
        se, pe = oracle_errors(got, ref3)
        assert se <= 1e-13 and max(pe) <= TOL_PLANE, (wg, d, se, pe)
    se, pe = oracle_errors(got, oref)
    assert se <= TOL and max(pe) <= TOL_PLANE, (se, pe)


def test_waveform_and_counters():
    say("case blocked waveform")
    prob = S.Problem(-2, 2, 0.999, 190, 12, -30.0, 50.0)
    o = S.TeukOracle(prob)
    dt = 0.4 * o.dt_bound(1.0)
    u0 = W.random_state(prob.nr, prob.nth, seed=5, smooth=True)
    kw = dict(x_extract=10.0, extract_every=2, max_samples=8)
    g3, i3, (t3, w3) = run(prob, dt, u0, 7, "rk3", **kw)
    gb, ib, (tb, wb) = run(prob, dt, u0, 7, "rk3_blocked", **kw)
    se, pe = oracle_errors(gb, g3)
    assert se <= 1e-13 and max(pe) <= TOL_PLANE, (se, pe)
    assert float(np.max(np.abs(wb - w3))) <= 1e-13 * float(np.max(np.abs(w3)))
    assert np.array_equal(tb, t3)
    assert ib.steps == i3.steps == 7 and ib.samples == i3.samples


def test_c2_full_size():
    wl = W.C2
    say("case blocked C2 full size")
    prob = S.Problem(wl.s, wl.m, wl.a, wl.nr, wl.nth, wl.x_min, wl.x_max)
    u0 = W.gaussian_pulse(wl)
    g3, i3, _ = run(prob, 0.0, u0, 3, "rk3")
    gb, ib, _ = run(prob, 0.0, u0, 3, "rk3_blocked")
    say("  tiles", ib.workgroups, "max diff", float(np.max(np.abs(gb - g3))))
    assert ib.dt == i3.dt
    se, pe = oracle_errors(gb, g3)
    assert se <= 1e-13 and max(pe) <= TOL_PLANE, (se, pe)
    oref, _ = S.TeukOracle(prob).evolve(u0, i3.dt, 3)
    se, pe = oracle_errors(gb, oref)
    assert se <= TOL and max(pe) <= TOL_PLANE, (se, pe)


@pytest.mark.parametrize("grid", [GRIDS[1], GRIDS[3], GRIDS[5], GRIDS[8]])
def test_fp32_weights_against_three_launch(grid):
    nr, nth, s, m, a = grid
    say("case blocked fp32", grid)
    prob = S.Problem(s, m, a, nr, nth, -30.0, 50.0)
    dt = 0.4 * S.TeukOracle(prob).dt_bound(1.0)
    u0 = W.random_state(nr, nth, seed=nr + 7 * nth, smooth=True)
    ref3, _, _ = run(prob, dt, u0, 3, "rk3", weight_prec="fp32")
    got, inf, _ = run(prob, dt, u0, 3, "rk3_blocked", weight_prec="fp32")
    rel = float(np.max(np.abs(got - ref3))) / float(np.max(np.abs(ref3)))
    say("  tiles", inf.workgroups, "max |blocked - three-launch| / max", rel)
    assert rel <= 1e-9, rel


def test_fp32_weights_c2_full_size():
    wl = W.C2
    say("case blocked fp32 C2 full size")
    prob = S.Problem(wl.s, wl.m, wl.a, wl.nr, wl.nth, wl.x_min, wl.x_max)
    u0 = W.gaussian_pulse(wl)
    g3, i3, _ = run(prob, 0.0, u0, 3, "rk3", weight_prec="fp32")
    gb, ib, _ = run(prob, 0.0, u0, 3, "rk3_blocked", weight_prec="fp32")
    rel = float(np.max(np.abs(gb - g3))) / float(np.max(np.abs(g3)))
    say("  tiles", ib.workgroups, "max |blocked - three-launch| / max", rel)
    assert ib.dt == i3.dt and rel <= 1e-9, rel
    oref, _ = S.TeukOracle(prob).evolve(u0, i3.dt, 3)
    assert float(np.max(np.abs(gb - oref))) / float(np.max(np.abs(oref))) <= 1e-6


def test_fp32_weights_reduced_precision_bar():
    say("case blocked fp32 against the oracle")
    wl = W.C1.with_(nr=400, nth=24)
    prob = S.Problem(wl.s, wl.m, wl.a, wl.nr, wl.nth, wl.x_min, wl.x_max)
    o = S.TeukOracle(prob)
    dt = o.dt_bound(0.5)
    u0 = W.gaussian_pulse(wl)
    ref, _ = o.evolve(u0, dt, 200)
    got, _, _ = run(prob, dt, u0, 200, "rk3_blocked", weight_prec="fp32")
    err = float(np.max(np.abs(got - ref))) / float(np.max(np.abs(ref)))
    say("  error", err)
    assert err <= 1e-6, err


def test_not_offered():
    say("case blocked unsupported")
    prob = S.Problem(0, 0, 0.5, 64, 4, -10.0, 10.0)
    for kw in (dict(weight_prec="fp16"), dict(weight_prec="bf16"), dict(scheme="weno3"),
               dict(state="dd", weight_prec="dd")):
        with pytest.raises(T.TeukError) as ei:
            T.teuk_create(cfg_for(prob, 0.0, "rk3_blocked", **kw))
        assert ei.value.status == T.TEUK_ERR_UNSUPPORTED
    ch = T.make_config(s=-2, m=0, a=1.0, nr=101, ntheta=8, x_min=20 / 21, x_max=19.0, chart="H",
                       integrator="rk3_blocked")
    with pytest.raises(T.TeukError) as ei:
        T.teuk_create(ch)
    assert ei.value.status == T.TEUK_ERR_UNSUPPORTED
