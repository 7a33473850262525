"""GPU: the SSP-RK(10,4) integrator (Sec. 3.2) against the FP64 oracle.

The library runs the paper's ten stages in three state buffers (the fifth
stage writes two outputs, the last combines in place); the oracle runs the
stages as printed.  Same bar as the SSP-RK(3,3) parity tests: whole-state
max-norm relative error <= 1e-12 and each plane <= 5e-12 of its own scale.
Cases: ragged tortoise-chart grids with FP64 and FP32 weights, the
hyperboloidal chart, the waveform samples, the default step (cfl x 6 x the
stability bound), the C2 grid at full size, and the configurations that are
not offered (double-double state, group members)."""
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
                         x_max=prob.x_max, M=prob.M, dt=dt, weno_eps=prob.eps, integrator="rk104",
                         chart=prob.chart, S=prob.S, **kw)


CASES = [(7, 2, 0, 0, 0.5), (63, 5, -2, 2, 0.999), (64, 4, 0, 1, 1.0), (127, 9, -2, 3, 0.9),
         (200, 17, -2, 1, 0.7)]


@pytest.mark.parametrize("nr,nth,s,m,a", CASES)
def test_random_state_steps(nr, nth, s, m, a):
    say("case rk104 random", nr, nth, s, m, a)
    prob = S.Problem(s, m, a, nr, nth, -30.0, 50.0)
    o = S.TeukOracle(prob)
    dt = 1.5 * o.dt_bound(1.0)
    u0 = W.random_state(nr, nth, seed=nr * 7 + nth, smooth=True)
    for n in (1, 3):
        ref, _ = o.evolve(u0, dt, n, integrator="rk104")
        with T.Solver(cfg_for(prob, dt)) as sv:
            sv.set_initial(u0)
            sv.step(n)
            got = sv.state()
        se, pe = errors(got, ref)
        say("  steps", n, "error", se, max(pe))
        assert se <= TOL and max(pe) <= TOL_PLANE, (n, se, pe)


def test_fp32_weights_within_the_reduced_precision_bar():
    say("case rk104 fp32 weights")
    wl = W.C1
    prob = S.Problem(wl.s, wl.m, wl.a, wl.nr, wl.nth, wl.x_min, wl.x_max)
    o = S.TeukOracle(prob)
    dt = 3.0 * o.dt_bound(1.0)
    u0 = W.gaussian_pulse(wl)
    n = 60
    ref, wref = o.evolve(u0, dt, n, x_e=wl.x_e, every=2, integrator="rk104")
    with T.Solver(cfg_for(prob, dt, weight_prec="fp32", x_extract=wl.x_e, extract_every=2,
                          max_samples=n // 2 + 1)) as sv:
        sv.set_initial(u0)
        sv.step(n)
        _, w = sv.waveform()
    err = float(np.linalg.norm(w - wref) / np.linalg.norm(wref))
    say("  waveform rel-L2", err)
    assert err <= 1e-6


def test_hyperboloidal_chart():
    say("case rk104 chart H")
    prob = S.Problem(-2, 0, 1.0, 150, 8, 20.0 / 21.0, 19.5, chart="H", S=20.0)
    o = S.TeukOracle(prob)
    dt = 1.5 * o.dt_bound(1.0)
    u0 = W.random_state(prob.nr, prob.nth, seed=3, smooth=True)
    ref, _ = o.evolve(u0, dt, 3, integrator="rk104")
    with T.Solver(cfg_for(prob, dt)) as sv:
        sv.set_initial(u0)
        sv.step(3)
        got = sv.state()
    se, pe = errors(got, ref)
    say("  error", se, max(pe))
    assert se <= TOL and max(pe) <= TOL_PLANE


def test_waveform_and_default_step():
    say("case rk104 waveform + default dt")
    prob = S.Problem(-2, 2, 0.999, 190, 12, -30.0, 50.0)
    o = S.TeukOracle(prob)
    cfg = cfg_for(prob, 0.0, x_extract=10.0, extract_every=2, max_samples=8)
    with T.Solver(cfg) as sv:
        inf = sv.info()
        assert inf.dt == pytest.approx(0.5 * 6.0 * inf.dt_bound, rel=1e-15)
        assert inf.dt_bound == pytest.approx(o.dt_bound(1.0), rel=1e-12)
        u0 = W.random_state(prob.nr, prob.nth, seed=6, smooth=True)
        sv.set_initial(u0)
        sv.step(6)
        t, w = sv.waveform()
        got = sv.state()
        dt = inf.dt
    ref, wref = o.evolve(u0, dt, 6, x_e=10.0, every=2, integrator="rk104")
    se, pe = errors(got, ref)
    assert se <= TOL and max(pe) <= TOL_PLANE
    assert w.shape == wref.shape
    assert float(np.max(np.abs(w - wref))) <= TOL * float(np.max(np.abs(wref)))
    np.testing.assert_allclose(t, dt * np.arange(0, 7, 2), rtol=1e-15)


def test_c2_full_size():
    wl = W.C2
    say("case rk104 C2 full size")
    prob = S.Problem(wl.s, wl.m, wl.a, wl.nr, wl.nth, wl.x_min, wl.x_max)
    o = S.TeukOracle(prob)
    u0 = W.gaussian_pulse(wl)
    with T.Solver(cfg_for(prob, 0.0)) as sv:
        dt = sv.info().dt
        sv.set_initial(u0)
        sv.step(2)
        got = sv.state()
    ref, _ = o.evolve(u0, dt, 2, integrator="rk104")
    se, pe = errors(got, ref)
    say("  error", se, max(pe))
    assert se <= TOL and max(pe) <= TOL_PLANE


def test_not_offered():
    say("case rk104 unsupported")
    prob = S.Problem(0, 0, 0.5, 64, 4, -10.0, 10.0)
    with pytest.raises(T.TeukError) as ei:
        T.teuk_create(cfg_for(prob, 0.0, state="dd", weight_prec="dd"))
    assert ei.value.status == T.TEUK_ERR_UNSUPPORTED
    with T.Solver(cfg_for(prob, 0.0)) as sv, T.Group(2) as g:
        sv.set_initial(W.random_state(64, 4, seed=1))
        with pytest.raises(T.TeukError) as ei:
            g.add(sv)
        assert ei.value.status == T.TEUK_ERR_UNSUPPORTED
