"""GPU: the comparison schemes of Sec. 3.1 (WENO3; FD6 with KO8 dissipation)
against the FP64 oracle, through the C ABI.

Same bar as the WENO5 parity tests: whole-state max-norm relative error
<= 1e-12 and each plane <= 5e-12 of its own scale.  Cases: ragged
tortoise-chart grids (strip boundaries, the smallest grid, odd pole parity,
a = M) with both integrators, the hyperboloidal chart, F(u) alone, the C2
grid at full size, and the configurations that are not offered."""
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


def cfg_for(prob, dt, integrator="rk3", **kw):
    return T.make_config(s=prob.s, m=prob.m, a=prob.a, nr=prob.nr, ntheta=prob.nth, x_min=prob.x_min,
                         x_max=prob.x_max, M=prob.M, dt=dt, weno_eps=prob.eps, chart=prob.chart, S=prob.S,
                         scheme=prob.scheme, ko_sigma=prob.ko_sigma, integrator=integrator, **kw)


GRIDS = [(7, 2, 0, 0, 0.5), (63, 5, -2, 2, 0.999), (64, 4, 0, 1, 1.0), (130, 9, -2, 3, 0.9), (200, 17, -2, 1, 0.7)]


@pytest.mark.parametrize("scheme", ["weno3", "fd6ko8"])
@pytest.mark.parametrize("grid", GRIDS)
def test_steps_match_the_oracle(scheme, grid):
    nr, nth, s, m, a = grid
    say("case scheme", scheme, grid)
    prob = S.Problem(s, m, a, nr, nth, -30.0, 50.0, scheme=scheme, ko_sigma=0.3)
    o = S.TeukOracle(prob)
    u0 = W.random_state(nr, nth, seed=nr + 11 * nth, smooth=True)
    for integ, k, n in (("rk3", 0.4, 3), ("rk104", 1.5, 2)):
        dt = k * o.dt_bound(1.0)
        ref, _ = o.evolve(u0, dt, n, integrator=integ)
        with T.Solver(cfg_for(prob, dt, integ)) as sv:
            sv.set_initial(u0)
            sv.step(n)
            got = sv.state()
        se, pe = errors(got, ref)
        say("  ", integ, "error", se, max(pe))
        assert se <= TOL and max(pe) <= TOL_PLANE, (integ, se, pe)


@pytest.mark.parametrize("scheme", ["weno3", "fd6ko8"])
def test_rhs_and_hyperboloidal_chart(scheme):
    say("case scheme rhs + chart H", scheme)
    prob = S.Problem(-2, 0, 1.0, 150, 8, 20.0 / 21.0, 19.5, chart="H", S=20.0, scheme=scheme)
    o = S.TeukOracle(prob)
    u0 = W.random_state(prob.nr, prob.nth, seed=4, smooth=True)
    dt = 0.4 * o.dt_bound(1.0)
    ref, _ = o.evolve(u0, dt, 3)
    F = o.rhs(u0)
    with T.Solver(cfg_for(prob, dt)) as sv:
        sv.set_initial(u0)
        gF = sv.rhs()
        sv.step(3)
        got = sv.state()
    se, pe = errors(gF, F)
    assert se <= TOL and max(pe) <= TOL_PLANE, ("rhs", se, pe)
    se, pe = errors(got, ref)
    say("  error", se, max(pe))
    assert se <= TOL and max(pe) <= TOL_PLANE


@pytest.mark.parametrize("scheme", ["weno3", "fd6ko8"])
def test_c2_full_size(scheme):
    wl = W.C2
    say("case scheme C2 full size", scheme)
    prob = S.Problem(wl.s, wl.m, wl.a, wl.nr, wl.nth, wl.x_min, wl.x_max, scheme=scheme)
    o = S.TeukOracle(prob)
    u0 = W.gaussian_pulse(wl)
    with T.Solver(cfg_for(prob, 0.0)) as sv:
        dt = sv.info().dt
        sv.set_initial(u0)
        sv.step(3)
        got = sv.state()
    ref, _ = o.evolve(u0, dt, 3)
    se, pe = errors(got, ref)
    say("  error", se, max(pe))
    assert se <= TOL and max(pe) <= TOL_PLANE


def test_not_offered():
    say("case schemes unsupported")
    prob = S.Problem(0, 0, 0.5, 64, 4, -10.0, 10.0, scheme="weno3")
    for kw in (dict(weight_prec="fp32"), dict(state="dd", weight_prec="dd")):
        with pytest.raises(T.TeukError) as ei:
            T.teuk_create(cfg_for(prob, 0.0, **kw))
        assert ei.value.status == T.TEUK_ERR_UNSUPPORTED
    with T.Solver(cfg_for(prob, 0.0)) as sv, T.Group(2) as g:
        sv.set_initial(W.random_state(64, 4, seed=1))
        with pytest.raises(T.TeukError) as ei:
            g.add(sv)
        assert ei.value.status == T.TEUK_ERR_UNSUPPORTED
    c = cfg_for(prob, 0.0)
    c.ko_sigma = 2.0
    assert T.teuk_footprint_bytes(c) == 0
