"""Fourth-order theta differences (theta_order = 4) on the GPU against the
oracle's fourth-order option.

The stage kernel reads Phi on two rows ahead from its LDS ring and keeps two
rows behind in registers; beyond a pole the ghost rows are the mirrored rows
times (-1)^(m+s).  Bars as for the second-order path: whole state <= 1e-12
and each plane <= 5e-12 of its own scale (the fourth-order second difference
sums |weights| 64/12 = 5.3 against 4 at second order, so the amplification of
one-ulp differences by 1/dtheta^2 grows by 4/3; the measured errors sit far
below the bar).

Cases: ragged radial tails and every small theta count (2 .. 9 rows, where
segments are a row or two long and both ahead rows can be ghosts), F(u)
itself, the C1 workload in full, the C2 grid at full size in the benchmarked
launch shape, FP32, FP16 and BF16 weights to their reduced-precision bars, SSP-RK(10,4) (its
dual-output stage), a group with second- and fourth-order members, graph
mode, the tuner, the stability bound, and the combinations that are refused.
"""
import numpy as np
import pytest
import torch

import paper_2010_04760_amd as T
import workloads as W
from oracle import solver as S

pytestmark = pytest.mark.gpu

TOL = 1e-12
TOL_PLANE = 5e-12


def say(*a):
    print(*a, flush=True)


def assert_parity(g, o, tol=TOL, what=""):
    big = max(float(np.max(np.abs(o))), 1e-300)
    se = float(np.max(np.abs(g - o))) / big
    errs = []
    for p in range(o.shape[0]):
        ref = float(np.max(np.abs(o[p])))
        errs.append(float(np.max(np.abs(g[p] - o[p]))) / (ref if ref > 0 else big))
    assert se <= tol, (what, se, errs)
    assert max(errs) <= TOL_PLANE, (what, se, errs)
    return se, errs


def prob4(s, m, a, nr, nth, x_min, x_max):
    return S.Problem(s, m, a, nr, nth, x_min, x_max, theta_order=4)


def cfg_for(prob, dt, **kw):
    return T.make_config(s=prob.s, m=prob.m, a=prob.a, nr=prob.nr, ntheta=prob.nth, x_min=prob.x_min,
                         x_max=prob.x_max, M=prob.M, dt=dt, weno_eps=prob.eps, theta_order=4, **kw)


def run_gpu(cfg, u0, nsteps):
    with T.Solver(cfg) as sv:
        sv.set_initial(u0)
        sv.step(nsteps)
        return sv.state()


RAGGED = [(7, 2, 0, 0, 0.5), (8, 3, -2, 2, 0.999), (62, 4, -2, 1, 0.7), (63, 5, 0, 1, 1.0),
          (64, 6, -2, 0, 0.3), (65, 7, 1, -1, 0.9), (126, 9, -2, 3, 1.0), (127, 16, 0, 0, 0.0),
          (200, 17, -2, 2, 0.999), (513, 33, 0, 2, 0.5)]


@pytest.mark.parametrize("nr,nth,s,m,a", RAGGED)
def test_random_state_steps(nr, nth, s, m, a):
    say("case theta4 random", nr, nth, s, m, a)
    prob = prob4(s, m, a, nr, nth, -30.0, 50.0)
    o = S.TeukOracle(prob)
    dt = 0.3 * o.dt_bound(1.0)
    u0 = W.random_state(nr, nth, seed=nr * 100 + nth + 1)
    for n in (1, 3):
        ref, _ = o.evolve(u0, dt, n)
        got = run_gpu(cfg_for(prob, dt), u0, n)
        assert_parity(got, ref, what=(nr, nth, n))


@pytest.mark.parametrize("nr,nth,s,m,a", RAGGED)
@pytest.mark.parametrize("workgroups", [0, 1])
def test_rhs_random_state(nr, nth, s, m, a, workgroups):
    # workgroups = 1: one theta segment per strip (the whole column in one march);
    # 0: as many segments as rows allow, down to one row each
    say("case theta4 rhs", nr, nth, s, m, a, workgroups)
    prob = prob4(s, m, a, nr, nth, -30.0, 50.0)
    o = S.TeukOracle(prob)
    u0 = W.random_state(nr, nth, seed=nr * 7 + nth + 1)
    with T.Solver(cfg_for(prob, 0.01, workgroups=workgroups * ((nr + 62) // 63))) as sv:
        sv.set_initial(u0)
        F = sv.rhs()
    assert_parity(F, o.rhs(u0), what=("rhs", nr, nth))


def test_segments_of_one_row():
    # a workgroup budget that cuts every strip into one-row segments: every
    # march takes both ahead rows from the ring past its own segment
    say("case theta4 one-row segments")
    prob = prob4(-2, 2, 0.9, 130, 12, -30.0, 50.0)
    o = S.TeukOracle(prob)
    dt = 0.4 * o.dt_bound(1.0)
    u0 = W.random_state(130, 12, seed=21, smooth=True)
    ref, _ = o.evolve(u0, dt, 4)
    outs = [run_gpu(cfg_for(prob, dt, workgroups=wg), u0, 4) for wg in (3, 3 * 12, 3 * 5)]
    for g in outs:
        assert_parity(g, ref, what="segments")
    for g in outs[1:]:
        assert np.array_equal(g, outs[0])


def test_c1_workload_full_run():
    wl = W.C1
    say("case theta4 C1 full", wl.name)
    prob = prob4(wl.s, wl.m, wl.a, wl.nr, wl.nth, wl.x_min, wl.x_max)
    o = S.TeukOracle(prob)
    dt = o.dt_bound(0.5)
    u0 = W.gaussian_pulse(wl)
    ref, wref = o.evolve(u0, dt, wl.steps, wl.x_e, wl.every)
    cfg = cfg_for(prob, dt, x_extract=wl.x_e, extract_every=wl.every, max_samples=wl.steps // wl.every + 1)
    with T.Solver(cfg) as sv:
        sv.set_initial(u0)
        sv.step(wl.steps)
        got = sv.state()
        _, wave = sv.waveform()
    say("C1 theta4 state errors", assert_parity(got, ref, what="C1 state"))
    assert np.max(np.abs(wave - wref)) / np.max(np.abs(wref)) <= TOL


def test_c2_grid_full_size():
    wl = W.C2
    say("case theta4 C2 full grid", wl.name)
    prob = prob4(wl.s, wl.m, wl.a, wl.nr, wl.nth, wl.x_min, wl.x_max)
    o = S.TeukOracle(prob)
    dt = o.dt_bound(0.5)
    u0 = W.gaussian_pulse(wl)
    ref, _ = o.evolve(u0, dt, 3)
    got = run_gpu(cfg_for(prob, dt), u0, 3)
    say("C2 theta4 errors", assert_parity(got, ref, what="C2"))


@pytest.mark.parametrize("prec,bar", [("fp32", 1e-6), ("fp16", 1e-3), ("bf16", 1e-2)])
def test_reduced_precision_weights_within_their_bars(prec, bar):
    # the bars of the second-order path's reduced-precision tests, on the
    # state after 200 steps of a Gaussian pulse
    say("case theta4 weights", prec)
    wl = W.C1.with_(nr=400, nth=24)
    prob = prob4(wl.s, wl.m, wl.a, wl.nr, wl.nth, wl.x_min, wl.x_max)
    o = S.TeukOracle(prob)
    dt = o.dt_bound(0.5)
    u0 = W.gaussian_pulse(wl)
    ref, _ = o.evolve(u0, dt, 200)
    got = run_gpu(cfg_for(prob, dt, weight_prec=prec), u0, 200)
    err = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    say("  error", err)
    assert err <= bar, err


def test_rk104():
    say("case theta4 rk104")
    prob = prob4(-2, 2, 0.999, 300, 20, -40.0, 60.0)
    o = S.TeukOracle(prob)
    dt = 2.0 * o.dt_bound(1.0)
    u0 = W.random_state(300, 20, seed=8, smooth=True)
    ref, _ = o.evolve(u0, dt, 5, integrator="rk104")
    got = run_gpu(cfg_for(prob, dt, integrator="rk104"), u0, 5)
    assert_parity(got, ref, what="rk104")


def test_stability_bound():
    say("case theta4 dt bound")
    for (s, m, a) in ((-2, 2, 0.999), (0, 0, 1.0)):
        prob = prob4(s, m, a, 700, 24, -150.0, 300.0)
        o = S.TeukOracle(prob)
        with T.Solver(cfg_for(prob, 0.0, cfl=0.5)) as sv:
            inf = sv.info()
        assert inf.dt_bound == pytest.approx(o.dt_bound(1.0), rel=1e-12)
        # and the fourth-order bound is the tighter one
        with T.Solver(T.make_config(s=s, m=m, a=a, nr=700, ntheta=24, x_min=-150.0, x_max=300.0)) as sv2:
            assert sv2.info().dt_bound > inf.dt_bound


def test_group_mixes_orders_bitwise():
    say("case theta4 group")
    specs = [(W.C2.with_(nr=300, nth=24, x_min=-60.0, x_max=100.0, seed=41), 4),
             (W.C1.with_(nr=200, nth=16, seed=42), 2),
             (W.C2.with_(nr=260, nth=9, x_min=-60.0, x_max=100.0, seed=43), 4)]
    g = T.Group(3)
    alone, members = [], []
    for wl, order in specs:
        cfg = T.make_config(s=wl.s, m=wl.m, a=wl.a, nr=wl.nr, ntheta=wl.nth, x_min=wl.x_min, x_max=wl.x_max,
                            theta_order=order)
        u0 = W.gaussian_pulse(wl)
        sv = T.Solver(cfg)
        sv.set_initial(u0)
        g.add(sv)
        members.append(sv)
        a = T.Solver(cfg)
        a.set_initial(u0)
        a.step(30)
        alone.append(a.state())
        a.close()
    assert g.info().classes == 2
    g.step(30)
    for sv, ref in zip(members, alone):
        assert np.array_equal(sv.state(), ref)
    g.close()
    for sv in members:
        sv.close()


def test_graph_mode_and_tuner_bitwise():
    say("case theta4 graph + tune")
    wl = W.C2.with_(nr=500, nth=32, x_min=-100.0, x_max=200.0)
    prob = prob4(wl.s, wl.m, wl.a, wl.nr, wl.nth, wl.x_min, wl.x_max)
    dt = S.TeukOracle(prob).dt_bound(0.5)
    cfg = cfg_for(prob, dt, extract_every=5, max_samples=20, x_extract=30.0)
    u0 = W.gaussian_pulse(wl)
    with T.Solver(cfg) as a, T.Solver(cfg) as b:
        a.set_initial(u0)
        b.set_initial(u0)
        a.set_graph(10)
        for n in (20, 7, 13):
            a.step(n)
            b.step(n)
            assert np.array_equal(a.state(), b.state())
            assert np.array_equal(a.waveform()[1], b.waveform()[1])
    T.teuk_tune_forget()
    info = T.teuk_tune(cfg, 4)
    assert info.workgroups > 0
    with T.Solver(cfg) as c:                      # created with the tuned budget
        c.set_initial(u0)
        c.step(40)
        tuned = c.state()
    T.teuk_tune_forget()
    assert np.array_equal(tuned, run_gpu(cfg, u0, 40))


def test_refused_combinations():
    say("case theta4 refused")
    base = dict(s=0, m=0, a=0.5, nr=128, ntheta=8, x_min=-20.0, x_max=20.0, theta_order=4)
    for kw in (dict(integrator="rk3_blocked"), dict(integrator="rk3_pipelined"), dict(state="dd"),
               dict(scheme="weno3"), dict(chart="H", x_min=0.5, x_max=19.0, a=0.5)):
        cfg = T.make_config(**{**base, **kw})
        with pytest.raises(T.TeukError) as ei:
            T.Solver(cfg)
        assert ei.value.status == T.TEUK_ERR_UNSUPPORTED, kw
    with pytest.raises(T.TeukError) as ei:
        T.Solver(T.make_config(**{**base, "theta_order": 3}))
    assert ei.value.status == T.TEUK_ERR_INVALID_ARG
    torch.cuda.synchronize()
