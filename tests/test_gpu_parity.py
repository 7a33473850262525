"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.

Bar (<= 1e-12 max relative error): max |g - o| / max |o| with the
max taken over the whole state u = {Phi_R, Phi_I, pi_R, pi_I} <= 1e-12.  Each
plane is also held to its own scale, max |g_p - o_p| / max |o_p| <= 5e-12: the
centred theta second difference amplifies one-ulp differences between two
correct FP64 evaluations by ~1/dtheta^2, and on the 256-row C2 grid the oracle
rebuilt with FMA contraction differs from itself by 1.1e-12 in pi_R after three
steps from pi(0) = 0 (see tests/test_parity_conditioning.py).

Cases cover ragged radial tails around the 63-point strip, minimum grids,
extremal Kerr, the C1 workload in full, the C2 grid at full size, launch-shape
invariance, the waveform ring buffer, checkpoint/resume, error paths and the
stability-bound reduction."""
import numpy as np
import pytest
import torch

import paper_2010_04760_amd as T
import workloads as W
from oracle import solver as S

pytestmark = pytest.mark.gpu

TOL = 1e-12          # whole-state max-norm relative error
TOL_PLANE = 5e-12    # each plane against its own max


def say(*a):
    print(*a, flush=True)


def state_error(g, o):
    return float(np.max(np.abs(g - o))) / max(float(np.max(np.abs(o))), 1e-300)


def plane_errors(g, o):
    big = max(float(np.max(np.abs(o))), 1e-300)
    errs = []
    for p in range(o.shape[0]):
        ref = float(np.max(np.abs(o[p])))
        errs.append(float(np.max(np.abs(g[p] - o[p]))) / (ref if ref > 0 else big))
    return errs


def assert_parity(g, o, tol=TOL, what=""):
    se = state_error(g, o)
    errs = plane_errors(g, o)
    assert se <= tol, (what, se, errs)
    assert max(errs) <= TOL_PLANE, (what, se, errs)
    return se, errs


def cfg_for(prob: S.Problem, dt, **kw):
    return T.make_config(s=prob.s, m=prob.m, a=prob.a, nr=prob.nr, ntheta=prob.nth, x_min=prob.x_min,
                         x_max=prob.x_max, M=prob.M, dt=dt, weno_eps=prob.eps, **kw)


def run_gpu(cfg, u0, nsteps):
    with T.Solver(cfg) as sv:
        sv.set_initial(u0)
        sv.step(nsteps)
        return sv.state()


RAGGED = [(7, 2, 0, 0, 0.5), (8, 3, -2, 2, 0.999), (62, 4, -2, 1, 0.7), (63, 5, 0, 1, 1.0),
          (64, 4, -2, 0, 0.3), (65, 7, 1, -1, 0.9), (126, 9, -2, 3, 1.0), (127, 16, 0, 0, 0.0),
          (200, 17, -2, 2, 0.999), (513, 33, 0, 2, 0.5)]


@pytest.mark.parametrize("nr,nth,s,m,a", RAGGED)
def test_random_state_steps(nr, nth, s, m, a):
    say("case random", nr, nth, s, m, a)
    prob = S.Problem(s, m, a, nr, nth, -30.0, 50.0)
    o = S.TeukOracle(prob)
    dt = 0.3 * o.dt_bound(1.0)
    u0 = W.random_state(nr, nth, seed=nr * 100 + nth)
    for n in (1, 3):
        ref, _ = o.evolve(u0, dt, n)
        got = run_gpu(cfg_for(prob, dt), u0, n)
        assert_parity(got, ref, what=(nr, nth, n))


@pytest.mark.parametrize("nr,nth,s,m,a", RAGGED)
def test_rhs_random_state(nr, nth, s, m, a):
    # F(u) itself (TEUK_X_RHS evaluates it with the stage kernel) against the oracle
    say("case rhs", nr, nth, s, m, a)
    prob = S.Problem(s, m, a, nr, nth, -30.0, 50.0)
    o = S.TeukOracle(prob)
    u0 = W.random_state(nr, nth, seed=nr * 7 + nth)
    with T.Solver(cfg_for(prob, 0.01)) as sv:
        sv.set_initial(u0)
        F = sv.rhs()
        assert np.array_equal(sv.state(), u0)          # the state is untouched
    assert_parity(F, o.rhs(u0), what=("rhs", nr, nth))


def test_c1_workload_full_run():
    wl = W.C1
    say("case C1 full", wl.name)
    prob = S.Problem(wl.s, wl.m, wl.a, wl.nr, wl.nth, wl.x_min, wl.x_max)
    o = S.TeukOracle(prob)
    dt = o.dt_bound(0.5)
    u0 = W.gaussian_pulse(wl)
    ref, wref = o.evolve(u0, dt, wl.steps, wl.x_e, wl.every)
    cfg = cfg_for(prob, dt, x_extract=wl.x_e, extract_every=wl.every, max_samples=wl.steps // wl.every + 1)
    with T.Solver(cfg) as sv:
        sv.set_initial(u0)
        sv.step(wl.steps)
        got = sv.state()
        t, wave = sv.waveform()
        inf = sv.info()
    errs = assert_parity(got, ref, what="C1 state")
    say("C1 state errors", errs)
    assert wave.shape == wref.shape
    werr = np.max(np.abs(wave - wref)) / np.max(np.abs(wref))
    assert werr <= TOL, werr
    np.testing.assert_allclose(t, np.arange(wave.shape[0]) * wl.every * dt, rtol=1e-15)
    assert inf.steps == wl.steps and inf.samples == wave.shape[0]
    assert inf.j_extract == o.extract_index(wl.x_e)


@pytest.mark.parametrize("nsteps", [3, 40])
def test_c2_grid_full_size(nsteps):
    wl = W.C2
    say("case C2 full grid", wl.name, nsteps)
    prob = S.Problem(wl.s, wl.m, wl.a, wl.nr, wl.nth, wl.x_min, wl.x_max)
    o = S.TeukOracle(prob)
    dt = o.dt_bound(0.5)
    u0 = W.gaussian_pulse(wl)
    ref, _ = o.evolve(u0, dt, nsteps)
    got = run_gpu(cfg_for(prob, dt), u0, nsteps)      # default launch shape, as benchmarked
    errs = assert_parity(got, ref, what="C2")
    say("C2 errors", errs)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_c3_grid_full_size(prec):
    """The extremal-Kerr sweep grid (16384 x 128, a = M) at full size, 3 steps:
    FP64 weights against the oracle to the parity bar; FP32 weights against
    the oracle to 1e-6 (the reduced-precision bar)."""
    wl = W.C3
    say("case C3 full grid", wl.name, prec)
    prob = S.Problem(wl.s, wl.m, wl.a, wl.nr, wl.nth, wl.x_min, wl.x_max)
    o = S.TeukOracle(prob)
    dt = o.dt_bound(0.5)
    u0 = W.gaussian_pulse(wl)
    ref, _ = o.evolve(u0, dt, 3)
    got = run_gpu(cfg_for(prob, dt, weight_prec=prec), u0, 3)
    if prec == "fp64":
        errs = assert_parity(got, ref, what="C3")
    else:
        errs = state_error(got, ref)
        assert errs <= 1e-6, errs
    say("C3 errors", errs)


def test_launch_shape_invariance():
    say("case rows invariance")
    prob = S.Problem(-2, 2, 0.999, 300, 37, -50.0, 80.0)
    o = S.TeukOracle(prob)
    dt = 0.4 * o.dt_bound(1.0)
    u0 = W.random_state(300, 37, seed=5, smooth=True)
    outs = [run_gpu(cfg_for(prob, dt, workgroups=r), u0, 4) for r in (1, 3, 8, 37, 64)]
    for g in outs[1:]:
        assert np.array_equal(g, outs[0])


def test_dt_bound_and_coefficients_match_oracle():
    say("case dt bound / coefficients")
    for (s, m, a) in ((-2, 2, 0.999), (0, 0, 1.0), (0, 3, 0.5)):
        prob = S.Problem(s, m, a, 700, 24, -150.0, 300.0)
        o = S.TeukOracle(prob)
        cfg = cfg_for(prob, 0.0, cfl=0.5)
        with T.Solver(cfg) as sv:
            inf = sv.info()
            coef = sv.coefficients()
        assert inf.dt_bound == pytest.approx(o.dt_bound(1.0), rel=1e-12)
        assert inf.dt == pytest.approx(0.5 * o.dt_bound(1.0), rel=1e-12)
        names = ["lam1", "m3r", "m3i", "btr", "bti", "cr", "ci", "ath", "bth"]
        scale = max(np.max(np.abs(o.tab[n])) for n in names)
        for i, n in enumerate(names):
            err = np.max(np.abs(coef[i] - o.tab[n]))
            assert err <= 1e-13 * np.max(np.abs(o.tab[n])) + 1e-15 * scale, (n, err)


def test_waveform_ring_buffer():
    say("case ring buffer")
    prob = S.Problem(0, 0, 0.5, 256, 8, -40.0, 60.0)
    o = S.TeukOracle(prob)
    dt = 0.5 * o.dt_bound(1.0)
    wl = W.C1.with_(nr=256, nth=8, x_min=-40.0, x_max=60.0)
    u0 = W.gaussian_pulse(wl)
    _, wref = o.evolve(u0, dt, 20, 30.0, 3)           # samples at steps 0,3,...,18 (7 samples)
    cfg = cfg_for(prob, dt, x_extract=30.0, extract_every=3, max_samples=4)
    with T.Solver(cfg) as sv:
        sv.set_initial(u0)
        sv.step(11)
        sv.step(9)
        t, wave = sv.waveform()
        assert sv.info().samples == 7
    assert wave.shape == (4, 8, 2)
    np.testing.assert_allclose(t, np.array([9, 12, 15, 18]) * dt, rtol=1e-15)
    assert np.max(np.abs(wave - wref[3:])) <= TOL * np.max(np.abs(wref))


def test_checkpoint_resume_is_bitwise():
    say("case checkpoint")
    prob = S.Problem(-2, 2, 0.999, 400, 20, -60.0, 100.0)
    o = S.TeukOracle(prob)
    dt = 0.5 * o.dt_bound(1.0)
    wl = W.C2.with_(nr=400, nth=20, x_min=-60.0, x_max=100.0)
    u0 = W.gaussian_pulse(wl)
    straight = run_gpu(cfg_for(prob, dt), u0, 40)
    mid = run_gpu(cfg_for(prob, dt), u0, 20)
    resumed = run_gpu(cfg_for(prob, dt), mid, 20)
    assert np.array_equal(straight, resumed)


def test_device_initial_data_and_library_owned_memory():
    say("case device input")
    prob = S.Problem(0, 1, 0.6, 150, 10, -30.0, 40.0)
    o = S.TeukOracle(prob)
    dt = 0.5 * o.dt_bound(1.0)
    u0 = W.random_state(150, 10, seed=9, smooth=True)
    ref, _ = o.evolve(u0, dt, 5)
    h = T.teuk_create(cfg_for(prob, dt), None)       # library allocates with hipMalloc
    try:
        ud = torch.from_numpy(u0).cuda()
        torch.cuda.synchronize()
        T.teuk_set_initial(h, ud)
        T.teuk_step(h, 5)
        got = T.teuk_extract(h, T.TEUK_X_STATE, u0.size).reshape(u0.shape)
    finally:
        T.teuk_destroy(h)
    assert_parity(got, ref)


def test_side_stream():
    say("case side stream")
    prob = S.Problem(-2, 2, 0.999, 200, 12, -40.0, 60.0)
    o = S.TeukOracle(prob)
    dt = 0.5 * o.dt_bound(1.0)
    u0 = W.random_state(200, 12, seed=3, smooth=True)
    ref, _ = o.evolve(u0, dt, 6)
    st = torch.cuda.Stream()
    with T.Solver(cfg_for(prob, dt), stream=st) as sv:
        sv.set_initial(u0)
        sv.step(6)
        got = sv.state()
    assert_parity(got, ref)


def test_error_paths():
    say("case errors")
    prob = S.Problem(0, 0, 0.5, 64, 4, -10.0, 10.0)
    cfg = cfg_for(prob, 0.01)
    with T.Solver(cfg) as sv:
        with pytest.raises(T.TeukError) as ei:
            sv.step(1)
        assert ei.value.status == T.TEUK_ERR_STATE
        bad = np.zeros((4, 4, 64))
        bad[2, 1, 7] = np.nan
        with pytest.raises(T.TeukError) as ei:
            sv.set_initial(bad)
        assert ei.value.status == T.TEUK_ERR_NONFINITE
        bad_dev = torch.from_numpy(bad).cuda()
        with pytest.raises(T.TeukError) as ei:
            sv.set_initial(bad_dev)
        assert ei.value.status == T.TEUK_ERR_NONFINITE
        with pytest.raises(T.TeukError) as ei:
            T.teuk_step(sv.h, -1)
        assert ei.value.status == T.TEUK_ERR_INVALID_ARG
        sv.set_initial(np.zeros((4, 4, 64)))
        with pytest.raises(T.TeukError) as ei:
            T.teuk_extract(sv.h, T.TEUK_X_STATE, 10)
        assert ei.value.status == T.TEUK_ERR_CAPACITY
        sv.check_finite()
    nb = T.teuk_footprint_bytes(cfg)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    ctx = T.teuk_device_ctx(None, ws.data_ptr(), nb - 256)
    with pytest.raises(T.TeukError) as ei:
        T.teuk_create(cfg, ctx)
    assert ei.value.status == T.TEUK_ERR_OUT_OF_MEMORY
