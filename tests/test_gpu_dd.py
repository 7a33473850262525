"""GPU: the double-double state path (the paper's quad baseline, Sec. 3.1.3)
against the binary128 oracle.

Both weight variants are compared element by element with the oracle run in
the same variant (double-double weights vs binary128 weights; the mixed
variant's double weights vs the oracle's double weights, which the two sides
form from the same rounded stencil by the same printed operations).  The bar
is 1e-26 of the state's largest value: double-double carries about 32 digits,
binary128 34, and an FP64 path misses it by ten orders.  Cases: random smooth
and rough data over several strips with a ragged tail, the smallest grids,
strip-boundary sizes, odd pole parity, the extremal hole, F(u) alone, the
waveform samples, the streamed coefficient table, device initial data, and
one step of the full 8192 x 256 grid sampled in windows."""
import math

import numpy as np
import pytest
import torch

import paper_2010_04760_amd as T
import workloads as W
from oracle import quad as Q
from oracle import solver as S

pytestmark = pytest.mark.gpu

BAR = 1e-26


def say(*a):
    print(*a, flush=True)


def dd_err(got, ref):
    """max |(hi+lo)_got - (hi+lo)_ref| / max |ref|, formed without losing the lo parts."""
    d = (got[..., 0] - ref[..., 0]) + (got[..., 1] - ref[..., 1])
    return float(np.max(np.abs(d))) / max(float(np.max(np.abs(ref[..., 0]))), 1e-300)


def solver_for(prob, weights, dt, **kw):
    cfg = T.make_config(s=prob.s, m=prob.m, a=prob.a, nr=prob.nr, ntheta=prob.nth, x_min=prob.x_min,
                        x_max=prob.x_max, dt=dt, state="dd", weight_prec="dd" if weights == "quad" else "fp64", **kw)
    return T.Solver(cfg)


CASES = [  # s, m, a, nr, nth, x_min, x_max, smooth
    (-2, 2, 0.999, 150, 10, -30.0, 50.0, True),
    (-2, 2, 0.999, 150, 10, -30.0, 50.0, False),
    (0, 1, 0.5, 7, 2, -10.0, 10.0, False),
    (-2, 3, 1.0, 63, 5, -20.0, 40.0, True),
    (0, 0, 0.9, 64, 3, -25.0, 25.0, False),
    (-2, 1, 0.7, 127, 4, -40.0, 60.0, True),
]


@pytest.mark.parametrize("weights", ["quad", "fp64"])
@pytest.mark.parametrize("case", CASES)
def test_steps_match_the_binary128_oracle(case, weights):
    s, m, a, nr, nth, x0, x1, smooth = case
    say("case dd steps", case, weights)
    prob = S.Problem(s, m, a, nr, nth, x0, x1)
    dt = 0.4 * S.TeukOracle(prob).dt_bound(1.0)
    o = Q.TeukOracleQ(prob, weights=weights)
    u0 = Q.promote(W.random_state(nr, nth, seed=31 + nr, smooth=smooth))
    nsteps = 4
    ref, _ = o.evolve(u0, dt, nsteps)
    with solver_for(prob, weights, dt) as sv:
        sv.set_initial(u0)
        sv.step(nsteps)
        got = sv.state()
    err = dd_err(got, ref)
    say("  state error", err)
    assert err <= BAR


def test_rhs_and_waveform_match():
    say("case dd rhs + waveform")
    prob = S.Problem(-2, 2, 0.999, 190, 12, -30.0, 50.0)
    dt = 0.4 * S.TeukOracle(prob).dt_bound(1.0)
    o = Q.TeukOracleQ(prob)
    u0 = Q.promote(W.random_state(prob.nr, prob.nth, seed=5, smooth=True))
    x_e = 10.0
    ref, wref = o.evolve(u0, dt, 6, x_e=x_e, every=2)
    F = o.rhs(u0)
    with solver_for(prob, "quad", dt, x_extract=x_e, extract_every=2, max_samples=8) as sv:
        sv.set_initial(u0)
        got_F = sv.rhs()
        sv.step(6)
        t, w = sv.waveform()
        got = sv.state()
    assert got_F.shape == F.shape
    assert dd_err(got_F, F) <= BAR
    assert dd_err(got, ref) <= BAR
    assert w.shape == wref.shape == (4, prob.nth, 2, 2)
    assert dd_err(w, wref) <= BAR
    np.testing.assert_allclose(t, dt * np.arange(0, 7, 2), rtol=1e-15)


def test_streamed_table_and_normalised_device_input():
    say("case dd table + device input")
    cfg = T.make_config(s=-2, m=2, a=0.999, nr=100, ntheta=6, x_min=-20.0, x_max=30.0, state="dd", weight_prec="dd")
    host = T.teuk_host_coefficients(cfg)
    rng = np.random.default_rng(2)
    hi = rng.standard_normal((4, 6, 100))
    lo = rng.standard_normal((4, 6, 100)) * 1e-3          # far from normalised
    u = np.stack([hi, lo], axis=-1)
    with T.Solver(cfg) as sv:
        assert np.array_equal(sv.coefficients(), host)
        sv.set_initial(torch.from_numpy(u).cuda())
        st = sv.state()
    # the same values, stored as TwoSum pairs: hi = fl(hi + lo), the rest in lo
    np.testing.assert_array_equal(st[..., 0], hi + lo)
    for a, b, c, d in zip(st[..., 0].ravel(), st[..., 1].ravel(), hi.ravel(), lo.ravel()):
        assert math.fsum([a, b, -c, -d]) == 0.0
    assert np.all(np.abs(st[..., 1]) <= 0.5 * np.spacing(np.abs(st[..., 0])))


def test_weight_variants_differ_only_by_double_rounded_weights():
    say("case dd mixed vs dd weights")
    prob = S.Problem(-2, 2, 0.999, 150, 10, -30.0, 50.0)
    dt = 0.4 * S.TeukOracle(prob).dt_bound(1.0)
    u0 = W.random_state(prob.nr, prob.nth, seed=8, smooth=True)
    out = {}
    for wv in ("quad", "fp64"):
        with solver_for(prob, wv, dt) as sv:
            sv.set_initial(u0)
            sv.step(10)
            out[wv] = sv.state()
    cfg = T.make_config(s=prob.s, m=prob.m, a=prob.a, nr=prob.nr, ntheta=prob.nth, x_min=prob.x_min,
                        x_max=prob.x_max, dt=dt)
    with T.Solver(cfg) as sv:
        sv.set_initial(u0)
        sv.step(10)
        u64 = sv.state()
    d = dd_err(out["fp64"], out["quad"])
    assert 0 < d <= 1e-14
    assert np.max(np.abs(out["quad"][..., 0] - u64)) <= 1e-13 * np.max(np.abs(u64))


@pytest.mark.parametrize("weights", ["quad", "fp64"])
def test_full_grid_step_sampled_in_windows(weights):
    # One SSP-RK3 step of the 8192 x 256 grid (the benchmark's launch shape);
    # the oracle solves windows of the grid alone and is compared inside a
    # margin of 9 radial nodes and 3 theta rows (one step's reach).
    wl = W.C2
    say("case dd full grid", wl.nr, wl.nth, weights)
    prob = S.Problem(wl.s, wl.m, wl.a, wl.nr, wl.nth, wl.x_min, wl.x_max)
    u0 = W.random_state(wl.nr, wl.nth, seed=12, smooth=True)      # every window holds data
    cfg = T.make_config(s=wl.s, m=wl.m, a=wl.a, nr=wl.nr, ntheta=wl.nth, x_min=wl.x_min, x_max=wl.x_max,
                        state="dd", weight_prec="dd" if weights == "quad" else "fp64")
    with T.Solver(cfg) as sv:
        dt = sv.info().dt
        sv.set_initial(u0)
        sv.step(1)
        got = sv.state()
    u0p = Q.promote(u0)
    # windows: the inner edge and pole, the middle, a strip boundary, the outer edge and pole
    for j0, k0 in ((0, 0), (4000, 120), (63 * 70 - 12, 200), (wl.nr - 26, wl.nth - 8)):
        nw, kw = 26, 8
        o = Q.TeukOracleQ(prob, weights=weights, window=(j0, k0, nw, kw))
        ref, _ = o.evolve(u0p[:, k0:k0 + kw, j0:j0 + nw], dt, 1)
        jl = 0 if j0 == 0 else 9
        jh = nw if j0 + nw == wl.nr else nw - 9
        kl = 0 if k0 == 0 else 3
        kh = kw if k0 + kw == wl.nth else kw - 3
        g = got[:, k0:k0 + kw, j0:j0 + nw][:, kl:kh, jl:jh]
        r = ref[:, kl:kh, jl:jh]
        scale = float(np.max(np.abs(got[..., 0])))
        err = float(np.max(np.abs((g[..., 0] - r[..., 0]) + (g[..., 1] - r[..., 1])))) / scale
        say("  window", j0, k0, "error", err)
        assert err <= BAR
