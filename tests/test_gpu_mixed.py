"""Reduced-precision WENO weights (paper Sec. 3.1.3) on the GPU.

The smoothness indicators and weights are computed in FP32, FP16 or BF16 from
FP64 stencil differences; omega_2 is the FP64 complement, so the weights sum to
one in FP64 and every candidate-flux combination stays consistent.  Checks:

* weights-sum-to-one identity: every candidate stencil is exact for
  quadratics, so on data quadratic in x the low-precision and FP64 paths give
  the same F(u) to FP64 rounding at every point whose stencil avoids the
  boundary ghosts, while on rough data they differ (the low path is in use);
* error against the FP64 oracle of a full C1 run (1000 steps), waveform
  relative L2: FP32 <= 1e-6 (the bar set for the method), FP16 and BF16 held
  to the looser bars below, which sit above the measured errors;
* every epsilon the configuration accepts, on data whose smoothness
  indicators run through every magnitude down to exact zeros: F(u) stays
  finite, equals the FP64 path's where the data are flat, and stays within
  the bars below of it elsewhere.
"""
import numpy as np
import pytest

import paper_2010_04760_amd as T
import workloads as W
from oracle import solver as S

pytestmark = pytest.mark.gpu

LOW = ["fp32", "fp16", "bf16"]
WAVE_BAR = {"fp32": 1e-6, "fp16": 1e-3, "bf16": 1e-2}


def say(*a):
    print(*a, flush=True)


def cfg_for(prob, dt, **kw):
    return T.make_config(s=prob.s, m=prob.m, a=prob.a, nr=prob.nr, ntheta=prob.nth, x_min=prob.x_min,
                         x_max=prob.x_max, dt=dt, **kw)


def rhs(prob, u, prec, **kw):
    with T.Solver(cfg_for(prob, 0.01, weight_prec=prec, **kw)) as sv:
        sv.set_initial(u)
        return sv.rhs()


@pytest.mark.parametrize("prec", LOW)
def test_weights_sum_to_one_identity(prec):
    say("case quadratic identity", prec)
    prob = S.Problem(-2, 2, 0.9, 300, 12, -20.0, 40.0)
    x = prob.x()
    th = prob.theta()
    ang = W.angular_profile(-2, 2, th)
    u = np.zeros((4, prob.nth, prob.nr))
    for p, (c0, c1, c2) in enumerate([(1.0, 0.3, -0.02), (-0.5, 0.1, 0.01), (0.2, -0.05, 0.003),
                                      (0.7, 0.02, -0.004)]):
        u[p] = ang[:, None] * (c0 + c1 * x + c2 * x * x)[None, :]
    F64 = rhs(prob, u, "fp64")
    Flo = rhs(prob, u, prec)
    inner = slice(3, prob.nr - 3)
    scale = np.max(np.abs(F64[:, :, inner]))
    assert np.max(np.abs(Flo[:, :, inner] - F64[:, :, inner])) <= 1e-13 * scale
    # rough data: the low-precision weights do change F
    ur = W.random_state(prob.nr, prob.nth, seed=11)
    d = np.max(np.abs(rhs(prob, ur, prec) - rhs(prob, ur, "fp64")))
    assert d > 1e-12 * np.max(np.abs(rhs(prob, ur, "fp64")))


@pytest.fixture(scope="module")
def c1_reference():
    wl = W.C1
    prob = S.Problem(wl.s, wl.m, wl.a, wl.nr, wl.nth, wl.x_min, wl.x_max)
    o = S.TeukOracle(prob)
    dt = o.dt_bound(0.5)
    u0 = W.gaussian_pulse(wl)
    ref, wref = o.evolve(u0, dt, wl.steps, wl.x_e, wl.every)
    return wl, prob, dt, u0, ref, wref


@pytest.mark.parametrize("prec", LOW)
def test_c1_waveform_error_against_fp64_oracle(prec, c1_reference):
    wl, prob, dt, u0, ref, wref = c1_reference
    say("case C1 mixed", prec)
    cfg = cfg_for(prob, dt, weight_prec=prec, x_extract=wl.x_e, extract_every=wl.every,
                  max_samples=wl.steps // wl.every + 1)
    with T.Solver(cfg) as sv:
        sv.set_initial(u0)
        sv.step(wl.steps)
        _, w = sv.waveform()
    err = np.linalg.norm(w - wref) / np.linalg.norm(wref)
    say("C1", prec, "waveform rel L2", err)
    assert err <= WAVE_BAR[prec], err


@pytest.mark.parametrize("prec", LOW)
def test_flat_stencil_next_to_a_jump_stays_finite(prec):
    """A flat sub-stencil beside a large jump: after the power-of-two scaling of
    the 16-bit paths eps underflows to zero, so tau_min = 0 while a
    neighbouring tau_k is tiny but nonzero.  The weights must stay finite (the
    ratio tau_min / tau_k is formed without the reciprocal of tau_k)."""
    say("case flat stencil beside a jump", prec)
    prob = S.Problem(0, 0, 0.5, 200, 8, -20.0, 40.0)
    prof = np.zeros(prob.nr)
    prof[100] = 2.0
    prof[101:] = 1000.0
    u = np.zeros((4, prob.nth, prob.nr))
    for p in range(4):
        u[p] = prof[None, :] * (1.0 + 0.1 * p)
    F64 = rhs(prob, u, "fp64")
    Flo = rhs(prob, u, prec)
    assert np.all(np.isfinite(Flo))
    assert np.max(np.abs(Flo - F64)) <= 0.1 * np.max(np.abs(F64))


# measured over the sweep: FP32 <= 2e-10, FP16 1.2e-6, BF16 1.1e-5 of max |F|; the
# bars leave a factor of about 100 to the weights' rounding (2^-23, 2^-10, 2^-7
# relative, times corrections that are a small part of F)
EPS_BAR = {"fp32": 1e-7, "fp16": 1e-4, "bf16": 1e-3}


@pytest.mark.parametrize("prec", LOW)
@pytest.mark.parametrize("eps", [1e-30, 1e-13, 1e-11, 1e-10, 1e-8, 1e-6, 1e2, 1e30])
def test_every_eps_stays_finite_and_close(prec, eps):
    """The FP32 weights' common denominator is at least 2560 eps^4 on a flat
    stencil, which is subnormal or zero in FP32 for eps below about 4e-9
    (its reciprocal would overflow); there the lane must take the FP64
    weights.  The data: a Gaussian whose tails take IS_k through every
    magnitude down to ~1e-50, then exact zeros over the outer third."""
    say("case eps sweep", prec, eps)
    prob = S.Problem(-2, 2, 0.9, 400, 12, -40.0, 60.0, eps=eps)
    x = prob.x()
    prof = np.exp(-(x / 4.0) ** 2)
    prof[x > 30.0] = 0.0
    ang = W.angular_profile(-2, 2, prob.theta())
    u = np.zeros((4, prob.nth, prob.nr))
    for p in range(4):
        u[p] = ang[:, None] * prof[None, :] * (1.0 + 0.25 * p)
    F64 = rhs(prob, u, "fp64", weno_eps=eps)
    Flo = rhs(prob, u, prec, weno_eps=eps)
    assert np.all(np.isfinite(Flo)), (prec, eps)
    flat = x > 31.0                        # every radial stencil reads zeros only
    assert np.array_equal(Flo[:, :, flat], F64[:, :, flat])
    rel = float(np.max(np.abs(Flo - F64))) / float(np.max(np.abs(F64)))
    say("eps sweep", prec, eps, "max |F_low - F_64| / max |F_64|", rel)
    assert rel <= EPS_BAR[prec], (prec, eps, rel)
