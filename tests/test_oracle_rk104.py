"""Pins of the oracle's SSP-RK(10,4) step (paper Sec. 3.2), against what the
method's published definition fixes:
- on u' = lambda u, one step equals the stability polynomial of the same method
  written in its low-storage form (Ketcheson, SIAM J. Sci. Comput. 30 (2008)):
      q1 = q2 = u;  q1 += dt/6 F(q1) five times;  q2 = q2/25 + 9 q1/25;
      q1 = 15 q2 - 5 q1;  q1 += dt/6 F(q1) four times;  u = q2 + 3/5 q1 + dt/10 F(q1),
  expanded here symbolically, a different arrangement of the paper's stages;
- fourth-order convergence on a nonlinear ODE;
- the SSP coefficient C = 6: with first-order upwinding, whose forward Euler
  step obeys the maximum principle for dt <= dx/|a|, a square wave stays within
  its bounds at dt = 6 dx/|a| and overshoots well above it;
- on the Teukolsky system, SSP-RK(10,4) and SSP-RK(3,3) approach each other as
  dt shrinks, at the rate of the third-order method."""
import numpy as np
import pytest
import sympy as sp

import workloads as W
from oracle import solver as S


def low_storage_polynomial():
    z = sp.Symbol("z")
    q1 = sp.Integer(1)
    q2 = sp.Integer(1)
    for _ in range(5):
        q1 = q1 + z / 6 * q1
    q2 = q2 / 25 + sp.Rational(9, 25) * q1
    q1 = 15 * q2 - 5 * q1
    for _ in range(4):
        q1 = q1 + z / 6 * q1
    return sp.Poly(sp.expand(q2 + sp.Rational(3, 5) * q1 + z / 10 * q1), z), z


def test_amplification_equals_the_low_storage_form():
    P, z = low_storage_polynomial()
    # fourth order: agrees with exp(z) through z^4 and not at z^5
    coeffs = P.all_coeffs()[::-1]
    for k in range(5):
        assert coeffs[k] == sp.Rational(1, sp.factorial(k))
    assert coeffs[5] != sp.Rational(1, 120)
    assert P.degree() == 10
    for lam in (-1.0, -3.7, 0.5, 2.0, -12.0):
        dt = 0.3
        got = S.ssprk104_step(np.array([1.0, -2.0]), dt, lambda u: lam * u)
        want = float(P.eval(lam * dt))
        np.testing.assert_allclose(got, want * np.array([1.0, -2.0]), rtol=1e-13)
    # imaginary axis: u = (x, y), u' = omega (-y, x)
    om, dt = 1.1, 0.9
    got = S.ssprk104_step(np.array([0.7, -0.2]), dt, lambda u: om * np.array([-u[1], u[0]]))
    Rz = complex(P.eval(sp.I * om * dt)) * (0.7 - 0.2j)
    np.testing.assert_allclose(got, [Rz.real, Rz.imag], rtol=1e-13)


def test_fourth_order_on_a_nonlinear_ode():
    # u' = -u^2, u(0) = 1  ->  u(1) = 1/2
    errs = []
    for n in (5, 10, 20, 40):
        u = np.array([1.0])
        for _ in range(n):
            u = S.ssprk104_step(u, 1.0 / n, lambda v: -v * v)
        errs.append(abs(u[0] - 0.5))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 3.8) and np.all(orders < 4.3), (errs, orders)


def _upwind(u):
    # u_t + u_x = 0 on a periodic unit grid (dx = 1): F = -(u_j - u_{j-1})
    return -(u - np.roll(u, 1))


@pytest.mark.parametrize("ratio,holds", [(6.0, True), (5.0, True), (8.0, False)])
def test_ssp_coefficient_six(ratio, holds):
    u = np.zeros(60)
    u[10:25] = 1.0
    lo, hi = 0.0, 1.0
    worst = 0.0
    for _ in range(40):
        u = S.ssprk104_step(u, ratio, _upwind)
        worst = max(worst, float(np.max(u)) - hi, lo - float(np.min(u)))
    if holds:
        assert worst <= 1e-13, worst
    else:
        assert worst > 1e-3, worst


def test_teukolsky_integrators_agree_as_dt_shrinks():
    wl = W.C1.with_(nr=160, nth=8, x_min=-30.0, x_max=40.0)
    prob = S.Problem(wl.s, wl.m, wl.a, wl.nr, wl.nth, wl.x_min, wl.x_max)
    o = S.TeukOracle(prob)
    b = o.dt_bound(1.0)
    u0 = W.gaussian_pulse(wl)
    T_end = 6.0
    diffs = []
    for k in (0.4, 0.2, 0.1):
        n3 = int(round(T_end / (k * b)))
        dt = T_end / n3
        u3, _ = o.evolve(u0, dt, n3, integrator="rk3")
        u4, _ = o.evolve(u0, dt, n3, integrator="rk104")
        diffs.append(float(np.max(np.abs(u3 - u4))))
    rates = np.log2(np.array(diffs[:-1]) / np.array(diffs[1:]))
    assert np.all(rates > 2.7), (diffs, rates)
