"""Pins of the oracle's comparison schemes (Sec. 3.1): third-order WENO and
the sixth-order centred difference with eighth-order Kreiss-Oliger
dissipation, against what the mathematics fixes:
- WENO3 weights and fluxes against the Jiang-Shu definitions (linear
  candidates matching two cell averages, smoothness as the integral of the
  squared derivative, ideal weights from the three-cell quadratic) in exact
  rational arithmetic; this also pins the reading of the printed f^- flux as
  the mirror image of f^+ about j + 1/2;
- the mirror identity, third order with linear weights, convergence and the
  non-oscillatory square wave with the nonlinear weights;
- FD6 exact to degree six and not seven, sixth-order convergence;
- KO8: zero on polynomials of degree <= 7, the Fourier symbol
  sigma sin^8(k dx/2)/dx with the dissipative sign;
- the Teukolsky right-hand side of a static solution vanishing at each
  scheme's order."""
from fractions import Fraction as Fr

import numpy as np
import pytest
import sympy as sp

from oracle import solver as S

X = sp.Symbol("x")


def _linear(avgs, cells):
    c0, c1 = sp.symbols("c0 c1")
    p = c0 + c1 * X
    eqs = [sp.integrate(p, (X, sp.Rational(2 * c - 1, 2), sp.Rational(2 * c + 1, 2))) - a for c, a in zip(cells, avgs)]
    return p.subs(sp.solve(eqs, (c0, c1), dict=True)[0])


def _exact_weno3(f, side, eps):
    """(omega, flux) of f^+_{j+1/2} (side=+1, f at cells -1, 0, 1) or of its
    mirror f^-_{j+1/2} (side=-1, f at cells 0, 1, 2), the reconstruction at
    x = 1/2 from the upwind cell."""
    if side > 0:
        cells, base, upwind = [(-1, 0), (0, 1)], -1, 0
    else:
        cells, base, upwind = [(1, 2), (0, 1)], 0, 1
    vals = {base + i: sp.Rational(Fr(float(v))) for i, v in enumerate(f)}
    edge = sp.Rational(1, 2)
    # ideal weights from the three-cell quadratic
    fs = sp.symbols("g0:3")
    look = dict(zip(sorted(vals), fs))
    qs = [_linear([look[c] for c in cs], cs).subs(X, edge) for cs in cells]
    k0, k1, k2 = sp.symbols("k0:3")
    P = k0 + k1 * X + k2 * X**2
    eqs = [sp.integrate(P, (X, sp.Rational(2 * c - 1, 2), sp.Rational(2 * c + 1, 2))) - look[c] for c in sorted(vals)]
    Pe = P.subs(sp.solve(eqs, (k0, k1, k2), dict=True)[0]).subs(X, edge)
    d = sp.symbols("d0:2")
    expr = sp.expand(d[0] * qs[0] + d[1] * qs[1] - Pe)
    dsol = sp.solve([expr.coeff(g) for g in fs], d, dict=True)[0]
    dk = [dsol[d[0]], dsol[d[1]]]
    alph, cand = [], []
    for k, cs in enumerate(cells):
        p = _linear([vals[c] for c in cs], cs)
        lo, hi = sp.Rational(2 * upwind - 1, 2), sp.Rational(2 * upwind + 1, 2)
        IS = sp.integrate(sp.diff(p, X) ** 2, (X, lo, hi))
        alph.append(dk[k] / (sp.Rational(Fr(eps)) + IS) ** 2)
        cand.append(p.subs(X, edge))
    tot = sum(alph)
    om = [a / tot for a in alph]
    return om, sum(o * q for o, q in zip(om, cand)), dk


@pytest.mark.parametrize("side", [+1, -1])
def test_weno3_from_the_jiang_shu_definitions(side):
    rng = np.random.default_rng(3 + side)
    for trial in range(8):
        f = rng.standard_normal(3) * 10.0 ** rng.integers(-2, 2)
        eps = 1e-6 if trial % 2 else 1e-2
        om, flux, dk = _exact_weno3(f, side, eps)
        assert dk == [sp.Rational(1, 3), sp.Rational(2, 3)]
        w = S.weno3_weights(f, side, eps)
        np.testing.assert_allclose(w, [float(om[0]), float(om[1])], rtol=2e-15, atol=1e-16)
        got = S.weno3_flux(f, side, eps)
        assert got == pytest.approx(float(flux), rel=1e-14, abs=1e-15 * np.max(np.abs(f)))


def test_weno3_mirror_identity():
    rng = np.random.default_rng(9)
    for _ in range(20):
        g = rng.standard_normal(3)
        assert S.weno3_flux(g, -1) == S.weno3_flux(g[::-1].copy(), +1)


def test_weno3_linear_weights_exact_to_cubics():
    dx = 0.3
    x = dx * np.arange(-4, 5)
    for deg in range(4):
        row = x ** deg
        want = deg * 0.0 ** (deg - 1) if deg > 0 else 0.0
        for speed in (+1.0, -1.0):
            assert S.radial_derivative(row, 4, dx, speed, "weno3", eps=1e150) == pytest.approx(want, abs=1e-12)
    assert abs(S.radial_derivative(x ** 4, 4, dx, 1.0, "weno3", eps=1e150)) > 1e-4


def _sine_errors(scheme, ns, eps=1e-6, sigma=0.01, T=0.5):
    errs = []
    for n in ns:
        dx = 1.0 / n
        x = dx * np.arange(n)
        u0 = np.sin(2 * np.pi * x)
        # time error below the spatial one: dt ~ dx^2 for the sixth-order scheme
        dt = {"fd6ko8": 2.0 * dx * dx, "weno3": 0.4 * dx}.get(scheme, 0.5 * dx ** (5 / 3))
        nsteps = int(np.ceil(T / dt))
        dt = T / nsteps
        u = S.advect1d_scheme(u0, dx, 1.0, dt, nsteps, scheme, sigma=sigma, eps=eps)
        errs.append(float(np.mean(np.abs(u - np.sin(2 * np.pi * (x - T))))))
    return np.array(errs)


def test_weno3_third_order_with_linear_weights_and_convergent_otherwise():
    lin = _sine_errors("weno3", (40, 80, 160), eps=1e150)
    o_lin = np.log2(lin[:-1] / lin[1:])
    assert np.all(np.abs(o_lin - 3.0) < 0.15), (lin, o_lin)
    nl = _sine_errors("weno3", (40, 80, 160, 320))
    o_nl = np.log2(nl[:-1] / nl[1:])
    assert np.all(o_nl > 1.8) and o_nl[-1] > 2.7 and nl[-1] < 2e-4, (nl, o_nl)


def test_weno3_square_wave_is_essentially_non_oscillatory():
    n = 200
    dx = 1.0 / n
    x = dx * np.arange(n)
    u0 = ((x > 0.2) & (x < 0.5)).astype(float)
    u = S.advect1d_scheme(u0, dx, 1.0, 0.4 * dx, 100, "weno3")
    assert u.max() < 1.0 + 2e-3 and u.min() > -2e-3


def test_fd6_exact_to_degree_six():
    dx = 0.21
    x = dx * np.arange(-4, 5)
    for deg in range(7):
        want = deg * 0.0 ** (deg - 1) if deg > 0 else 0.0
        assert S.radial_derivative(x ** deg, 4, dx, 1.0, "fd6ko8") == pytest.approx(want, abs=1e-11)
    assert abs(S.radial_derivative(x ** 7, 4, dx, 1.0, "fd6ko8")) > 1e-6


def test_fd6ko8_sixth_order_convergence():
    e = _sine_errors("fd6ko8", (16, 32, 64), T=0.25)
    o = np.log2(e[:-1] / e[1:])
    assert np.all(o > 5.6), (e, o)


def test_ko8_symbol_and_sign():
    # speed 0: u_t = -Q u.  For u = cos(k x) on a periodic grid Q u =
    # sigma sin^8(k dx / 2) / dx u, so the mode decays at that rate.
    n, sigma = 16, 0.7
    dx = 1.0 / n
    x = dx * np.arange(n)
    for kk in (1, 3, 7):
        k = 2 * np.pi * kk
        lam = sigma * np.sin(k * dx / 2) ** 8 / dx
        u0 = np.cos(k * x)
        T, nsteps = 0.05, 2000
        u = S.advect1d_scheme(u0, dx, 0.0, T / nsteps, nsteps, "fd6ko8", sigma=sigma)
        np.testing.assert_allclose(u, np.exp(-lam * T) * u0, rtol=1e-9, atol=1e-12)
        assert np.max(np.abs(u)) < 1.0


def test_ko8_vanishes_on_degree_seven():
    from oracle.solver import Problem, TeukOracle
    # through the full RHS: the difference between sigma and sigma = 0 on a
    # plane that is a degree-7 polynomial in x is zero away from the ghosts
    prob = Problem(0, 0, 0.5, 40, 4, -5.0, 5.0, scheme="fd6ko8", ko_sigma=0.5)
    prob0 = Problem(0, 0, 0.5, 40, 4, -5.0, 5.0, scheme="fd6ko8", ko_sigma=0.0)
    o, o0 = TeukOracle(prob), TeukOracle(prob0)
    x = prob.x()
    for deg, zero in ((7, True), (8, False)):
        u = np.zeros((4, 4, 40))
        u[0] = (x / 5.0) ** deg
        d = o.rhs(u) - o0.rhs(u)
        inner = d[:, :, 4:-4]
        if zero:
            assert np.max(np.abs(inner)) < 1e-15      # rounding of the eight-term difference
        else:
            # delta^8 (x/5)^8 = 8! (dx/5)^8, and the RHS receives -sigma delta^8 / (256 dx)
            dx = prob.dx
            want = -0.5 * 40320.0 * (dx / 5.0) ** 8 / (256.0 * dx)
            np.testing.assert_allclose(inner[0], want, rtol=1e-6)
            assert np.max(np.abs(inner[1:])) == 0.0


@pytest.mark.parametrize("scheme,order,grids", [("weno3", 1.8, (201, 401, 801)), ("fd6ko8", 5.5, (101, 201, 401))])
def test_static_solution_rhs_vanishes_at_the_scheme_order(scheme, order, grids):
    # Psi = 1, s = m = 0: Phi = r(x), pi = b d_x Phi (as for WENO5); the FD6
    # grids stop before FP64 rounding (1e-13 here) flattens the last ratio
    errs = []
    for nr in grids:
        prob = S.Problem(s=0, m=0, a=0.5, nr=nr, nth=4, x_min=-10.0, x_max=30.0, scheme=scheme)
        o = S.TeukOracle(prob)
        x = prob.x()
        r = o.r
        drdx = o.Delta / (r * r + 0.25)
        u = np.zeros((4, prob.nth, nr))
        u[0] = r[None, :]
        u[2] = o.tab["lam1"] * drdx[None, :]
        F = o.rhs(u)
        interior = (x > -5) & (x < 25)
        errs.append(np.max(np.abs(F[:, :, interior])))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > order), (errs, orders)
