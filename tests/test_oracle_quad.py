"""Pins of the binary128 ("quad", Sec. 3.1.3) build of the oracle.

The quad build is the FP64 oracle's source with a wider working type, so its
logic is pinned by the FP64 tests; what these tests pin is that every step
really carries binary128 precision and that the mixed-weight variant is the
paper's:
- WENO5 weights and fluxes against the Jiang-Shu definitions (candidate
  polynomials matching cell averages, smoothness as the integral of squared
  derivatives, ideal weights from the five-cell polynomial) in exact rational
  arithmetic, both sides;
- the mixed variant: omega_0, omega_1 bit-equal to the FP64 oracle's weights on
  the rounded stencil, omega_2 the exact complement, exact derivatives of
  quadratics (which needs the weights to sum to one in binary128);
- SSP-RK3 against its stability polynomial to 1e-30;
- the coefficient tables at 45 digits: r(x) round trip, agreement with the FP64
  tables, and static solutions of the first-order system to 1e-30;
- the Teukolsky right-hand side exact on quadratic data to 1e-27 and equal to
  the FP64 oracle's to FP64 rounding.
"""
from fractions import Fraction as Fr

import mpmath as mp
import numpy as np
import pytest
import sympy as sp

from oracle import coefficients as C
from oracle import quad as Q
from oracle import solver as S

X = sp.Symbol("x")


def _candidate(avgs, cells):
    """Quadratic whose averages over unit cells [c-1/2, c+1/2] (c in cells) are avgs."""
    c0, c1, c2 = sp.symbols("c0 c1 c2")
    p = c0 + c1 * X + c2 * X**2
    eqs = [sp.integrate(p, (X, sp.Rational(2 * c - 1, 2), sp.Rational(2 * c + 1, 2))) - a
           for c, a in zip(cells, avgs)]
    sol = sp.solve(eqs, (c0, c1, c2), dict=True)[0]
    return p.subs(sol)


def _smoothness(p):
    """Jiang-Shu: sum over l = 1, 2 of the integral over cell 0 of (d^l p)^2 (unit dx)."""
    half = sp.Rational(1, 2)
    return sum(sp.integrate(sp.diff(p, X, l) ** 2, (X, -half, half)) for l in (1, 2))


def _ideal_weights(cell_sets, edge):
    """d_k with sum_k d_k q_k = P(edge) for every five-cell average vector."""
    fs = sp.symbols("f0:5")
    all_cells = sorted({c for cs in cell_sets for c in cs})
    lookup = dict(zip(all_cells, fs))
    qs = [_candidate([lookup[c] for c in cs], cs).subs(X, edge) for cs in cell_sets]
    # five-cell quartic
    cs_ = sp.symbols("k0:5")
    P = sum(cs_[i] * X**i for i in range(5))
    eqs = [sp.integrate(P, (X, sp.Rational(2 * c - 1, 2), sp.Rational(2 * c + 1, 2))) - lookup[c] for c in all_cells]
    Psol = P.subs(sp.solve(eqs, cs_, dict=True)[0]).subs(X, edge)
    d = sp.symbols("d0:3")
    expr = sp.expand(sum(di * qi for di, qi in zip(d, qs)) - Psol)
    sol = sp.solve([expr.coeff(f) for f in fs], d, dict=True)[0]
    return [sol[di] for di in d]


def _exact_weno(f, side, eps):
    """Exact (omega, flux) of f^+_{j+1/2} (side=+1, f at cells -2..2 relative to j)
    or f^-_{j+1/2} (side=-1, f at cells -1..3), ordered as the oracle orders them."""
    if side > 0:
        cells = [(-2, -1, 0), (-1, 0, 1), (0, 1, 2)]
        base = -2
    else:
        cells = [(1, 2, 3), (0, 1, 2), (-1, 0, 1)]        # omega_0 pairs with the far-right stencil
        base = -1
    edge = sp.Rational(1, 2)
    d = _ideal_weights(cells, edge)
    vals = {base + i: sp.Rational(Fr(float(v))) for i, v in enumerate(f)}
    alph, qs = [], []
    for k, cs in enumerate(cells):
        p = _candidate([vals[c] for c in cs], cs)
        # the smoothness integral is over the cell of the reconstruction point's
        # upwind side: cell 0 for f^+, cell 1 for f^- (shift x -> x + 1)
        IS = _smoothness(p if side > 0 else p.subs(X, X + 1))
        alph.append(d[k] / (sp.Rational(Fr(eps)) + IS) ** 2)
        qs.append(p.subs(X, edge))
    tot = sum(alph)
    om = [al / tot for al in alph]
    return om, sum(o * q for o, q in zip(om, qs)), d


def _mpf(x):
    return mp.mpf(sp.Rational(x).p) / mp.mpf(sp.Rational(x).q)


@pytest.mark.parametrize("side", [+1, -1])
def test_weights_and_flux_from_the_jiang_shu_definitions(side):
    mp.mp.dps = 50
    rng = np.random.default_rng(11 + side)
    for trial in range(6):
        f = rng.standard_normal(5) * (10.0 ** rng.integers(-3, 3))
        eps = 1e-6 if trial % 2 == 0 else 1e-2
        om, flux, d = _exact_weno(f, side, eps)
        if trial == 0:
            assert [sp.nsimplify(v) for v in d] == [sp.Rational(1, 10), sp.Rational(3, 5), sp.Rational(3, 10)]
        w = Q.weno5_weights(Q.promote(f), side, eps=eps)
        for k in range(3):
            assert abs(Q.to_mpf(w[k]) - _mpf(om[k])) <= mp.mpf("1e-32"), (k, w[k])
        got = Q.to_mpf(Q.weno5_flux(Q.promote(f), side, eps=eps))
        scale = max(abs(float(v)) for v in f)
        assert abs(got - _mpf(flux)) <= mp.mpf("1e-31") * scale


@pytest.mark.parametrize("side", [+1, -1])
def test_mixed_weights_are_double_weights_with_a_binary128_complement(side):
    rng = np.random.default_rng(5)
    for _ in range(20):
        hi = rng.standard_normal(5)
        lo = hi * rng.uniform(-1, 1, 5) * 2.0**-54      # below half an ulp: hi is the rounded value
        f = np.stack([hi, lo], axis=-1)
        w = Q.weno5_weights(f, side, weights="fp64")
        ref = S.weno5_weights_plus(hi) if side > 0 else S.weno5_weights_minus(hi)
        assert w[0, 0] == ref[0] and w[0, 1] == 0.0
        assert w[1, 0] == ref[1] and w[1, 1] == 0.0
        comp = Fr(1) - Fr(ref[0]) - Fr(ref[1])
        got2 = Fr(w[2, 0]) + Fr(w[2, 1])
        assert abs(got2 - comp) <= Fr(2) ** -112 * abs(comp)
        # and the FP64 oracle's printed omega_2 differs from the complement
        # only by double rounding
        assert abs(float(comp) - ref[2]) <= 4e-16


@pytest.mark.parametrize("weights", ["quad", "fp64"])
@pytest.mark.parametrize("side", [+1, -1])
def test_derivative_of_quadratics_exact_in_binary128(weights, side):
    mp.mp.dps = 50
    rng = np.random.default_rng(7)
    dx = mp.mpf(3) / 7
    dxp = Q.split(dx)
    for _ in range(5):
        c = [mp.mpf(float(v)) for v in rng.standard_normal(3)]
        x0 = mp.mpf(float(rng.uniform(-2, 2)))
        xs = [x0 + (i - 3) * dx for i in range(7)]
        # cell averages of h over [x-dx/2, x+dx/2] are the samples of f = c0 + c1 x + c2 x^2,
        # and the flux-difference derivative is exact for f' (the average of h' is f')
        row = np.array([Q.split(c[0] + c[1] * xv + c[2] * xv * xv) for xv in xs])
        got = Q.to_mpf(Q.derivative(row, 3, dxp, side, weights=weights))
        want = c[1] + 2 * c[2] * x0
        assert abs(got - want) <= mp.mpf("1e-29") * (abs(c[1]) + abs(c[2]) * 4 + 1), (got, want)


def test_rk3_reproduces_its_stability_polynomial():
    mp.mp.dps = 50
    for lam, dt, n in ((-1.0, 0.01, 100), (-3.7, 1e-3, 700), (0.5, 0.25, 12)):
        z = mp.mpf(lam) * mp.mpf(dt)
        want = (1 + z + z**2 / 2 + z**3 / 6) ** n
        got = Q.to_mpf(Q.ode_rk3(lam, (dt, 0.0), n))
        assert abs(got - want) <= mp.mpf("1e-31") * abs(want) * n, (lam, got, want)


def test_rk3_third_order_below_double_precision():
    # u' = -u to t = 1: the global error ~ dt^3 / 24 e^-1 falls below one FP64
    # ulp of the answer at the finest steps, where only binary128 still sees it.
    mp.mp.dps = 50
    errs = []
    for n in (20000, 40000, 80000):
        got = Q.to_mpf(Q.ode_rk3(-1.0, Q.split(mp.mpf(1) / n), n))
        errs.append(abs(got - mp.e ** -1))
    assert errs[-1] < 2.0**-53 * 0.37
    orders = [float(mp.log(errs[i] / errs[i + 1], 2)) for i in range(2)]
    assert all(2.95 < o < 3.05 for o in orders), orders


# ----------------------------------------------------------------------------- tables at 45 digits
def _tortoise_mp(r, a):
    M = mp.mpf(1)
    d = mp.sqrt(max(M * M - a * a, mp.mpf(0)))
    rp, rm = M + d, M - d
    if rp - rm > 0:
        return r + 2 * M * rp / (rp - rm) * mp.log((r - rp) / (2 * M)) - 2 * M * rm / (rp - rm) * mp.log((r - rm) / (2 * M))
    return r + 2 * M * mp.log((r - M) / M) - 2 * M * M / (r - M)


@pytest.mark.parametrize("a", [0.5, 0.999, 1.0])
def test_radial_nodes_round_trip(a):
    with mp.workdps(60):
        x = [mp.mpf(v) for v in (-40, -3.25, 0, 7.5, 80)]
        rs, Ds = Q._r_at_nodes(x, 1.0, a)
        am = mp.mpf(a)
        for xv, r, D in zip(x, rs, Ds):
            assert abs(_tortoise_mp(r, am) - xv) < mp.mpf("1e-40") * (1 + abs(xv))
            assert abs(D - (r * r - 2 * r + am * am)) <= mp.mpf("1e-45") * (r * r)


def test_tables_agree_with_the_fp64_tables():
    prob = S.Problem(-2, 2, 0.999, 40, 6, -30.0, 50.0)
    tq = Q.first_order_tables_mp(prob)
    t64 = S.TeukOracle(prob).tab
    for n, v in t64.items():
        scale = max(float(np.max(np.abs(v))), 1e-300)
        assert np.max(np.abs(tq[n][..., 0] - v)) <= 8e-15 * scale, n


@pytest.mark.parametrize("a", [0.5, 1.0])
@pytest.mark.parametrize("kind", ["const", "dipole"])
def test_static_solutions_of_the_first_order_system(a, kind):
    # s = m = 0.  Psi = 1 (Phi = r) and Psi = (r - M) cos(theta) (Phi = r (r-M) cos)
    # are static, so pi = b d_x Phi and the pi rows of eq. evln vanish:
    #   b d_x(b d_x Phi) - m3 d_x Phi + B~t b d_x Phi + A~thth Phi_thth + B~th Phi_th + C~ Phi = 0.
    prob = S.Problem(0, 0, a, 5, 3, -6.0, 12.0)
    tq = Q.first_order_tables_mp(prob)
    keys, fn = Q._mp_lambdified()
    with mp.workdps(Q.DPS + 10):
        am = mp.mpf(a)
        x = [mp.mpf(prob.x_min) + j * (mp.mpf(prob.x_max) - mp.mpf(prob.x_min)) / (prob.nr - 1)
             for j in range(prob.nr)]
        rs, _ = Q._r_at_nodes(x, 1.0, a)
        Dl = lambda r: r * r - 2 * r + am * am
        for k in range(prob.nth):
            th = (k + mp.mpf(1) / 2) * mp.pi / prob.nth
            cs, sn = mp.cos(th), mp.sin(th)
            ang = (1, 0, 0) if kind == "const" else (cs, -sn, -cs)     # Theta, Theta', Theta''
            radial = (lambda r: r) if kind == "const" else (lambda r: r * (r - 1))

            def b_of_r(r):
                return fn(r, Dl(r), cs, sn, mp.mpf(1), am, 0, 0)[0]

            for j, r in enumerate(rs):
                xr = Dl(r) / (r * r + am * am)                     # dx -> dr factor
                phi_x = xr * mp.diff(radial, r)
                pi_ = lambda rr: b_of_r(rr) * Dl(rr) / (rr * rr + am * am) * mp.diff(radial, rr)
                dpi_x = xr * mp.diff(pi_, r)
                v = {n: Q.to_mpf(tq[n][k, j]) for n in tq}
                res = (v["lam1"] * dpi_x * ang[0] - v["m3r"] * phi_x * ang[0]
                       + v["btr"] * v["lam1"] * phi_x * ang[0]
                       + v["ath"] * radial(r) * ang[2] + v["bth"] * radial(r) * ang[1] + v["cr"] * radial(r) * ang[0])
                scale = abs(v["lam1"] * dpi_x) + abs(v["cr"] * radial(r)) + abs(v["ath"] * radial(r)) + abs(
                    v["m3r"] * phi_x)
                assert abs(res) <= mp.mpf("1e-30") * scale, (kind, a, j, k, res, scale)
                assert abs(v["lam2"] + v["lam1"]) == 0 and v["m3i"] == 0 and v["bti"] == 0 and v["ci"] == 0


# ----------------------------------------------------------------------------- the Teukolsky RHS
def _quadratic_state(prob, rng):
    """Each plane P(x) + Q(theta) with random quadratics; values as pairs, plus
    the exact first derivative in x and derivatives in theta at the nodes."""
    nr, nth = prob.nr, prob.nth
    u = np.zeros((4, nth, nr, 2))
    dx = (mp.mpf(prob.x_max) - mp.mpf(prob.x_min)) / (nr - 1)
    dth = mp.pi / nth
    ders = []
    for p in range(4):
        a0, a1, a2, b1, b2 = [mp.mpf(float(v)) for v in rng.standard_normal(5)]
        dp = {}
        for k in range(nth):
            th = (k + mp.mpf(1) / 2) * dth
            for j in range(nr):
                x = mp.mpf(prob.x_min) + j * dx
                u[p, k, j] = Q.split(a0 + a1 * x + a2 * x * x + b1 * th + b2 * th * th)
                dp[k, j] = (a1 + 2 * a2 * x, b1 + 2 * b2 * th, 2 * b2, a0 + a1 * x + a2 * x * x + b1 * th + b2 * th * th)
        ders.append(dp)
    return u, ders


def test_teuk_rhs_exact_on_quadratic_data():
    # A quadratic in x is differentiated exactly by WENO5 (any weights), and a
    # quadratic in theta by the centred differences, so away from the ghosts
    # the discrete F equals eq. evln with exact derivatives.  With the
    # coefficients read from the same tables, only rounding separates them.
    mp.mp.dps = 50
    prob = S.Problem(-2, 2, 0.999, 24, 6, -20.0, 30.0)
    rng = np.random.default_rng(3)
    u, ders = _quadratic_state(prob, rng)
    for weights in ("quad", "fp64"):
        oq = Q.TeukOracleQ(prob, weights=weights, tables=None if weights == "quad" else tab)
        tab = oq.tab
        F = oq.rhs(u)
        for k in range(1, prob.nth - 1):
            for j in range(3, prob.nr - 3):
                v = {n: Q.to_mpf(tab[n][k, j]) for n in tab}
                dPhR, tPhR, ttPhR, PhR = ders[0][k, j]
                dPhI, tPhI, ttPhI, PhI = ders[1][k, j]
                dPiR, _, _, PiR = ders[2][k, j]
                dPiI, _, _, PiI = ders[3][k, j]
                want = [
                    PiR - v["lam1"] * dPhR,
                    PiI - v["lam1"] * dPhI,
                    -v["lam2"] * dPiR - (v["m3r"] * dPhR - v["m3i"] * dPhI) + (v["btr"] * PiR - v["bti"] * PiI)
                    + v["ath"] * ttPhR + v["bth"] * tPhR + (v["cr"] * PhR - v["ci"] * PhI),
                    -v["lam2"] * dPiI - (v["m3r"] * dPhI + v["m3i"] * dPhR) + (v["btr"] * PiI + v["bti"] * PiR)
                    + v["ath"] * ttPhI + v["bth"] * tPhI + (v["cr"] * PhI + v["ci"] * PhR),
                ]
                for p in range(4):
                    got = Q.to_mpf(F[p, k, j])
                    assert abs(got - want[p]) <= mp.mpf("1e-27") * (1 + abs(want[p])), (weights, p, k, j)


def test_teuk_rhs_and_steps_agree_with_the_fp64_oracle():
    import workloads as W
    prob = S.Problem(-2, 2, 0.999, 70, 8, -30.0, 50.0)
    o = S.TeukOracle(prob)
    oq = Q.TeukOracleQ(prob)
    u0 = W.random_state(prob.nr, prob.nth, seed=4, smooth=True)
    F = o.rhs(u0)
    Fq = oq.rhs(Q.promote(u0))
    assert np.max(np.abs(Fq[..., 0] - F)) <= 1e-13 * np.max(np.abs(F))
    dt = 0.4 * o.dt_bound(1.0)
    u, _ = o.evolve(u0, dt, 4)
    uq, _ = oq.evolve(Q.promote(u0), dt, 4)
    assert np.max(np.abs(uq[..., 0] - u)) <= 1e-13 * np.max(np.abs(u))
    # and the two weight variants differ only at the level of double-rounded weights
    oqm = Q.TeukOracleQ(prob, weights="fp64", tables=oq.tab)
    um, _ = oqm.evolve(Q.promote(u0), dt, 4)
    diff = np.max(np.abs((um[..., 0] - uq[..., 0]) + (um[..., 1] - uq[..., 1])))
    assert 0 < diff <= 1e-14 * np.max(np.abs(u))


def test_window_solve_matches_the_full_grid_inside():
    # The window oracle (used for sampled checks of large grids) solves a block
    # as if it were the whole grid; one step moves information 9 radial nodes
    # and 3 theta rows, so inside that margin it must equal the full solve.
    import workloads as W
    prob = S.Problem(-2, 2, 0.999, 60, 12, -30.0, 50.0)
    full = Q.TeukOracleQ(prob)
    u0 = Q.promote(W.random_state(prob.nr, prob.nth, seed=9, smooth=True))
    dt = 0.4 * S.TeukOracle(prob).dt_bound(1.0)
    uf, _ = full.evolve(u0, dt, 1)
    j0, k0, nw, kw = 17, 3, 30, 8
    win = Q.TeukOracleQ(prob, window=(j0, k0, nw, kw))
    for n in win.tab:
        assert np.array_equal(win.tab[n], full.tab[n][k0:k0 + kw, j0:j0 + nw]), n
    uw, _ = win.evolve(u0[:, k0:k0 + kw, j0:j0 + nw], dt, 1)
    inner = (slice(None), slice(3, kw - 3), slice(9, nw - 9))
    assert np.array_equal(uw[inner], uf[:, k0:k0 + kw, j0:j0 + nw][inner])
    assert not np.array_equal(uw, uf[:, k0:k0 + kw, j0:j0 + nw])
