"""Pins of the oracle's hyperboloidal chart (chart H, paper Sec. 2.2-2.3).

* eq. teuk0 applied numerically (mpmath derivatives of Psi(t, r, theta, phi)
  built from the paper's definitions of tau, rho, t~ and phi~, with r_* and
  k(r) by quadrature) equals the derived eq. near_final coefficients applied to
  Phi, at points outside and inside the horizon and far out towards null
  infinity;
* the first-order tables reproduce eq. final for an arbitrary smooth Phi with
  pi = Phi_tau + b Phi_rho and d_rho b taken numerically (pins lam2 and m3);
* static Kerr solutions Psi = 1 and Psi = (r - M) cos(theta) (s = 0) make the
  continuum operator vanish and the discrete right-hand side converge to zero
  at the WENO order;
* the speeds: lam1 <= 0 everywhere, lam2 has the sign of Delta;
* the horizon interpolation weights are exact on cubics, and so is the
  horizon sampler (Phi_H, d_rho Phi_H at rho_H) on fields cubic in rho.
"""
import mpmath as mp
import numpy as np
import pytest

from oracle import coefficients as C
from oracle import hyperboloidal as H
from oracle import solver as S

SS = 20.0


def _phi_test():
    al, kap = mp.mpc(-0.3, 0.7), mp.mpc(0.05, 0.2)

    def Fm(t, x, th):
        return mp.exp(al * t + kap * x - mp.mpf("0.01") * x * x) * (1 + mp.mpf("0.4") * mp.cos(th)
                                                                   + mp.mpf("0.2") * mp.sin(th) ** 2)

    def partials(t, x, th):
        F = Fm(t, x, th)
        gx = kap - mp.mpf("0.02") * x
        cs, sn = mp.cos(th), mp.sin(th)
        ang = 1 + mp.mpf("0.4") * cs + mp.mpf("0.2") * sn**2
        return {
            "F": F, "Ft": al * F, "Ftt": al * al * F, "Fx": gx * F, "Fxx": (gx * gx - mp.mpf("0.02")) * F,
            "Ftx": al * gx * F,
            "Fth": F / ang * (-mp.mpf("0.4") * sn + mp.mpf("0.4") * sn * cs),
            "Fthth": F / ang * (-mp.mpf("0.4") * cs + mp.mpf("0.4") * (cs * cs - sn * sn)),
        }
    return Fm, partials


def _bl_check_H(a, s, m, r0, th0, t0=0.3, dps=40):
    mp.mp.dps = dps
    M = mp.mpf(1)
    a_ = mp.mpf(a)
    Sm = mp.mpf(SS)
    Dl = lambda rr: rr * rr - 2 * M * rr + a_ * a_
    r0m = mp.mpf(r0)
    Fm, partials = _phi_test()

    def rstar(rr):                      # r_* up to a constant
        return mp.quad(lambda u: (u * u + a_ * a_) / Dl(u), [r0m, rr])

    def kr(rr):
        return mp.quad(lambda u: a_ / Dl(u), [r0m, rr])

    def tau(t, rr):                     # tau = t~ - r^2/(r+S) + 4M ln(S/(r+S)), t~ = t - r + r_*
        return t - rr + rstar(rr) - rr**2 / (rr + Sm) + 4 * M * mp.log(Sm / (rr + Sm))

    def rho(rr):
        return rr / (1 + rr / Sm)

    def Psi(t, rr, th):                 # at phi = 0; phi-dependence exp(i m phi)
        return mp.exp(1j * m * kr(rr)) * rr ** (-1) * Dl(rr) ** (-s) * Fm(tau(t, rr), rho(rr), th)

    t0m, th = mp.mpf(t0), mp.mpf(th0)
    P = Psi(t0m, r0m, th)
    P_t = mp.diff(lambda t: Psi(t, r0m, th), t0m)
    P_tt = mp.diff(lambda t: Psi(t, r0m, th), t0m, 2)
    P_th = mp.diff(lambda u: Psi(t0m, r0m, u), th)
    P_thth = mp.diff(lambda u: Psi(t0m, r0m, u), th, 2)
    inner = lambda rr: Dl(rr) ** (s + 1) * mp.diff(lambda v: Psi(t0m, v, th), rr)
    radial = Dl(r0m) ** (-s) * mp.diff(inner, r0m)
    D0 = Dl(r0m)
    sn, cs = mp.sin(th), mp.cos(th)
    I = 1j
    op = (-((r0m**2 + a_**2) ** 2 / D0 - a_**2 * sn**2) * P_tt
          - 4 * M * a_ * r0m / D0 * (I * m) * P_t
          - 2 * s * (r0m - M * (r0m**2 - a_**2) / D0 + I * a_ * cs) * P_t
          + radial
          + (1 / sn) * (cs * P_th + sn * P_thth)
          + (1 / sn**2 - a_**2 / D0) * (-m * m) * P
          + 2 * s * (a_ * (r0m - M) / D0 + I * cs / sn**2) * (I * m) * P
          - (s**2 * cs**2 / sn**2 - s) * P)
    lhs = op / (r0m ** (-1) * D0 ** (-s))       # k(r0) = 0 by construction

    d = partials(tau(t0m, r0m), rho(r0m), th)
    c = H.second_order_point(r0, th0, 1.0, a, s, m, SS)
    terms = [c["Att"] * d["Ftt"], c["Atx"] * d["Ftx"], c["Axx"] * d["Fxx"], c["Ath"] * d["Fthth"],
             c["Bt"] * d["Ft"], c["Bx"] * d["Fx"], c["Bth"] * d["Fth"], c["C"] * d["F"]]
    rhs = sum(terms)
    scale = max(abs(x) for x in terms)
    return complex(lhs), complex(rhs), float(scale)


@pytest.mark.parametrize("a,s,m", [(1.0, -2, 0), (1.0, 0, 0), (0.5, -2, 2), (0.999, 0, 3), (0.0, -2, 1)])
def test_bl_operator_identity_chart_H(a, s, m):
    rp, rm = C.horizons(1.0, a)
    pts = [(rp + 0.3, 0.4), (6.0, 2.1), (80.0, 1.2)]
    if rp - rm > 0.5:
        pts.append((0.5 * (rp + rm), 0.9))      # between the horizons
    for r0, th0 in pts:
        lhs, rhs, scale = _bl_check_H(a, s, m, r0, th0)
        assert abs(lhs - rhs) < 1e-12 * scale, (r0, th0, lhs, rhs, scale)


def _b_of(rho_, th_, a, s, m):
    """b by the printed root from the undivided coefficients at (rho, theta)."""
    rr = rho_ * SS / (SS - rho_)
    c = H.second_order_point(rr, th_, 1.0, a, s, m, SS)
    W = -c["Att"]
    T, R = c["Atx"] / W, c["Axx"] / W
    return -(T + mp.sqrt(T * T + 4 * R)) / 2, c


@pytest.mark.parametrize("a,s,m", [(1.0, -2, 0), (0.7, -2, 2), (0.3, 0, 1)])
def test_first_order_tables_reproduce_the_second_order_equation(a, s, m):
    mp.mp.dps = 40
    rp, _ = C.horizons(1.0, a)
    rho_h = SS * rp / (rp + SS)
    rho = np.array([rho_h + 0.013, 3.3, 11.7, 19.2])
    th = np.array([0.35, 1.9])
    tab = H.first_order_tables(rho, th, 1.0, a, s, m, SS)
    _, partials = _phi_test()
    for k, t in enumerate(th):
        for j, x in enumerate(rho):
            xm, tm = mp.mpf(float(x)), mp.mpf(float(t))
            b, c = _b_of(xm, tm, a, s, m)
            b_rho = mp.diff(lambda v: _b_of(v, tm, a, s, m)[0], xm)
            d = partials(mp.mpf("0.2"), xm, tm)
            W = -c["Att"]
            # second-order residual of eq. final
            res2 = d["Ftt"] - (c["Atx"] * d["Ftx"] + c["Axx"] * d["Fxx"] + c["Ath"] * d["Fthth"]
                               + c["Bt"] * d["Ft"] + c["Bx"] * d["Fx"] + c["Bth"] * d["Fth"] + c["C"] * d["F"]) / W
            # first-order form with pi = Phi_tau + b Phi_rho
            pi = d["Ft"] + b * d["Fx"]
            pi_t = d["Ftt"] + b * d["Ftx"]
            pi_x = d["Ftx"] + b_rho * d["Fx"] + b * d["Fxx"]
            g = {n: tab[n][k, j] for n in tab}
            m3 = g["m3r"] + 1j * g["m3i"]
            Bt = g["btr"] + 1j * g["bti"]
            Cc = g["cr"] + 1j * g["ci"]
            res1 = (pi_t + g["lam2"] * pi_x + m3 * d["Fx"] - Bt * pi - g["ath"] * d["Fthth"]
                    - g["bth"] * d["Fth"] - Cc * d["F"])
            assert abs(float(g["lam1"]) - float(mp.re(b))) < 1e-14 * max(1.0, abs(float(mp.re(b))))
            scale = max(abs(d["Ftt"]), abs(pi_t), abs(m3 * d["Fx"]), abs(Cc * d["F"]), abs(g["lam2"] * pi_x))
            assert abs(complex(res1) - complex(res2)) < 1e-12 * float(scale), (x, t, res1, res2)


def _phi_static(kind, v, u):
    """Static s = 0, m = 0 Kerr solutions Psi = 1 and Psi = (r - M) cos(theta)
    (M = 1), as Phi = r Psi in chart H (Psi = r^-1 Phi), at rho = v, theta = u."""
    rr = v * SS / (SS - v)
    return rr if kind == "one" else rr * (rr - 1) * mp.cos(u)


@pytest.mark.parametrize("a,kind", [(1.0, "one"), (0.6, "one"), (1.0, "dipole"), (0.9, "dipole")])
def test_static_solutions_continuum_chart_H(a, kind):
    mp.mp.dps = 40
    for x, t in ((1.3, 0.7), (5.0, 1.4), (17.5, 2.6)):
        xm, tm = mp.mpf(x), mp.mpf(t)
        rr = xm * SS / (SS - xm)
        F = _phi_static(kind, xm, tm)
        Fx = mp.diff(lambda v: _phi_static(kind, v, tm), xm)
        Fxx = mp.diff(lambda v: _phi_static(kind, v, tm), xm, 2)
        Fth = mp.diff(lambda u: _phi_static(kind, xm, u), tm)
        Fthth = mp.diff(lambda u: _phi_static(kind, xm, u), tm, 2)
        c = H.second_order_point(rr, tm, 1.0, a, 0, 0, SS)
        terms = [c["Axx"] * Fxx, c["Bx"] * Fx, c["Ath"] * Fthth, c["Bth"] * Fth, c["C"] * F]
        assert abs(sum(terms)) < 1e-25 * max(abs(v) for v in terms)


@pytest.mark.parametrize("a", [1.0, 0.8])
def test_static_solution_discrete_rhs_converges_chart_H(a):
    """Psi = (r - M) cos(theta), s = m = 0, is static: Phi = r (r - M) cos(theta),
    pi = b Phi_rho.  The discrete right-hand side must vanish at the radial
    WENO order (theta is exact for this l = 1 profile up to the second-order
    centred error, which does not change with the radial grid)."""
    errs = []
    for nr in (96, 192):
        prob = S.Problem(0, 0, a, nr, 4, 1.5, 6.0, chart="H", S=SS)
        o = S.TeukOracle(prob)
        x = prob.x()
        th = prob.theta()
        rr = x * SS / (SS - x)
        drdx = SS**2 / (SS - x) ** 2
        phi = (rr * (rr - 1.0))[None, :] * np.cos(th)[:, None]
        dphi = ((2 * rr - 1.0) * drdx)[None, :] * np.cos(th)[:, None]
        u = np.zeros((4, prob.nth, nr))
        u[0] = phi
        u[2] = o.tab["lam1"] * dphi
        F = o.rhs(u)
        inner = slice(8, nr - 8)
        # Phi rows: F = pi - lam1 D Phi, pure radial truncation error
        errs.append(np.max(np.abs(F[0][:, inner])))
    order = np.log2(errs[0] / errs[1])
    assert order > 4.0, (errs, order)


@pytest.mark.parametrize("a", [1.0, 0.5])
def test_speeds_chart_H(a):
    rp, _ = C.horizons(1.0, a)
    rho_h = SS * rp / (rp + SS)
    x0 = 0.6 * rho_h
    prob = S.Problem(-2, 0, a, 97, 6, x0, SS - 0.1, chart="H", S=SS)
    o = S.TeukOracle(prob)
    x = prob.x()
    rr = x * SS / (SS - x)
    Delta = (rr - rp) * (rr - C.horizons(1.0, a)[1])
    assert np.all(o.tab["lam1"] <= 0.0)
    assert np.all(np.sign(o.tab["lam2"]) == np.sign(Delta)[None, :])


def test_horizon_stencil_one_sided_exact_on_cubics():
    rng = np.random.default_rng(2)
    for f, nr in ((0.0, 50), (0.3, 50), (-0.4, 50), (48.2, 50), (7.6, 50)):
        j0, w, dw = H.horizon_stencil(f, nr)
        assert 0 <= j0 <= nr - 4
        c = rng.standard_normal(4)
        p = lambda z: c[0] + c[1] * z + c[2] * z * z + c[3] * z**3
        dp = lambda z: c[1] + 2 * c[2] * z + 3 * c[3] * z * z
        vals = np.array([p(float(j0 + i)) for i in range(4)])
        assert abs(vals @ w - p(f)) < 1e-9 * max(1.0, abs(p(f)))
        assert abs(vals @ dw - dp(f)) < 1e-9 * max(1.0, abs(dp(f)))


def test_coefficients_a_hair_from_the_horizon():
    """A node within rounding of the extremal horizon (the grid that starts on
    it): the extra working precision keeps the tables equal to their limit,
    i.e. continuous with the neighbouring nodes."""
    rho_h = 20.0 / 21.0
    rho = np.array([rho_h, rho_h + 1e-9, rho_h + 1e-6])
    tab = H.first_order_tables(rho, np.array([0.6]), 1.0, 1.0, -2, 0, SS)
    for k, v in tab.items():
        assert np.all(np.isfinite(v)), k
        assert abs(v[0, 0] - v[0, 1]) <= 1e-7 * max(1.0, abs(v[0, 2])), (k, v)


def test_horizon_weights_exact_on_cubics():
    rng = np.random.default_rng(1)
    for xi in (0.0, 0.25, 0.5, 0.9):
        w, dw = H.horizon_weights(xi)
        for _ in range(3):
            c = rng.standard_normal(4)
            p = lambda z: c[0] + c[1] * z + c[2] * z * z + c[3] * z**3
            dp = lambda z: c[1] + 2 * c[2] * z + 3 * c[3] * z * z
            vals = np.array([p(z) for z in (-1.0, 0.0, 1.0, 2.0)])
            assert abs(vals @ w - p(xi)) < 1e-13
            assert abs(vals @ dw - dp(xi)) < 1e-13


@pytest.mark.parametrize("a, start_on_horizon", [(1.0, True), (0.6, False)])
def test_horizon_samples_exact_on_cubic_fields(a, start_on_horizon):
    """Phi_H and d_rho Phi_H of the oracle's horizon sampler, for a field that
    is a cubic in rho on every theta row, against the cubic's value and
    derivative at rho_H = S r+ / (r+ + S), r+ = M + sqrt(M^2 - a^2) (the outer
    Kerr horizon, M = 1): pins the horizon location, the node offset, the
    division by the radial step and the pairing of the real and imaginary
    planes."""
    rp = 1.0 + np.sqrt(1.0 - a * a)
    rho_h = SS * rp / (rp + SS)
    x0 = rho_h if start_on_horizon else 0.7 * rho_h
    prob = S.Problem(-2, 0, a, 81, 5, x0, SS - 0.5, chart="H", S=SS)
    o = S.TeukOracle(prob)
    x = prob.x()
    rng = np.random.default_rng(7)
    cr = rng.standard_normal((prob.nth, 4))
    ci = rng.standard_normal((prob.nth, 4))

    def cubic(c, z):
        return c[:, 0:1] + c[:, 1:2] * z + c[:, 2:3] * z**2 + c[:, 3:4] * z**3

    def dcubic(c, z):
        return c[:, 1] + 2 * c[:, 2] * z + 3 * c[:, 3] * z**2

    u = np.zeros((4, prob.nth, prob.nr))
    u[0] = cubic(cr, x[None, :])
    u[1] = cubic(ci, x[None, :])
    u[2] = rng.standard_normal((prob.nth, prob.nr))
    u[3] = rng.standard_normal((prob.nth, prob.nr))
    ph, dph = o.horizon(u)
    want = cubic(cr, np.array([[rho_h]]))[:, 0] + 1j * cubic(ci, np.array([[rho_h]]))[:, 0]
    dwant = dcubic(cr, rho_h) + 1j * dcubic(ci, rho_h)
    scale = 1.0 + float(np.max(np.abs(want)))
    assert np.max(np.abs(ph - want)) < 1e-12 * scale
    assert np.max(np.abs(dph - dwant)) < 1e-10 * scale
