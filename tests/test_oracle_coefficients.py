"""Pins of the oracle's chart-T coefficients (paper Sec. 2.1-2.3) against
mathematics that does not go through the oracle's derivation:

* a = 0 reduces to the Regge-Wheeler form (b = 1, m3 = 0, A~thth = f/r^2, ...).
* eq. teuk0 evaluated independently by mpmath numerical differentiation (nested
  radial derivative, r_* and k(r) by quadrature) on a complex test field agrees
  with the derived second-order coefficients at Kerr points up to extremal.
* Psi = 1 and Psi = (r - M) cos(theta) are static s = 0, m = 0 solutions for any
  a, so the continuum operator annihilates them and the discrete first-order
  right-hand side converges to zero at the scheme's order.
* at a = 0 the angular terms are the spin-weighted spherical Laplacian, whose
  eigenfunctions (Goldberg's formula) have eigenvalue -(l - s)(l + s + 1);
  the discrete theta operator converges to it at second order up to the poles.
"""
import numpy as np
import pytest
import sympy as sp
import mpmath as mp

from oracle import coefficients as C
from oracle import solver as S


# ----------------------------------------------------------------------------- Regge-Wheeler
@pytest.mark.parametrize("s", [-2, -1, 0, 1, 2])
@pytest.mark.parametrize("m", [0, 1, 3])
def test_schwarzschild_reduction(s, m):
    M = 1.0
    r = np.array([2.0001, 2.5, 3.0, 7.0, 40.0])[None, :]
    D = r * (r - 2 * M)
    th = np.array([0.2, 1.1, 2.9])[:, None]
    c = C.first_order_coefficients(r, D, th, M, 0.0, s, m)
    f = D / r**2          # 1 - 2M/r, formed without cancellation
    np.testing.assert_allclose(c["lam1"], 1.0, rtol=1e-14)
    np.testing.assert_allclose(c["lam2"], -1.0, rtol=1e-14)
    assert np.max(np.abs(c["m3"])) < 1e-13
    np.testing.assert_allclose(c["Ath"], np.broadcast_to(f / r**2, c["Ath"].shape), rtol=1e-13)
    np.testing.assert_allclose(c["Bth"], f / r**2 / np.tan(th), rtol=1e-13)
    if s == 0:
        np.testing.assert_allclose(c["C"].real, -2 * M * f / r**3 - f * m * m / (r * np.sin(th)) ** 2,
                                   rtol=1e-12, atol=1e-15)
        assert np.max(np.abs(c["C"].imag)) < 1e-15
        assert np.max(np.abs(c["Bt"])) < 1e-15


def test_tortoise_closed_forms_have_the_right_derivative():
    # dr_*/dr = (r^2 + a^2)/Delta for the closed forms used by the oracle
    for a in (0.0, 0.5, 0.999, 1.0):
        rp, rm = C.horizons(1.0, a)
        for y in (1e-3, 0.3, 5.0, 200.0):
            h = 1e-6 * max(y, 1e-3)
            dxdr = (C.tortoise_of_y(y + h, 1.0, a) - C.tortoise_of_y(y - h, 1.0, a)) / (2 * h)
            r = rp + y
            want = (r * r + a * a) / (y * (r - rm))
            assert dxdr == pytest.approx(want, rel=1e-7)


def test_inversion_round_trip():
    for a in (0.0, 0.5, 0.999, 1.0):
        x = np.linspace(-400.0, 800.0, 1001)
        r, y, D = C.r_of_tortoise(x, 1.0, a)
        assert np.max(np.abs(C.tortoise_of_y(y, 1.0, a) - x)) < 1e-11 * 800
        assert np.all(y > 0) and np.all(D > 0)


# ----------------------------------------------------------------------------- BL operator
def _bl_check(a, s, m, r0, th0, t0=0.3, dps=30):
    """Return (lhs, rhs): eq. teuk0 applied numerically vs the derived coefficients."""
    mp.mp.dps = dps
    M = mp.mpf(1)
    a_ = mp.mpf(a)
    q = 2 * s + 1
    Dl = lambda rr: rr * rr - 2 * M * rr + a_ * a_
    r0m = mp.mpf(r0)

    al, kap = mp.mpc(-0.3, 0.7), mp.mpc(0.05, 0.2)

    def Fm(t, x, th):
        return mp.exp(al * t + kap * x - mp.mpf("0.01") * x * x) * (1 + mp.mpf("0.4") * mp.cos(th)
                                                                   + mp.mpf("0.2") * mp.sin(th) ** 2)

    def xr(rr):
        return mp.quad(lambda u: (u * u + a_ * a_) / Dl(u), [r0m, rr])

    def kr(rr):
        return mp.quad(lambda u: a_ / Dl(u), [r0m, rr])

    def Psi(t, rr, th):     # at phi = 0; phi-dependence exp(i m phi)
        return mp.exp(1j * m * kr(rr)) * rr ** (-q) * Fm(t, xr(rr), th)

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
    # eq. teuk0 with d_phi -> i m
    op = (-((r0m**2 + a_**2) ** 2 / D0 - a_**2 * sn**2) * P_tt
          - 4 * M * a_ * r0m / D0 * (I * m) * P_t
          - 2 * s * (r0m - M * (r0m**2 - a_**2) / D0 + I * a_ * cs) * P_t
          + radial
          + (1 / sn) * (cs * P_th + sn * P_thth)
          + (1 / sn**2 - a_**2 / D0) * (-m * m) * P
          + 2 * s * (a_ * (r0m - M) / D0 + I * cs / sn**2) * (I * m) * P
          - (s**2 * cs**2 / sn**2 - s) * P)
    Sig2 = (r0m**2 + a_**2) ** 2 - a_**2 * D0 * sn**2
    lhs = op / (mp.exp(1j * m * kr(r0m)) * r0m ** (-q)) / (Sig2 / D0)

    # right-hand side from the derived coefficients, F derivatives in closed form
    x0 = mp.mpf(0)   # x(r0) = 0 by construction
    F = Fm(t0m, x0, th)
    F_t, F_tt = al * F, al * al * F
    gx = kap - mp.mpf("0.02") * x0
    F_x = gx * F
    F_xx = (gx * gx - mp.mpf("0.02")) * F
    ang = 1 + mp.mpf("0.4") * cs + mp.mpf("0.2") * sn**2
    F_th = F / ang * (-mp.mpf("0.4") * sn + mp.mpf("0.4") * sn * cs)
    F_thth = F / ang * (-mp.mpf("0.4") * cs + mp.mpf("0.4") * (cs * cs - sn * sn))
    c = C.second_order_coefficients(np.array(float(r0)), np.array(float(D0)), np.array(float(th0)),
                                    1.0, a, s, m)
    cv = {k: complex(v) for k, v in c.items()}
    rhs = (-F_tt + cv["Axx"] * F_xx + cv["Ath"] * F_thth + cv["Bt"] * F_t + cv["Bx"] * F_x
           + cv["Bth"] * F_th + cv["C"] * F)
    scale = max(abs(F_tt), abs(cv["Axx"] * F_xx), abs(cv["C"] * F), abs(cv["Bt"] * F_t), 1e-30)
    return complex(lhs), complex(rhs), float(scale)


@pytest.mark.parametrize("a,s,m", [(0.0, -2, 2), (0.5, 0, 1), (0.999, -2, 2), (1.0, -2, 0),
                                   (0.7, 1, -1), (0.999, 0, 4), (1.0, -2, 3)])
def test_bl_operator_identity(a, s, m):
    rp, _ = C.horizons(1.0, a)
    for r0, th0 in ((rp + 0.3, 0.4), (6.0, 2.1)):
        lhs, rhs, scale = _bl_check(a, s, m, r0, th0)
        assert abs(lhs - rhs) < 1e-9 * scale, (lhs, rhs, scale)


# ----------------------------------------------------------------------------- static solutions
def _static_phi(kind, r, th, M=1.0):
    """Phi = r Psi (s = 0: q = 1) and its r, theta derivatives for a static Psi."""
    if kind == "const":
        return r + 0 * th, 1.0 + 0 * th, 0 * th + 0 * r, 0 * r * th, 0 * r * th
    # Psi = (r - M) cos(theta):  Phi = r (r - M) cos(theta)
    cs, sn = np.cos(th), np.sin(th)
    return r * (r - M) * cs, (2 * r - M) * cs, 2 * cs + 0 * r, -r * (r - M) * sn, -r * (r - M) * cs


@pytest.mark.parametrize("a", [0.3, 0.999, 1.0])
@pytest.mark.parametrize("kind", ["const", "dipole"])
def test_static_solutions_continuum(a, kind):
    M = 1.0
    x = np.linspace(-30, 60, 37)
    r, y, D = C.r_of_tortoise(x, M, a)
    r, D = r[None, :], D[None, :]
    th = np.array([0.3, 1.3, 2.6])[:, None]
    Phi, Pr, Prr, Pth, Pthth = _static_phi(kind, r, th)
    h = D / (r * r + a * a)                                   # dx/dr inverse
    hp = (2 * (r - M) * (r * r + a * a) - 2 * r * D) / (r * r + a * a) ** 2
    Px = h * Pr
    Pxx = h * (hp * Pr + h * Prr)
    c = C.second_order_coefficients(r, D, th, M, a, 0, 0)
    res = c["Axx"] * Pxx + c["Ath"] * Pthth + c["Bx"] * Px + c["Bth"] * Pth + c["C"] * Phi
    scale = np.abs(c["Axx"] * Pxx) + np.abs(c["C"] * Phi) + np.abs(c["Bx"] * Px) + 1e-300
    assert np.max(np.abs(res) / scale) < 1e-12


@pytest.mark.parametrize("a", [0.5, 1.0])
def test_static_solution_discrete_rhs_converges(a):
    # Psi = 1, s = m = 0: Phi = r(x), pi = b d_x Phi; F -> 0 at fifth order in dx.
    errs = []
    for nr in (201, 401, 801):
        prob = S.Problem(s=0, m=0, a=a, nr=nr, nth=4, x_min=-10.0, x_max=30.0)
        o = S.TeukOracle(prob)
        x = prob.x()
        r = o.r
        drdx = o.Delta / (r * r + a * a)
        u = np.zeros((4, prob.nth, nr))
        u[0] = r[None, :]
        u[2] = o.tab["lam1"] * drdx[None, :]
        F = o.rhs(u)
        interior = (x > -5) & (x < 25)
        errs.append(np.max(np.abs(F[:, :, interior])))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 4.5), (errs, orders)


# ----------------------------------------------------------------------------- spin-weighted harmonics
def _goldberg(s, l, m):
    """_sY_lm(theta) up to normalisation and the e^{i m phi} factor (Goldberg et al. 1967)."""
    th = sp.Symbol("theta")
    tot = 0
    for r_ in range(0, l - s + 1):
        k = r_ + s - m
        if k < 0 or k > l + s:
            continue
        tot += (sp.binomial(l - s, r_) * sp.binomial(l + s, k) * (-1) ** (l - r_ - s)
                * sp.cot(th / 2) ** (2 * r_ + s - m))
    Y = sp.sin(th / 2) ** (2 * l) * tot
    return th, Y


@pytest.mark.parametrize("s,m", [(0, 0), (0, 2), (-2, 0), (-2, 1), (-2, 2), (-2, 4)])
def test_spin_weighted_eigenvalues_continuum(s, m):
    # G = (Ath Y'' + Bth Y' + C Y)/Y must not depend on theta (separation) and
    # G_l - G_l' = -(Delta/r^4) [(l-s)(l+s+1) - (l'-s)(l'+s+1)].
    M = 1.0
    r = np.array([[2.5, 4.0, 12.0]])
    D = r * (r - 2 * M)
    ls = [l for l in range(max(abs(s), abs(m)), max(abs(s), abs(m)) + 3)]
    thv = np.array([0.35, 0.9, 1.7, 2.5])[:, None]
    c = C.second_order_coefficients(r, D, thv, M, 0.0, s, m)
    G = {}
    for l in ls:
        th, Y = _goldberg(s, l, m)
        f0, f1, f2 = (sp.lambdify(th, e, "numpy") for e in (Y, sp.diff(Y, th), sp.diff(Y, th, 2)))
        Yv, Y1, Y2 = f0(thv), f1(thv), f2(thv)
        g = (c["Ath"] * Y2 + c["Bth"] * Y1 + c["C"] * Yv) / Yv
        assert np.max(np.abs(g - g[0:1])) < 1e-10 * np.max(np.abs(g))      # separation
        G[l] = g[0]
    lam = lambda l: (l - s) * (l + s + 1)
    for l in ls[1:]:
        want = -(D / r**4)[0] * (lam(l) - lam(ls[0]))
        np.testing.assert_allclose((G[l] - G[ls[0]]).real, want, rtol=1e-10)


@pytest.mark.parametrize("s,m,pole", [(-2, 2, 0), (2, -2, 0), (-1, 1, 0), (-2, -2, 1), (2, 2, 1)])
def test_angular_potential_accurate_at_the_pole(s, m, pole):
    # For m = -s (theta -> 0) or m = s (theta -> pi) the angular potential
    # (m + s cos)^2 / sin^2 stays finite while eq. teuk0 assembles it from
    # O(m^2 / sin^2) pieces.  The separated operator applied to the l = |s|
    # harmonic must give the same G as in the interior to ~1e-12 at 2e-3 and
    # 1e-2 from the pole (harmonic derivatives in 40-digit arithmetic).
    M = 1.0
    l = max(abs(s), abs(m))
    r = np.array([[2.5, 4.0, 12.0]])
    D = r * (r - 2 * M)
    near = np.array([0.002, 0.01]) if pole == 0 else np.pi - np.array([0.002, 0.01])
    thv = np.concatenate([[1.1], near])[:, None]
    c = C.second_order_coefficients(r, D, thv, M, 0.0, s, m)
    th, Y = _goldberg(s, l, m)
    mp.mp.dps = 40
    Yd = [sp.lambdify(th, e, "mpmath") for e in (Y, sp.diff(Y, th), sp.diff(Y, th, 2))]
    vals = np.array([[complex(f(mp.mpf(float(t)))) for f in Yd] for t in thv[:, 0]])
    Yv, Y1, Y2 = (vals[:, i][:, None] for i in range(3))
    g = (c["Ath"] * Y2 + c["Bth"] * Y1 + c["C"] * Yv) / Yv
    assert np.max(np.abs(g - g[0:1])) < 2e-12 * np.max(np.abs(g)), np.abs(g - g[0:1])


@pytest.mark.parametrize("s,m,l", [(0, 0, 2), (-2, 2, 2), (-2, 1, 3), (-2, 0, 2), (0, 1, 1), (-2, 3, 3)])
def test_spin_weighted_discrete_theta_operator(s, m, l):
    # Oracle RHS on Phi = g(x) Y(theta), pi = 0 at a = 0: F_pi = g (Ath D2 + Bth D1 + C) Y.
    # Against the continuum value the error is second order away from the poles;
    # at the pole rows the cot(theta) term leaves O(dtheta) for fields odd about the
    # pole, so there the bar is first order.  A wrong (-1)^(m+s) ghost does not
    # converge at all at the pole rows.
    th_s, Y = _goldberg(s, l, m)
    fY, f1, f2 = (sp.lambdify(th_s, e, "numpy") for e in (Y, sp.diff(Y, th_s), sp.diff(Y, th_s, 2)))
    e_in, e_all = [], []
    for nth in (16, 32, 64, 128):
        prob = S.Problem(s=s, m=m, a=0.0, nr=64, nth=nth, x_min=0.0, x_max=20.0)
        o = S.TeukOracle(prob)
        th = prob.theta()
        g = np.exp(-((prob.x() - 10.0) / 3.0) ** 2)
        u = np.zeros((4, nth, prob.nr))
        u[0] = fY(th)[:, None] * g[None, :]
        F = o.rhs(u)
        t = o.tab
        want = (t["ath"] * f2(th)[:, None] + t["bth"] * f1(th)[:, None] + t["cr"] * fY(th)[:, None]) * g
        scale = np.max(np.abs(want))
        err = np.abs(F[2] - want) / scale
        inner = (th > 0.4) & (th < np.pi - 0.4)
        e_in.append(err[inner].max())
        e_all.append(err.max())
        assert np.max(np.abs(F[3])) < 1e-12 * scale
    o_in = np.log2(np.array(e_in[:-1]) / np.array(e_in[1:]))
    o_all = np.log2(np.array(e_all[:-1]) / np.array(e_all[1:]))
    assert np.all(o_in > 1.6) and np.all(o_in[1:] > 1.8), (e_in, o_in)
    assert np.all(o_all > 0.9), (e_all, o_all)


@pytest.mark.parametrize("s,m,l", [(0, 0, 2), (-2, 2, 2), (-2, 2, 3)])
def test_wrong_pole_parity_does_not_converge(s, m, l):
    # The same check with the ghost sign flipped (planted in the oracle's input)
    # must fail to converge at the pole rows: this is what the check above guards.
    # On the cell-centred grid the ghost enters the first row of
    # d_thth + cot d_th with weight 1/h^2 - cot(h/2)/(2h) = 1/12 + O(h^2), so its
    # sign matters at leading order only where the field is nonzero on the pole
    # (m + s = 0 at theta = 0, m - s = 0 at theta = pi).
    th_s, Y = _goldberg(s, l, m)
    fY, f1, f2 = (sp.lambdify(th_s, e, "numpy") for e in (Y, sp.diff(Y, th_s), sp.diff(Y, th_s, 2)))
    errs = []
    for nth in (32, 64, 128):
        prob = S.Problem(s=s, m=m, a=0.0, nr=64, nth=nth, x_min=0.0, x_max=20.0)
        o = S.TeukOracle(prob)
        o._s.parity = -o._s.parity
        th = prob.theta()
        g = np.exp(-((prob.x() - 10.0) / 3.0) ** 2)
        u = np.zeros((4, nth, prob.nr))
        u[0] = fY(th)[:, None] * g[None, :]
        F = o.rhs(u)
        t = o.tab
        want = (t["ath"] * f2(th)[:, None] + t["bth"] * f1(th)[:, None] + t["cr"] * fY(th)[:, None]) * g
        errs.append(np.max(np.abs(F[2] - want)) / np.max(np.abs(want)))
    assert errs[-1] > 0.5 * errs[0], errs
