"""Pins of the oracle's WENO5 operator (paper Sec. 3.1.2) against what the
mathematics fixes: linear weights on smooth data, the linear fifth-order limit,
exactness for quadratics with arbitrary weights that sum to one, the mirror
identity between the two sides, fifth-order convergence, conservation and the
essentially non-oscillatory property on a square wave."""
import numpy as np
import pytest

from oracle import solver as S

D_LINEAR = np.array([0.1, 0.6, 0.3])


def test_constant_data_gives_linear_weights():
    for c in (0.0, 1.0, -3.5):
        f = np.full(5, c)
        np.testing.assert_allclose(S.weno5_weights_plus(f), D_LINEAR, rtol=0, atol=1e-15)
        np.testing.assert_allclose(S.weno5_weights_minus(f), D_LINEAR, rtol=0, atol=1e-15)


def test_linear_data_gives_linear_weights():
    # f = c x: every smoothness indicator equals c^2 dx^2, so omega = d exactly.
    for c in (1.0, -2.0, 1e-3):
        f = c * np.arange(-2.0, 3.0)
        np.testing.assert_allclose(S.weno5_weights_plus(f), D_LINEAR, rtol=0, atol=2e-15)
        np.testing.assert_allclose(S.weno5_weights_minus(f), D_LINEAR, rtol=0, atol=2e-15)


def test_large_eps_gives_linear_fifth_order_flux():
    # eps -> infinity forces omega = d: f^+ = (2, -13, 47, 27, -3)/60 on j-2..j+2.
    rng = np.random.default_rng(0)
    for _ in range(20):
        f = rng.standard_normal(5)
        want = np.dot([2, -13, 47, 27, -3], f) / 60.0
        assert S.weno5_flux_plus(f, eps=1e150) == pytest.approx(want, abs=1e-14)
        # mirrored for f^-: (−3, 27, 47, −13, 2)/60 on j-1..j+3
        want_m = np.dot([-3, 27, 47, -13, 2], f) / 60.0
        assert S.weno5_flux_minus(f, eps=1e150) == pytest.approx(want_m, abs=1e-14)


def test_linear_limit_derivative_is_exact_for_quintics():
    # With omega = d, D^+ = (-2, 15, -60, 20, 30, -3)/(60 dx) on j-3..j+2, exact
    # for polynomials of degree <= 5.
    dx = 0.1
    x = dx * np.arange(-3, 4)
    for p in range(6):
        f = x**p
        pad = np.concatenate([[0.0, 0.0, 0.0], f[:], [0.0, 0.0, 0.0]])  # row point j=3 is x=0
        want = p * 0.0 ** (p - 1) if p > 0 else 0.0
        dp = S.derivative(pad, 3, dx, +1, eps=1e150)
        dm = S.derivative(pad, 3, dx, -1, eps=1e150)
        assert dp == pytest.approx(want, abs=1e-9)
        assert dm == pytest.approx(want, abs=1e-9)
    # and it is not exact at degree 6 (so the order is exactly five)
    f = x**6
    pad = np.concatenate([[0.0] * 3, f, [0.0] * 3])
    assert abs(S.derivative(pad, 3, dx, +1, eps=1e150)) > 1e-8


def test_quadratics_exact_with_arbitrary_weights():
    # Every candidate stencil is exact for quadratics, so any weights summing to
    # one at j+1/2 and (independently) at j-1/2 give D f = f' exactly.
    rng = np.random.default_rng(1)
    dx = 0.37
    x = dx * np.arange(-3, 4)
    for _ in range(20):
        c0, c1, c2 = rng.standard_normal(3)
        f = c0 + c1 * x + c2 * x * x
        wp = rng.uniform(0, 1, 3)
        wp /= wp.sum()
        wm = rng.uniform(0, 1, 3)
        wm /= wm.sum()
        d = (S.weno5_combine_plus(f[1:6], wp) - S.weno5_combine_plus(f[0:5], wm)) / dx
        assert d == pytest.approx(c1, abs=1e-12)
        # a weight-sum defect delta gives an O(delta f / dx) error
        bad = wp * (1 + 1e-4)
        d_bad = (S.weno5_combine_plus(f[1:6], bad) - S.weno5_combine_plus(f[0:5], wm)) / dx
        assert abs(d_bad - c1) > 1e-6 * abs(S.weno5_combine_plus(f[1:6], wp)) / dx


def test_nonlinear_weights_on_quadratic_still_exact():
    dx = 0.05
    x = dx * np.arange(-3, 4) + 0.3
    f = 2.0 - 3.0 * x + 7.0 * x * x
    pad = np.concatenate([[0.0] * 3, f, [0.0] * 3])
    for side in (+1, -1):
        assert S.derivative(pad, 3, dx, side) == pytest.approx(-3.0 + 14.0 * 0.3, abs=1e-11)


def test_mirror_identity():
    # f^- on data reversed about j+1/2 equals f^+: weights and flux.
    rng = np.random.default_rng(2)
    for _ in range(50):
        f = rng.standard_normal(5) * rng.uniform(0.01, 10)
        assert S.weno5_flux_minus(f[::-1]) == pytest.approx(S.weno5_flux_plus(f), rel=1e-14, abs=1e-15)
        np.testing.assert_allclose(S.weno5_weights_minus(f[::-1]), S.weno5_weights_plus(f), rtol=1e-14,
                                   atol=1e-16)


def _advect(N, periods=1.0, u0fn=lambda x: np.sin(np.pi * x), speed=1.0):
    dx = 2.0 / N
    x = -1 + dx * np.arange(N)
    u0 = u0fn(x)
    dt = 0.5 * dx ** (5.0 / 3.0)
    T = 2.0 * periods
    n = int(np.ceil(T / dt))
    dt = T / n
    return x, u0, S.advect1d(u0, dx, speed, dt, n)


def test_advection_fifth_order_convergence():
    errs = []
    Ns = [40, 80, 160, 320]
    for N in Ns:
        _, u0, u = _advect(N)
        errs.append(np.mean(np.abs(u - u0)))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 4.8), (errs, orders)
    assert errs[0] < 1e-4


def test_advection_negative_speed_uses_other_side():
    N = 160
    _, u0, u = _advect(N, speed=-1.0)
    assert np.mean(np.abs(u - u0)) < 1e-7


def test_advection_conserves_sum():
    _, u0, u = _advect(160)
    assert abs(u.sum() - u0.sum()) < 1e-12


def test_square_wave_is_essentially_non_oscillatory():
    sq = lambda x: np.where(np.abs(x) < 0.5, 1.0, 0.0)
    _, u0, u = _advect(200, u0fn=sq)
    assert u.max() < 1.01
    assert u.min() > -0.01
