"""Pins of the oracle's SSP-RK(3,3) step (paper Sec. 3.2): on u' = lambda u the
Shu-Osher stages must reproduce the third-order Taylor amplification factor
R(z) = 1 + z + z^2/2 + z^3/6 exactly (up to rounding)."""
import numpy as np
import pytest

from oracle import solver as S


def R(z):
    return 1 + z + z * z / 2 + z**3 / 6


@pytest.mark.parametrize("lam", [-1.0, -3.7, 0.5, 2.0])
def test_real_amplification(lam):
    dt = 0.3
    u0 = np.array([1.0, -2.0, 0.25])
    u1 = S.ssprk3_step(u0, dt, lambda u: lam * u)
    np.testing.assert_allclose(u1, R(lam * dt) * u0, rtol=1e-14)


def test_imaginary_axis_amplification():
    # u = (x, y), u' = omega (-y, x): eigenvalues +- i omega.
    om, dt = 1.3, 0.4
    u0 = np.array([0.7, -0.2])
    u1 = S.ssprk3_step(u0, dt, lambda u: om * np.array([-u[1], u[0]]))
    z = R(1j * om * dt) * (u0[0] + 1j * u0[1])
    np.testing.assert_allclose(u1, [z.real, z.imag], rtol=1e-14)


def test_order_three_on_nonlinear_ode():
    # u' = -u^2, u(0) = 1  ->  u(T) = 1/(1+T); global error O(dt^3).
    errs = []
    for n in (10, 20, 40, 80):
        dt = 1.0 / n
        u = np.array([1.0])
        for _ in range(n):
            u = S.ssprk3_step(u, dt, lambda v: -v * v)
        errs.append(abs(u[0] - 0.5))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(orders - 3.0) < 0.15), orders
