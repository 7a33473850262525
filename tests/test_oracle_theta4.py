"""Oracle pins for the fourth-order theta differences (theta_order = 4).

Sec. 3.1 takes centred differences in theta without stating their order; the
oracle builds second order by default and, as an option, the fourth-order
centred stencils

    D1 u = (-u_{k+2} + 8 u_{k+1} - 8 u_{k-1} + u_{k-2}) / (12 dth),
    D2 u = (-u_{k+2} + 16 u_{k+1} - 30 u_k + 16 u_{k-1} - u_{k-2}) / (12 dth^2),

with two ghost rows per pole, each (-1)^(m+s) times the row mirrored across
the pole.  Pinned here against what the mathematics fixes:

* exactness: D1 and D2 of a quartic in theta are its derivatives at every row
  whose stencil stays inside the grid (second order is not exact there);
* the separated angular operator A~thth D2 + B~th D1 + C~ on spin-weighted
  harmonics (Goldberg's closed form) converges at fourth order away from the
  poles and at third order on the pole rows, where cot(theta) ~ 2/dth
  multiplies the O(dth^4) error of D1 for fields odd about the pole.  Replacing
  the second ghost row's mirror (row 1) by row 0 leaves an O(1) error at the
  pole rows (measured: the error stops converging), so this check guards the
  two-row mirror; a flipped pole parity fails it the same way;
* a whole evolution converges at fourth order in dth on nested cell-centred
  grids (nth = 6, 18, 54 share every third row), with the same radial grid and
  time step for all three, while the second-order option converges at second;
* the time-step bound's constants are the largest moduli of the stencils'
  Fourier symbols, found here by brute force over the wavenumbers.
"""
import numpy as np
import pytest
import sympy as sp

import workloads as W
from oracle import solver as S
from test_oracle_coefficients import _goldberg


def test_symbol_maxima_brute_force():
    xi = np.linspace(0.0, np.pi, 400001)
    for order, d2, d1 in ((2, 2.0 * np.cos(xi) - 2.0, np.sin(xi)),
                          (4, (-2.0 * np.cos(2 * xi) + 32.0 * np.cos(xi) - 30.0) / 12.0,
                           (8.0 * np.sin(xi) - np.sin(2 * xi)) / 6.0)):
        c2, c1 = S.theta_symbol_maxima(order)
        assert abs(c2 - np.max(np.abs(d2))) < 1e-12, order
        assert abs(c1 - np.max(np.abs(d1))) < 1e-9, order


def _theta_part(prob, Y, dY, d2Y):
    """F_pi of the oracle on Phi = Y(theta) (constant in x), pi = 0, and the
    continuum value A~thth Y'' + B~th Y' + C~ Y (a = 0: m3 vanishes)."""
    o = S.TeukOracle(prob)
    th = prob.theta()
    u = np.zeros((4, prob.nth, prob.nr))
    u[0] = Y(th)[:, None]
    F = o.rhs(u)
    t = o.tab
    want = t["ath"] * d2Y(th)[:, None] + t["bth"] * dY(th)[:, None] + t["cr"] * Y(th)[:, None]
    return F, want


def test_exact_on_quartics():
    c = np.array([1.0, 0.3, -0.7, 0.25, -0.05])
    Y = lambda t: np.polyval(c[::-1], t)
    dY = lambda t: np.polyval(np.polyder(c[::-1]), t)
    d2Y = lambda t: np.polyval(np.polyder(c[::-1], 2), t)
    for nth in (12, 40):
        errs = {}
        for order in (2, 4):
            prob = S.Problem(s=0, m=0, a=0.0, nr=16, nth=nth, x_min=0.0, x_max=20.0, theta_order=order)
            F, want = _theta_part(prob, Y, dY, d2Y)
            inner = slice(2, nth - 2)
            errs[order] = np.max(np.abs(F[2][inner] - want[inner])) / np.max(np.abs(want[inner]))
            assert np.max(np.abs(F[3])) == 0.0
        assert errs[4] < 1e-11, (nth, errs)
        assert errs[2] > 1e-5, (nth, errs)


def _operator_errors(s, m, l, parity_flip=False):
    th_s, Ys = _goldberg(s, l, m)
    fY, f1, f2 = (sp.lambdify(th_s, e, "numpy") for e in (Ys, sp.diff(Ys, th_s), sp.diff(Ys, th_s, 2)))
    e_in, e_all = [], []
    for nth in (16, 32, 64, 128):
        prob = S.Problem(s=s, m=m, a=0.0, nr=32, nth=nth, x_min=0.0, x_max=20.0, theta_order=4)
        o = S.TeukOracle(prob)
        if parity_flip:
            o._s.parity = -o._s.parity
        th = prob.theta()
        u = np.zeros((4, nth, prob.nr))
        u[0] = fY(th)[:, None]
        F = o.rhs(u)
        t = o.tab
        want = t["ath"] * f2(th)[:, None] + t["bth"] * f1(th)[:, None] + t["cr"] * fY(th)[:, None]
        err = np.abs(F[2] - want) / np.max(np.abs(want))
        inner = (th > 0.4) & (th < np.pi - 0.4)
        e_in.append(err[inner].max())
        e_all.append(err.max())
    return np.array(e_in), np.array(e_all)


@pytest.mark.parametrize("s,m,l", [(0, 0, 2), (-2, 2, 2), (-2, 1, 3), (-2, 0, 2), (0, 1, 1), (-2, 3, 3)])
def test_spin_weighted_operator_fourth_order(s, m, l):
    e_in, e_all = _operator_errors(s, m, l)
    o_in = np.log2(e_in[:-1] / e_in[1:])
    o_all = np.log2(e_all[:-1] / e_all[1:])
    assert np.all(o_in > 3.6) and np.all(o_in[1:] > 3.8), (e_in, o_in)
    assert np.all(o_all > 2.8), (e_all, o_all)


@pytest.mark.parametrize("s,m,l", [(0, 0, 2), (-2, 2, 2)])
def test_wrong_pole_parity_fails_at_fourth_order(s, m, l):
    # the parity sign planted in the oracle's input: no convergence on the pole rows
    _, e_all = _operator_errors(s, m, l, parity_flip=True)
    assert e_all[-1] > 0.5 * e_all[0], e_all


def _nested_evolution_order(order, s, m, a, T=6.0):
    nths = (6, 18, 54)
    probs = {n: S.Problem(s=s, m=m, a=a, nr=121, nth=n, x_min=-20.0, x_max=40.0, theta_order=order)
             for n in nths}
    dt = min(S.TeukOracle(p).dt_bound(0.5) for p in probs.values())
    nsteps = int(np.ceil(T / dt))
    dt = T / nsteps
    out = {}
    for n, p in probs.items():
        wl = W.C1.with_(s=s, m=m, a=a, nr=121, nth=n, x_min=-20.0, x_max=40.0, angular="lowest", seed=7)
        out[n], _ = S.TeukOracle(p).evolve(W.gaussian_pulse(wl), dt, nsteps)
    ref = out[54][:, 4::9, :]                  # the rows of the nth = 6 grid
    e_c = np.max(np.abs(out[6] - ref))
    e_f = np.max(np.abs(out[18][:, 1::3, :] - ref))
    return np.log(e_c / e_f) / np.log(3.0)


@pytest.mark.parametrize("s,m,a", [(-2, 2, 0.7), (0, 0, 0.5)])
def test_evolution_converges_at_the_theta_order(s, m, a):
    S.set_threads(4)
    p4 = _nested_evolution_order(4, s, m, a)
    p2 = _nested_evolution_order(2, s, m, a)
    assert 3.6 < p4 < 4.4, p4
    assert 1.8 < p2 < 2.4, p2
