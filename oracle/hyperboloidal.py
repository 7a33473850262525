"""Oracle: the first-order Teukolsky system in the hyperboloidal chart.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module;
only the tests, the smoke check and the CPU-baseline leg of the benchmark do.

Chart H (paper Sec. 2.2): ingoing-Kerr time t~ = t - r + r_* and azimuth
phi~ = phi + k(r) (k' = a/Delta), then the hyperboloidal time and compactified
radius

    tau = t~ - r^2/(r+S) + 4M ln(S/(r+S)),     rho = r / (1 + r/S),

so that rho in [0, S) covers r in [0, oo) and t = tau - H(r) with

    H(r) = r_* - r - r^2/(r+S) + 4M ln(S/(r+S)).

(The paper writes "4 ln" in units M = 1.)  The field ansatz is

    Psi(t, r, theta, phi) = exp(i m phi~) r^-1 Delta^-s Phi(tau, rho, theta),

which for s = -2 is the paper's Phi = (r / Delta^2) Psi of Sec. 4.

What is computed:

* eq. teuk0 is applied to the ansatz by the chain rule (d_t = d_tau,
  d_r|_t = H' d_tau + rho' d_rho, d_phi = i m); the coefficients of
  Phi_tautau, Phi_taurho, Phi_rhorho, Phi_thth, Phi_tau, Phi_rho, Phi_th and Phi
  are those of eq. near_final.  The theta-dependent terms of eq. teuk0 pass
  through the radial change of variables untouched, so each coefficient is a
  radial expression (derived symbolically here, evaluated per radial node in
  50-digit arithmetic) plus the printed angular terms.
* They are divided by -A^tautau (eq. final) and reduced to first order as in
  Sec. 2.3 with the printed root

      b = -(A~trho + sqrt(A~trho^2 + 4 A~rhorho)) / 2,

  giving the speeds lam1 = b (Phi rows) and lam2 = -(A~trho + b) (pi rows) and
  m3 = (A~trho + b) d_rho b + b B~tau - B~rho.  Each row is then upwinded by the
  sign of its own speed at the point (Sec. 3.1.2).

Everything per point is done in mpmath (50 digits, more for nodes a hair from
the horizon, where the chain rule's 1/Delta^2 terms cancel) and rounded once to
FP64.  A node exactly on the horizon (Delta = 0) is refused: the divided
coefficients are 0/0 there as written; they are regular, and the library's
closed forms are, but the oracle keeps the printed construction.
"""
from __future__ import annotations

import functools

import mpmath as mp
import numpy as np
import sympy as sp

from .coefficients import Dl, DlP, Mb, ab, d_dr, mb, r, sb

Sb = sp.Symbol("S", positive=True)
F, Ft, Ftt, Fx, Fxx, Ftx = sp.symbols("F F_t F_tt F_x F_xx F_tx")

DPS = 50


@functools.lru_cache(maxsize=None)
def _radial_symbolic():
    """Radial parts of the eq. near_final coefficients in chart H.

    Returns a dict of sympy expressions in (r, Delta, M, a, s, m, S):
    Rtt, Rtx, Rxx, Rt, Rx, RF (coefficients of Phi_tautau, Phi_taurho,
    Phi_rhorho, Phi_tau, Phi_rho, Phi from the terms of eq. teuk0 without
    theta dependence) and dRtt, dRtx, dRxx (their total r-derivatives).
    """
    I = sp.I
    # E(r) = exp(i m k(r)) r^-1 Delta^-s,  g = E'/E
    g = I * mb * ab / Dl - 1 / r - sb * DlP / Dl
    gp = d_dr(g)
    rho_p = Sb**2 / (r + Sb) ** 2                      # d rho / dr
    rho_pp = sp.diff(rho_p, r)
    Hp = (r**2 + ab**2) / Dl - 1 - sp.diff(r**2 / (r + Sb), r) - 4 * Mb / (r + Sb)
    Hpp = d_dr(Hp)

    # Partials of Psi divided by exp(i m phi~) E(r), in terms of Phi's partials.
    Psi = F
    Psi_t, Psi_tt = Ft, Ftt
    Psi_r = g * F + Hp * Ft + rho_p * Fx
    Psi_rr = ((gp + g**2) * F + 2 * g * (Hp * Ft + rho_p * Fx) + Hpp * Ft + rho_pp * Fx
              + Hp**2 * Ftt + 2 * Hp * rho_p * Ftx + rho_p**2 * Fxx)
    Psi_ph = I * mb * F
    Psi_phph = -mb**2 * F
    Psi_tph = I * mb * Ft

    # eq. teuk0, the terms with no theta dependence (the angular ones are added
    # per point below, as printed): Delta^-s d_r(Delta^(s+1) d_r Psi) is written out
    # by the product rule as Delta Psi_rr + (s+1) Delta' Psi_r.
    op = (
        -((r**2 + ab**2) ** 2 / Dl) * Psi_tt
        - 4 * Mb * ab * r / Dl * Psi_tph
        - 2 * sb * (r - Mb * (r**2 - ab**2) / Dl) * Psi_t
        + Dl * Psi_rr + (sb + 1) * DlP * Psi_r
        + (-ab**2 / Dl) * Psi_phph
        + 2 * sb * (ab * (r - Mb) / Dl) * Psi_ph
    )
    out = {}
    for name, sym in (("Rtt", Ftt), ("Rtx", Ftx), ("Rxx", Fxx), ("Rt", Ft), ("Rx", Fx), ("RF", F)):
        out[name] = sp.diff(op, sym)                  # op is linear in Phi's partials
    for name in ("Rtt", "Rtx", "Rxx"):
        out["d" + name] = d_dr(out[name])
    return out


@functools.lru_cache(maxsize=None)
def _radial_fns():
    args = (r, Dl, Mb, ab, sb, mb, Sb)
    return {k: sp.lambdify(args, v, modules="mpmath") for k, v in _radial_symbolic().items()}


def horizons_mp(M, a):
    M, a = mp.mpf(M), mp.mpf(a)
    d = mp.sqrt(max(M * M - a * a, mp.mpf(0)))
    return M + d, M - d


def radial_values(rho, M, a, s, m, S):
    """Radial coefficient parts at the nodes rho (1D array of floats), in
    50-digit arithmetic: r = rho S / (S - rho), Delta = (r - r+)(r - r-)."""
    fns = _radial_fns()
    out = []
    for x in np.asarray(rho, dtype=np.float64):
        with mp.workdps(DPS):
            rp, rm = horizons_mp(M, a)
            xr = mp.mpf(float(x))
            D0 = (xr * mp.mpf(S) / (mp.mpf(S) - xr) - rp) * (xr * mp.mpf(S) / (mp.mpf(S) - xr) - rm)
        if D0 == 0:
            raise ValueError("a radial node lies exactly on the horizon (0/0 in the printed construction)")
        # the chain rule leaves terms up to 1/Delta^2 that cancel: carry enough
        # digits for nodes a hair from the horizon
        extra = int(max(0.0, -2.0 * float(mp.log10(abs(D0))))) + 5
        with mp.workdps(DPS + extra):
            Sm = mp.mpf(S)
            rp, rm = horizons_mp(M, a)
            xr = mp.mpf(float(x))
            rr = xr * Sm / (Sm - xr)
            D = (rr - rp) * (rr - rm)
            vals = {k: f(rr, D, mp.mpf(M), mp.mpf(a), int(s), int(m), Sm) for k, f in fns.items()}
            vals["r"], vals["Delta"] = rr, D
            vals["rho_p"] = Sm**2 / (rr + Sm) ** 2
            vals = {k: +v for k, v in vals.items()}
        out.append(vals)
    return out


def first_order_tables(rho, theta, M, a, s, m, S):
    """Per-point tables of the first-order system in chart H.

    Returns a dict of float64 arrays of shape [nth][nr]: lam1, lam2, m3r, m3i,
    btr, bti, cr, ci, ath, bth, with

        d_tau Phi = pi - lam1 d_rho Phi
        d_tau pi  = -lam2 d_rho pi - m3 d_rho Phi + B~tau pi + A~thth Phi_thth + B~th Phi_th + C~ Phi
    """
    rad = radial_values(rho, M, a, s, m, S)
    nth, nr = len(theta), len(rho)
    names = ("lam1", "lam2", "m3r", "m3i", "btr", "bti", "cr", "ci", "ath", "bth")
    tab = {k: np.empty((nth, nr)) for k in names}
    with mp.workdps(DPS):
        am, sm, mm = mp.mpf(a), int(s), int(m)
        for k, th in enumerate(np.asarray(theta, dtype=np.float64)):
            t = mp.mpf(float(th))
            c, sn = mp.cos(t), mp.sin(t)
            # angular terms of eq. teuk0, as printed
            att_ang = am**2 * sn**2                                   # coefficient of Phi_tautau
            bt_ang = -2 * sm * 1j * am * c                            # coefficient of Phi_tau
            cf_ang = (-(mm**2) / sn**2 + 2 * sm * (1j * c / sn**2) * (1j * mm)
                      - (sm**2 * c**2 / sn**2 - sm))                   # coefficient of Phi
            for j, v in enumerate(rad):
                Att = v["Rtt"] + att_ang
                W = -Att                                               # -A^tautau
                T = v["Rtx"] / W
                R = v["Rxx"] / W
                Wr = -v["dRtt"]
                Tr = (v["dRtx"] * W - v["Rtx"] * Wr) / W**2
                Rr = (v["dRxx"] * W - v["Rxx"] * Wr) / W**2
                q = mp.sqrt(T * T + 4 * R)
                b = -(T + q) / 2
                b_r = -(Tr + (T * Tr + 2 * Rr) / q) / 2
                b_rho = b_r / v["rho_p"]
                Bt = (v["Rt"] + bt_ang) / W
                Bx = v["Rx"] / W
                Cc = (v["RF"] + cf_ang) / W
                m3 = (T + b) * b_rho + b * Bt - Bx
                tab["lam1"][k, j] = float(mp.re(b))
                tab["lam2"][k, j] = float(mp.re(-(T + b)))
                tab["m3r"][k, j] = float(mp.re(m3))
                tab["m3i"][k, j] = float(mp.im(m3))
                tab["btr"][k, j] = float(mp.re(Bt))
                tab["bti"][k, j] = float(mp.im(Bt))
                tab["cr"][k, j] = float(mp.re(Cc))
                tab["ci"][k, j] = float(mp.im(Cc))
                tab["ath"][k, j] = float(mp.re(1 / W))
                tab["bth"][k, j] = float(mp.re(c / sn / W))
    return tab


def second_order_point(r_, theta_, M, a, s, m, S):
    """Undivided eq. near_final coefficients (complex mpf) at one point (r, theta),
    for the operator-identity checks: Att, Atx, Axx, Ath, Bt, Bx, Bth, C."""
    fns = _radial_fns()
    with mp.workdps(max(DPS, mp.mp.dps)):       # never below the caller's precision
        rr = mp.mpf(r_)
        rp, rm = horizons_mp(M, a)
        D = (rr - rp) * (rr - rm)
        v = {k: f(rr, D, mp.mpf(M), mp.mpf(a), int(s), int(m), mp.mpf(S)) for k, f in fns.items()}
        t = mp.mpf(theta_)
        c, sn = mp.cos(t), mp.sin(t)
        am, sm, mm = mp.mpf(a), int(s), int(m)
        return {
            "Att": v["Rtt"] + am**2 * sn**2,
            "Atx": v["Rtx"], "Axx": v["Rxx"], "Ath": mp.mpf(1),
            "Bt": v["Rt"] - 2 * sm * 1j * am * c, "Bx": v["Rx"], "Bth": c / sn,
            "C": v["RF"] - (mm**2) / sn**2 + 2 * sm * (1j * c / sn**2) * (1j * mm) - (sm**2 * c**2 / sn**2 - sm),
        }


def rho_of_r(r_, S):
    return r_ / (1.0 + r_ / S)


def horizon_stencil(f, nr):
    """Nodes and weights for the horizon at fractional node position f (the
    horizon sits at x_min + f dx): the four nodes j0 .. j0+3 with
    j0 = floor(f) - 1, shifted to stay inside the grid (one-sided next to its
    ends), and the 4-point Lagrange weights for the value and for the
    derivative (per unit step) at f."""
    j0 = int(np.floor(f)) - 1
    j0 = min(max(j0, 0), nr - 4)
    nodes = [float(j0 + i) for i in range(4)]
    w, dw = [], []
    for i, zi in enumerate(nodes):
        others = [z for k, z in enumerate(nodes) if k != i]
        den = np.prod([zi - z for z in others])
        w.append(np.prod([f - z for z in others]) / den)
        d = 0.0
        for k in range(3):
            d += np.prod([f - z for kk, z in enumerate(others) if kk != k])
        dw.append(d / den)
    return j0, np.array(w), np.array(dw)


def horizon_weights(xi):
    """Weights on the nodes at offsets -1, 0, 1, 2 for the value and the
    derivative at offset xi in [0, 1) (an interior horizon)."""
    j0, w, dw = horizon_stencil(1.0 + xi, 10**6)
    return w, dw
