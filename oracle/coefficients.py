"""Oracle: coefficients of the first-order Teukolsky system, derived symbolically.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module;
only the tests, the smoke check and the CPU-baseline leg of the benchmark do.

What is derived here (paper Sec. 2.1-2.3):

* The Boyer-Lindquist Teukolsky master equation (eq. teuk0) is applied to the
  field ansatz

      Psi(t, r, theta, phi) = exp(i m phi~) r^-(2s+1) Phi(t, x, theta),
      phi~ = phi + k(r),  k'(r) = a / Delta,   x = r_*(r),  dx/dr = (r^2+a^2)/Delta,

  i.e. the ingoing-Kerr azimuth of Sec. 2.2 and the tortoise coordinate r_* as
  the radial chart ("chart T": the (r_*, theta) grid).  The factor r^-(2s+1)
  makes Phi O(1) at large r for outgoing radiation.
* The coefficients of Phi_tt, Phi_t, Phi_xx, Phi_x, Phi_thth, Phi_th, Phi are
  collected and divided by minus the Phi_tt coefficient, which is the step that
  turns eq. near_final into eq. final (Sec. 2.3).  In chart T there is no
  Phi_tx term (A~^{tx} = 0).
* The first-order reduction of Sec. 2.3 (pi = Phi_t + b Phi_x, eq. evln with
  the matrices M, A, L) is then taken in the general form

      b      = (-A~tx + sqrt(A~tx^2 + 4 A~xx)) / 2        (speed of the Phi rows)
      lam2   = -(A~tx + b)                               (speed of the pi rows)
      m3     = (A~tx + b) d_x b + b B~t - B~x            (complex; m31 = Re m3, m32 = -Im m3)

  which with A~tx = 0 gives lam2 = -b, the diagonal of the paper's M.  The
  root with b > 0 is taken because the paper upwinds the first two rows as a
  positive-speed flux (Sec. 3.1.2); the printed root differs only in sign
  and gives an equally exact reduction (see the design notes' reading list).

Delta = r^2 - 2Mr + a^2 is carried as an independent symbol and supplied
numerically from an accurate value (Delta = y (r - r_-), y = r - r_+), because
forming it from r loses every digit near the horizon.
"""
from __future__ import annotations

import functools

import numpy as np
import sympy as sp

# ----------------------------------------------------------------------------- symbols
r = sp.Symbol("r", positive=True)
cth, sth = sp.symbols("cth sth", real=True)        # cos(theta), sin(theta)
Mb, ab = sp.symbols("M a", nonnegative=True)
sb, mb = sp.symbols("s m", integer=True)
Dl = sp.Symbol("Delta", positive=True)              # Delta, kept symbolic
DlP = 2 * (r - Mb)                                  # dDelta/dr

# Phi and its partial derivatives in (t, x, theta), as plain symbols
F, Ft, Ftt, Fx, Fxx, Fth, Fthth = sp.symbols("F F_t F_tt F_x F_xx F_th F_thth")


def d_dr(expr):
    """Total r-derivative of an expression in (r, Delta): d/dr = d_r + Delta' d_Delta."""
    return sp.diff(expr, r) + DlP * sp.diff(expr, Dl)


@functools.lru_cache(maxsize=None)
def _chart_T_symbolic():
    """Divided second-order coefficients in chart T, as sympy expressions.

    Returns a dict with keys Axx, Ath, Bt, Bx, Bth, C (eq. final with
    tau -> t, rho -> x = r_*), each an expression in r, Delta, cth, sth and the
    parameters M, a, s, m.
    """
    I = sp.I
    q = 2 * sb + 1
    # E(r) = exp(i m k(r)) r^-q ;  g = E'/E
    g = I * mb * ab / Dl - q / r
    gp = d_dr(g)
    xp = (r**2 + ab**2) / Dl                         # dx/dr
    xpp = d_dr(xp)

    # Partials of Psi, each divided by exp(i m phi~) E(r).  phi-derivatives act
    # as i m because phi~ - phi depends on r only.
    Psi = F
    Psi_t, Psi_tt = Ft, Ftt
    Psi_r = g * F + xp * Fx
    Psi_rr = (gp + g**2) * F + (2 * g * xp + xpp) * Fx + xp**2 * Fxx
    Psi_th, Psi_thth = Fth, Fthth
    Psi_ph = I * mb * F
    Psi_phph = -mb**2 * F
    Psi_tph = I * mb * Ft

    # eq. teuk0, term by term.  Delta^-s d_r(Delta^(s+1) d_r Psi) is written out
    # by the product rule as Delta Psi_rr + (s+1) Delta' Psi_r, and
    # (1/sin) d_th(sin d_th Psi) as Psi_thth + cot Psi_th.
    op = (
        -((r**2 + ab**2) ** 2 / Dl - ab**2 * sth**2) * Psi_tt
        - 4 * Mb * ab * r / Dl * Psi_tph
        - 2 * sb * (r - Mb * (r**2 - ab**2) / Dl + I * ab * cth) * Psi_t
        + Dl * Psi_rr + (sb + 1) * DlP * Psi_r
        + Psi_thth + cth / sth * Psi_th
        + (1 / sth**2 - ab**2 / Dl) * Psi_phph
        + 2 * sb * (ab * (r - Mb) / Dl + I * cth / sth**2) * Psi_ph
        - (sb**2 * cth**2 / sth**2 - sb) * Psi
    )
    # Multiplying by Delta^2 clears every 1/Delta, so that each coefficient below
    # is a ratio of polynomials in Delta and stays finite for Delta down to the
    # smallest normal double (no 1/Delta^2 overflow deep in the horizon region).
    op = sp.expand(op * Dl**2)
    coef = {sym: op.coeff(sym) for sym in (Ftt, Ft, Fxx, Fx, Fthth, Fth, F)}
    norm = -coef[Ftt]                                  # -A^tt Delta^2
    out = {
        "Axx": coef[Fxx] / norm,
        "Ath": coef[Fthth] / norm,
        "Bt": coef[Ft] / norm,
        "Bx": coef[Fx] / norm,
        "Bth": coef[Fth] / norm,
        "C": coef[F] / norm,
    }
    return out


@functools.lru_cache(maxsize=None)
def _chart_T_reduction_symbolic():
    """First-order reduction (Sec. 2.3) of the chart-T equation, symbolically.

    Returns expressions for lam1 = b, lam2, m3 (complex) plus the pass-through
    coefficients Bt, C, Ath, Bth.
    """
    c = _chart_T_symbolic()
    Atx = sp.Integer(0)                                # no Phi_tx term in chart T
    b = (-Atx + sp.sqrt(Atx**2 + 4 * c["Axx"])) / 2
    d_dx = lambda e: Dl / (r**2 + ab**2) * d_dr(e)   # d/dx at fixed t, theta
    lam2 = -(Atx + b)
    m3 = (Atx + b) * d_dx(b) + b * c["Bt"] - c["Bx"]
    return {"lam1": b, "lam2": lam2, "m3": m3, "Bt": c["Bt"], "C": c["C"],
            "Ath": c["Ath"], "Bth": c["Bth"], "Axx": c["Axx"], "Bx": c["Bx"]}


@functools.lru_cache(maxsize=None)
def _lambdified(kind: str):
    exprs = _chart_T_symbolic() if kind == "second_order" else _chart_T_reduction_symbolic()
    args = (r, Dl, cth, sth, Mb, ab, sb, mb)
    return {k: sp.lambdify(args, v, modules="numpy") for k, v in exprs.items()}


def _eval(fn, rr, Dd, th, M, a, s, m):
    """Evaluate a lambdified coefficient in x87 extended precision, then round.

    The expressions keep eq. teuk0's terms as printed; its three angular terms
    (1/sin^2 d_phph, 2 i s cos/sin^2 d_ph, -s^2 cot^2) combine into
    -(m + s cos)^2 / sin^2, which for m = -s (or m = s) nearly vanishes at the
    pole and is formed from O(m^2/sin^2) pieces.  Evaluating in long double
    (64-bit significand) and rounding once makes the FP64 tables accurate to
    about an ulp there as well.
    """
    ld = np.longdouble
    rr, Dd, th = (np.asarray(v, dtype=ld) for v in (rr, Dd, th))
    val = fn(rr, Dd, np.cos(th), np.sin(th), ld(M), ld(a), int(s), int(m))
    val = np.asarray(val)
    return np.broadcast_to(val.astype(np.complex128), np.broadcast(rr, th).shape).copy()


def second_order_coefficients(r_, Delta_, theta_, M, a, s, m):
    """Coefficients of eq. final in chart T at points (r, Delta, theta).

    r_, Delta_ and theta_ broadcast against each other.  Returns complex
    arrays Axx, Ath, Bt, Bx, Bth, C.
    """
    fns = _lambdified("second_order")
    return {k: _eval(f, r_, Delta_, theta_, M, a, s, m) for k, f in fns.items()}


def first_order_coefficients(r_, Delta_, theta_, M, a, s, m):
    """Per-point coefficients of the first-order system (eq. evln) in chart T.

    Returns real arrays lam1, lam2, Ath, Bth and complex arrays m3, Bt, C:

        d_t Phi = pi - lam1 d_x Phi
        d_t pi  = -lam2 d_x pi - m3 d_x Phi + Bt pi + Ath Phi_thth + Bth Phi_th + C Phi
    """
    fns = _lambdified("first_order")
    out = {}
    for k, f in fns.items():
        v = _eval(f, r_, Delta_, theta_, M, a, s, m)
        out[k] = v.real.copy() if k in ("lam1", "lam2", "Ath", "Bth", "Axx") else v
    return out


# ----------------------------------------------------------------------------- background
def horizons(M, a):
    """Outer and inner horizon radii r_+- = M +- sqrt(M^2 - a^2)."""
    d = np.sqrt(max(M * M - a * a, 0.0))
    return M + d, M - d


def tortoise_of_y(y, M, a):
    """r_*(r) with y = r - r_+ (Sec. 2.2: r_* = int (r^2+a^2)/Delta dr).

    The integration constant is fixed by the closed forms
      a < M:  r_* = r + 2M r+/(r+ - r-) ln((r - r+)/2M) - 2M r-/(r+ - r-) ln((r - r-)/2M)
      a = M:  r_* = r + 2M ln((r - M)/M) - 2M^2/(r - M)
    """
    rp, rm = horizons(M, a)
    rr = rp + y
    if rp - rm > 0:
        return (rr + 2 * M * rp / (rp - rm) * np.log(y / (2 * M))
                - 2 * M * rm / (rp - rm) * np.log((rr - rm) / (2 * M)))
    return rr + 2 * M * np.log(y / M) - 2 * M * M / y


def r_of_tortoise(x, M, a, iters=90):
    """Invert r_*(r) = x by bisection in u = ln(r - r_+).

    r_* is strictly increasing in u, so bisection on a bracket that covers every
    representable y is slow but cannot fail.  Returns (r, y, Delta) with
    Delta = y (r - r_-) formed without cancellation.
    """
    x = np.asarray(x, dtype=np.float64)
    lo = np.full_like(x, -700.0)
    hi = np.full_like(x, np.log(np.abs(x).max() + 100.0 * M + 10.0))
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        above = tortoise_of_y(np.exp(mid), M, a) > x
        hi = np.where(above, mid, hi)
        lo = np.where(above, lo, mid)
    y = np.exp(0.5 * (lo + hi))
    rp, rm = horizons(M, a)
    rr = rp + y
    Delta = y * (rr - rm)
    return rr, y, Delta


def kerr_k_of_y(y, M, a):
    """phi~ - phi = k(r), k' = a/Delta (used only to interpret Phi)."""
    rp, rm = horizons(M, a)
    if rp - rm > 0:
        return a / (rp - rm) * np.log(y / (y + rp - rm))
    return -a / y
