"""Oracle: Python driver for the plain FP64 Teukolsky solver in teuk_oracle.c.

(The binary128 build of the same source is driven by ``oracle.quad``.)

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark import this module; the product path never does.

It builds the chart-T grid (uniform in x = r_*, cell-centred in theta), the
per-point coefficient tables from the symbolic derivation in
``oracle.coefficients``, the time-step bound, and calls the C routines for the
WENO5 right-hand side and SSP-RK(3,3) steps.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

from . import coefficients as coeffs

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "teuk_oracle.c")
_LIB = os.path.join(_HERE, "_liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)


_LIBQ = os.path.join(_HERE, "_liboracle_q.so")


def _compile(out: str, defines, verbose: bool):
    cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
           *defines, "-shared", _SRC, "-o", out + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)


def build_oracle(verbose: bool = False) -> str:
    """Compile teuk_oracle.c with gcc (rounding exactly as written: no
    contraction, no fast math), once with FP64 and once with binary128 as the
    working precision.  Returns the FP64 library path."""
    _compile(_LIB, [], verbose)
    _compile(_LIBQ, ["-DORACLE_QUAD"], verbose)
    return _LIB


class _OracleTeuk(ctypes.Structure):
    _fields_ = [("nr", ctypes.c_long), ("nth", ctypes.c_long),
                ("dx", ctypes.c_double), ("dx_lo", ctypes.c_double),
                ("dth", ctypes.c_double), ("dth_lo", ctypes.c_double), ("eps", ctypes.c_double),
                ("parity", ctypes.c_double), ("wmode", ctypes.c_int), ("scheme", ctypes.c_int),
                ("ko_sigma", ctypes.c_double)] + [
                (n, ctypes.c_void_p) for n in ("lam1", "lam2", "m3r", "m3i", "btr", "bti", "cr", "ci", "ath", "bth")] + [
                ("theta_order", ctypes.c_int)]


RHS_FN = ctypes.CFUNCTYPE(None, _dp, _dp, ctypes.c_void_p)

_lib_handle = None


def lib() -> ctypes.CDLL:
    """Load the oracle library, building it first if it is not there."""
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            _compile(_LIB, [], False)
        L = ctypes.CDLL(_LIB)
        L.oracle_weno5_weights_plus.argtypes = [_dp, ctypes.c_double, _dp]
        L.oracle_weno5_weights_minus.argtypes = [_dp, ctypes.c_double, _dp]
        for fn in ("oracle_weno5_flux_plus", "oracle_weno5_flux_minus"):
            getattr(L, fn).argtypes = [_dp, ctypes.c_double]
            getattr(L, fn).restype = ctypes.c_double
        for fn in ("oracle_weno5_combine_plus", "oracle_weno5_combine_minus"):
            getattr(L, fn).argtypes = [_dp, _dp]
            getattr(L, fn).restype = ctypes.c_double
        for fn in ("oracle_dplus", "oracle_dminus"):
            getattr(L, fn).argtypes = [_dp, ctypes.c_long, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_int]
            getattr(L, fn).restype = ctypes.c_double
        L.oracle_ssprk3_step.argtypes = [_dp, ctypes.c_long, ctypes.c_double, RHS_FN, ctypes.c_void_p, _dp]
        L.oracle_ssprk104_step.argtypes = [_dp, ctypes.c_long, ctypes.c_double, RHS_FN, ctypes.c_void_p, _dp]
        L.oracle_teuk_evolve_rk.argtypes = [ctypes.POINTER(_OracleTeuk), _dp, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_long, ctypes.c_long, ctypes.c_long, _dp, ctypes.c_long,
                                            ctypes.c_int]
        L.oracle_teuk_evolve_rk.restype = ctypes.c_long
        L.oracle_advect1d.argtypes = [_dp, ctypes.c_long, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_long, ctypes.c_double,
                                      ctypes.c_int]
        L.oracle_teuk_rhs.argtypes = [ctypes.POINTER(_OracleTeuk), _dp, _dp]
        for fn in ("oracle_weno3_weights_plus", "oracle_weno3_weights_minus"):
            getattr(L, fn).argtypes = [_dp, ctypes.c_double, _dp]
        for fn in ("oracle_weno3_flux_plus", "oracle_weno3_flux_minus"):
            getattr(L, fn).argtypes = [_dp, ctypes.c_double]
            getattr(L, fn).restype = ctypes.c_double
        L.oracle_radial_d.argtypes = [_dp, ctypes.c_long, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_int]
        L.oracle_radial_d.restype = ctypes.c_double
        L.oracle_advect1d_scheme.argtypes = [_dp, ctypes.c_long, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_long, ctypes.c_double, ctypes.c_int, ctypes.c_double]
        L.oracle_teuk_evolve.argtypes = [ctypes.POINTER(_OracleTeuk), _dp, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_long, ctypes.c_long, ctypes.c_long, _dp, ctypes.c_long]
        L.oracle_teuk_evolve.restype = ctypes.c_long
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        _lib_handle = L
    return _lib_handle


def ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


# ----------------------------------------------------------------------------- 1D helpers
def weno5_weights_plus(f5, eps=1e-6):
    f = np.ascontiguousarray(f5, dtype=np.float64)
    w = np.zeros(3)
    lib().oracle_weno5_weights_plus(ptr(f), eps, ptr(w))
    return w


def weno5_weights_minus(f5, eps=1e-6):
    f = np.ascontiguousarray(f5, dtype=np.float64)
    w = np.zeros(3)
    lib().oracle_weno5_weights_minus(ptr(f), eps, ptr(w))
    return w


def weno5_flux_plus(f5, eps=1e-6):
    f = np.ascontiguousarray(f5, dtype=np.float64)
    return lib().oracle_weno5_flux_plus(ptr(f), eps)


def weno5_flux_minus(f5, eps=1e-6):
    f = np.ascontiguousarray(f5, dtype=np.float64)
    return lib().oracle_weno5_flux_minus(ptr(f), eps)


def weno5_combine_plus(f5, w):
    f = np.ascontiguousarray(f5, dtype=np.float64)
    ww = np.ascontiguousarray(w, dtype=np.float64)
    return lib().oracle_weno5_combine_plus(ptr(f), ptr(ww))


def derivative(p_padded, j, dx, side, eps=1e-6):
    """D^+ (side=+1) or D^- (side=-1) at point j of a row padded by 3 each side."""
    p = np.ascontiguousarray(p_padded, dtype=np.float64)
    base = p.ctypes.data + 3 * 8
    pp = ctypes.cast(base, _dp)
    fn = lib().oracle_dplus if side > 0 else lib().oracle_dminus
    return fn(pp, j, dx, 0.0, eps, 0)


SCHEMES = {"weno5": 0, "weno3": 1, "fd6ko8": 2}


def weno3_weights(f3, side, eps=1e-6):
    """omega_1, omega_2 of f^+_{j+1/2} (side=+1, f_{j-1..j+1}) or f^- (side=-1, f_{j..j+2})."""
    f = np.ascontiguousarray(f3, dtype=np.float64)
    w = np.zeros(2)
    (lib().oracle_weno3_weights_plus if side > 0 else lib().oracle_weno3_weights_minus)(ptr(f), eps, ptr(w))
    return w


def weno3_flux(f3, side, eps=1e-6):
    f = np.ascontiguousarray(f3, dtype=np.float64)
    return (lib().oracle_weno3_flux_plus if side > 0 else lib().oracle_weno3_flux_minus)(ptr(f), eps)


def radial_derivative(row, j, dx, speed, scheme, eps=1e-6):
    """Radial derivative at index j of `row` (entries j-4 .. j+4 must exist)."""
    p = np.ascontiguousarray(row, dtype=np.float64)
    return lib().oracle_radial_d(ptr(p), j, speed, dx, 0.0, eps, SCHEMES[scheme])


def advect1d_scheme(u0, dx, speed, dt, nsteps, scheme, sigma=0.01, eps=1e-6):
    """Periodic u_t + speed u_x = 0 by the chosen radial scheme and SSP-RK3."""
    u = np.ascontiguousarray(u0, dtype=np.float64).copy()
    lib().oracle_advect1d_scheme(ptr(u), u.size, dx, speed, dt, nsteps, eps, SCHEMES[scheme], sigma)
    return u


def advect1d(u0, dx, speed, dt, nsteps, eps=1e-6):
    u = np.ascontiguousarray(u0, dtype=np.float64).copy()
    lib().oracle_advect1d(ptr(u), u.size, dx, 0.0, speed, dt, 0.0, nsteps, eps, 0)
    return u


INTEGRATORS = {"rk3": 0, "rk104": 1}


def ssprk3_step(u0, dt, rhs):
    """One SSP-RK(3,3) step of the oracle with a Python right-hand side rhs(u)->F."""
    return _rk_step(u0, dt, rhs, "oracle_ssprk3_step", 3)


def ssprk104_step(u0, dt, rhs):
    """One SSP-RK(10,4) step of the oracle with a Python right-hand side rhs(u)->F."""
    return _rk_step(u0, dt, rhs, "oracle_ssprk104_step", 5)


def _rk_step(u0, dt, rhs, name, nwork):
    u = np.ascontiguousarray(u0, dtype=np.float64).copy()
    n = u.size
    work = np.zeros(nwork * n)

    def cb(up, Fp, _ctx):
        uu = np.ctypeslib.as_array(up, shape=(n,))
        FF = np.ctypeslib.as_array(Fp, shape=(n,))
        FF[:] = rhs(uu.copy())

    f = RHS_FN(cb)
    getattr(lib(), name)(ptr(u), n, dt, f, None, ptr(work))
    return u


# ----------------------------------------------------------------------------- Teukolsky
@dataclass
class Problem:
    """One solve: background (M, a), field (s, m), chart and grid.

    chart "T": x = r_* (tortoise); chart "H": x = rho, the compactified
    hyperboloidal radius with parameter S (paper Sec. 2.2).  In both charts
    the radial nodes are x_j = x_min + j (x_max - x_min)/(nr - 1).
    """
    s: int
    m: int
    a: float
    nr: int
    nth: int
    x_min: float
    x_max: float
    M: float = 1.0
    eps: float = 1e-6
    chart: str = "T"
    S: float = 20.0
    scheme: str = "weno5"        # radial scheme: "weno5", "weno3" or "fd6ko8" (Sec. 3.1)
    ko_sigma: float = 0.01       # Kreiss-Oliger sigma (fd6ko8)
    theta_order: int = 2         # order of the centred theta differences: 2 or 4 (Sec. 3.1 leaves it open)

    @property
    def dx(self):
        return (self.x_max - self.x_min) / (self.nr - 1)

    @property
    def dth(self):
        return np.pi / self.nth

    def x(self):
        """Radial nodes x_j = x_min + j dx (x = r_*)."""
        return self.x_min + self.dx * np.arange(self.nr)

    def theta(self):
        """Cell-centred polar nodes theta_k = (k + 1/2) pi / nth; no node on a pole."""
        return (np.arange(self.nth) + 0.5) * self.dth

    def parity(self):
        return -1.0 if (self.m + self.s) % 2 else 1.0


def theta_symbol_maxima(order):
    """(max |dth^2 D2 symbol|, max |dth D1 symbol|) over the wavenumbers.

    Second order: D2 -> (2 cos xi - 2), D1 -> i sin xi: (4, 1).  Fourth order:
    D2 -> (32 cos xi - 2 cos 2xi - 30)/12, largest at xi = pi: 16/3; D1 ->
    i (8 sin xi - sin 2xi)/6, whose derivative 8 cos xi - 2 cos 2xi vanishes
    at cos xi = 1 - sqrt(3/2), where it equals sin xi (4 - cos xi)/3.
    """
    if order == 4:
        c = 1.0 - np.sqrt(1.5)
        return 16.0 / 3.0, float(np.sqrt(1.0 - c * c) * (4.0 - c) / 3.0)
    return 4.0, 1.0


class TeukOracle:
    """Chart-T oracle for one Problem: coefficient tables plus the C solver."""

    def __init__(self, prob: Problem):
        if prob.theta_order not in (2, 4):
            raise ValueError("theta_order must be 2 or 4")
        if prob.nth < prob.theta_order // 2:
            raise ValueError("fourth-order theta differences need nth >= 2")
        self.prob = prob
        x = prob.x()
        th = prob.theta()
        if prob.chart == "H":
            from . import hyperboloidal as hyp
            self.r = x * prob.S / (prob.S - x)
            tab = hyp.first_order_tables(x, th, prob.M, prob.a, prob.s, prob.m, prob.S)
            self.tab = {k: np.ascontiguousarray(v, dtype=np.float64) for k, v in tab.items()}
        else:
            self.r, self.y, self.Delta = coeffs.r_of_tortoise(x, prob.M, prob.a)
            R = self.r[None, :]
            D = self.Delta[None, :]
            T = th[:, None]
            c = coeffs.first_order_coefficients(R, D, T, prob.M, prob.a, prob.s, prob.m)
            shp = (prob.nth, prob.nr)
            f = lambda v: np.ascontiguousarray(np.broadcast_to(v, shp), dtype=np.float64)
            self.tab = {
                "lam1": f(c["lam1"]), "lam2": f(c["lam2"]),
                "m3r": f(c["m3"].real), "m3i": f(c["m3"].imag),
                "btr": f(c["Bt"].real), "bti": f(c["Bt"].imag),
                "cr": f(c["C"].real), "ci": f(c["C"].imag),
                "ath": f(c["Ath"]), "bth": f(c["Bth"]),
            }
        self._s = _OracleTeuk(prob.nr, prob.nth, prob.dx, 0.0, prob.dth, 0.0, prob.eps, prob.parity(), 0,
                              SCHEMES[prob.scheme], prob.ko_sigma,
                              *[self.tab[n].ctypes.data for n in ("lam1", "lam2", "m3r", "m3i", "btr",
                                                                  "bti", "cr", "ci", "ath", "bth")],
                              prob.theta_order)

    # a8: stability bound (reading of the SSP framework of Sec. 3.2)
    def dt_bound(self, cfl=0.5):
        """dt = cfl / max_points( max(|lam1|,|lam2|)/dx + sqrt(c2 Ath/dth^2 + c1 |Bth|/dth + |C|) ).

        The square root bounds the frequency of the theta part (Gershgorin on
        the centred theta operator acting through the Phi-pi coupling); the
        first term is the radial upwind speed over dx.  c2 and c1 are the
        largest moduli of the Fourier symbols of dth^2 D2 and dth D1 (see
        theta_symbol_maxima).
        """
        p, t = self.prob, self.tab
        c2, c1 = theta_symbol_maxima(p.theta_order)
        lam = np.maximum(np.abs(t["lam1"]), np.abs(t["lam2"]))
        om = np.sqrt(c2 * t["ath"] / p.dth**2 + c1 * np.abs(t["bth"]) / p.dth + np.hypot(t["cr"], t["ci"]))
        return cfl / float(np.max(lam / p.dx + om))

    def rhs(self, u):
        """F(u) for u of shape [4][nth][nr]."""
        u = np.ascontiguousarray(u, dtype=np.float64)
        F = np.empty_like(u)
        lib().oracle_teuk_rhs(ctypes.byref(self._s), ptr(u), ptr(F))
        return F

    def extract_index(self, x_e):
        p = self.prob
        return int(np.floor((x_e - p.x_min) / p.dx + 0.5))

    def horizon(self, u):
        """Phi and d_rho Phi on the horizon rho_H = S r+ / (r+ + S) (chart H),
        per theta row, by 4-point Lagrange interpolation on the nodes around it
        (one-sided at the grid's inner end).  Returns complex arrays
        (Phi_H[nth], dPhi_H[nth])."""
        from . import hyperboloidal as hyp
        p = self.prob
        rp, _ = coeffs.horizons(p.M, p.a)
        rho_h = p.S * rp / (rp + p.S)
        f = (rho_h - p.x_min) / p.dx
        j0, w, dw = hyp.horizon_stencil(f, p.nr)
        ph = u[0] + 1j * u[1]
        win = ph[:, j0:j0 + 4]
        return win @ w, (win @ dw) / p.dx

    def evolve(self, u0, dt, nsteps, x_e=None, every=0, max_samples=0, integrator="rk3"):
        """Run nsteps steps of SSP-RK(3,3) (integrator "rk3") or SSP-RK(10,4)
        ("rk104").  Returns (u, wave[n][nth][2] or None)."""
        u = np.ascontiguousarray(u0, dtype=np.float64).copy()
        wave = None
        j_e = 0
        if x_e is not None and every > 0:
            j_e = self.extract_index(x_e)
            if max_samples <= 0:
                max_samples = nsteps // every + 1
            wave = np.zeros((max_samples, self.prob.nth, 2))
        n = lib().oracle_teuk_evolve_rk(ctypes.byref(self._s), ptr(u), dt, 0.0, nsteps, j_e, every,
                                        ptr(wave) if wave is not None else None, max_samples,
                                        INTEGRATORS[integrator])
        if wave is not None:
            wave = wave[:n]
        return u, wave


def set_threads(n: int):
    lib().oracle_set_threads(int(n))


def num_threads() -> int:
    return int(lib().oracle_num_threads())
