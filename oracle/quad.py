"""Oracle: Python driver for the binary128 ("quad") build of teuk_oracle.c.

TEST INFRASTRUCTURE ONLY.  Only the tests and the benchmark's checks import
this module; the product path never does.

The paper's baseline precision is quad (Sec. 3.1.3: about 30 significant
digits), with a mixed variant that forms the WENO weights in double.  This
driver runs the same plain solver as ``oracle.solver`` with IEEE binary128 as
its working precision, on coefficient tables evaluated from the symbolic chart-T
derivation of ``oracle.coefficients`` at 45 significant digits (mpmath), and
with the weights either in binary128 (``weights="quad"``) or in the paper's
mixed form (``weights="fp64"``).

Values cross the Python boundary as (hi, lo) pairs of doubles, value = hi + lo
(106 significant bits), in arrays whose last axis has length 2.
"""
from __future__ import annotations

import ctypes
import functools
import os

import mpmath as mp
import numpy as np
import sympy as sp

from . import coefficients as coeffs
from . import solver as S

DPS = 45
_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p

_lib_handle = None


def lib() -> ctypes.CDLL:
    """Load the binary128 oracle library, building it first if needed."""
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(S._LIBQ) or os.path.getmtime(S._LIBQ) < os.path.getmtime(S._SRC):
            S._compile(S._LIBQ, ["-DORACLE_QUAD"], False)
        L = ctypes.CDLL(S._LIBQ)
        for fn in ("oracle_weno5_weights_plus_q", "oracle_weno5_weights_minus_q",
                   "oracle_weno5_weights_plus_w64_q", "oracle_weno5_weights_minus_w64_q"):
            getattr(L, fn).argtypes = [_vp, ctypes.c_double, _vp]
        L.oracle_advect1d_q.argtypes = [_vp, ctypes.c_long, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_long, ctypes.c_double,
                                        ctypes.c_int]
        L.oracle_teuk_rhs_q.argtypes = [ctypes.POINTER(S._OracleTeuk), _vp, _vp]
        L.oracle_teuk_evolve_q.argtypes = [ctypes.POINTER(S._OracleTeuk), _vp, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_long, ctypes.c_long, ctypes.c_long, _vp, ctypes.c_long]
        L.oracle_teuk_evolve_q.restype = ctypes.c_long
        L.oracle_ode_rk3_q.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_long, _dp]
        L.oracle_weno5_flux_pair_q.argtypes = [_vp, ctypes.c_double, ctypes.c_int, ctypes.c_int, _dp]
        L.oracle_dside_pair_q.argtypes = [_vp, ctypes.c_long, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_int, ctypes.c_int, _dp]
        L.oracle_q_from_pairs.argtypes = [_dp, _vp, ctypes.c_long]
        L.oracle_q_to_pairs.argtypes = [_vp, _dp, ctypes.c_long]
        _lib_handle = L
    return _lib_handle


# ----------------------------------------------------------------------------- pairs <-> binary128
class QBuf:
    """A 16-byte-aligned buffer of n binary128 values."""

    def __init__(self, n: int):
        self.n = int(n)
        self._raw = np.zeros(2 * self.n + 2, dtype=np.float64)
        off = (-self._raw.ctypes.data) % 16
        self.addr = self._raw.ctypes.data + off

    @classmethod
    def from_pairs(cls, p) -> "QBuf":
        p = np.ascontiguousarray(p, dtype=np.float64)
        assert p.shape[-1] == 2
        q = cls(p.size // 2)
        lib().oracle_q_from_pairs(p.ctypes.data_as(_dp), q.addr, q.n)
        return q

    def pairs(self, shape=None) -> np.ndarray:
        out = np.empty((self.n, 2), dtype=np.float64)
        lib().oracle_q_to_pairs(self.addr, out.ctypes.data_as(_dp), self.n)
        return out.reshape(tuple(shape) + (2,)) if shape is not None else out


def split(v) -> tuple[float, float]:
    """An mpmath (or exact) value as a (hi, lo) pair of doubles."""
    hi = float(v)
    lo = float(mp.mpf(v) - mp.mpf(hi))
    return hi, lo


def to_mpf(pair) -> mp.mpf:
    return mp.mpf(float(pair[0])) + mp.mpf(float(pair[1]))


def promote(u: np.ndarray) -> np.ndarray:
    """FP64 values as exact pairs (lo = 0)."""
    u = np.asarray(u, dtype=np.float64)
    return np.stack([u, np.zeros_like(u)], axis=-1)


# ----------------------------------------------------------------------------- 1D helpers
def weno5_weights(f5_pairs, side: int, eps=1e-6, weights="quad"):
    """omega_0..2 of f^+ (side=+1, f_{j-2..j+2}) or f^- (side=-1, f_{j-1..j+3}), as pairs."""
    f = QBuf.from_pairs(np.asarray(f5_pairs).reshape(5, 2))
    w = QBuf(3)
    name = "oracle_weno5_weights_" + ("plus" if side > 0 else "minus") + ("_w64" if weights == "fp64" else "") + "_q"
    getattr(lib(), name)(f.addr, eps, w.addr)
    return w.pairs()


def weno5_flux(f5_pairs, side: int, eps=1e-6, weights="quad"):
    """f^+_{j+1/2} (side=+1) or f^-_{j+1/2} (side=-1) as a pair."""
    f = QBuf.from_pairs(np.asarray(f5_pairs).reshape(5, 2))
    out = np.zeros(2)
    lib().oracle_weno5_flux_pair_q(f.addr, eps, side, 1 if weights == "fp64" else 0, out.ctypes.data_as(_dp))
    return out


def derivative(row_pairs, j, dx_pair, side, eps=1e-6, weights="quad"):
    """D^+ (side=+1) or D^- (side=-1) at index j of a row (pairs) whose
    entries j-3 .. j+3 exist; returns a pair."""
    row = QBuf.from_pairs(row_pairs)
    out = np.zeros(2)
    lib().oracle_dside_pair_q(row.addr, j, dx_pair[0], dx_pair[1], eps, side, 1 if weights == "fp64" else 0,
                              out.ctypes.data_as(_dp))
    return out


def advect1d(u0_pairs, dx_pair, speed, dt_pair, nsteps, eps=1e-6, weights="quad"):
    """Periodic WENO5 + SSP-RK3 advection u_t + speed u_x = 0 in binary128."""
    u = QBuf.from_pairs(u0_pairs)
    lib().oracle_advect1d_q(u.addr, u.n, dx_pair[0], dx_pair[1], speed, dt_pair[0], dt_pair[1], nsteps, eps,
                            1 if weights == "fp64" else 0)
    return u.pairs()


def ode_rk3(lam, dt_pair, nsteps):
    out = np.zeros(2)
    lib().oracle_ode_rk3_q(lam, dt_pair[0], dt_pair[1], nsteps, out.ctypes.data_as(_dp))
    return out


# ----------------------------------------------------------------------------- chart-T tables at 45 digits
@functools.lru_cache(maxsize=None)
def _mp_lambdified():
    ex = coeffs._chart_T_reduction_symbolic()
    args = (coeffs.r, coeffs.Dl, coeffs.cth, coeffs.sth, coeffs.Mb, coeffs.ab, coeffs.sb, coeffs.mb)
    keys = ("lam1", "lam2", "m3", "Bt", "C", "Ath", "Bth")
    return keys, sp.lambdify(args, [ex[k] for k in keys], modules="mpmath")


def first_order_tables_mp(prob: S.Problem, window=None):
    """Per-point first-order coefficients (eq. evln, chart T) at DPS digits,
    as (hi, lo) pair arrays [nth][nr][2] keyed like the FP64 oracle's tables.
    window = (j0, k0, nr_w, nth_w) restricts them to those nodes of prob's grid."""
    keys, fn = _mp_lambdified()
    j0, k0, nr, nth = window if window is not None else (0, 0, prob.nr, prob.nth)
    with mp.workdps(DPS):
        x = [mp.mpf(prob.x_min) + (j0 + j) * (mp.mpf(prob.x_max) - mp.mpf(prob.x_min)) / (prob.nr - 1)
             for j in range(nr)]
    # the x nodes are formed at DPS digits; their double values only seed the
    # Newton solve for r, which is taken at the exact node.
    names = ("lam1", "lam2", "m3r", "m3i", "btr", "bti", "cr", "ci", "ath", "bth")
    tab = {n: np.zeros((nth, nr, 2)) for n in names}
    with mp.workdps(DPS + 10):
        rs, Ds = _r_at_nodes(x, prob.M, prob.a)
        dth = mp.pi / prob.nth
        for k in range(nth):
            th = (k0 + k + mp.mpf(1) / 2) * dth
            c, s_ = mp.cos(th), mp.sin(th)
            for j in range(nr):
                v = dict(zip(keys, fn(rs[j], Ds[j], c, s_, mp.mpf(prob.M), mp.mpf(prob.a), prob.s, prob.m)))
                vals = {"lam1": v["lam1"], "lam2": v["lam2"], "m3r": mp.re(v["m3"]), "m3i": mp.im(v["m3"]),
                        "btr": mp.re(v["Bt"]), "bti": mp.im(v["Bt"]), "cr": mp.re(v["C"]), "ci": mp.im(v["C"]),
                        "ath": mp.re(v["Ath"]), "bth": mp.re(v["Bth"])}
                for n in names:
                    tab[n][k, j] = split(vals[n])
    return tab


def _r_at_nodes(x_mp, M, a):
    """r and Delta at the exact nodes x_mp (Newton at DPS+10 digits)."""
    rr0, y0, _ = coeffs.r_of_tortoise(np.array([float(v) for v in x_mp]), M, a)
    Mm, am = mp.mpf(M), mp.mpf(a)
    d = mp.sqrt(max(Mm * Mm - am * am, mp.mpf(0)))
    rp, rm = Mm + d, Mm - d
    out_r, out_D = [], []
    for xm, yv in zip(x_mp, y0):
        u = mp.log(mp.mpf(float(yv)))
        for _ in range(60):
            y = mp.exp(u)
            r = rp + y
            if rp - rm > 0:
                f = (r + 2 * Mm * rp / (rp - rm) * mp.log(y / (2 * Mm))
                     - 2 * Mm * rm / (rp - rm) * mp.log((r - rm) / (2 * Mm)))
                df = (r * r + am * am) / (r - rm)
            else:
                f = r + 2 * Mm * mp.log(y / Mm) - 2 * Mm * Mm / y
                df = (r * r + am * am) / y
            du = (f - xm) / df
            u -= du
            if abs(du) < mp.mpf(10) ** (-(DPS + 5)):
                break
        y = mp.exp(u)
        out_r.append(rp + y)
        out_D.append(y * (rp + y - rm))
    return out_r, out_D


# ----------------------------------------------------------------------------- solver
class TeukOracleQ:
    """Chart-T oracle in binary128 for one Problem.

    weights="quad": IS, alpha, omega in binary128 as printed.
    weights="fp64": the paper's mixed variant (Sec. 3.1.3): stencil values
    rounded to double, weights in double, omega_2 the binary128 complement.
    """

    NAMES = ("lam1", "lam2", "m3r", "m3i", "btr", "bti", "cr", "ci", "ath", "bth")

    def __init__(self, prob: S.Problem, weights: str = "quad", tables=None, window=None):
        """window = (j0, k0, nr_w, nth_w): solve on that block of prob's grid
        alone, its edges taken as grid ends (ghosts by the usual rules), so
        that values away from the block's edges equal the full grid's."""
        assert prob.chart == "T", "the binary128 oracle covers the tortoise chart"
        assert prob.theta_order == 2, "the binary128 oracle takes second-order theta differences"
        assert weights in ("quad", "fp64")
        self.prob = prob
        self.weights = weights
        self.window = window if window is not None else (0, 0, prob.nr, prob.nth)
        self.nr, self.nth = self.window[2], self.window[3]
        self.tab = tables if tables is not None else first_order_tables_mp(prob, window)
        self._q = {n: QBuf.from_pairs(self.tab[n]) for n in self.NAMES}
        with mp.workdps(DPS):
            dx = split((mp.mpf(prob.x_max) - mp.mpf(prob.x_min)) / (prob.nr - 1))
            dth = split(mp.pi / prob.nth)
        self.dx_pair, self.dth_pair = dx, dth
        self._s = S._OracleTeuk(self.nr, self.nth, dx[0], dx[1], dth[0], dth[1], prob.eps, prob.parity(),
                                1 if weights == "fp64" else 0, S.SCHEMES[prob.scheme], prob.ko_sigma,
                                *[self._q[n].addr for n in self.NAMES])

    def shape(self):
        return (4, self.nth, self.nr)

    def rhs(self, u_pairs):
        """F(u) for u of shape [4][nth][nr][2] (pairs); returns pairs."""
        u = QBuf.from_pairs(u_pairs)
        F = QBuf(u.n)
        lib().oracle_teuk_rhs_q(ctypes.byref(self._s), u.addr, F.addr)
        return F.pairs(self.shape())

    def extract_index(self, x_e):
        p = self.prob
        return int(np.floor((x_e - p.x_min) / p.dx + 0.5)) - self.window[0]

    def evolve(self, u0_pairs, dt, nsteps, x_e=None, every=0, max_samples=0):
        """nsteps SSP-RK3 steps of size dt (a double, or a (hi, lo) pair).
        Returns (u pairs [4][nth][nr][2], wave pairs [n][nth][2][2] or None)."""
        dtp = (float(dt), 0.0) if np.isscalar(dt) else (float(dt[0]), float(dt[1]))
        u = QBuf.from_pairs(u0_pairs)
        wave = None
        j_e = 0
        if x_e is not None and every > 0:
            j_e = self.extract_index(x_e)
            if max_samples <= 0:
                max_samples = nsteps // every + 1
            wave = QBuf(max_samples * self.nth * 2)
        n = lib().oracle_teuk_evolve_q(ctypes.byref(self._s), u.addr, dtp[0], dtp[1], nsteps, j_e, every,
                                       wave.addr if wave is not None else None, max_samples)
        w = None
        if wave is not None:
            w = wave.pairs((max_samples, self.nth, 2))[:n]
        return u.pairs(self.shape()), w
