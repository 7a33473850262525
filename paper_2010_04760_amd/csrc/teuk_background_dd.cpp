// Double-double coefficient table for the tortoise chart, evaluated in IEEE
// binary128 (libquadmath) and stored as (hi, lo) pairs of doubles.
//
// The double-double state path (the paper's quad baseline of Sec. 3.1.3)
// needs the per-point coefficients to about 32 significant digits; the FP64
// radial / polar tables of teuk_background.cpp carry 16.  This file repeats
// their closed forms (teuk_coef.h) in binary128:
//   - r(x) from x = r_*: Newton steps in u = ln(r - r_+) at binary128, started
//     from the FP64 solve, on the closed forms of the tortoise coordinate
//     (Sec. 2.2); Delta = y (y + r_+ - r_-) keeps its relative precision;
//   - the radial factors P, Q, T0..T2, A0, A1, H0, G1, G2, X1 and the polar
//     factors sin^2, cos, cot, (m + s cos)^2 / sin^2 (half-angle form);
//   - the per-point combination with v = 1/Sigma.
// Compiled by the host C++ compiler (it needs quadmath.h), not by hipcc.
#include <quadmath.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <thread>
#include <vector>

#include "teuk_dd_tables.h"

namespace teuk {

namespace {

typedef __float128 Q;

void put(double* dst, Q v)
{
    const double hi = (double)v;
    dst[0] = hi;
    dst[1] = (double)(v - (Q)hi);
}

struct KerrQ {
    Q M, a, rp, rm;
    bool extremal;
};

// x = r_*(y) and d x / d ln y at y = r - r_+.
void tortoise_q(const KerrQ& k, Q y, Q* xs, Q* dxs)
{
    const Q r = k.rp + y;
    if (!k.extremal) {
        const Q w = k.rp - k.rm;
        *xs = r + 2 * k.M * k.rp / w * logq(y / (2 * k.M)) - 2 * k.M * k.rm / w * logq((y + w) / (2 * k.M));
        *dxs = (r * r + k.a * k.a) / (y + w);
    } else {
        *xs = r + 2 * k.M * logq(y / k.M) - 2 * k.M * k.M / y;
        *dxs = (r * r + k.a * k.a) / y;
    }
}

}  // namespace

bool build_tables_dd(const teuk_config& c, std::vector<double>& dtab, DDScalars* sc, std::string& err)
{
    const int nr = c.nr, nth = c.ntheta;
    const size_t plane = (size_t)nr * nth;
    KerrQ K;
    K.M = c.M;
    K.a = c.a;
    const Q d2 = K.M * K.M - K.a * K.a;
    const Q d = d2 > 0 ? sqrtq(d2) : (Q)0;
    K.rp = K.M + d;
    K.rm = K.M - d;
    K.extremal = !(d > 0);
    const Q M = K.M, a = K.a, s = c.s, m = c.m, q = 2 * (Q)c.s + 1;
    const Q dx = ((Q)c.x_max - (Q)c.x_min) / (nr - 1);
    const Q dth = M_PIq / nth;

    // radial factors per node, in binary128
    enum { Dl, P, Qf, Ra2, T0, T1, T2, A0, A1, H0, G1, G2, X1, NR };
    std::vector<Q> R((size_t)NR * nr);
    for (int j = 0; j < nr; ++j) {
        const Q x = (Q)c.x_min + dx * j;
        double u0 = tortoise_lny(c, (double)x);
        Q u = u0;
        for (int it = 0; it < 12; ++it) {
            Q f, df;
            tortoise_q(K, expq(u), &f, &df);
            const Q du = (f - x) / df;
            u -= du;
            if (fabsq(du) <= 1e-33Q * fmaxq(1, fabsq(u))) break;
        }
        const Q y = expq(u);
        const Q r = K.rp + y;
        const Q D = y * (y + (K.rp - K.rm));
        if (!(D > 1e-280Q) || !(r == r)) {
            err = "radial node x = " + std::to_string((double)x) +
                  " lies too deep toward the horizon for FP64 (Delta underflows); raise x_min";
            return false;
        }
        const Q ra2 = r * r + a * a;
        Q* Rj = R.data() + (size_t)j * NR;
        Rj[Dl] = D;
        Rj[P] = ra2 * ra2;
        Rj[Qf] = a * a * D;
        Rj[Ra2] = ra2;
        Rj[T0] = -2 * s * (r * D - M * (r * r - a * a));
        Rj[T1] = -4 * M * a * m * r;
        Rj[T2] = -2 * s * a * D;
        Rj[A0] = D * (q * (q + 1) * D / (r * r) - 2 * (s + 1) * q * (r - M) / r + s);
        Rj[A1] = -2 * m * a * q * D / r + 4 * s * m * a * (r - M);
        const Q X0 = -2 * q * D * ra2 / r + 2 * r * D + 2 * s * (r - M) * ra2;
        Rj[H0] = 2 * r * D - X0;
        Rj[G1] = 2 * r * D * ra2 * ra2;
        Rj[G2] = D * ra2 * a * a * (r - M);
        Rj[X1] = 2 * m * a * ra2;
    }

    dtab.assign((size_t)kNDD * plane * 2, 0.0);
    auto rows = [&](int k0, int k1) {
        for (int k = k0; k < k1; ++k) {
            const Q th = ((Q)k + 0.5Q) * dth;
            const Q sn = sinq(th), cs = cosq(th);
            const Q sn2 = sn * sn, cot = cs / sn;
            const Q hs = sinq(th / 2), hc = cosq(th / 2);
            const Q mc = (m + s) * hc * hc + (m - s) * hs * hs;
            const Q tp = mc * mc / sn2;
            for (int j = 0; j < nr; ++j) {
                const Q* Rj = R.data() + (size_t)j * NR;
                const Q v = 1 / sqrtq(Rj[P] - Rj[Qf] * sn2);
                const Q w = v * v;
                const Q b = Rj[Ra2] * v;
                const Q ath = Rj[Dl] * w;
                const Q btr = w * Rj[T0];
                const Q bti = w * (Rj[T1] + Rj[T2] * cs);
                const Q vals[kNDD] = {
                    b,
                    b * btr + w * (Rj[H0] - w * (Rj[G1] - Rj[G2] * sn2)),
                    b * bti - w * Rj[X1],
                    btr,
                    bti,
                    w * (Rj[A0] - Rj[Dl] * tp),
                    w * Rj[A1],
                    ath,
                    ath * cot,
                };
                const size_t i = (size_t)k * nr + j;
                for (int t = 0; t < kNDD; ++t) put(dtab.data() + 2 * ((size_t)t * plane + i), vals[t]);
            }
        }
    };
    unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if ((size_t)nr * nth < 65536) nt = 1;
    if (nt > (unsigned)nth) nt = nth;
    std::vector<std::thread> pool;
    for (unsigned t = 0; t < nt; ++t) pool.emplace_back(rows, (int)((long long)nth * t / nt), (int)((long long)nth * (t + 1) / nt));
    for (auto& th : pool) th.join();

    put(sc->inv_dx, 1 / dx);
    put(sc->ih1, 1 / (2 * dth));
    put(sc->ih2, 1 / (dth * dth));
    put(sc->third, (Q)1 / 3);
    put(sc->two_thirds, (Q)2 / 3);
    put(sc->d[0], (Q)1 / 10);
    put(sc->d[1], (Q)6 / 10);
    put(sc->d[2], (Q)3 / 10);
    put(sc->c13_3, (Q)13 / 3);
    put(sc->sixth, (Q)1 / 6);
    return true;
}

}  // namespace teuk
