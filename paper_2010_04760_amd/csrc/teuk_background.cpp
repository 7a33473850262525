// Host-side background for the tortoise chart: r(x) from x = r_*, Delta without
// cancellation, and the radial / polar coefficient tables of teuk_coef.h.
//
// Kerr background (paper Sec. 2.1-2.2): Delta = r^2 - 2Mr + a^2 with roots
// r_+- = M +- sqrt(M^2 - a^2); the tortoise coordinate r_* = int (r^2+a^2)/Delta dr
// is fixed here, up to its free constant, by
//     a < M:  r_* = r + 2M r+/(r+ - r-) ln((r-r+)/2M) - 2M r-/(r+ - r-) ln((r-r-)/2M)
//     a = M:  r_* = r + 2M ln((r-M)/M) - 2M^2/(r-M).
// The unknown solved for is y = r - r_+ > 0, so that Delta = y (y + r_+ - r_-)
// keeps full relative precision as r -> r_+ (x -> -infinity).
#include <cmath>
#include <string>
#include <vector>

#include "teuk_coef.h"
#include "teuk_dd_tables.h"
#include "teuk_internal.h"

namespace teuk {

namespace {

struct Kerr {
    double M, a, rp, rm;
    bool extremal;
};

Kerr make_kerr(double M, double a)
{
    Kerr k;
    k.M = M;
    k.a = a;
    const double d2 = M * M - a * a;
    const double d = d2 > 0.0 ? std::sqrt(d2) : 0.0;
    k.rp = M + d;
    k.rm = M - d;
    k.extremal = !(d > 0.0);
    return k;
}

// r_*(y) and d r_* / d ln y, with y = r - r_+.
void tortoise(const Kerr& k, double y, double* xs, double* dxs_dlny)
{
    const double r = k.rp + y;
    if (!k.extremal) {
        const double w = k.rp - k.rm;
        *xs = r + 2.0 * k.M * k.rp / w * std::log(y / (2.0 * k.M)) -
              2.0 * k.M * k.rm / w * std::log((y + w) / (2.0 * k.M));
        // y dr_*/dr = y (r^2+a^2)/(y (r - r_-)) = (r^2+a^2)/(r - r_-)
        *dxs_dlny = (r * r + k.a * k.a) / (y + w);
    } else {
        *xs = r + 2.0 * k.M * std::log(y / k.M) - 2.0 * k.M * k.M / y;
        *dxs_dlny = (r * r + k.a * k.a) / y;
    }
}

// Solve r_*(y) = x for u = ln y.  r_* is strictly increasing in u, so keep a
// bracket [lo, hi] and take Newton steps, falling back to bisection whenever
// the Newton step leaves the bracket or fails to halve the step before last
// (deep in the extremal throat r_* ~ -2M^2/y Newton alone gains only one unit
// of ln y per step).
double solve_lny(const Kerr& k, double x)
{
    double lo = -740.0, hi = std::log(std::fabs(x) + 100.0 * k.M + 10.0);
    double u = 0.5 * (lo + hi);
    double dxold = hi - lo, dx = dxold;
    double f, df;
    tortoise(k, std::exp(u), &f, &df);
    f -= x;
    for (int it = 0; it < 300; ++it) {
        const bool out = ((u - hi) * df - f) * ((u - lo) * df - f) > 0.0;
        if (out || !std::isfinite(f) || std::fabs(2.0 * f) > std::fabs(dxold * df)) {
            dxold = dx;
            dx = 0.5 * (hi - lo);
            u = lo + dx;
        } else {
            dxold = dx;
            dx = f / df;
            u -= dx;
        }
        if (std::fabs(dx) <= 4e-16 * std::fmax(1.0, std::fabs(u))) break;
        tortoise(k, std::exp(u), &f, &df);
        f -= x;
        if (f < 0.0) lo = u; else hi = u;
    }
    return u;
}

}  // namespace

double tortoise_lny(const teuk_config& c, double x)
{
    return solve_lny(make_kerr(c.M, c.a), x);
}

bool build_tables(const teuk_config& c, std::vector<double>& rtab, std::vector<double>& ttab,
                  std::string& err)
{
    const int nr = c.nr, nth = c.ntheta;
    const Kerr K = make_kerr(c.M, c.a);
    const double M = c.M, a = c.a;
    const double s = c.s, m = c.m, q = 2.0 * c.s + 1.0;
    const double dx = (c.x_max - c.x_min) / (nr - 1);
    rtab.assign((size_t)kNRT * nr, 0.0);
    ttab.assign((size_t)kNTT * nth, 0.0);
    for (int j = 0; j < nr; ++j) {
        const double x = c.x_min + dx * j;
        const double y = std::exp(solve_lny(K, x));
        const double r = K.rp + y;
        const double Dl = y * (y + (K.rp - K.rm));
        if (!(Dl > 1e-280) || !std::isfinite(r)) {
            err = "radial node x = " + std::to_string(x) +
                  " lies too deep toward the horizon for FP64 (Delta underflows); raise x_min";
            return false;
        }
        const double ra2 = r * r + a * a;
        double* R = rtab.data();
        auto put = [&](int row, double v) { R[(size_t)row * nr + j] = v; };
        put(kDl, Dl);
        put(kP, ra2 * ra2);
        put(kQ, a * a * Dl);
        put(kRa2, ra2);
        put(kT0, -2.0 * s * (r * Dl - M * (r * r - a * a)));
        put(kT1, -4.0 * M * a * m * r);
        put(kT2, -2.0 * s * a * Dl);
        put(kA0, Dl * (q * (q + 1.0) * Dl / (r * r) - 2.0 * (s + 1.0) * q * (r - M) / r + s));
        put(kA1, -2.0 * m * a * q * Dl / r + 4.0 * s * m * a * (r - M));
        const double X0 = -2.0 * q * Dl * ra2 / r + 2.0 * r * Dl + 2.0 * s * (r - M) * ra2;
        put(kH0, 2.0 * r * Dl - X0);
        put(kG1, 2.0 * r * Dl * ra2 * ra2);
        put(kG2, Dl * ra2 * a * a * (r - M));
        put(kX1, 2.0 * m * a * ra2);
    }
    const double dth = M_PI / nth;
    for (int k = 0; k < nth; ++k) {
        const double th = (k + 0.5) * dth;
        const double sn = std::sin(th), cs = std::cos(th);
        ttab[(size_t)kSn2 * nth + k] = sn * sn;
        ttab[(size_t)kCs * nth + k] = cs;
        ttab[(size_t)kCot * nth + k] = cs / sn;
        // m + s cos(theta) = (m + s) cos^2(theta/2) + (m - s) sin^2(theta/2): no
        // cancellation at either pole when m = -s or m = s, where the pole
        // factor (m + s cos)^2 / sin^2 stays finite.
        const double hs = std::sin(0.5 * th), hc = std::cos(0.5 * th);
        const double mc = (m + s) * hc * hc + (m - s) * hs * hs;
        ttab[(size_t)kTh * nth + k] = mc * mc / (sn * sn);
    }
    return true;
}

// ---------------------------------------------------------------- chart H
// Hyperboloidal chart (paper Sec. 2.2): tau = t~ - r^2/(r+S) + 4M ln(S/(r+S)),
// rho = r S/(r + S), with t~ the ingoing-Kerr time and Psi = exp(i m phi~)
// r^-1 Delta^-s Phi.  With u = r + S, rho' = S^2/u^2 and
//     h   = H' - (r^2+a^2)/Delta = -2 + eps,   eps = (S^2 - 4 M u)/u^2,
//     K   = Delta H' = r^2 + a^2 + Delta h = -u^2 + G,
//     G   = 2 u S - S^2 + 4 M r - a^2 + Delta eps,
//     P   = -2 (r^2+a^2) h - Delta h^2
//         = 2 r S (4 M u + r S)/u^2 + eps (2a^2 - 8 M r) - Delta eps^2,
// the coefficients of eq. near_final are, all regular through the horizon:
//     A^tautau = -(P - a^2 sin^2),   A^taurho = 2 K rho' = 2 S^2 (G/u^2 - 1),
//     A^rhorho = Delta rho'^2,       A^thth = 1,   B^th = cot(theta),
//     B^tau = -4sM - s eps Delta' - 4M + 2a^2/r + eps (2M - 2a^2/r) + Delta eps'
//             + i [2 m a (eps - 1) - 2 s a cos(theta)],
//     B^rho = rho' (-2 Delta/r + (1-s) Delta') + Delta rho'' + 2 i m a rho',
//     C     = 2 Delta/r^2 + (s-1) Delta'/r - s - (m + s cos)^2/sin^2 - 2 i m a/r.
// (The 1/Delta terms of the chain rule cancel exactly; the forms above are
// arranged so that no large terms cancel near null infinity either.)  Divided
// by W = P - a^2 sin^2 (eq. final) and reduced as in Sec. 2.3 with the printed
// root b = -(A~taurho + sqrt(A~taurho^2 + 4 A~rhorho))/2: with A = A^taurho,
// R = A^rhorho, Q = sqrt(A^2 + 4 R W),
//     lam1 = b       = -(A + Q)/(2W)   (A >= 0),   -2R/(Q - A)   (A < 0),
//     lam2 = -(A/W + b) = 2R/(Q + A)   (A >= 0),   (Q - A)/(2W)  (A < 0),
// each the form without cancellation, and m3 = -lam2 d_rho b + b B~tau - B~rho
// with d_rho b = (d_r b)/rho'.  Evaluated in long double and rounded once.
bool build_tables_H(const teuk_config& c, std::vector<double>& ctab, std::string& err)
{
    (void)err;   // every node is admissible: the forms are regular through the horizon
    typedef long double L;
    const int nr = c.nr, nth = c.ntheta;
    const L M = c.M, a = c.a, S = c.S, s = c.s, m = c.m;
    const L d = (L)c.M * c.M - (L)c.a * c.a > 0 ? std::sqrt((L)c.M * c.M - (L)c.a * c.a) : 0.0L;
    const L rp = M + d, rm = M - d;
    const L rho_h = S * rp / (rp + S);
    const double dx = (c.x_max - c.x_min) / (nr - 1);
    const size_t plane = (size_t)nr * nth;
    ctab.assign((size_t)kNCH * plane, 0.0);
    const double dth = M_PI / nth;
    for (int j = 0; j < nr; ++j) {
        const double xj = c.x_min + dx * j;           // the node, as in every other table
        const L x = xj;
        const L r = x * S / (S - x);
        const L y = S * S * (x - rho_h) / ((S - x) * (S - rho_h));   // r - r+
        const L D = y * (y + (rp - rm));
        const L Dp = 2 * (r - M);
        const L u = r + S;
        const L r1 = S * S / (u * u), r2 = -2 * S * S / (u * u * u);
        const L eps = (S * S - 4 * M * u) / (u * u), epsp = (4 * M * u - 2 * S * S) / (u * u * u);
        const L N = 4 * M * r * u + r * r * S, Np = 4 * M * u + 4 * M * r + 2 * r * S;
        const L P = 2 * S * N / (u * u) + eps * (2 * a * a - 8 * M * r) - D * eps * eps;
        const L Pp = 2 * S * (Np * u - 2 * N) / (u * u * u) + epsp * (2 * a * a - 8 * M * r) - 8 * M * eps -
                     Dp * eps * eps - 2 * D * eps * epsp;
        const L G = 2 * u * S - S * S + 4 * M * r - a * a + D * eps;
        const L Gp = 2 * S + 4 * M + Dp * eps + D * epsp;
        const L A = 2 * S * S * (G / (u * u) - 1);
        const L Ap = 2 * S * S * (Gp * u - 2 * G) / (u * u * u);
        const L R = D * r1 * r1;
        const L Rp = Dp * r1 * r1 + 2 * D * r1 * r2;
        const L btr0 = -4 * s * M - s * eps * Dp - 4 * M + 2 * a * a / r + eps * (2 * M - 2 * a * a / r) + D * epsp;
        const L bti0 = 2 * m * a * (eps - 1);
        const L bxr = r1 * (-2 * D / r + (1 - s) * Dp) + D * r2;
        const L bxi = 2 * m * a * r1;
        const L cr0 = 2 * D / (r * r) + (s - 1) * Dp / r - s;
        const L ci0 = -2 * m * a / r;
        for (int k = 0; k < nth; ++k) {
            const L th = (k + 0.5) * (L)dth;
            const L sn = std::sin(th), cs = std::cos(th);
            const L hs = std::sin(th / 2), hc = std::cos(th / 2);
            const L mc = (m + s) * hc * hc + (m - s) * hs * hs;
            const L V = mc * mc / (sn * sn);
            const L W = P - a * a * sn * sn;
            const L Q = std::sqrt(A * A + 4 * R * W);
            const L Qp = (A * Ap + 2 * Rp * W + 2 * R * Pp) / Q;
            L lam1, lam2, bp;
            if (A >= 0) {
                lam1 = -(A + Q) / (2 * W);
                lam2 = 2 * R / (Q + A);
                bp = -((Ap + Qp) * W - (A + Q) * Pp) / (2 * W * W);
            } else {
                lam1 = -2 * R / (Q - A);
                lam2 = (Q - A) / (2 * W);
                bp = -2 * (Rp * (Q - A) - R * (Qp - Ap)) / ((Q - A) * (Q - A));
            }
            const L brho = bp / r1;
            const L Btr = btr0 / W, Bti = (bti0 - 2 * s * a * cs) / W;
            const L Bxr = bxr / W, Bxi = bxi / W;
            const size_t i = (size_t)k * nr + j;
            double* T = ctab.data();
            T[kHLam1 * plane + i] = (double)lam1;
            T[kHLam2 * plane + i] = (double)lam2;
            T[kHM3r * plane + i] = (double)(-lam2 * brho + lam1 * Btr - Bxr);
            T[kHM3i * plane + i] = (double)(lam1 * Bti - Bxi);
            T[kHBtr * plane + i] = (double)Btr;
            T[kHBti * plane + i] = (double)Bti;
            T[kHCr * plane + i] = (double)((cr0 - V) / W);
            T[kHCi * plane + i] = (double)(ci0 / W);
            T[kHAth * plane + i] = (double)(1 / W);
            T[kHBth * plane + i] = (double)(cs / sn / W);
        }
    }
    return true;
}

}  // namespace teuk
