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

}  // namespace teuk
