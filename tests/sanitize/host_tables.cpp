// Host-side table builders of libteuk run under AddressSanitizer and
// UndefinedBehaviorSanitizer (built by tests/test_host_sanitizers.py with g++):
// the chart-T radial and polar tables, the chart-H per-point table and the
// double-double table, on grids from the smallest accepted (7 x 2) to a few
// thousand points, spins a = 0 .. M, |m| up to 8, and radial ranges reaching
// deep towards the horizon.  Every table that is built must be finite.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "teuk_coef.h"
#include "teuk_dd_tables.h"
#include "teuk_internal.h"

namespace {

teuk_config base(int s, int m, double a, int nr, int nth, double x0, double x1)
{
    teuk_config c;
    std::memset(&c, 0, sizeof(c));
    c.abi_version = TEUK_ABI_VERSION;
    c.s = s;
    c.m = m;
    c.a = a;
    c.M = 1.0;
    c.nr = nr;
    c.ntheta = nth;
    c.x_min = x0;
    c.x_max = x1;
    c.chart = TEUK_CHART_TORTOISE;
    c.weno_eps = 1e-6;
    c.cfl = 0.5;
    c.S = 20.0;
    c.theta_order = 2;
    return c;
}

bool finite_all(const std::vector<double>& v)
{
    for (double x : v)
        if (!std::isfinite(x)) return false;
    return true;
}

}  // namespace

int main()
{
    int cases = 0, built = 0, failures = 0;
    const double spins[] = {0.0, 0.5, 0.9, 0.999, 1.0};
    const int sw[] = {-2, -1, 0, 2};
    const int ms[] = {-8, 0, 1, 8};
    const int grids[][2] = {{7, 2}, {64, 3}, {1000, 33}, {4097, 16}};
    const double ranges[][2] = {{-30.0, 50.0}, {-400.0, 800.0}, {-5.0, 5.0}};
    for (double a : spins)
        for (int s : sw)
            for (int m : ms)
                for (const auto& g : grids)
                    for (const auto& r : ranges) {
                        teuk_config c = base(s, m, a, g[0], g[1], r[0], r[1]);
                        std::vector<double> rt, tt;
                        std::string err;
                        ++cases;
                        if (teuk::build_tables(c, rt, tt, err)) {
                            ++built;
                            if (rt.size() != (size_t)teuk::kNRT * c.nr || tt.size() != (size_t)teuk::kNTT * c.ntheta ||
                                !finite_all(rt) || !finite_all(tt)) {
                                std::printf("chart T table wrong: a=%g s=%d m=%d %dx%d\n", a, s, m, g[0], g[1]);
                                ++failures;
                            }
                        }
                    }
    // chart H: the grid from the horizon rho_H = S r+/(r+ + S) outwards
    for (double a : {0.5, 0.8, 0.999, 1.0})
        for (int s : {-2, 0})
            for (const auto& g : grids) {
                const double rp = 1.0 + std::sqrt(std::fmax(0.0, 1.0 - a * a));
                const double rho_h = 20.0 * rp / (rp + 20.0);
                teuk_config c = base(s, 0, a, g[0], g[1], rho_h, 19.99);
                c.chart = TEUK_CHART_HYPERBOLOIDAL;
                std::vector<double> ct;
                std::string err;
                ++cases;
                if (teuk::build_tables_H(c, ct, err)) {
                    ++built;
                    if (ct.size() != (size_t)teuk::kNCH * c.nr * c.ntheta || !finite_all(ct)) {
                        std::printf("chart H table wrong: a=%g s=%d %dx%d\n", a, s, g[0], g[1]);
                        ++failures;
                    }
                }
            }
    // double-double tables (tortoise chart, binary128 on the host)
    for (double a : {0.0, 0.7, 1.0})
        for (int m : {0, 2}) {
            teuk_config c = base(-2, m, a, 70, 5, -30.0, 50.0);
            c.state_prec = TEUK_S_DD;
            std::vector<double> dt;
            teuk::DDScalars sc{};
            std::string err;
            ++cases;
            if (teuk::build_tables_dd(c, dt, &sc, err)) {
                ++built;
                if (!finite_all(dt)) {
                    std::printf("double-double table not finite: a=%g m=%d\n", a, m);
                    ++failures;
                }
            }
        }
    std::printf("cases %d built %d failures %d\n", cases, built, failures);
    return failures == 0 && built > 0 ? 0 : 1;
}
