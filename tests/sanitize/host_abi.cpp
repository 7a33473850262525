// The host side of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer:
// configuration validation (every field pushed past its limits), footprints,
// the host evaluation of the per-point coefficients, and teuk_create's error
// paths on a machine whose runtime offers no GPU (or on one that does, the
// create and destroy of a small solver).  Only host code is compiled (the
// kernels are not built in), so every launch the library would make fails
// cleanly instead.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "teuk.h"

namespace {

teuk_config good()
{
    teuk_config c;
    teuk_default_config(&c);
    c.s = -2;
    c.m = 2;
    c.a = 0.9;
    c.nr = 300;
    c.ntheta = 12;
    c.x_min = -40.0;
    c.x_max = 60.0;
    return c;
}

}  // namespace

int main()
{
    int checks = 0, failures = 0;
    auto expect = [&](bool ok, const char* what) {
        ++checks;
        if (!ok) {
            std::printf("failed: %s\n", what);
            ++failures;
        }
    };
    // validation: each field out of range on an otherwise valid configuration
    {
        teuk_config c = good();
        expect(teuk_footprint_bytes(&c) > 0, "valid configuration has a footprint");
        expect(teuk_footprint_bytes(nullptr) == 0, "NULL configuration");
    }
    struct Bad { const char* what; void (*set)(teuk_config&); };
    const Bad bad[] = {
        {"abi", [](teuk_config& c) { c.abi_version = 0; }},
        {"s", [](teuk_config& c) { c.s = 3; }},
        {"m", [](teuk_config& c) { c.m = -9; }},
        {"nr small", [](teuk_config& c) { c.nr = 6; }},
        {"nr large", [](teuk_config& c) { c.nr = (1 << 24) + 1; }},
        {"ntheta", [](teuk_config& c) { c.ntheta = 1; }},
        {"ntheta large", [](teuk_config& c) { c.ntheta = 65537; }},
        {"points", [](teuk_config& c) { c.nr = 1 << 24; c.ntheta = 65536; }},
        {"weights", [](teuk_config& c) { c.weight_prec = 9; }},
        {"state", [](teuk_config& c) { c.state_prec = 5; }},
        {"integrator", [](teuk_config& c) { c.integrator = -1; }},
        {"scheme", [](teuk_config& c) { c.scheme = 7; }},
        {"theta order", [](teuk_config& c) { c.theta_order = 3; }},
        {"M", [](teuk_config& c) { c.M = 0.0; }},
        {"a", [](teuk_config& c) { c.a = 1.5; }},
        {"a NaN", [](teuk_config& c) { c.a = std::nan(""); }},
        {"range", [](teuk_config& c) { c.x_max = c.x_min; }},
        {"eps", [](teuk_config& c) { c.weno_eps = 1e-40; }},
        {"chart", [](teuk_config& c) { c.chart = 4; }},
        {"chart H range", [](teuk_config& c) { c.chart = TEUK_CHART_HYPERBOLOIDAL; c.x_min = -1.0; }},
        {"samples", [](teuk_config& c) { c.extract_every = 5; c.max_samples = -1; }},
    };
    for (const Bad& b : bad) {
        teuk_config c = good();
        b.set(c);
        expect(teuk_footprint_bytes(&c) == 0, b.what);
        teuk_solver* h = reinterpret_cast<teuk_solver*>(1);
        expect(teuk_create(&c, nullptr, &h) == TEUK_ERR_INVALID_ARG && h == nullptr, b.what);
        expect(std::strlen(teuk_last_error(nullptr)) > 0, "error message");
    }
    // host coefficients: chart T, chart H from the horizon, double-double pairs, too small an array
    {
        teuk_config c = good();
        std::vector<double> out((size_t)TEUK_NCOEF * c.ntheta * c.nr);
        expect(teuk_host_coefficients(&c, out.data(), out.size()) == TEUK_OK, "chart T coefficients");
        bool fin = true;
        for (double v : out) fin = fin && std::isfinite(v);
        expect(fin, "chart T coefficients finite");
        expect(teuk_host_coefficients(&c, out.data(), out.size() - 1) != TEUK_OK, "too small an array");
        teuk_config h = c;
        h.chart = TEUK_CHART_HYPERBOLOIDAL;
        h.a = 1.0;
        h.s = -2;
        h.m = 0;
        h.S = 20.0;
        h.x_min = 20.0 / 21.0;
        h.x_max = 19.99;
        expect(teuk_host_coefficients(&h, out.data(), out.size()) == TEUK_OK, "chart H coefficients");
        teuk_config d = c;
        d.state_prec = TEUK_S_DD;
        std::vector<double> dd(2 * out.size());
        expect(teuk_host_coefficients(&d, dd.data(), dd.size()) == TEUK_OK, "double-double coefficients");
    }
    // teuk_create on the host only: succeeds where a GPU answers, else fails cleanly
    {
        teuk_config c = good();
        teuk_solver* h = nullptr;
        const teuk_status st = teuk_create(&c, nullptr, &h);
        expect((st == TEUK_OK) == (h != nullptr), "create result and handle agree");
        if (h) teuk_destroy(h);
    }
    std::printf("checks %d failures %d\n", checks, failures);
    return failures == 0 ? 0 : 1;
}
