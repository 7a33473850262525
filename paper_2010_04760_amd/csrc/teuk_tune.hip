// Launch-shape autotuner of libteuk (declared in include/teuk.h).
//
// A stage launch of a single solve runs nstrips x segs workgroups: the grid's
// radial strips of 63 points, each cut into segs theta segments (the blocked
// step: strips of 114 points).  teuk_create derives segs from a workgroup
// budget, by default the number of stage workgroups the GPU holds at once.
// teuk_tune times the stage kernels of one configuration over a set of budgets
// around that default, on a scratch solver of the same grid (no
// waveform ring, a smooth synthetic state), and remembers the fastest budget per device and launch
// class; later solvers of that class created with workgroups = 0 use it.  Only
// the tiling changes between candidates: every point runs the same arithmetic,
// so the results do not depend on the choice.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "teuk_internal.h"

namespace {

// What a tuned budget applies to: device, launch class (chart and theta
// order), weight and state precision, integrator, scheme and grid.
typedef std::tuple<int, int, int, int, int, int, int, int> TuneKey;

std::mutex g_tune_mutex;
std::map<TuneKey, int> g_tuned;
thread_local std::string g_tune_err;

TuneKey key_of(const teuk_config& c, int device)
{
    return TuneKey(device, teuk::kernel_chart(c), c.weight_prec, c.state_prec, c.integrator, c.scheme, c.nr,
                   c.ntheta);
}

// Theta segments per strip that a workgroup budget gives (the rule of
// teuk_create: at most one per row; for the three-launch step an even count
// when more than one, so that neighbouring segments pair up).
int segs_for(long long budget, int nstrips, int nth, bool even)
{
    long long segs = budget / nstrips;
    if (segs > nth) segs = nth;
    if (even && segs > 1) segs &= ~1LL;
    if (segs < 1) segs = 1;
    return (int)segs;
}

teuk_status tfail(teuk_status st, const std::string& msg)
{
    g_tune_err = msg;
    return st;
}

// Microseconds per step of cfg with the given workgroup budget: the best of
// three timed runs of `steps` steps after two warm-up steps.
teuk_status time_budget(const teuk_config& base, int budget, int steps, hipStream_t stream,
                        const std::vector<double>& zeros, double* us)
{
    teuk_config c = base;
    c.workgroups = budget;
    c.extract_every = 0;
    c.max_samples = 0;
    teuk_device_ctx ctx{stream, nullptr, 0};
    teuk_solver* h = nullptr;
    teuk_status st = teuk_create(&c, &ctx, &h);
    if (st != TEUK_OK) return tfail(st, std::string("scratch solver: ") + teuk_last_error(nullptr));
    st = teuk_set_initial(h, zeros.data(), 0);
    if (st == TEUK_OK) st = teuk_step(h, 2);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int e = 0;
    if (st == TEUK_OK) {
        e = (int)hipEventCreate(&e0);
        if (!e) e = (int)hipEventCreate(&e1);
    }
    double best = 0.0;
    for (int rep = 0; rep < 3 && st == TEUK_OK && !e; ++rep) {
        e = (int)hipEventRecord(e0, stream);
        if (!e) st = teuk_step(h, steps);
        if (!e && st == TEUK_OK) e = (int)hipEventRecord(e1, stream);
        if (!e && st == TEUK_OK) e = (int)hipEventSynchronize(e1);
        float ms = 0.0f;
        if (!e && st == TEUK_OK) e = (int)hipEventElapsedTime(&ms, e0, e1);
        const double t = 1e3 * (double)ms / steps;
        if (!e && st == TEUK_OK && (rep == 0 || t < best)) best = t;
    }
    std::string msg = st != TEUK_OK ? std::string(teuk_last_error(h)) : std::string();
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    teuk_destroy(h);
    if (st != TEUK_OK) return tfail(st, "timing run: " + msg);
    if (e) return tfail(TEUK_ERR_DEVICE, std::string("timing events: ") + hipGetErrorString((hipError_t)e));
    *us = best;
    return TEUK_OK;
}

}  // namespace

namespace teuk {

int tuned_workgroups(const teuk_config& c)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    auto it = g_tuned.find(key_of(c, dev));
    return it == g_tuned.end() ? 0 : it->second;
}

}  // namespace teuk

extern "C" {

teuk_status teuk_tune(const teuk_config* cfg, int32_t steps, teuk_tune_info_t* out)
{
    if (!cfg || !out) return tfail(TEUK_ERR_INVALID_ARG, "cfg and out must not be NULL");
    if (steps < 0) return tfail(TEUK_ERR_INVALID_ARG, "steps must be >= 0");
    std::memset(out, 0, sizeof(*out));
    if (cfg->state_prec != TEUK_S_FP64)
        return tfail(TEUK_ERR_UNSUPPORTED, "the double-double kernel has a fixed launch shape (one wave per strip and row)");
    if (teuk_footprint_bytes(cfg) == 0) {
        teuk_solver* h = nullptr;
        const teuk_status st = teuk_create(cfg, nullptr, &h);   // reports why cfg is invalid
        return tfail(st == TEUK_OK ? TEUK_ERR_INVALID_ARG : st, teuk_last_error(nullptr));
    }
    int dev = 0;
    int e = (int)hipGetDevice(&dev);
    if (e) return tfail(TEUK_ERR_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString((hipError_t)e));
    const bool blocked = cfg->integrator == TEUK_RK_SSP33_BLOCKED;
    const int strip = blocked ? teuk::kBlockedPoints : teuk::kStripPoints;
    const int nstrips = (cfg->nr + strip - 1) / strip;
    const long long resident = blocked ? teuk::blocked_grid(cfg->weight_prec) : teuk::stage_grid(cfg->weight_prec, false, teuk::kernel_chart(*cfg));
    if (resident <= 0) return tfail(TEUK_ERR_UNSUPPORTED, "occupancy query failed");

    // candidate budgets around the resident count, one per distinct segment
    // count, and on grids too small to fill the GPU (where every budget near
    // the resident count gives one segment per row) longer segments of 2, 4
    // and 8 rows
    const double mult[] = {0.25, 0.375, 0.5, 0.625, 0.75, 0.875, 1.0, 1.25, 1.5, 2.0, 3.0, 4.0};
    std::vector<long long> raw;
    for (double f : mult) raw.push_back(std::max(1LL, (long long)(f * (double)resident)));
    for (int rows : {2, 4, 8})
        if (cfg->ntheta >= 2 * rows) raw.push_back((long long)nstrips * (cfg->ntheta / rows));
    std::vector<int> budgets;
    std::vector<int> seen;
    for (long long b : raw) {
        const int s = segs_for(b, nstrips, cfg->ntheta, !blocked);
        if (std::find(seen.begin(), seen.end(), s) != seen.end()) continue;
        seen.push_back(s);
        budgets.push_back((int)std::min<long long>(b, (1LL << 31) - 1));
    }
    const int default_segs = segs_for(resident, nstrips, cfg->ntheta, !blocked);

    hipStream_t stream = nullptr;
    e = (int)hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
    if (e) return tfail(TEUK_ERR_DEVICE, std::string("hipStreamCreateWithFlags: ") + hipGetErrorString((hipError_t)e));
    // a smooth state of order one (not zeros: the FP64 units draw less power
    // on zero data and the clock, which bounds these kernels, runs higher)
    const size_t plane = (size_t)cfg->nr * (size_t)cfg->ntheta;
    std::vector<double> zeros(4 * plane);
    for (size_t p = 0; p < 4; ++p)
        for (int k = 0; k < cfg->ntheta; ++k)
            for (int j = 0; j < cfg->nr; ++j)
                zeros[p * plane + (size_t)k * cfg->nr + j] =
                    std::sin(0.37 * j + 0.11 * k + (double)p) * std::cos(0.013 * j - 0.7 * (double)p);
    teuk_config base = *cfg;
    teuk_status st = TEUK_OK;
    int n = steps;
    if (n == 0) {
        // aim at about 2 ms per timed run
        double us = 0.0;
        st = time_budget(base, (int)resident, 4, stream, zeros, &us);
        n = st == TEUK_OK ? (int)std::min(2000.0, std::max(4.0, 2000.0 / std::max(us, 1e-3))) : 0;
    }
    double best_us = 0.0, default_us = 0.0;
    int best = 0;
    for (size_t i = 0; i < budgets.size() && st == TEUK_OK; ++i) {
        double us = 0.0;
        st = time_budget(base, budgets[i], n, stream, zeros, &us);
        if (st != TEUK_OK) break;
        if (seen[i] == default_segs) default_us = us;
        if (best == 0 || us < best_us) {
            best = budgets[i];
            best_us = us;
        }
    }
    (void)hipStreamDestroy(stream);
    if (st != TEUK_OK) return st;
    {
        std::lock_guard<std::mutex> lock(g_tune_mutex);
        g_tuned[key_of(*cfg, dev)] = best;
    }
    out->workgroups = best;
    out->segs = segs_for(best, nstrips, cfg->ntheta, !blocked);
    out->default_workgroups = (int32_t)std::min<long long>(resident, (1LL << 31) - 1);
    out->default_segs = default_segs;
    out->candidates = (int32_t)budgets.size();
    out->steps = n;
    out->us_per_step = best_us;
    out->us_per_step_default = default_us;
    return TEUK_OK;
}

void teuk_tune_forget(void)
{
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tuned.clear();
}

const char* teuk_tune_last_error(void)
{
    return g_tune_err.c_str();
}

}  // extern "C"
