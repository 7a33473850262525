// C ABI of libteuk (declared in include/teuk.h): validation, device buffers,
// the SSP-RK(3,3) step loop, waveform ring buffer, guard and extraction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <array>
#include <vector>

#include "teuk_coef.h"
#include "teuk_dd_tables.h"
#include "teuk_internal.h"

using namespace teuk;

struct teuk_solver {
    teuk_config cfg;
    hipStream_t stream = nullptr;
    bool owns = false;
    void* base = nullptr;
    size_t bytes = 0;
    double* u[3] = {nullptr, nullptr, nullptr};   // u^n, u^(1), u^(2)
    double* rtab = nullptr;
    double* ttab = nullptr;
    double* ctab = nullptr;                         // chart H per-point table
    bool dd = false;                                // double-double state
    double* dtab = nullptr;                         // double-double per-point table (pairs)
    DDScalars ddk{};                                // double-double constants
    long long vals = 0;                             // doubles in the state (4 planes, x2 for pairs)
    double* wave = nullptr;
    double* hwave = nullptr;                        // chart H horizon ring [samples][nth][4]
    int j_h = 0;                                    // chart H: first of the four horizon-stencil nodes
    double hw[4] = {0, 0, 0, 0}, hdw[4] = {0, 0, 0, 0};   // horizon value / derivative weights
    unsigned long long* cell = nullptr;             // dt-bound reduction cell
    int* flag = nullptr;                            // non-finite flag
    unsigned long long* scount = nullptr;           // samples recorded (FP64 state; device copy of `samples`)
    int* perr = nullptr;                            // pipelined step: a dependency wait timed out
    long long* pdone = nullptr;                     // pipelined step: stages completed per tile
    int pgrid = 0;                                  // pipelined step: workgroups per launch
    double dx = 0, dth = 0, dt = 0, dt_bound = 0;
    int j_e = 0;
    int nstrips = 0;
    int segs[2] = {0, 0};                           // theta segments per strip: stage 1, stages 2-3
    int bstrips = 0, bsegs = 0;                     // temporal blocking: tiles per launch = bstrips * bsegs
    long long plane = 0;
    long long steps = 0, samples = 0;
    bool have_init = false;
    int device = 0;
    teuk_group* group = nullptr;                    // group holding this solver, if any
    // graph mode: teuk_step replays a captured graph of graph_chunk steps
    int graph_chunk = 0;                            // 0: off
    hipStream_t cap_stream = nullptr;               // private stream the chunk is captured on
    hipGraphExec_t gexec = nullptr;                 // the captured chunk, or null
    long long graph_phase = -1;                     // steps % extract_every when it was captured
    const double* graph_u0 = nullptr;               // the state buffer u[0] when it was captured
    std::string err;
};

constexpr int kClasses = 12;  // (weight precision, launch class) pairs: 4 x (T, H, T with 4th-order theta)
constexpr int kMaxGraphChunk = 4096;   // steps per captured graph
constexpr long long kPipeSpinTicks = 200000000;   // 2 s of the 100 MHz real-time counter

// Group members are stepped in cache blocks: consecutive members of one
// (weight precision, chart) class whose solver footprints sum to at most this
// many bytes (a member larger than that is a block of its own).  A block runs
// all of a teuk_group_step's steps before the next block starts, so much of
// its state stays in the GPU's 256 MB last-level cache from one stage launch
// to the next instead of streaming from HBM at every stage.  Measured on the
// 64-solve batched workload (9.2 GB of footprint): 96 MiB blocks 5.04e10
// point-updates/s, 224 MiB 5.44e10, 256 MiB 5.56e10, 320 MiB 5.54e10, 448 MiB
// 5.17e10, one block per class 5.38e10.  Smaller blocks lose more to launches
// that do not fill the GPU than they gain in cache hits.
#ifndef TEUK_GROUP_BLOCK_MB
#define TEUK_GROUP_BLOCK_MB 256
#endif
constexpr long long kGroupBlockBytes = (long long)TEUK_GROUP_BLOCK_MB << 20;

// A cache block whose every member fills the GPU by itself (strips x rows at
// least the stage kernel's resident workgroups) is stepped by its members' own
// stage launches, member after member within each stage, instead of the
// batched launch (unless the caller fixed the batched launch's workgroup
// count): the single-solve launch keeps every workgroup resident from
// the start and carries the issue-priority steps and the DPP flux shift, which
// the batched launch, dispatching short tiles as slots free up, cannot use.
// Same arithmetic at every point, so the results are bitwise those of the
// batched launch.
#ifndef TEUK_GROUP_SOLO
#define TEUK_GROUP_SOLO 1
#endif

// One cache block: members [first, first + n) of the class order (their stage
// descriptors are consecutive in d_args), tile prefix sums from d_start + start.
struct GroupBlock {
    int cls = 0;
    int first = 0, n = 0;
    long long tiles = 0, units = 0;
    size_t start = 0;
    int grid = 0;
    bool solo = false;   // members stepped by their own single-solve launches
    long long solo_wg = 0;   // their stage-2/3 workgroups, summed over the members
};

struct teuk_group {
    hipStream_t stream = nullptr;
    int device = 0;
    int cap = 0;                                    // max members
    int workgroups = 0;                             // per stage launch; 0 = one per tile
    int rows = 8;                                   // theta rows per tile (target)
    long long block_bytes = kGroupBlockBytes;       // cache-block size (member footprints)
    std::vector<teuk_solver*> mem;                  // insertion order
    StageArgs* d_args = nullptr;                    // [3][cap]: per stage, members by weight precision
    long long* d_start = nullptr;                   // [2 cap + 2]: each block's tile prefix sums, from 0
    std::vector<StageArgs> h_args;
    std::vector<long long> h_start;
    std::vector<teuk_solver*> order;                // members in class order, block by block
    std::vector<GroupBlock> blocks;                 // class c = weight_prec + 4 * chart
    long long points = 0;
    // graph mode: each cache block replays a captured graph of graph_chunk steps
    int graph_chunk = 0;                            // 0: off
    hipStream_t cap_stream = nullptr;
    std::vector<hipGraphExec_t> gexec;              // per block, or null
    std::vector<std::vector<long long>> gphase;     // per block: its members' steps % extract_every at capture
    std::string err;
};

namespace {

thread_local std::string g_err;

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t u, rtab, ttab, ctab, dtab, wave, hwave, pipe, cells, total;
};

Layout layout_of(const teuk_config& c)
{
    Layout L;
    const size_t plane = (size_t)c.nr * (size_t)c.ntheta;
    const bool DD = c.state_prec == TEUK_S_DD;
    const size_t pv = DD ? 2 : 1;                      // doubles per value
    L.u = align_up(4 * plane * pv * sizeof(double));
    const bool H = c.chart == TEUK_CHART_HYPERBOLOIDAL;
    L.rtab = H ? 0 : align_up((size_t)kNRT * c.nr * sizeof(double));
    L.ttab = H ? 0 : align_up((size_t)kNTT * c.ntheta * sizeof(double));
    L.ctab = H ? align_up((size_t)kNCH * plane * sizeof(double)) : 0;
    L.dtab = DD ? align_up((size_t)kNDD * plane * 2 * sizeof(double)) : 0;
    const size_t ns = c.extract_every > 0 ? (size_t)c.max_samples : 0;
    L.wave = align_up(ns * (size_t)c.ntheta * 2 * pv * sizeof(double));
    L.hwave = H ? align_up(ns * (size_t)c.ntheta * 4 * sizeof(double)) : 0;
    // pipelined step: one stage counter per tile (at most one tile per strip and row)
    const size_t nstrips = ((size_t)c.nr + kStripPoints - 1) / kStripPoints;
    L.pipe = c.integrator == TEUK_RK_SSP33_PIPELINED ? align_up(nstrips * (size_t)c.ntheta * sizeof(long long)) : 0;
    L.cells = kAlign;
    L.total = 3 * L.u + L.rtab + L.ttab + L.ctab + L.dtab + L.wave + L.hwave + L.pipe + L.cells;
    return L;
}

// Horizon of the hyperboloidal chart, rho_H = S r+ / (r+ + S), at fractional
// node position f = (rho_H - x_min)/dx: the four nodes j0 .. j0+3 around it
// (j0 = floor(f) - 1, shifted to stay inside the grid, i.e. one-sided when the
// grid starts on the horizon) and the 4-point Lagrange weights for the value
// (w) and the rho-derivative (dw, divided by dx).  False unless
// -1/2 <= f <= nr - 3/2 (at most half a step of extrapolation at either end).
bool horizon_stencil(const teuk_config& c, int* j0, double* w, double* dw)
{
    const double d2 = c.M * c.M - c.a * c.a;
    const double rp = c.M + (d2 > 0.0 ? std::sqrt(d2) : 0.0);
    const double rho_h = c.S * rp / (rp + c.S);
    const double dx = (c.x_max - c.x_min) / (c.nr - 1);
    const double f = (rho_h - c.x_min) / dx;
    if (!(f >= -0.5) || !(f <= c.nr - 1.5) || c.nr < 4) return false;
    int jj = (int)std::floor(f) - 1;
    if (jj < 0) jj = 0;
    if (jj > c.nr - 4) jj = c.nr - 4;
    for (int i = 0; i < 4; ++i) {
        const double zi = jj + i;
        double num = 1.0, den = 1.0, dsum = 0.0;
        for (int k = 0; k < 4; ++k) {
            if (k == i) continue;
            const double zk = jj + k;
            num *= f - zk;
            den *= zi - zk;
            double prod = 1.0;                                 // d/df of the product, factor k left out
            for (int q = 0; q < 4; ++q)
                if (q != i && q != k) prod *= f - (jj + q);
            dsum += prod;
        }
        w[i] = num / den;
        dw[i] = dsum / den / dx;
    }
    *j0 = jj;
    return true;
}

bool validate(const teuk_config* c, std::string& err)
{
    if (!c) { err = "cfg is NULL"; return false; }
    if (c->abi_version != TEUK_ABI_VERSION) { err = "abi_version must be " + std::to_string(TEUK_ABI_VERSION); return false; }
    if (c->chart != TEUK_CHART_TORTOISE && c->chart != TEUK_CHART_HYPERBOLOIDAL) { err = "chart must be a TEUK_CHART_* value"; return false; }
    if (c->s < -2 || c->s > 2) { err = "spin weight s must satisfy |s| <= 2"; return false; }
    if (c->m < -8 || c->m > 8) { err = "azimuthal number m must satisfy |m| <= 8"; return false; }
    if (c->nr < 7 || c->nr > (1 << 24)) { err = "nr must be in [7, 2^24]"; return false; }
    if (c->ntheta < 2 || c->ntheta > 65536) { err = "ntheta must be in [2, 65536]"; return false; }
    if ((long long)c->nr * c->ntheta > (1LL << 34)) { err = "nr * ntheta too large"; return false; }
    if (c->weight_prec < TEUK_W_FP64 || c->weight_prec > TEUK_W_DD) { err = "weight_prec must be a TEUK_W_* value"; return false; }
    if (c->state_prec != TEUK_S_FP64 && c->state_prec != TEUK_S_DD) { err = "state_prec must be a TEUK_S_* value"; return false; }
    if (c->integrator < TEUK_RK_SSP33 || c->integrator > TEUK_RK_SSP33_PIPELINED) { err = "integrator must be a TEUK_RK_* value"; return false; }
    if (c->scheme < TEUK_SCHEME_WENO5 || c->scheme > TEUK_SCHEME_FD6KO8) { err = "scheme must be a TEUK_SCHEME_* value"; return false; }
    if (c->theta_order != 0 && c->theta_order != 2 && c->theta_order != 4) { err = "theta_order must be 0, 2 or 4"; return false; }
    if (!(c->ko_sigma >= 0.0) || !(c->ko_sigma <= 1.0)) { err = "ko_sigma must lie in [0, 1]"; return false; }
    if (c->weight_prec == TEUK_W_DD && c->state_prec != TEUK_S_DD) { err = "TEUK_W_DD weights need the TEUK_S_DD state"; return false; }
    if (!(c->M > 0.0) || !std::isfinite(c->M)) { err = "M must be positive and finite"; return false; }
    if (!(c->a >= 0.0) || !(c->a <= c->M)) { err = "spin a must satisfy 0 <= a <= M"; return false; }
    if (!std::isfinite(c->x_min) || !std::isfinite(c->x_max) || !(c->x_min < c->x_max)) { err = "need finite x_min < x_max"; return false; }
    if (!(c->weno_eps >= 1e-30) || !(c->weno_eps <= 1e30)) { err = "weno_eps must lie in [1e-30, 1e30]"; return false; }
    if (!std::isfinite(c->dt)) { err = "dt must be finite"; return false; }
    if (c->dt <= 0.0 && (!(c->cfl > 0.0) || !std::isfinite(c->cfl))) { err = "cfl must be positive when dt <= 0"; return false; }
    if (c->extract_every < 0 || c->max_samples < 0) { err = "extract_every and max_samples must be >= 0"; return false; }
    if (c->extract_every > 0) {
        if (c->max_samples < 1) { err = "max_samples must be >= 1 when extract_every > 0"; return false; }
        if (!(c->x_extract >= c->x_min && c->x_extract <= c->x_max)) { err = "x_extract must lie in [x_min, x_max]"; return false; }
    }
    if (c->workgroups < 0) { err = "workgroups must be >= 0"; return false; }
    if (c->chart == TEUK_CHART_HYPERBOLOIDAL) {
        if (!(c->S > 0.0) || !std::isfinite(c->S)) { err = "S must be positive and finite"; return false; }
        if (!(c->x_min > 0.0) || !(c->x_max < c->S)) { err = "hyperboloidal chart needs 0 < x_min and x_max < S"; return false; }
        int jh;
        double w[4], dw[4];
        if (!horizon_stencil(*c, &jh, w, dw)) {
            err = "hyperboloidal chart needs the horizon rho_H = S r+/(r+ + S) on the grid (at most half a "
                  "step outside it) and nr >= 4";
            return false;
        }
    }
    return true;
}

// Theta segments per radial strip: as many as fit the workgroups the GPU holds
// at once (or the caller's workgroup count), an even number when more than
// one so that neighbouring segments pair up, and at most one per theta row.
int pick_segs(const teuk_config& c, int nstrips, int weight_prec, bool first)
{
    // The stages of a solve take the same tiling (consecutive launches then
    // march the same tiles and meet at the same rows, whose lines are still in
    // L2), sized for the stage kernel that holds the fewer workgroups at once,
    // when the two stage kernels hold nearly as many (FP32 weights: stage 1
    // fits 17 workgroups per CU by LDS, stages 2-3 16 by VGPRs); when they
    // differ by a whole wave per SIMD (BF16 weights: 4 and 3), each stage
    // fills the GPU with its own count, which measured faster there.
    long long cap = c.workgroups;
    if (cap <= 0) {
        const long long g1 = stage_grid(weight_prec, true, kernel_chart(c));
        const long long g2 = stage_grid(weight_prec, false, kernel_chart(c));
        const long long lo = g1 < g2 ? g1 : g2, hi = g1 < g2 ? g2 : g1;
        cap = 8 * hi <= 9 * lo ? lo : (first ? g1 : g2);
    }
    if (cap <= 0) return 0;
    long long segs = cap / nstrips;
    if (segs > c.ntheta) segs = c.ntheta;
    if (segs > 1) segs &= ~1LL;
    if (segs < 1) segs = 1;
    return (int)segs;
}

teuk_status fail(teuk_solver* h, teuk_status st, const std::string& msg)
{
    if (h) h->err = msg; else g_err = msg;
    return st;
}

teuk_status hip_fail(teuk_solver* h, int e, const char* what)
{
    return fail(h, TEUK_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString((hipError_t)e));
}

// Destroy the solver's captured graph (after the work already enqueued on its
// stream, which may still be replaying it, has finished).
void drop_graph(teuk_solver* h)
{
    if (h->gexec) {
        (void)hipStreamSynchronize(h->stream);
        (void)hipGraphExecDestroy(h->gexec);
        h->gexec = nullptr;
    }
    h->graph_phase = -1;
    h->graph_u0 = nullptr;
}

void free_solver(teuk_solver* h)
{
    if (!h) return;
    drop_graph(h);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    if (h->owns && h->base) (void)hipFree(h->base);
    delete h;
}

teuk_status run_guard(teuk_solver* h)
{
    int e = (int)hipMemsetAsync(h->flag, 0, sizeof(int), h->stream);
    if (e) return hip_fail(h, e, "hipMemsetAsync(flag)");
    e = launch_guard(h->u[0], h->vals, h->flag, h->stream);
    if (e) return hip_fail(h, e, "guard launch");
    int f = 0;
    e = (int)hipMemcpyAsync(&f, h->flag, sizeof(int), hipMemcpyDeviceToHost, h->stream);
    if (e) return hip_fail(h, e, "hipMemcpyAsync(flag)");
    e = (int)hipStreamSynchronize(h->stream);
    if (e) return hip_fail(h, e, "hipStreamSynchronize");
    if (h->pdone) {
        int pe = 0;
        e = (int)hipMemcpy(&pe, h->perr, sizeof(int), hipMemcpyDeviceToHost);
        if (e) return hip_fail(h, e, "hipMemcpy(pipeline flag)");
        if (pe) return fail(h, TEUK_ERR_DEVICE, "pipelined step: a wait for neighbouring tiles timed out");
    }
    if (f) return fail(h, TEUK_ERR_NONFINITE, "non-finite value (NaN or Inf) in the state");
    return TEUK_OK;
}

teuk_status record_sample(teuk_solver* h)
{
    if (h->cfg.extract_every <= 0) return TEUK_OK;
    int e;
    if (h->dd) {
        const long long slot = h->samples % h->cfg.max_samples;
        e = launch_dd_extract(h->u[0], h->plane, h->cfg.nr, h->cfg.ntheta, h->j_e,
                              h->wave + (size_t)slot * h->cfg.ntheta * 4, h->stream);
    } else {
        // the slot is taken from the device copy of the sample count, so that a
        // captured chunk of steps samples into the right slots on every replay
        e = launch_sample(h->u[0], h->plane, h->cfg.nr, h->cfg.ntheta, h->j_e, h->wave, h->hwave, h->j_h, h->hw,
                          h->hdw, h->cfg.max_samples, h->scount, h->stream);
    }
    if (e) return hip_fail(h, e, "sample launch");
    ++h->samples;
    return TEUK_OK;
}

// Double-double table [kNDD][plane][2] -> TEUK_X_COEFFS order, pairs:
// lam1 = b, Re m3, Im m3, Re B~t, Im B~t, Re C~, Im C~, A~thth, B~th, lam2 = -b.
void dd_coeff_order(const double* t, long long plane, double* out)
{
    const int src[TEUK_NCOEF] = {kDB, kDM3r, kDM3i, kDBtr, kDBti, kDCr, kDCi, kDAth, kDBth, kDB};
    const size_t n = (size_t)plane * 2;
    for (int q = 0; q < TEUK_NCOEF; ++q) {
        const double* a = t + (size_t)src[q] * n;
        double* o = out + (size_t)q * n;
        if (q == TEUK_NCOEF - 1)
            for (size_t i = 0; i < n; ++i) o[i] = -a[i];
        else
            std::memcpy(o, a, n * sizeof(double));
    }
}

}  // namespace

extern "C" {

void teuk_default_config(teuk_config* c)
{
    if (!c) return;
    std::memset(c, 0, sizeof(*c));
    c->abi_version = TEUK_ABI_VERSION;
    c->chart = TEUK_CHART_TORTOISE;
    c->weight_prec = TEUK_W_FP64;
    c->M = 1.0;
    c->cfl = 0.5;
    c->weno_eps = 1e-6;
    c->S = 20.0;
    c->ko_sigma = 0.01;
    c->theta_order = 2;
}

size_t teuk_footprint_bytes(const teuk_config* cfg)
{
    std::string err;
    if (!validate(cfg, err)) return 0;
    return layout_of(*cfg).total;
}

teuk_status teuk_create(const teuk_config* cfg, const teuk_device_ctx* ctx, teuk_solver** out)
{
    if (!out) return fail(nullptr, TEUK_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    std::string err;
    if (!validate(cfg, err)) return fail(nullptr, TEUK_ERR_INVALID_ARG, err);
    const bool chartH = cfg->chart == TEUK_CHART_HYPERBOLOIDAL;
    const bool dd = cfg->state_prec == TEUK_S_DD;
    if (dd && (chartH || (cfg->weight_prec != TEUK_W_DD && cfg->weight_prec != TEUK_W_FP64)))
        return fail(nullptr, TEUK_ERR_UNSUPPORTED,
                    "double-double state: tortoise chart with TEUK_W_DD or TEUK_W_FP64 weights only");
    if (dd && cfg->integrator != TEUK_RK_SSP33)
        return fail(nullptr, TEUK_ERR_UNSUPPORTED, "double-double state: SSP-RK(3,3) only");
    if (cfg->scheme != TEUK_SCHEME_WENO5 && (dd || cfg->weight_prec != TEUK_W_FP64))
        return fail(nullptr, TEUK_ERR_UNSUPPORTED, "comparison schemes: FP64 state and weights only");
    if (cfg->integrator == TEUK_RK_SSP33_BLOCKED &&
        (chartH || dd || cfg->scheme != TEUK_SCHEME_WENO5 ||
         (cfg->weight_prec != TEUK_W_FP64 && cfg->weight_prec != TEUK_W_FP32)))
        return fail(nullptr, TEUK_ERR_UNSUPPORTED,
                    "temporal blocking: tortoise chart, FP64 state, WENO5 with FP64 or FP32 weights only");
    if (cfg->integrator == TEUK_RK_SSP33_PIPELINED &&
        (chartH || dd || cfg->scheme != TEUK_SCHEME_WENO5 || cfg->weight_prec == TEUK_W_DD))
        return fail(nullptr, TEUK_ERR_UNSUPPORTED, "pipelined steps: tortoise chart, FP64 state, WENO5 only");
    if (cfg->theta_order == 4 &&
        (chartH || dd || cfg->scheme != TEUK_SCHEME_WENO5 ||
         (cfg->integrator != TEUK_RK_SSP33 && cfg->integrator != TEUK_RK_SSP104)))
        return fail(nullptr, TEUK_ERR_UNSUPPORTED,
                    "fourth-order theta differences: tortoise chart, FP64 state, WENO5, "
                    "SSP-RK(3,3) or SSP-RK(10,4) stepped stage by stage");
    std::vector<double> rtab, ttab, ctab, dtab;
    DDScalars ddk{};
    if (chartH ? !build_tables_H(*cfg, ctab, err) : !build_tables(*cfg, rtab, ttab, err))
        return fail(nullptr, TEUK_ERR_INVALID_ARG, err);
    if (dd && !build_tables_dd(*cfg, dtab, &ddk, err)) return fail(nullptr, TEUK_ERR_INVALID_ARG, err);

    teuk_solver* h = new (std::nothrow) teuk_solver();
    if (!h) return fail(nullptr, TEUK_ERR_OUT_OF_MEMORY, "host allocation failed");
    h->cfg = *cfg;
    h->stream = ctx ? (hipStream_t)ctx->stream : nullptr;
    (void)hipGetDevice(&h->device);
    const Layout L = layout_of(*cfg);
    h->bytes = L.total;
    if (ctx && ctx->workspace) {
        if (ctx->workspace_bytes < L.total) {
            delete h;
            return fail(nullptr, TEUK_ERR_OUT_OF_MEMORY,
                        "workspace holds " + std::to_string(ctx->workspace_bytes) + " bytes, solver needs " +
                            std::to_string(L.total));
        }
        if (((uintptr_t)ctx->workspace) % kAlign) {
            delete h;
            return fail(nullptr, TEUK_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
        }
        h->base = ctx->workspace;
        h->owns = false;
    } else {
        int e = (int)hipMalloc(&h->base, L.total);
        if (e) {
            h->base = nullptr;
            delete h;
            (void)hipGetLastError();
            return fail(nullptr, e == (int)hipErrorOutOfMemory ? TEUK_ERR_OUT_OF_MEMORY : TEUK_ERR_DEVICE,
                        std::string("hipMalloc: ") + hipGetErrorString((hipError_t)e));
        }
        h->owns = true;
    }
    char* p = (char*)h->base;
    for (int i = 0; i < 3; ++i) { h->u[i] = (double*)p; p += L.u; }
    h->rtab = L.rtab ? (double*)p : nullptr; p += L.rtab;
    h->ttab = L.ttab ? (double*)p : nullptr; p += L.ttab;
    h->ctab = L.ctab ? (double*)p : nullptr; p += L.ctab;
    h->dtab = L.dtab ? (double*)p : nullptr; p += L.dtab;
    h->dd = dd;
    h->ddk = ddk;
    h->wave = (double*)p; p += L.wave;
    h->hwave = L.hwave ? (double*)p : nullptr; p += L.hwave;
    h->pdone = L.pipe ? (long long*)p : nullptr; p += L.pipe;
    if (chartH) (void)horizon_stencil(*cfg, &h->j_h, h->hw, h->hdw);
    h->cell = (unsigned long long*)p;
    h->flag = (int*)(p + 64);
    h->scount = (unsigned long long*)(p + 128);
    h->perr = (int*)(p + 192);

    h->plane = (long long)cfg->nr * cfg->ntheta;
    h->vals = 4 * h->plane * (dd ? 2 : 1);
    h->dx = (cfg->x_max - cfg->x_min) / (cfg->nr - 1);
    h->dth = M_PI / cfg->ntheta;
    h->nstrips = (cfg->nr + kStripPoints - 1) / kStripPoints;
    // the caller's workgroup budget, else the one teuk_tune found for this
    // launch class on this device, else (0) all the GPU holds at once
    teuk_config eff = *cfg;
    if (eff.workgroups == 0) eff.workgroups = tuned_workgroups(*cfg);
    // (the double-double kernel runs one wave per strip and theta row)
    h->segs[0] = dd ? 1 : pick_segs(eff, h->nstrips, cfg->weight_prec, true);
    h->segs[1] = dd ? 1 : pick_segs(eff, h->nstrips, cfg->weight_prec, false);
    if (h->segs[0] <= 0 || h->segs[1] <= 0 || (long long)h->nstrips * h->segs[0] > (1LL << 31) - 1 ||
        (long long)h->nstrips * h->segs[1] > (1LL << 31) - 1) {
        free_solver(h);
        return fail(nullptr, TEUK_ERR_UNSUPPORTED, "weight precision not built (or occupancy query failed)");
    }
    if (cfg->integrator == TEUK_RK_SSP33_PIPELINED) {
        // every stage runs the later-stage tiling; all workgroups resident at once
        const long long tiles = (long long)h->nstrips * h->segs[1];
        const long long cap = pipe_grid(cfg->weight_prec);
        h->pgrid = (int)(cap < tiles ? cap : tiles);
        if (cap <= 0 || tiles > (1LL << 31) - 1) {
            free_solver(h);
            return fail(nullptr, TEUK_ERR_UNSUPPORTED, "pipelined steps: occupancy query failed");
        }
    }
    if (cfg->integrator == TEUK_RK_SSP33_BLOCKED) {
        h->bstrips = (cfg->nr + kBlockedPoints - 1) / kBlockedPoints;
        long long cap = eff.workgroups > 0 ? eff.workgroups : blocked_grid(cfg->weight_prec);
        long long segs = cap / h->bstrips;
        if (segs > cfg->ntheta) segs = cfg->ntheta;
        if (segs < 1) segs = 1;
        h->bsegs = (int)segs;
        if (cap <= 0 || (long long)h->bstrips * h->bsegs > (1LL << 31) - 1) {
            free_solver(h);
            return fail(nullptr, TEUK_ERR_UNSUPPORTED, "temporal blocking: occupancy query failed");
        }
    }
    h->j_e = cfg->extract_every > 0 ? (int)std::floor((cfg->x_extract - cfg->x_min) / h->dx + 0.5) : 0;
    if (h->j_e > cfg->nr - 1) h->j_e = cfg->nr - 1;

    int e = 0;
    if (chartH) {
        e = (int)hipMemcpyAsync(h->ctab, ctab.data(), ctab.size() * sizeof(double), hipMemcpyHostToDevice, h->stream);
    } else {
        e = (int)hipMemcpyAsync(h->rtab, rtab.data(), rtab.size() * sizeof(double), hipMemcpyHostToDevice, h->stream);
        if (!e) e = (int)hipMemcpyAsync(h->ttab, ttab.data(), ttab.size() * sizeof(double), hipMemcpyHostToDevice, h->stream);
    }
    if (!e && dd)
        e = (int)hipMemcpyAsync(h->dtab, dtab.data(), dtab.size() * sizeof(double), hipMemcpyHostToDevice, h->stream);
    if (!e) e = (int)hipMemsetAsync(h->cell, 0, sizeof(unsigned long long), h->stream);
    if (!e) e = (int)hipMemsetAsync(h->perr, 0, sizeof(int), h->stream);
    if (!e) e = launch_dt_bound(h->rtab, h->ttab, h->ctab, cfg->nr, cfg->ntheta, h->dx, h->dth, cfg->theta_order,
                                h->cell, h->stream);
    unsigned long long bits = 0;
    if (!e) e = (int)hipMemcpyAsync(&bits, h->cell, sizeof(bits), hipMemcpyDeviceToHost, h->stream);
    if (!e) e = (int)hipStreamSynchronize(h->stream);
    if (e) {
        std::string msg = std::string("device setup: ") + hipGetErrorString((hipError_t)e);
        free_solver(h);
        return fail(nullptr, TEUK_ERR_DEVICE, msg);
    }
    double mx;
    std::memcpy(&mx, &bits, sizeof(mx));
    if (!(mx > 0.0) || !std::isfinite(mx)) {
        free_solver(h);
        return fail(nullptr, TEUK_ERR_NONFINITE, "stability bound is not finite");
    }
    h->dt_bound = 1.0 / mx;
    const double ssp_c = cfg->integrator == TEUK_RK_SSP104 ? 6.0 : 1.0;   // SSP coefficient (Sec. 3.2)
    h->dt = cfg->dt > 0.0 ? cfg->dt : cfg->cfl * ssp_c * h->dt_bound;
    *out = h;
    return TEUK_OK;
}

teuk_status teuk_set_initial(teuk_solver* h, const double* u, int32_t on_device)
{
    if (!h) return fail(nullptr, TEUK_ERR_INVALID_ARG, "solver is NULL");
    if (!u) return fail(h, TEUK_ERR_INVALID_ARG, "u is NULL");
    const size_t n = (size_t)h->vals;
    std::vector<double> norm;
    if (!on_device) {
        for (size_t i = 0; i < n; ++i)
            if (!std::isfinite(u[i])) return fail(h, TEUK_ERR_NONFINITE, "initial data contain NaN or Inf");
        if (h->dd) {
            // store each pair normalised: TwoSum(hi, lo)
            norm.resize(n);
            for (size_t i = 0; i < n; i += 2) {
                const double a = u[i], b = u[i + 1];
                const double s = a + b, bb = s - a;
                norm[i] = s;
                norm[i + 1] = (a - (s - bb)) + (b - bb);
            }
            u = norm.data();
        }
    }
    int e = (int)hipMemcpyAsync(h->u[0], u, n * sizeof(double),
                                on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, h->stream);
    if (e) return hip_fail(h, e, "hipMemcpyAsync(initial state)");
    if (on_device && h->dd) {
        e = launch_dd_normalise(h->u[0], (long long)n / 2, h->stream);
        if (e) return hip_fail(h, e, "normalise launch");
    }
    if (!on_device) {
        e = (int)hipStreamSynchronize(h->stream);   // host array may be released after return
        if (e) return hip_fail(h, e, "hipStreamSynchronize");
    } else {
        teuk_status st = run_guard(h);
        if (st != TEUK_OK) return st;
    }
    h->steps = 0;
    h->samples = 0;
    if (h->pdone) {
        e = (int)hipMemsetAsync(h->pdone, 0, (size_t)h->nstrips * h->segs[1] * sizeof(long long), h->stream);
        if (e) return hip_fail(h, e, "hipMemsetAsync(stage counters)");
    }
    if (!h->dd && h->cfg.extract_every > 0) {
        static const unsigned long long kZero = 0;
        e = (int)hipMemcpyAsync(h->scount, &kZero, sizeof(kZero), hipMemcpyHostToDevice, h->stream);
        if (e) return hip_fail(h, e, "hipMemcpyAsync(sample count)");
    }
    h->have_init = true;
    return record_sample(h);
}

static DDStageArgs dd_args(const teuk_solver* h)
{
    const teuk_config& c = h->cfg;
    DDStageArgs a{};
    a.ctab = h->dtab;
    a.plane = h->plane;
    a.nr = c.nr;
    a.nth = c.ntheta;
    a.nstrips = h->nstrips;
    auto cp = [](double* d, const double* s) { d[0] = s[0]; d[1] = s[1]; };
    cp(a.inv_dx, h->ddk.inv_dx);
    cp(a.ih1, h->ddk.ih1);
    cp(a.ih2, h->ddk.ih2);
    cp(a.sixth, h->ddk.sixth);
    cp(a.c13_3, h->ddk.c13_3);
    for (int q = 0; q < 3; ++q) cp(a.d[q], h->ddk.d[q]);
    a.ca[0] = a.ca[1] = a.cb[1] = 0.0;
    a.cb[0] = 1.0;
    a.dt = h->dt;
    a.eps = c.weno_eps;
    a.parity = ((c.m + c.s) % 2 != 0) ? -1.0 : 1.0;
    a.uk = a.un = h->u[0];
    a.out = h->u[1];
    return a;
}

// One SSP-RK(3,3) step of the double-double state, the same three stages as
// the FP64 path with the combination coefficients as double-double pairs.
static int dd_step(teuk_solver* h)
{
    DDStageArgs a = dd_args(h);
    const int wp = h->cfg.weight_prec;
    a.uk = h->u[0]; a.un = h->u[0]; a.out = h->u[1];
    int e = launch_dd_stage(a, 1, wp, h->stream);
    if (!e) {
        a.uk = h->u[1]; a.out = h->u[2];
        a.ca[0] = 0.75; a.cb[0] = 0.25;
        e = launch_dd_stage(a, 2, wp, h->stream);
    }
    if (!e) {
        a.uk = h->u[2]; a.out = h->u[0];
        a.ca[0] = h->ddk.third[0]; a.ca[1] = h->ddk.third[1];
        a.cb[0] = h->ddk.two_thirds[0]; a.cb[1] = h->ddk.two_thirds[1];
        e = launch_dd_stage(a, 3, wp, h->stream);
    }
    return e;
}

static StageArgs stage_args(const teuk_solver* h)
{
    const teuk_config& c = h->cfg;
    StageArgs a;
    a.rtab = h->rtab;
    a.ttab = h->ttab;
    a.ctab = h->ctab;
    a.plane = h->plane;
    a.nr = c.nr;
    a.nth = c.ntheta;
    a.nstrips = h->nstrips;
    a.segs = h->segs[0];
    a.grid = h->nstrips * h->segs[0];
    a.inv6dx = 1.0 / (6.0 * h->dx);
    theta_scales(c.theta_order, h->dth, &a.ih1, &a.ih2);
    a.dt = h->dt;
    a.ca = 0.0;
    a.cb = 1.0;
    a.out2 = nullptr;
    a.ca2 = a.cb2 = 0.0;
    a.inv_dx = 1.0 / h->dx;
    a.ko_sigma = c.ko_sigma;
    a.eps = c.weno_eps;
    a.parity = ((c.m + c.s) % 2 != 0) ? -1.0 : 1.0;
    a.flip = 0;
    a.uk = a.un = h->u[0];
    a.out = h->u[1];
    return a;
}

// Stage `stage` (1..3) of one SSP-RK(3,3) step of h, from a = stage_args(h).
// Consecutive launches march their theta segments in opposite directions (flip
// alternates with the launch count 3 steps + stage), so that a stage starts on
// the rows the previous one wrote last, which are still in the XCD's L2.  The
// arithmetic of every point is the same either way.
static void rk3_stage(const teuk_solver* h, StageArgs& a, int stage)
{
    const int flip = (int)(h->steps & 1);
    if (stage == 1) {            // u1 = u + dt F(u)
        a.uk = h->u[0]; a.un = h->u[0]; a.out = h->u[1]; a.ca = 0.0; a.cb = 1.0;
        a.segs = h->segs[0]; a.flip = flip;
    } else if (stage == 2) {     // u2 = 3/4 u + 1/4 (u1 + dt F(u1))
        a.uk = h->u[1]; a.un = h->u[0]; a.out = h->u[2]; a.ca = 0.75; a.cb = 0.25;
        a.segs = h->segs[1]; a.flip = flip ^ 1;
    } else {                     // u = 1/3 u + 2/3 (u2 + dt F(u2)), in place (u^n read at the own point only)
        a.uk = h->u[2]; a.un = h->u[0]; a.out = h->u[0]; a.ca = 1.0 / 3.0; a.cb = 2.0 / 3.0;
        a.segs = h->segs[1]; a.flip = flip;
    }
    a.grid = h->nstrips * a.segs;
}

// One temporally blocked SSP-RK(3,3) step of h on `stream`: u^n in u[0], u^{n+1}
// written to u[1], then the two buffers trade roles.
static int blocked_step_once(teuk_solver* h, hipStream_t stream)
{
    StageArgs a = stage_args(h);
    a.nstrips = h->bstrips;
    a.segs = h->bsegs;
    a.grid = h->bstrips * h->bsegs;
    a.ca = 0.0;
    a.cb = 1.0;
    a.uk = h->u[0];
    a.un = h->u[0];
    a.out = h->u[1];
    const int e = launch_blocked_step(a, h->cfg.weight_prec, stream);
    if (!e) std::swap(h->u[0], h->u[1]);             // u^{n+1} is the new state buffer
    return e;
}

// One stage launch of the solver's radial scheme.
static int run_stage(const teuk_solver* h, const StageArgs& a, int stage)
{
    const teuk_config& c = h->cfg;
    if (c.scheme != TEUK_SCHEME_WENO5) return launch_cmp_stage(a, stage, c.scheme, c.chart, h->stream);
    return launch_stage(a, stage, c.weight_prec, kernel_chart(c), h->stream);
}

// One SSP-RK(10,4) step (Sec. 3.2) in the three state buffers U = u^n,
// A = u[1], B = u[2]: stages 1-4 ping-pong U -> A -> B -> A -> B (= u(4)) with
// out = u + dt/6 F(u); stage 5 reads B and u^n and writes u(5) = 3/5 u^n + 2/5 v
// into A and q = 1/25 u^n + 9/25 v over U (v = u(4) + dt/6 F(u(4)), u^n read at
// the own point only); stages 6-9 ping-pong A -> B -> A -> B -> A (= u(9));
// stage 10 writes u^{n+1} = q + 3/5 (u(9) + dt/6 F(u(9))) over U.
static int rk104_step(teuk_solver* h, StageArgs a)
{
    double* U = h->u[0];
    double* AB[2] = {h->u[1], h->u[2]};
    a.dt = h->dt / 6.0;
    a.segs = h->segs[0];
    a.grid = h->nstrips * h->segs[0];
    a.ca = 0.0;
    a.cb = 1.0;
    int e = 0;
    const double* in = U;
    for (int st = 1; st <= 4 && !e; ++st) {
        a.uk = in;
        a.un = in;
        a.out = AB[(st - 1) & 1];   // A, B, A, B
        e = run_stage(h, a, 1);
        in = a.out;
    }
    if (e) return e;
    a.segs = h->segs[1];
    a.grid = h->nstrips * h->segs[1];
    a.uk = AB[1];
    a.un = U;
    a.out = AB[0];
    a.ca = 3.0 / 5.0;
    a.cb = 2.0 / 5.0;
    a.out2 = U;
    a.ca2 = 1.0 / 25.0;
    a.cb2 = 9.0 / 25.0;
    e = run_stage(h, a, 4);
    a.out2 = nullptr;
    a.segs = h->segs[0];
    a.grid = h->nstrips * h->segs[0];
    a.ca = 0.0;
    a.cb = 1.0;
    in = AB[0];
    for (int st = 6; st <= 9 && !e; ++st) {
        a.uk = in;
        a.un = in;
        a.out = AB[(st - 5) & 1];   // B, A, B, A
        e = run_stage(h, a, 1);
        in = a.out;
    }
    if (e) return e;
    a.segs = h->segs[1];
    a.grid = h->nstrips * h->segs[1];
    a.uk = in;                 // u(9), in A
    a.un = U;                  // q
    a.out = U;
    a.ca = 1.0;
    a.cb = 3.0 / 5.0;
    return run_stage(h, a, 2);
}

// nsteps steps launch by launch on h->stream.
static teuk_status step_eager(teuk_solver* h, int64_t nsteps)
{
    const teuk_config& c = h->cfg;
    if (h->dd) {
        for (int64_t n = 0; n < nsteps; ++n) {
            const int e = dd_step(h);
            if (e) return hip_fail(h, e, "stage launch");
            ++h->steps;
            if (c.extract_every > 0 && h->steps % c.extract_every == 0) {
                teuk_status st = record_sample(h);
                if (st != TEUK_OK) return st;
            }
        }
        return TEUK_OK;
    }
    StageArgs a = stage_args(h);
    if (c.integrator == TEUK_RK_SSP33_BLOCKED) {
        for (int64_t n = 0; n < nsteps; ++n) {
            const int e = blocked_step_once(h, h->stream);
            if (e) return hip_fail(h, e, "blocked step launch");
            ++h->steps;
            if (c.extract_every > 0 && h->steps % c.extract_every == 0) {
                teuk_status st = record_sample(h);
                if (st != TEUK_OK) return st;
            }
        }
        return TEUK_OK;
    }
    if (c.integrator == TEUK_RK_SSP33_PIPELINED) {
        StageArgs st[3];
        a.segs = h->segs[1];
        a.grid = h->pgrid;
        st[0] = a; st[0].uk = h->u[0]; st[0].un = h->u[0]; st[0].out = h->u[1]; st[0].ca = 0.0; st[0].cb = 1.0;
        st[1] = a; st[1].uk = h->u[1]; st[1].un = h->u[0]; st[1].out = h->u[2]; st[1].ca = 0.75; st[1].cb = 0.25;
        st[2] = a; st[2].uk = h->u[2]; st[2].un = h->u[0]; st[2].out = h->u[0]; st[2].ca = 1.0 / 3.0; st[2].cb = 2.0 / 3.0;
        for (int64_t left = nsteps; left > 0;) {
            // up to the next waveform sample, at most 1000 steps per launch
            int64_t k = left < 1000 ? left : 1000;
            if (c.extract_every > 0) {
                const int64_t to_sample = c.extract_every - h->steps % c.extract_every;
                if (k > to_sample) k = to_sample;
            }
            const int e = launch_pipe(st, h->pdone, h->perr, 3 * h->steps, (int)k, h->pgrid, kPipeSpinTicks,
                                      c.weight_prec, h->stream);
            if (e) return hip_fail(h, e, "pipelined launch");
            h->steps += k;
            left -= k;
            if (c.extract_every > 0 && h->steps % c.extract_every == 0) {
                teuk_status st2 = record_sample(h);
                if (st2 != TEUK_OK) return st2;
            }
        }
        return TEUK_OK;
    }
    if (c.integrator == TEUK_RK_SSP104) {
        for (int64_t n = 0; n < nsteps; ++n) {
            const int e = rk104_step(h, a);
            if (e) return hip_fail(h, e, "stage launch");
            ++h->steps;
            if (c.extract_every > 0 && h->steps % c.extract_every == 0) {
                teuk_status st = record_sample(h);
                if (st != TEUK_OK) return st;
            }
        }
        return TEUK_OK;
    }
    for (int64_t n = 0; n < nsteps; ++n) {
        int e = 0;
        for (int stage = 1; stage <= 3 && !e; ++stage) {
            rk3_stage(h, a, stage);
            e = run_stage(h, a, stage);
        }
        if (e) return hip_fail(h, e, "stage launch");
        ++h->steps;
        if (c.extract_every > 0 && h->steps % c.extract_every == 0) {
            teuk_status st = record_sample(h);
            if (st != TEUK_OK) return st;
        }
    }
    return TEUK_OK;
}

// Capture graph_chunk steps of h into a graph (on the solver's private
// capture stream, with the host counters and buffer roles restored after) and
// instantiate it; the captured launches are the ones step_eager enqueues.
static teuk_status capture_chunk(teuk_solver* h)
{
    const long long every = h->cfg.extract_every;
    const long long phase = every > 0 ? h->steps % every : 0;
    // the graph holds the buffer roles of its capture: the blocked step trades
    // u[0] and u[1] every step, so an odd number of eager steps since needs
    // a new capture even where the sampling phase is unchanged
    if (h->gexec && h->graph_phase == phase && h->graph_u0 == h->u[0]) return TEUK_OK;
    drop_graph(h);
    int e = 0;
    if (!h->cap_stream) {
        e = (int)hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking);
        if (e) {
            h->cap_stream = nullptr;
            return hip_fail(h, e, "hipStreamCreateWithFlags");
        }
    }
    const hipStream_t saved_stream = h->stream;
    const long long saved_steps = h->steps, saved_samples = h->samples;
    double* const saved_u[3] = {h->u[0], h->u[1], h->u[2]};
    e = (int)hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e) return hip_fail(h, e, "hipStreamBeginCapture");
    h->stream = h->cap_stream;
    const teuk_status st = step_eager(h, h->graph_chunk);
    h->stream = saved_stream;
    hipGraph_t graph = nullptr;
    e = (int)hipStreamEndCapture(h->cap_stream, &graph);
    h->steps = saved_steps;
    h->samples = saved_samples;
    for (int i = 0; i < 3; ++i) h->u[i] = saved_u[i];
    if (st != TEUK_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e || !graph) return hip_fail(h, e ? e : (int)hipErrorUnknown, "hipStreamEndCapture");
    e = (int)hipGraphInstantiate(&h->gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e) {
        h->gexec = nullptr;
        return hip_fail(h, e, "hipGraphInstantiate");
    }
    // move the graph's launch resources to the device now, so that the first
    // replay costs what later ones do
    e = (int)hipGraphUpload(h->gexec, h->stream);
    if (e) {
        (void)hipGraphExecDestroy(h->gexec);
        h->gexec = nullptr;
        return hip_fail(h, e, "hipGraphUpload");
    }
    h->graph_phase = phase;
    h->graph_u0 = h->u[0];
    return TEUK_OK;
}

teuk_status teuk_step(teuk_solver* h, int64_t nsteps)
{
    if (!h) return fail(nullptr, TEUK_ERR_INVALID_ARG, "solver is NULL");
    if (nsteps < 0) return fail(h, TEUK_ERR_INVALID_ARG, "nsteps must be >= 0");
    if (!h->have_init) return fail(h, TEUK_ERR_STATE, "teuk_step before teuk_set_initial");
    const int64_t chunk = h->graph_chunk;
    if (chunk > 0 && nsteps >= chunk) {
        teuk_status st = capture_chunk(h);
        if (st != TEUK_OK) return st;
        const long long every = h->cfg.extract_every;
        const long long per = every > 0 ? chunk / every : 0;   // chunk is a multiple of extract_every
        for (int64_t q = nsteps / chunk; q > 0; --q) {
            const int e = (int)hipGraphLaunch(h->gexec, h->stream);
            if (e) return hip_fail(h, e, "hipGraphLaunch");
            h->steps += chunk;
            h->samples += per;
        }
        return step_eager(h, nsteps % chunk);
    }
    return step_eager(h, nsteps);
}

teuk_status teuk_set_graph(teuk_solver* h, int32_t chunk_steps)
{
    if (!h) return fail(nullptr, TEUK_ERR_INVALID_ARG, "solver is NULL");
    if (chunk_steps < 0 || chunk_steps > kMaxGraphChunk)
        return fail(h, TEUK_ERR_INVALID_ARG, "chunk_steps must be in [0, " + std::to_string(kMaxGraphChunk) + "]");
    if (chunk_steps > 0) {
        if (h->dd) return fail(h, TEUK_ERR_UNSUPPORTED, "graph mode: FP64 state only");
        if (h->cfg.integrator == TEUK_RK_SSP33_PIPELINED)
            return fail(h, TEUK_ERR_UNSUPPORTED, "graph mode: the pipelined step is one cooperative launch already");
        if (h->cfg.extract_every > 0 && chunk_steps % h->cfg.extract_every != 0)
            return fail(h, TEUK_ERR_INVALID_ARG, "chunk_steps must be a multiple of extract_every");
        if (h->cfg.integrator == TEUK_RK_SSP33_BLOCKED && chunk_steps % 2 != 0)
            return fail(h, TEUK_ERR_INVALID_ARG, "the blocked step swaps two buffers per step: chunk_steps must be even");
    }
    drop_graph(h);
    h->graph_chunk = chunk_steps;
    // capture now, at the current sampling phase, so that the first replays
    // do not pay for it
    if (chunk_steps > 0 && h->have_init) return capture_chunk(h);
    return TEUK_OK;
}

teuk_status teuk_extract(teuk_solver* h, int32_t what, double* out, size_t capacity, size_t* written)
{
    if (written) *written = 0;
    if (!h) return fail(nullptr, TEUK_ERR_INVALID_ARG, "solver is NULL");
    if (!out) return fail(h, TEUK_ERR_INVALID_ARG, "out is NULL");
    const teuk_config& c = h->cfg;
    const long long nsamp = c.extract_every > 0 ? (h->samples < c.max_samples ? h->samples : c.max_samples) : 0;
    size_t need = 0;
    const size_t pv = h->dd ? 2 : 1;
    switch (what) {
    case TEUK_X_STATE: need = (size_t)h->vals; break;
    case TEUK_X_WAVEFORM: need = (size_t)nsamp * c.ntheta * 2 * pv; break;
    case TEUK_X_TIMES: need = (size_t)nsamp; break;
    case TEUK_X_COEFFS: need = (size_t)TEUK_NCOEF * h->plane * pv; break;
    case TEUK_X_RHS: need = (size_t)h->vals; break;
    case TEUK_X_HORIZON:
        if (!h->hwave) return fail(h, TEUK_ERR_UNSUPPORTED, "horizon samples need the hyperboloidal chart and a waveform cadence");
        need = (size_t)nsamp * c.ntheta * 4;
        break;
    default: return fail(h, TEUK_ERR_INVALID_ARG, "unknown extract kind");
    }
    if (capacity < need) return fail(h, TEUK_ERR_CAPACITY, "output holds " + std::to_string(capacity) +
                                                              " doubles, need " + std::to_string(need));
    if ((what == TEUK_X_STATE || what == TEUK_X_WAVEFORM || what == TEUK_X_RHS || what == TEUK_X_HORIZON) &&
        !h->have_init)
        return fail(h, TEUK_ERR_STATE, "no state: call teuk_set_initial first");
    int e = 0;
    teuk_status guard = TEUK_OK;
    if (what == TEUK_X_STATE) {
        guard = run_guard(h);
        if (guard == TEUK_ERR_DEVICE) return guard;
        e = (int)hipMemcpyAsync(out, h->u[0], need * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    } else if (what == TEUK_X_WAVEFORM) {
        const long long first = h->samples - nsamp;          // oldest sample kept
        const size_t per = (size_t)c.ntheta * 2 * pv;
        for (long long i = 0; i < nsamp && !e; ++i) {
            const long long slot = (first + i) % c.max_samples;
            e = (int)hipMemcpyAsync(out + i * per, h->wave + slot * per, per * sizeof(double),
                                    hipMemcpyDeviceToHost, h->stream);
        }
    } else if (what == TEUK_X_HORIZON) {
        const long long first = h->samples - nsamp;
        const size_t per = (size_t)c.ntheta * 4;
        for (long long i = 0; i < nsamp && !e; ++i) {
            const long long slot = (first + i) % c.max_samples;
            e = (int)hipMemcpyAsync(out + i * per, h->hwave + slot * per, per * sizeof(double),
                                    hipMemcpyDeviceToHost, h->stream);
        }
    } else if (what == TEUK_X_RHS) {
        // F(u^n) by the stage kernel itself, written into the u^(1) buffer
        // (scratch between steps), then copied out
        if (h->dd) {
            DDStageArgs a = dd_args(h);
            e = launch_dd_stage(a, 0, h->cfg.weight_prec, h->stream);
        } else {
            StageArgs a = stage_args(h);
            e = run_stage(h, a, 0);
        }
        if (!e) e = (int)hipMemcpyAsync(out, h->u[1], need * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    } else if (what == TEUK_X_TIMES) {
        const long long first = h->samples - nsamp;
        for (long long i = 0; i < nsamp; ++i) out[i] = (double)((first + i) * (long long)c.extract_every) * h->dt;
    } else if (h->dd) {
        // the streamed double-double table, rearranged into the TEUK_X_COEFFS order
        std::vector<double> t((size_t)kNDD * h->plane * 2);
        e = (int)hipMemcpyAsync(t.data(), h->dtab, t.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream);
        if (!e) e = (int)hipStreamSynchronize(h->stream);
        if (!e) dd_coeff_order(t.data(), h->plane, out);
    } else {
        double* tmp = nullptr;
        e = (int)hipMalloc(&tmp, need * sizeof(double));
        if (!e) e = launch_coef_dump(h->rtab, h->ttab, h->ctab, c.nr, c.ntheta, tmp, h->stream);
        if (!e) e = (int)hipMemcpyAsync(out, tmp, need * sizeof(double), hipMemcpyDeviceToHost, h->stream);
        if (!e) e = (int)hipStreamSynchronize(h->stream);
        if (tmp) (void)hipFree(tmp);
    }
    if (!e) e = (int)hipStreamSynchronize(h->stream);
    if (e) return hip_fail(h, e, "extract copy");
    if (written) *written = need;
    return guard;
}

teuk_status teuk_info(teuk_solver* h, teuk_info_t* info)
{
    if (!h) return fail(nullptr, TEUK_ERR_INVALID_ARG, "solver is NULL");
    if (!info) return fail(h, TEUK_ERR_INVALID_ARG, "info is NULL");
    int e = (int)hipStreamSynchronize(h->stream);
    if (e) return hip_fail(h, e, "hipStreamSynchronize");
    info->dt = h->dt;
    info->t = (double)h->steps * h->dt;
    info->steps = h->steps;
    info->samples = h->samples;
    info->j_extract = h->j_e;
    info->workgroups = h->cfg.integrator == TEUK_RK_SSP33_BLOCKED     ? h->bstrips * h->bsegs
                       : h->cfg.integrator == TEUK_RK_SSP33_PIPELINED ? h->pgrid
                                                                      : h->nstrips * h->segs[1];
    info->dt_bound = h->dt_bound;
    return TEUK_OK;
}

teuk_status teuk_check_finite(teuk_solver* h)
{
    if (!h) return fail(nullptr, TEUK_ERR_INVALID_ARG, "solver is NULL");
    if (!h->have_init) return fail(h, TEUK_ERR_STATE, "no state: call teuk_set_initial first");
    return run_guard(h);
}

void teuk_destroy(teuk_solver* h)
{
    if (!h) return;
    if (h->group) (void)teuk_group_remove(h->group, h);
    (void)hipStreamSynchronize(h->stream);
    free_solver(h);
}

const char* teuk_last_error(const teuk_solver* h)
{
    return h ? h->err.c_str() : g_err.c_str();
}

teuk_status teuk_host_coefficients(const teuk_config* cfg, double* out, size_t capacity)
{
    std::string err;
    if (!validate(cfg, err)) return fail(nullptr, TEUK_ERR_INVALID_ARG, err);
    if (!out) return fail(nullptr, TEUK_ERR_INVALID_ARG, "out is NULL");
    const size_t n = (size_t)cfg->nr * cfg->ntheta;
    if (cfg->state_prec == TEUK_S_DD) {
        if (cfg->chart != TEUK_CHART_TORTOISE)
            return fail(nullptr, TEUK_ERR_UNSUPPORTED, "double-double state: tortoise chart only");
        if (capacity < 2 * TEUK_NCOEF * n) return fail(nullptr, TEUK_ERR_CAPACITY, "out too small");
        std::vector<double> dtab;
        DDScalars sc;
        if (!build_tables_dd(*cfg, dtab, &sc, err)) return fail(nullptr, TEUK_ERR_INVALID_ARG, err);
        dd_coeff_order(dtab.data(), (long long)n, out);
        return TEUK_OK;
    }
    if (capacity < TEUK_NCOEF * n) return fail(nullptr, TEUK_ERR_CAPACITY, "out too small");
    if (cfg->chart == TEUK_CHART_HYPERBOLOIDAL) {
        std::vector<double> ctab;
        if (!build_tables_H(*cfg, ctab, err)) return fail(nullptr, TEUK_ERR_INVALID_ARG, err);
        const int order[TEUK_NCOEF] = {kHLam1, kHM3r, kHM3i, kHBtr, kHBti, kHCr, kHCi, kHAth, kHBth, kHLam2};
        for (int q = 0; q < TEUK_NCOEF; ++q)
            std::memcpy(out + (size_t)q * n, ctab.data() + (size_t)order[q] * n, n * sizeof(double));
        return TEUK_OK;
    }
    std::vector<double> rtab, ttab;
    if (!build_tables(*cfg, rtab, ttab, err)) return fail(nullptr, TEUK_ERR_INVALID_ARG, err);
    const int nr = cfg->nr, nth = cfg->ntheta;
    for (int k = 0; k < nth; ++k) {
        const double sn2 = ttab[kSn2 * nth + k], cs = ttab[kCs * nth + k];
        const double cot = ttab[kCot * nth + k], th = ttab[kTh * nth + k];
        for (int j = 0; j < nr; ++j) {
            double rt[kNRT];
            for (int t = 0; t < kNRT; ++t) rt[t] = rtab[(size_t)t * nr + j];
            const PointCoef c = point_coef(rt, sn2, cs, cot, th, 1.0 / std::sqrt(sigma2(rt, sn2)));
            const size_t i = (size_t)k * nr + j;
            out[0 * n + i] = c.b;
            out[1 * n + i] = c.m3r;
            out[2 * n + i] = c.m3i;
            out[3 * n + i] = c.btr;
            out[4 * n + i] = c.bti;
            out[5 * n + i] = c.cr;
            out[6 * n + i] = c.ci;
            out[7 * n + i] = c.ath;
            out[8 * n + i] = c.bth;
            out[9 * n + i] = -c.b;
        }
    }
    return TEUK_OK;
}

// ---------------------------------------------------------------- groups

static thread_local std::string g_group_err;

static teuk_status gfail(teuk_group* g, teuk_status st, const std::string& msg)
{
    if (g) g->err = msg; else g_group_err = msg;
    return st;
}

// Theta segments per strip when tiles should march about `rows` rows each (an
// even number when more than one, so that segments pair up at their shared
// boundary rows).
static int group_segs(int nth, int rows)
{
    int segs = nth / rows;
    if (segs > 1) segs &= ~1;
    if (segs < 1) segs = 1;
    return segs;
}

// Rebuild and upload the members' stage descriptors and tile prefix sums, cut
// each (precision, chart) class into cache blocks and size each block's launch.
// The caller has synchronised the group's stream.
static void drop_group_graphs(teuk_group* g);

static teuk_status group_upload(teuk_group* g)
{
    drop_group_graphs(g);
    const int cap = g->cap;
    int idx = 0;
    size_t soff = 0;
    g->points = 0;
    g->order.clear();
    g->blocks.clear();
    for (int c = 0; c < kClasses; ++c) {
        GroupBlock blk;
        long long bytes = 0;
        bool all_fill = true, blocked = false;
        // resident workgroups of the class's stage-2/3 kernel (class c = weight precision + 4 launch class)
        const long long resident = TEUK_GROUP_SOLO ? stage_grid(c % 4, false, c / 4) : 0;
        auto open_block = [&]() {
            blk = GroupBlock();
            blk.cls = c;
            blk.first = idx;
            blk.start = soff;
            g->h_start[soff] = 0;
            bytes = 0;
            all_fill = true;
            blocked = false;
        };
        auto close_block = [&]() {
            blk.grid = (int)(g->workgroups > 0 && g->workgroups < blk.tiles ? g->workgroups : blk.tiles);
            blk.solo = blocked || (TEUK_GROUP_SOLO && all_fill && g->workgroups == 0);
            g->blocks.push_back(blk);
            soff += (size_t)blk.n + 1;
        };
        open_block();
        for (teuk_solver* h : g->mem) {
            if (h->cfg.weight_prec + 4 * kernel_chart(h->cfg) != c) continue;
            // a member with the blocked step is a block of its own, stepped by its own launches
            const bool bl = h->cfg.integrator == TEUK_RK_SSP33_BLOCKED;
            if (blk.n > 0 && (bl || blocked || bytes + (long long)h->bytes > g->block_bytes)) {
                close_block();
                open_block();
            }
            blocked = bl;
            if (TEUK_GROUP_SOLO)
                all_fill = all_fill && resident > 0 && (long long)h->nstrips * h->cfg.ntheta >= resident;
            StageArgs a = stage_args(h);
            a.segs = group_segs(h->cfg.ntheta, g->rows);
            a.grid = 0;                                  // set per launch
            blk.tiles += (long long)h->nstrips * a.segs;
            blk.solo_wg += bl ? (long long)h->bstrips * h->bsegs : (long long)h->nstrips * h->segs[1];
            blk.units += (long long)h->nstrips * h->cfg.ntheta;
            if (blk.tiles > (1LL << 31) - 1)
                return gfail(g, TEUK_ERR_CAPACITY, "group block too large for one launch (2^31 - 1 tiles)");
            ++blk.n;
            g->h_start[soff + blk.n] = blk.tiles;
            bytes += (long long)h->bytes;
            // stage 1: u1 = u + dt F(u)
            a.uk = a.un = h->u[0]; a.out = h->u[1]; a.ca = 0.0; a.cb = 1.0;
            g->h_args[0 * (size_t)cap + idx] = a;
            // stage 2: u2 = 3/4 u + 1/4 (u1 + dt F(u1))
            a.uk = h->u[1]; a.un = h->u[0]; a.out = h->u[2]; a.ca = 0.75; a.cb = 0.25;
            g->h_args[1 * (size_t)cap + idx] = a;
            // stage 3: u = 1/3 u + 2/3 (u2 + dt F(u2)), in place
            a.uk = h->u[2]; a.un = h->u[0]; a.out = h->u[0]; a.ca = 1.0 / 3.0; a.cb = 2.0 / 3.0;
            g->h_args[2 * (size_t)cap + idx] = a;
            g->points += h->plane;
            g->order.push_back(h);
            ++idx;
        }
        if (blk.n > 0) close_block();
    }
    int e = (int)hipMemcpyAsync(g->d_args, g->h_args.data(), g->h_args.size() * sizeof(StageArgs),
                                hipMemcpyHostToDevice, g->stream);
    if (!e) e = (int)hipMemcpyAsync(g->d_start, g->h_start.data(), g->h_start.size() * sizeof(long long),
                                    hipMemcpyHostToDevice, g->stream);
    if (!e) e = (int)hipStreamSynchronize(g->stream);
    if (e) return gfail(g, TEUK_ERR_DEVICE, std::string("group upload: ") + hipGetErrorString((hipError_t)e));
    g->gexec.assign(g->blocks.size(), nullptr);
    g->gphase.assign(g->blocks.size(), std::vector<long long>());
    return TEUK_OK;
}

teuk_status teuk_group_create(const teuk_device_ctx* ctx, int32_t max_members, int32_t workgroups,
                              int32_t rows_per_tile, teuk_group** out)
{
    if (!out) return gfail(nullptr, TEUK_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (max_members < 1 || max_members > 65536) return gfail(nullptr, TEUK_ERR_INVALID_ARG, "max_members must be in [1, 65536]");
    if (workgroups < 0) return gfail(nullptr, TEUK_ERR_INVALID_ARG, "workgroups must be >= 0");
    if (rows_per_tile < 0) return gfail(nullptr, TEUK_ERR_INVALID_ARG, "rows_per_tile must be >= 0");
    teuk_group* g = new (std::nothrow) teuk_group();
    if (!g) return gfail(nullptr, TEUK_ERR_OUT_OF_MEMORY, "host allocation failed");
    g->stream = ctx ? (hipStream_t)ctx->stream : nullptr;
    (void)hipGetDevice(&g->device);
    g->cap = max_members;
    g->workgroups = workgroups;
    g->rows = rows_per_tile > 0 ? rows_per_tile : 8;
    g->h_args.assign(3 * (size_t)max_members, StageArgs{});
    g->h_start.assign(2 * (size_t)max_members + 2, 0);   // members + blocks + 1 entries at most
    int e = (int)hipMalloc(&g->d_args, g->h_args.size() * sizeof(StageArgs));
    if (!e) e = (int)hipMalloc(&g->d_start, g->h_start.size() * sizeof(long long));
    if (e) {
        if (g->d_args) (void)hipFree(g->d_args);
        (void)hipGetLastError();
        delete g;
        return gfail(nullptr, e == (int)hipErrorOutOfMemory ? TEUK_ERR_OUT_OF_MEMORY : TEUK_ERR_DEVICE,
                     std::string("hipMalloc: ") + hipGetErrorString((hipError_t)e));
    }
    *out = g;
    return TEUK_OK;
}

teuk_status teuk_group_add(teuk_group* g, teuk_solver* h)
{
    if (!g) return gfail(nullptr, TEUK_ERR_INVALID_ARG, "group is NULL");
    if (!h) return gfail(g, TEUK_ERR_INVALID_ARG, "solver is NULL");
    if (h->dd) return gfail(g, TEUK_ERR_UNSUPPORTED, "double-double solvers are not group members");
    if ((h->cfg.integrator != TEUK_RK_SSP33 && h->cfg.integrator != TEUK_RK_SSP33_BLOCKED) ||
        h->cfg.scheme != TEUK_SCHEME_WENO5)
        return gfail(g, TEUK_ERR_UNSUPPORTED, "group members step with SSP-RK(3,3), three-launch or blocked, and WENO5");
    if (h->group) return gfail(g, TEUK_ERR_INVALID_ARG, "solver already belongs to a group");
    if (h->stream != g->stream) return gfail(g, TEUK_ERR_INVALID_ARG, "solver and group use different streams");
    if (h->device != g->device) return gfail(g, TEUK_ERR_INVALID_ARG, "solver and group are on different devices");
    if (!h->have_init) return gfail(g, TEUK_ERR_STATE, "solver has no initial data");
    if ((int)g->mem.size() >= g->cap) return gfail(g, TEUK_ERR_CAPACITY, "group is full");
    int e = (int)hipStreamSynchronize(g->stream);
    if (e) return gfail(g, TEUK_ERR_DEVICE, std::string("hipStreamSynchronize: ") + hipGetErrorString((hipError_t)e));
    g->mem.push_back(h);
    teuk_status st = group_upload(g);
    if (st != TEUK_OK) {
        g->mem.pop_back();
        (void)group_upload(g);
        return st;
    }
    h->group = g;
    return TEUK_OK;
}

teuk_status teuk_group_remove(teuk_group* g, teuk_solver* h)
{
    if (!g) return gfail(nullptr, TEUK_ERR_INVALID_ARG, "group is NULL");
    if (!h || h->group != g) return gfail(g, TEUK_ERR_INVALID_ARG, "solver is not a member of this group");
    int e = (int)hipStreamSynchronize(g->stream);
    if (e) return gfail(g, TEUK_ERR_DEVICE, std::string("hipStreamSynchronize: ") + hipGetErrorString((hipError_t)e));
    for (size_t i = 0; i < g->mem.size(); ++i)
        if (g->mem[i] == h) {
            g->mem.erase(g->mem.begin() + (long)i);
            break;
        }
    h->group = nullptr;
    return group_upload(g);
}

// nsteps steps of cache block bi, launch by launch on `stream` (the members'
// samples too).
static teuk_status group_block_eager(teuk_group* g, size_t bi, int64_t nsteps, hipStream_t stream)
{
    const size_t cap = (size_t)g->cap;
    const GroupBlock& b = g->blocks[bi];
    const bool blocked = b.solo && g->order[(size_t)b.first]->cfg.integrator == TEUK_RK_SSP33_BLOCKED;
    for (int64_t n = 0; n < nsteps; ++n) {
        if (blocked) {   // a block of one member with the blocked step: one launch per step
            const int e = blocked_step_once(g->order[(size_t)b.first], stream);
            if (e) return gfail(g, TEUK_ERR_DEVICE, std::string("blocked step launch: ") +
                                                       hipGetErrorString((hipError_t)e));
        }
        for (int stage = 1; stage <= 3 && !blocked; ++stage) {
            int e = 0;
            if (b.solo) {
                for (int k = b.first; k < b.first + b.n && !e; ++k) {
                    const teuk_solver* h = g->order[(size_t)k];
                    StageArgs a = stage_args(h);
                    rk3_stage(h, a, stage);
                    e = launch_stage(a, stage, h->cfg.weight_prec, kernel_chart(h->cfg), stream);
                }
            } else {
                e = launch_group_stage(g->d_args + (stage - 1) * cap + b.first, g->d_start + b.start, b.n,
                                       b.tiles, b.grid, stage, b.cls % 4, b.cls / 4, stream);
            }
            if (e) return gfail(g, TEUK_ERR_DEVICE, std::string("group stage launch: ") +
                                                       hipGetErrorString((hipError_t)e));
        }
        for (int k = b.first; k < b.first + b.n; ++k) {
            teuk_solver* h = g->order[(size_t)k];
            ++h->steps;
            if (h->cfg.extract_every > 0 && h->steps % h->cfg.extract_every == 0) {
                const hipStream_t own = h->stream;
                h->stream = stream;
                teuk_status st = record_sample(h);
                h->stream = own;
                if (st != TEUK_OK) return gfail(g, st, h->err);
            }
        }
    }
    return TEUK_OK;
}

static void drop_group_graphs(teuk_group* g)
{
    bool any = false;
    for (hipGraphExec_t x : g->gexec) any = any || x;
    if (any) (void)hipStreamSynchronize(g->stream);
    for (hipGraphExec_t& x : g->gexec)
        if (x) {
            (void)hipGraphExecDestroy(x);
            x = nullptr;
        }
    g->gexec.assign(g->blocks.size(), nullptr);
    g->gphase.assign(g->blocks.size(), std::vector<long long>());
}

// The graph of graph_chunk steps of block bi, captured for its members'
// current sampling phases and state buffers (recaptured when they differ).
static teuk_status capture_block(teuk_group* g, size_t bi)
{
    const GroupBlock& b = g->blocks[bi];
    const int64_t chunk = g->graph_chunk;
    std::vector<long long> phase;
    for (int k = b.first; k < b.first + b.n; ++k) {
        const teuk_solver* h = g->order[(size_t)k];
        const long long every = h->cfg.extract_every;
        if (every > 0 && chunk % every != 0)
            return gfail(g, TEUK_ERR_INVALID_ARG, "graph mode: chunk_steps must be a multiple of every member's extract_every");
        if (h->cfg.integrator == TEUK_RK_SSP33_BLOCKED && chunk % 2 != 0)
            return gfail(g, TEUK_ERR_INVALID_ARG,
                         "graph mode: a member with the blocked step swaps two buffers per step: chunk_steps must be even");
        phase.push_back(every > 0 ? h->steps % every : 0);
        phase.push_back((long long)(uintptr_t)h->u[0]);   // buffer roles (the blocked step trades them)
    }
    if (g->gexec[bi] && g->gphase[bi] == phase) return TEUK_OK;
    int e = 0;
    if (g->gexec[bi]) {
        (void)hipStreamSynchronize(g->stream);
        (void)hipGraphExecDestroy(g->gexec[bi]);
        g->gexec[bi] = nullptr;
    }
    if (!g->cap_stream) {
        e = (int)hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking);
        if (e) {
            g->cap_stream = nullptr;
            return gfail(g, TEUK_ERR_DEVICE, std::string("hipStreamCreateWithFlags: ") + hipGetErrorString((hipError_t)e));
        }
    }
    std::vector<std::pair<long long, long long>> saved;
    std::vector<std::array<double*, 3>> saved_u;
    for (int k = b.first; k < b.first + b.n; ++k) {
        const teuk_solver* h = g->order[(size_t)k];
        saved.emplace_back(h->steps, h->samples);
        saved_u.push_back({h->u[0], h->u[1], h->u[2]});
    }
    e = (int)hipStreamBeginCapture(g->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e) return gfail(g, TEUK_ERR_DEVICE, std::string("hipStreamBeginCapture: ") + hipGetErrorString((hipError_t)e));
    const teuk_status st = group_block_eager(g, bi, chunk, g->cap_stream);
    hipGraph_t graph = nullptr;
    e = (int)hipStreamEndCapture(g->cap_stream, &graph);
    for (int k = b.first; k < b.first + b.n; ++k) {
        teuk_solver* h = g->order[(size_t)k];
        h->steps = saved[(size_t)(k - b.first)].first;
        h->samples = saved[(size_t)(k - b.first)].second;
        for (int i = 0; i < 3; ++i) h->u[i] = saved_u[(size_t)(k - b.first)][(size_t)i];
    }
    if (st != TEUK_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e || !graph)
        return gfail(g, TEUK_ERR_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString((hipError_t)(e ? e : (int)hipErrorUnknown)));
    e = (int)hipGraphInstantiate(&g->gexec[bi], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e) {
        g->gexec[bi] = nullptr;
        return gfail(g, TEUK_ERR_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString((hipError_t)e));
    }
    e = (int)hipGraphUpload(g->gexec[bi], g->stream);   // first replay as cheap as later ones
    if (e) {
        (void)hipGraphExecDestroy(g->gexec[bi]);
        g->gexec[bi] = nullptr;
        return gfail(g, TEUK_ERR_DEVICE, std::string("hipGraphUpload: ") + hipGetErrorString((hipError_t)e));
    }
    g->gphase[bi] = phase;
    return TEUK_OK;
}

teuk_status teuk_group_step(teuk_group* g, int64_t nsteps)
{
    if (!g) return gfail(nullptr, TEUK_ERR_INVALID_ARG, "group is NULL");
    if (nsteps < 0) return gfail(g, TEUK_ERR_INVALID_ARG, "nsteps must be >= 0");
    if (g->mem.empty()) return TEUK_OK;
    const int64_t chunk = g->graph_chunk;
    if (g->gexec.size() != g->blocks.size()) drop_group_graphs(g);
    // block by block: a block runs all nsteps steps before the next starts
    for (size_t bi = 0; bi < g->blocks.size(); ++bi) {
        int64_t left = nsteps;
        if (chunk > 0 && nsteps >= chunk) {
            teuk_status st = capture_block(g, bi);
            if (st != TEUK_OK) return st;
            const GroupBlock& b = g->blocks[bi];
            for (int64_t q = nsteps / chunk; q > 0; --q) {
                const int e = (int)hipGraphLaunch(g->gexec[bi], g->stream);
                if (e) return gfail(g, TEUK_ERR_DEVICE, std::string("hipGraphLaunch: ") + hipGetErrorString((hipError_t)e));
                for (int k = b.first; k < b.first + b.n; ++k) {
                    teuk_solver* h = g->order[(size_t)k];
                    h->steps += chunk;
                    if (h->cfg.extract_every > 0) h->samples += chunk / h->cfg.extract_every;
                }
            }
            left = nsteps % chunk;
        }
        teuk_status st = group_block_eager(g, bi, left, g->stream);
        if (st != TEUK_OK) return st;
    }
    return TEUK_OK;
}

teuk_status teuk_group_set_graph(teuk_group* g, int32_t chunk_steps)
{
    if (!g) return gfail(nullptr, TEUK_ERR_INVALID_ARG, "group is NULL");
    if (chunk_steps < 0 || chunk_steps > kMaxGraphChunk)
        return gfail(g, TEUK_ERR_INVALID_ARG, "chunk_steps must be in [0, " + std::to_string(kMaxGraphChunk) + "]");
    drop_group_graphs(g);
    g->graph_chunk = chunk_steps;
    // capture every block now, at its members' current sampling phases
    for (size_t bi = 0; chunk_steps > 0 && bi < g->blocks.size(); ++bi) {
        teuk_status st = capture_block(g, bi);
        if (st != TEUK_OK) return st;
    }
    return TEUK_OK;
}

// Microseconds per step of group t: the best of two timed runs of n steps
// after two warm-up steps, on t's stream.
static teuk_status time_group(teuk_group* t, int64_t n, double* us)
{
    teuk_status st = teuk_group_step(t, 2);
    if (st != TEUK_OK) return st;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int e = (int)hipEventCreate(&e0);
    if (!e) e = (int)hipEventCreate(&e1);
    double best = 0.0;
    for (int rep = 0; rep < 2 && !e && st == TEUK_OK; ++rep) {
        e = (int)hipEventRecord(e0, t->stream);
        if (!e) st = teuk_group_step(t, n);
        if (!e && st == TEUK_OK) e = (int)hipEventRecord(e1, t->stream);
        if (!e && st == TEUK_OK) e = (int)hipEventSynchronize(e1);
        float ms = 0.0f;
        if (!e && st == TEUK_OK) e = (int)hipEventElapsedTime(&ms, e0, e1);
        const double v = 1e3 * (double)ms / (double)n;
        if (!e && st == TEUK_OK && (rep == 0 || v < best)) best = v;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st != TEUK_OK) return st;
    if (e) return gfail(t, TEUK_ERR_DEVICE, std::string("timing events: ") + hipGetErrorString((hipError_t)e));
    *us = best;
    return TEUK_OK;
}

teuk_status teuk_group_tune(teuk_group* g, int32_t steps, teuk_group_tune_info_t* out)
{
    if (!g) return gfail(nullptr, TEUK_ERR_INVALID_ARG, "group is NULL");
    if (!out) return gfail(g, TEUK_ERR_INVALID_ARG, "out is NULL");
    if (steps < 0) return gfail(g, TEUK_ERR_INVALID_ARG, "steps must be >= 0");
    std::memset(out, 0, sizeof(*out));
    if (g->mem.empty()) return gfail(g, TEUK_ERR_STATE, "the group has no members to tune on");
    int e = (int)hipStreamSynchronize(g->stream);
    if (e) return gfail(g, TEUK_ERR_DEVICE, std::string("hipStreamSynchronize: ") + hipGetErrorString((hipError_t)e));
    hipStream_t ts = nullptr;
    e = (int)hipStreamCreateWithFlags(&ts, hipStreamNonBlocking);
    if (e) return gfail(g, TEUK_ERR_DEVICE, std::string("hipStreamCreateWithFlags: ") + hipGetErrorString((hipError_t)e));
    // clones of the members: same grids, classes and step sizes, no waveform
    // ring, starting from the members' current states
    std::vector<teuk_solver*> clones;
    teuk_group* tg = nullptr;
    teuk_status st = TEUK_OK;
    std::string why;
    for (teuk_solver* h : g->mem) {
        teuk_config c = h->cfg;
        c.extract_every = 0;
        c.max_samples = 0;
        c.dt = h->dt;
        teuk_device_ctx ctx{ts, nullptr, 0};
        teuk_solver* x = nullptr;
        st = teuk_create(&c, &ctx, &x);
        if (st != TEUK_OK) { why = std::string("clone: ") + teuk_last_error(nullptr); break; }
        clones.push_back(x);
        st = teuk_set_initial(x, h->u[0], 1);
        if (st != TEUK_OK) { why = std::string("clone state: ") + x->err; break; }
    }
    if (st == TEUK_OK) {
        teuk_device_ctx gctx{ts, nullptr, 0};
        st = teuk_group_create(&gctx, (int32_t)clones.size(), g->workgroups, g->rows, &tg);
        if (st != TEUK_OK) why = g_group_err;
        for (size_t i = 0; i < clones.size() && st == TEUK_OK; ++i) {
            st = teuk_group_add(tg, clones[i]);
            if (st != TEUK_OK) why = tg->err;
        }
    }
    const int rows_c[] = {4, 8, 16, 32, 64};
    // small blocks matter once members fill the GPU by themselves (solo blocks: a block
    // of one member runs all its steps alone, with its state in the last-level cache)
    const long long mib_c[] = {32, 64, 128, 256, 384, 512};
    int best_rows = g->rows;
    long long best_bytes = g->block_bytes;
    double best_us = 0.0, default_us = 0.0;
    int cand = 0;
    int64_t n = steps;
    if (st == TEUK_OK && n == 0) {
        // aim at about 20 ms per timed run
        double us = 0.0;
        st = time_group(tg, 1, &us);
        if (st != TEUK_OK) why = tg->err;
        n = (int64_t)std::min(200.0, std::max(2.0, 20000.0 / std::max(us, 1.0)));
    }
    auto try_shape = [&](int rows, long long bytes, double* us) {
        tg->rows = rows;
        tg->block_bytes = bytes;
        teuk_status s2 = group_upload(tg);
        if (s2 == TEUK_OK) s2 = time_group(tg, n, us);
        if (s2 != TEUK_OK) why = tg->err;
        return s2;
    };
    if (st == TEUK_OK) st = try_shape(g->rows, g->block_bytes, &default_us);
    if (st == TEUK_OK) {
        best_us = default_us;
        cand = 1;
    }
    for (int r : rows_c) {
        for (long long mb : mib_c) {
            if (st != TEUK_OK) break;
            if (r == g->rows && (mb << 20) == g->block_bytes) continue;
            double us = 0.0;
            st = try_shape(r, mb << 20, &us);
            if (st != TEUK_OK) break;
            ++cand;
            if (us < best_us) {
                best_us = us;
                best_rows = r;
                best_bytes = mb << 20;
            }
        }
    }
    if (tg) teuk_group_destroy(tg);
    for (teuk_solver* x : clones) teuk_destroy(x);
    (void)hipStreamDestroy(ts);
    if (st != TEUK_OK) return gfail(g, st, "group tuning: " + why);
    out->default_rows_per_tile = g->rows;
    out->default_block_mib = (int32_t)(g->block_bytes >> 20);
    g->rows = best_rows;
    g->block_bytes = best_bytes;
    st = group_upload(g);
    if (st != TEUK_OK) return st;
    out->rows_per_tile = best_rows;
    out->block_mib = (int32_t)(best_bytes >> 20);
    out->candidates = cand;
    out->steps = (int32_t)n;
    out->us_per_step = best_us;
    out->us_per_step_default = default_us;
    return TEUK_OK;
}

teuk_status teuk_group_info(const teuk_group* g, teuk_group_info_t* info)
{
    if (!g) return gfail(nullptr, TEUK_ERR_INVALID_ARG, "group is NULL");
    if (!info) return TEUK_ERR_INVALID_ARG;
    info->members = (int32_t)g->mem.size();
    info->classes = 0;
    info->workgroups = 0;
    info->tiles = 0;
    info->units = 0;
    bool seen[kClasses] = {};
    for (const GroupBlock& b : g->blocks) {
        info->classes += !seen[b.cls];
        seen[b.cls] = true;
        info->workgroups += b.solo ? b.solo_wg : b.grid;
        info->tiles += b.solo ? b.solo_wg : b.tiles;
        info->units += b.units;
    }
    info->points = g->points;
    return TEUK_OK;
}

void teuk_group_destroy(teuk_group* g)
{
    if (!g) return;
    drop_group_graphs(g);
    if (g->cap_stream) (void)hipStreamDestroy(g->cap_stream);
    (void)hipStreamSynchronize(g->stream);
    for (teuk_solver* h : g->mem) h->group = nullptr;
    if (g->d_args) (void)hipFree(g->d_args);
    if (g->d_start) (void)hipFree(g->d_start);
    delete g;
}

const char* teuk_group_last_error(const teuk_group* g)
{
    return g ? g->err.c_str() : g_group_err.c_str();
}

}  // extern "C"

// ---------------------------------------------------------------- allocation-free stepping
// teuk_step_noalloc keeps its device memory beyond the caller's state -- the
// two SSP-RK stage buffers u(1), u(2) and the chart-T radial and polar
// coefficient tables -- in one file-scope device array.  Every GPU the library
// runs on holds its own copy of the array from module load until the process
// ends.  Host code never passes the array's name to a kernel or a copy: it
// takes the array's device address on each device once (hipGetSymbolAddress)
// and uses that address.
namespace {
constexpr long long kNaMaxPoints = 1LL << 20;   // nr * ntheta
constexpr int kNaMaxNr = 1 << 15;
constexpr int kNaMaxNth = 1 << 12;
constexpr size_t kNaStateBytes = (size_t)kNaMaxPoints * 4 * sizeof(double);
constexpr size_t kNaOffU1 = 0;
constexpr size_t kNaOffU2 = kNaStateBytes;
constexpr size_t kNaOffR = 2 * kNaStateBytes;
constexpr size_t kNaOffT = kNaOffR + (size_t)kNRT * kNaMaxNr * sizeof(double);
constexpr size_t kNaBytes = kNaOffT + (size_t)kNTT * kNaMaxNth * sizeof(double);
static_assert(kNaOffR % 256 == 0 && kNaOffT % 256 == 0, "scratch regions stay 256-byte aligned");
constexpr int kNaMaxDevices = 64;

// What the resident coefficient tables were built from.
struct NaTableKey {
    int32_t s, m, nr, ntheta;
    double M, a, x_min, x_max;
};

struct NaDevice {
    char* ptr = nullptr;          // device address of `scratch` on this device
    bool tables = false;          // tables of `key` resident in the array
    NaTableKey key{};
};
std::mutex g_na_mutex;
NaDevice g_na[kNaMaxDevices];
}  // namespace

static __device__ __align__(256) char scratch[kNaBytes];

extern "C" teuk_status teuk_step_noalloc(const teuk_config* cfg, double* u, int64_t nsteps, void* stream)
{
    std::string err;
    if (!validate(cfg, err)) return fail(nullptr, TEUK_ERR_INVALID_ARG, err);
    if (!u) return fail(nullptr, TEUK_ERR_INVALID_ARG, "u is NULL");
    if (nsteps < 0) return fail(nullptr, TEUK_ERR_INVALID_ARG, "nsteps must be >= 0");
    if (cfg->chart != TEUK_CHART_TORTOISE || cfg->state_prec != TEUK_S_FP64 || cfg->integrator != TEUK_RK_SSP33 ||
        cfg->scheme != TEUK_SCHEME_WENO5 || cfg->weight_prec == TEUK_W_DD)
        return fail(nullptr, TEUK_ERR_UNSUPPORTED,
                    "teuk_step_noalloc: tortoise chart, FP64 state, SSP-RK(3,3), WENO5 only");
    if (!(cfg->dt > 0.0)) return fail(nullptr, TEUK_ERR_INVALID_ARG, "teuk_step_noalloc needs dt > 0");
    if (cfg->extract_every != 0) return fail(nullptr, TEUK_ERR_INVALID_ARG, "teuk_step_noalloc keeps no waveform: extract_every must be 0");
    if (cfg->nr > kNaMaxNr || cfg->ntheta > kNaMaxNth || (long long)cfg->nr * cfg->ntheta > kNaMaxPoints)
        return fail(nullptr, TEUK_ERR_INVALID_ARG,
                    "teuk_step_noalloc: grid " + std::to_string(cfg->nr) + " x " + std::to_string(cfg->ntheta) +
                        " exceeds its scratch limits (nr <= 32768, ntheta <= 4096, nr * ntheta <= 1048576)");
    if (nsteps == 0) return TEUK_OK;
    const hipStream_t st = (hipStream_t)stream;
    int dev = 0;
    int e = (int)hipGetDevice(&dev);
    if (e) return fail(nullptr, TEUK_ERR_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString((hipError_t)e));
    if (dev < 0 || dev >= kNaMaxDevices) return fail(nullptr, TEUK_ERR_UNSUPPORTED, "device index beyond 63");
    const NaTableKey key{cfg->s, cfg->m, cfg->nr, cfg->ntheta, cfg->M, cfg->a, cfg->x_min, cfg->x_max};
    char* base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_na_mutex);
        NaDevice& d = g_na[dev];
        if (!d.ptr) {
            void* p = nullptr;
            e = (int)hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e || !p)
                return fail(nullptr, TEUK_ERR_DEVICE,
                            std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString((hipError_t)e));
            d.ptr = (char*)p;
        }
        base = d.ptr;
        if (!d.tables || std::memcmp(&d.key, &key, sizeof(key)) != 0) {
            // A copy from host memory must not be recorded into a graph (its
            // source is released on return), so a capturing call needs the
            // tables of its configuration resident already.
            hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
            e = (int)hipStreamIsCapturing(st, &cs);
            if (e) return fail(nullptr, TEUK_ERR_DEVICE, std::string("hipStreamIsCapturing: ") + hipGetErrorString((hipError_t)e));
            if (cs != hipStreamCaptureStatusNone)
                return fail(nullptr, TEUK_ERR_STATE,
                            "teuk_step_noalloc under stream capture: call it once outside capture with this "
                            "configuration first, so that its coefficient tables are resident");
            std::vector<double> rtab, ttab;
            if (!build_tables(*cfg, rtab, ttab, err)) return fail(nullptr, TEUK_ERR_INVALID_ARG, err);
            d.tables = false;
            e = (int)hipMemcpyAsync(base + kNaOffR, rtab.data(), rtab.size() * sizeof(double), hipMemcpyHostToDevice, st);
            if (!e) e = (int)hipMemcpyAsync(base + kNaOffT, ttab.data(), ttab.size() * sizeof(double), hipMemcpyHostToDevice, st);
            if (!e) e = (int)hipStreamSynchronize(st);   // the host tables are released on return
            if (e) return fail(nullptr, TEUK_ERR_DEVICE, std::string("table upload: ") + hipGetErrorString((hipError_t)e));
            d.key = key;
            d.tables = true;
        }
    }
    const int nstrips = (cfg->nr + kStripPoints - 1) / kStripPoints;
    teuk_config eff = *cfg;
    if (eff.workgroups == 0) eff.workgroups = tuned_workgroups(*cfg);
    const int segs1 = pick_segs(eff, nstrips, cfg->weight_prec, true);
    const int segs23 = pick_segs(eff, nstrips, cfg->weight_prec, false);
    if (segs1 <= 0 || segs23 <= 0) return fail(nullptr, TEUK_ERR_UNSUPPORTED, "occupancy query failed");
    double* u1 = (double*)(base + kNaOffU1);
    double* u2 = (double*)(base + kNaOffU2);
    const double dx = (cfg->x_max - cfg->x_min) / (cfg->nr - 1);
    const double dth = M_PI / cfg->ntheta;
    StageArgs a;
    a.rtab = (const double*)(base + kNaOffR);
    a.ttab = (const double*)(base + kNaOffT);
    a.ctab = nullptr;
    a.plane = (long long)cfg->nr * cfg->ntheta;
    a.nr = cfg->nr;
    a.nth = cfg->ntheta;
    a.nstrips = nstrips;
    a.inv6dx = 1.0 / (6.0 * dx);
    theta_scales(cfg->theta_order, dth, &a.ih1, &a.ih2);
    a.dt = cfg->dt;
    a.out2 = nullptr;
    a.ca2 = a.cb2 = 0.0;
    a.inv_dx = 1.0 / dx;
    a.ko_sigma = cfg->ko_sigma;
    a.eps = cfg->weno_eps;
    a.parity = ((cfg->m + cfg->s) % 2 != 0) ? -1.0 : 1.0;
    const int kchart = kernel_chart(*cfg);
    for (int64_t n = 0; n < nsteps && !e; ++n) {
        // consecutive launches march their segments in opposite directions (see teuk_step)
        a.uk = u; a.un = u; a.out = u1; a.ca = 0.0; a.cb = 1.0; a.segs = segs1; a.grid = nstrips * segs1; a.flip = (int)(n & 1);
        e = launch_stage(a, 1, cfg->weight_prec, kchart, st);
        if (!e) { a.uk = u1; a.un = u; a.out = u2; a.ca = 0.75; a.cb = 0.25; a.segs = segs23; a.grid = nstrips * segs23;
                  a.flip ^= 1; e = launch_stage(a, 2, cfg->weight_prec, kchart, st); }
        if (!e) { a.uk = u2; a.un = u; a.out = u; a.ca = 1.0 / 3.0; a.cb = 2.0 / 3.0;
                  a.flip ^= 1; e = launch_stage(a, 3, cfg->weight_prec, kchart, st); }
    }
    if (e) return fail(nullptr, TEUK_ERR_DEVICE, std::string("stage launch: ") + hipGetErrorString((hipError_t)e));
    return TEUK_OK;
}
