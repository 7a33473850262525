// Internal declarations shared by the C ABI (teuk_api.hip), the host tables
// (teuk_background.cpp) and the device kernels (teuk_kernels.hip).
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "teuk.h"

namespace teuk {

// Build the radial [kNRT][nr] and polar [kNTT][ntheta] tables of teuk_coef.h
// for a validated chart-T configuration.  Returns false (with err) if a radial
// node is too close to the horizon for FP64.
bool build_tables(const teuk_config& c, std::vector<double>& rtab, std::vector<double>& ttab,
                  std::string& err);

// Build the chart-H per-point table [kNCH][ntheta][nr] of teuk_coef.h for a
// validated TEUK_CHART_HYPERBOLOIDAL configuration.
bool build_tables_H(const teuk_config& c, std::vector<double>& ctab, std::string& err);

// Launch class of the stage kernels: the chart (TEUK_CHART_*), with the
// tortoise chart at fourth-order theta differences a class of its own.
constexpr int kChartTortoise4 = 2;
inline int kernel_chart(const teuk_config& c)
{
    return (c.chart == TEUK_CHART_TORTOISE && c.theta_order == 4) ? kChartTortoise4 : c.chart;
}

// Scales of the centred theta differences as the stage kernels take them:
// 1/(2 dth) and 1/dth^2 at second order, 1/(12 dth) and 1/(12 dth^2) at fourth.
inline void theta_scales(int theta_order, double dth, double* ih1, double* ih2)
{
    const double d = theta_order == 4 ? 12.0 : 1.0;
    *ih1 = 1.0 / ((theta_order == 4 ? 12.0 : 2.0) * dth);
    *ih2 = 1.0 / (d * dth * dth);
}

// Points per radial strip of one stage workgroup (one wave of 64 lanes computes
// 64 interface fluxes and 63 point updates).
constexpr int kStripPoints = 63;

// Arguments of one fused SSP-RK stage launch.
struct StageArgs {
    const double* uk;      // u^(k): 4 planes [4][nth][nr]
    const double* un;      // u^n, read at the own point only (stages 2, 3)
    double* out;           // u^(k+1); may alias un (stage 3 writes in place)
    const double* rtab;    // radial table [kNRT][nr]
    const double* ttab;    // polar table [kNTT][nth]
    const double* ctab;    // chart H: per-point table [kNCH][nth][nr] (null in chart T)
    long long plane;       // nth * nr
    int nr, nth;
    int nstrips;           // radial strips of kStripPoints
    int segs;              // theta segments per strip (grid = nstrips * segs)
    int grid;              // workgroups launched
    double inv6dx;         // 1 / (6 dx): candidate fluxes are carried times 6
    double ih1, ih2;       // theta-difference scales (theta_scales)
    double dt, ca, cb;     // out = ca un + cb (uk + dt F)
    double* out2;          // dual stage: second output ca2 un + cb2 (uk + dt F); may alias un
    double ca2, cb2;
    double inv_dx;         // 1 / dx (comparison schemes)
    double ko_sigma;       // Kreiss-Oliger sigma (TEUK_SCHEME_FD6KO8)
    double eps, parity;    // WENO epsilon, (-1)^(m+s)
    int flip;              // 1: odd theta segments march upward and even ones downward
};

// Arguments of one stage of the double-double state path (tortoise chart).
// Every array holds (hi, lo) pairs: state [4][nth][nr], table [kNDD][nth][nr].
struct DDStageArgs {
    const double* uk;      // u^(k)
    const double* un;      // u^n, read at the own point only (stages 2, 3)
    double* out;           // u^(k+1); may alias un
    const double* ctab;    // double-double coefficient table
    long long plane;       // nth * nr (pairs)
    int nr, nth, nstrips;
    double inv_dx[2], ih1[2], ih2[2];
    double ca[2], cb[2];   // out = ca un + cb (uk + dt F) for stages 2, 3
    double sixth[2], c13_3[2], d[3][2];
    double dt, eps, parity;
};

// Workgroup budget that teuk_tune found fastest for c's launch class on the
// current device, or 0 if it has not been tuned.
int tuned_workgroups(const teuk_config& c);

// Resident workgroup count of a stage-kernel instantiation on the current
// device (0 if the weight precision is not built).  The launch uses
// nstrips * segs workgroups with segs chosen from it.
int stage_grid(int weight_prec, bool first, int chart);

// Launchers (all asynchronous on `stream`; they return the hipError_t as int).
// stage: 1 = out = u + dt F(u), 2/3 = later stages (ca u^n + cb (u^(k) + dt F)),
// 4 = dual (out and out2 from the same v = u^(k) + dt F), 0 = write F(u) only.
int launch_stage(const StageArgs& a, int stage, int weight_prec, int chart, void* stream);
// One stage (1, 2 or 3) of several solves in one launch of `grid` workgroups:
// args[0..nmem) are the members' stage arguments (segs = theta segments per
// strip), start[0..nmem] the prefix sums of their tile counts (nstrips * segs
// each), tiles = start[nmem].
int launch_group_stage(const StageArgs* args, const long long* start, int nmem, long long tiles, int grid,
                       int stage, int weight_prec, int chart, void* stream);
// Stability-bound reduction; theta_order picks the Fourier-symbol maxima of
// the theta differences.
int launch_dt_bound(const double* rtab, const double* ttab, const double* ctab, int nr, int nth, double dx,
                    double dth, int theta_order, unsigned long long* cell, void* stream);
int launch_guard(const double* u, long long n, int* flag, void* stream);
int launch_coef_dump(const double* rtab, const double* ttab, const double* ctab, int nr, int nth, double* out,
                     void* stream);
// Temporal blocking: one whole SSP-RK(3,3) step (tortoise chart, FP64 or
// FP32 weights) from a.uk into a.out (distinct buffers), tiles of
// kBlockedPoints radial points by a.nth / a.segs rows, a.grid = a.nstrips *
// a.segs workgroups.  blocked_grid(weight_prec) is the resident workgroup
// count (0 for a precision without a blocked kernel).
constexpr int kBlockedPoints = 114;
int blocked_grid(int weight_prec);
int launch_blocked_step(const StageArgs& a, int weight_prec, void* stream);
// Pipelined steps (tortoise chart, FP64 state, WENO5): nsteps SSP-RK(3,3)
// steps in one cooperative launch of `grid` workgroups (at most pipe_grid(),
// the resident count, and at most the tile count st[0].nstrips * st[0].segs);
// st[0..2] are the three stages' arguments (equal tiling), done[] the per-tile
// stage counters (absolute since the state was set, s0 of them done before
// this launch), *err is set if a dependency wait exceeds spin_ticks of the
// 100 MHz real-time counter.
int pipe_grid(int weight_prec);
int launch_pipe(const StageArgs st[3], long long* done, int* err, long long s0, int nsteps, int grid,
                long long spin_ticks, int weight_prec, void* stream);
// Comparison schemes (TEUK_SCHEME_WENO3 / TEUK_SCHEME_FD6KO8, FP64): one stage,
// same stage codes as launch_stage.
int launch_cmp_stage(const StageArgs& a, int stage, int scheme, int chart, void* stream);
// Double-double path: one stage (0 = F only, 1, 2, 3) with weights in FP64
// (TEUK_W_FP64, the mixed variant) or double-double (TEUK_W_DD); the waveform
// sample of one radial index ([nth][2] pairs); TwoSum normalisation of n pairs.
int launch_dd_stage(const DDStageArgs& a, int stage, int weight_prec, void* stream);
int launch_dd_extract(const double* u, long long plane, int nr, int nth, int j_e, double* slot, void* stream);
int launch_dd_normalise(double* u, long long n, void* stream);
// One ring sample of the FP64 state: the waveform [nth][2] at radial index j_e
// and, if hwave is not null, the horizon values [nth][4] (Phi and d_rho Phi,
// Re and Im, from the nodes j0 .. j0+3 with value weights w[4] and derivative
// weights dw[4], the latter divided by dx),
// into slot *counter % ring of the rings wave and hwave; then *counter += 1.
// One workgroup; the counter is device memory.
int launch_sample(const double* u, long long plane, int nr, int nth, int j_e, double* wave, double* hwave, int j0,
                  const double* w, const double* dw, long long ring, unsigned long long* counter, void* stream);

}  // namespace teuk
