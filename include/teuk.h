/*
 * teuk.h - C ABI of libteuk, a WENO5 / SSP-RK3 solver for the 2+1D first-order
 * Teukolsky system on one AMD Instinct MI355X (gfx950).
 *
 * Problem (paper Sec. 2): the Teukolsky master equation (eq. teuk0) for a field
 * of spin weight s and azimuthal number m on a Kerr background of mass M and
 * spin a (0 <= a <= M, a = M extremal), separated in the ingoing-Kerr azimuth
 * (Sec. 3: exp(i m phi~) dependence), divided by -A^tt (eq. final) and reduced
 * to first order in time (eq. evln):
 *
 *     d_t u + M d_x u + L u + A u = 0,   u = {Phi_R, Phi_I, pi_R, pi_I},
 *
 * with pi = d_t Phi + b d_x Phi.  The radial chart is the tortoise coordinate
 * x = r_* (Sec. 2.2) and Psi = exp(i m phi~) r^-(2s+1) Phi, so that Phi is O(1)
 * at large r.  The radial derivative is fifth-order WENO of Jiang and Shu
 * (Sec. 3.1.2), upwinded per row by the sign of its speed (+b for the Phi rows,
 * -b for the pi rows); theta derivatives are centred (Sec. 3.1, which leaves
 * their order open): second order by default, fourth order on request
 * (teuk_config.theta_order);
 * time stepping is SSP-RK(3,3) in Shu-Osher form (Sec. 3.2).  The WENO
 * smoothness indicators and weights may be computed in reduced precision with
 * the weights summing to one in FP64 (Sec. 3.1.3); candidate fluxes, flux
 * differences, the RK combination and extraction are always FP64.
 *
 * State precision (Sec. 3.1.3: the paper's baseline is quad precision, with a
 * mixed variant whose weights are computed in double): besides FP64, the state
 * may be carried in double-double (TEUK_S_DD), every value an unevaluated sum
 * hi + lo of two doubles (106 significant bits, about 32 digits), with every
 * operation of the right-hand side and the RK stages in double-double.  Its
 * weights are then TEUK_W_DD (double-double) or TEUK_W_FP64 (the paper's mixed
 * variant: the stencil values rounded to double, IS_k, alpha_k, omega_0 and
 * omega_1 formed in double as printed, omega_2 = 1 - omega_0 - omega_1 in
 * double-double).  Its coefficients are evaluated on the host in IEEE
 * binary128 and stored as double-double pairs.  Tortoise chart only.
 *
 * Grid: x_j = x_min + j (x_max - x_min)/(nr - 1), j = 0..nr-1;
 *       theta_k = (k + 1/2) pi / ntheta, k = 0..ntheta-1 (no node on a pole).
 * Boundaries: three ghost cells per radial side equal to the end value; in
 *       theta, ghost rows beyond each pole equal to (-1)^(m+s) times the row
 *       mirrored across it (row -1 - g mirrors row g, row ntheta + g mirrors
 *       row ntheta - 1 - g): one per pole at second order, two at fourth.
 * State layout (host arrays across this ABI): four FP64 planes
 *       [4][ntheta][nr] in the order Phi_R, Phi_I, pi_R, pi_I, radial index
 *       fastest, densely packed.  With TEUK_S_DD every value is a (hi, lo)
 *       pair of doubles, [4][ntheta][nr][2] (value = hi + lo), and so are the
 *       waveform samples and the per-point coefficients and F(u) below.
 *
 * Conventions for every call:
 *   - Every call returns a teuk_status; nothing aborts, throws or exits across
 *     the ABI.  On failure teuk_last_error() describes the cause.
 *   - Host pointers passed in are read (or written) only during the call and
 *     are never retained.
 *   - Device work is enqueued on the stream given at creation (the null stream
 *     if none).  teuk_step returns once the work is enqueued; teuk_extract and
 *     teuk_info synchronise that stream.
 *   - One solver must not be used from two threads at once; different solvers
 *     are independent.
 */
#ifndef TEUK_H
#define TEUK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TEUK_ABI_VERSION 2

typedef struct teuk_solver teuk_solver;   /* opaque; owned by the library */

typedef enum {
    TEUK_OK = 0,
    TEUK_ERR_INVALID_ARG = -1,    /* bad configuration, pointer or enum      */
    TEUK_ERR_OUT_OF_MEMORY = -2,  /* device allocation or workspace too small */
    TEUK_ERR_DEVICE = -3,         /* a HIP runtime call failed               */
    TEUK_ERR_STATE = -4,          /* call out of order (e.g. step before set_initial) */
    TEUK_ERR_NONFINITE = -5,      /* NaN or Inf found in the state or input   */
    TEUK_ERR_UNSUPPORTED = -6,    /* valid request the library does not offer */
    TEUK_ERR_CAPACITY = -7        /* output array smaller than the data       */
} teuk_status;

/* Radial chart.
 *   TEUK_CHART_TORTOISE:     x = r_* (Sec. 2.2), Psi = exp(i m phi~) r^-(2s+1) Phi(t, x, theta).
 *   TEUK_CHART_HYPERBOLOIDAL: x = rho = r/(1 + r/S), time tau = t~ - r^2/(r+S) + 4M ln(S/(r+S))
 *                            with t~ the ingoing-Kerr time (Sec. 2.2), and
 *                            Psi = exp(i m phi~) r^-1 Delta^-s Phi(tau, rho, theta) (for s = -2
 *                            the Phi = (r/Delta^2) Psi of Sec. 4).  The grid reaches through
 *                            the horizon towards null infinity (x_max < S).  Each row is
 *                            upwinded by the sign of its own speed at the point. */
enum { TEUK_CHART_TORTOISE = 0, TEUK_CHART_HYPERBOLOIDAL = 1 };

/* Precision of the WENO smoothness indicators and nonlinear weights
 * (Sec. 3.1.3).  The six stencil differences, the candidate fluxes and
 * everything after them stay FP64; omega_2 = 1 - omega_0 - omega_1 in FP64.
 * FP32 forms the weights over one common denominator; a point where that
 * denominator leaves [2^-100, 3e38] in FP32 (a flat stencil once weno_eps is
 * below about 4e-9, or differences above about 1e4) takes the FP64 weights.
 * FP16 and BF16 scale the differences by a power of two and form each weight
 * as a ratio, so they stay finite over the whole range of weno_eps. */
enum { TEUK_W_FP64 = 0, TEUK_W_FP32 = 1, TEUK_W_FP16 = 2, TEUK_W_BF16 = 3,
       TEUK_W_DD = 4 /* double-double weights: TEUK_S_DD only */ };

/* Precision of the state and of every operation on it.  TEUK_S_DD takes
 * TEUK_W_DD or TEUK_W_FP64 weights and the tortoise chart (else
 * UNSUPPORTED); it is not a group member. */
enum { TEUK_S_FP64 = 0, TEUK_S_DD = 1 };

/* Time integrator (Sec. 3.2), each step a sequence of fused stage kernels.
 *   TEUK_RK_SSP33:  SSP-RK(3,3) in Shu-Osher form, SSP coefficient C = 1.
 *   TEUK_RK_SSP104: the low-storage ten-stage fourth-order SSP-RK(10,4), C = 6:
 *       u(1) = u^n + dt/6 F(u^n), u(i) = u(i-1) + dt/6 F(u(i-1)) for i = 2..4,
 *       u(5) = 3/5 u^n + 2/5 u(4) + 1/15 dt F(u(4)), u(i) as before for i = 6..9,
 *       u^{n+1} = 1/25 u^n + 9/25 u(4) + 3/5 u(9) + 3/50 dt F(u(4)) + 1/10 dt F(u(9)),
 *     run in three state buffers: the fifth stage also writes
 *     q = 1/25 u^n + 9/25 (u(4) + dt/6 F(u(4))) over u^n, and the last is
 *     u^{n+1} = q + 3/5 (u(9) + dt/6 F(u(9))).  FP64 state, single solves only
 *     (UNSUPPORTED with TEUK_S_DD or in a group). */
enum { TEUK_RK_SSP33 = 0, TEUK_RK_SSP104 = 1, TEUK_RK_SSP33_BLOCKED = 2, TEUK_RK_SSP33_PIPELINED = 3 };
/* TEUK_RK_SSP33_BLOCKED: SSP-RK(3,3), each step one launch that computes all
 * three stages of a tile (temporal blocking): u(1) and u(2) stay in LDS and
 * HBM sees one read of u^n and one write of u^{n+1} per point.  Tiles are 114
 * radial points by about nth / segs rows (one workgroup of two waves); a tile recomputes the stage-1
 * values two rows and six points beyond its outputs and the stage-2 values one
 * row and three points beyond (workgroups, when > 0, sets the tile count).
 * The result is the same arithmetic as TEUK_RK_SSP33, point by point.
 * Tortoise chart, FP64 state, WENO5 with FP64 or FP32 weights.  In a group
 * such a solve is a cache block of its own, stepped by its own blocked
 * launches. */
/* TEUK_RK_SSP33_PIPELINED: SSP-RK(3,3), the steps between two waveform samples
 * (at most 1000) in one persistent cooperative launch.  Each workgroup takes
 * the tiles of the three-launch step (63-point strips by theta segments) of
 * stage after stage in order, and a tile's stage waits only until the nine
 * tiles around it have finished the previous stage (per-tile counters with
 * agent-scope release and acquire), instead of the whole grid waiting at each
 * launch boundary.  Bitwise the result of TEUK_RK_SSP33.  A dependency wait
 * that exceeds two seconds (it cannot under the cooperative launch's
 * residency guarantee) is reported as DEVICE by the next teuk_extract of the
 * state or teuk_check_finite, never as a hang.  Tortoise chart, FP64 state,
 * WENO5, any FP64/FP32/FP16/BF16 weights, single solves, no graph mode. */

/* Radial scheme (Sec. 3.1).  WENO5 is the hot path; the other two are the
 * paper's comparison schemes, run by a separate FP64 stage kernel (FP64 state
 * and weights, single solves; UNSUPPORTED otherwise):
 *   TEUK_SCHEME_WENO3:  third-order WENO, IS_1 = (f_j - f_{j-1})^2,
 *                       IS_2 = (f_{j+1} - f_j)^2, linear weights 1/3, 2/3; the f^-
 *                       flux is the mirror image of f^+ about j + 1/2.
 *   TEUK_SCHEME_FD6KO8: sixth-order centred difference
 *                       (u_{j+3} - 9 u_{j+2} + 45 u_{j+1} - 45 u_{j-1} + 9 u_{j-2} - u_{j-3})/(60 dx)
 *                       with eighth-order Kreiss-Oliger dissipation: every plane's
 *                       right-hand side receives -Q u, Q = ko_sigma dx^7 (D+ D-)^4 / 256,
 *                       the dissipative sign; four end-value ghosts per side. */
enum { TEUK_SCHEME_WENO5 = 0, TEUK_SCHEME_WENO3 = 1, TEUK_SCHEME_FD6KO8 = 2 };

/* What teuk_extract returns. */
enum {
    TEUK_X_STATE = 0,     /* [4][ntheta][nr] current state u^n                        */
    TEUK_X_WAVEFORM = 1,  /* [n][ntheta][2] (Phi_R, Phi_I) at x_extract, oldest first */
    TEUK_X_TIMES = 2,     /* [n] times of the waveform samples                        */
    TEUK_X_COEFFS = 3,    /* [TEUK_NCOEF][ntheta][nr] per-point coefficients as the
                             device evaluates them (diagnostic)                       */
    TEUK_X_RHS = 4,       /* [4][ntheta][nr] F(u^n) = -(M d_x u + L u + A u) of the
                             current state, by the stage kernel (diagnostic)           */
    TEUK_X_HORIZON = 5    /* [n][ntheta][4] (Phi_R, Phi_I, d_rho Phi_R, d_rho Phi_I) on the
                             horizon rho_H = S r+/(r+ + S), oldest first, sampled with
                             the waveform (hyperboloidal chart only)                  */
};

/* Per-point coefficients returned by TEUK_X_COEFFS / teuk_host_coefficients,
 * plane order: lam1, Re m3, Im m3, Re B~t, Im B~t, Re C~, Im C~, A~thth, B~th, lam2,
 * where (x the chart's radial coordinate, t its time)
 *   d_t Phi = pi - lam1 d_x Phi
 *   d_t pi  = -lam2 d_x pi - m3 d_x Phi + B~t pi + A~thth Phi_thth + B~th Phi_th + C~ Phi
 * (the paper's M, A, L entries: M11 = lam1, M33 = lam2, m31 = Re m3, m32 = -Im m3,
 *  a31 = -Re C~, a32 = Im C~, a33 = -Re B~t, a34 = Im B~t, l31 = -(A~thth d_thth + B~th d_th)).
 * Chart T: lam1 = b = (r^2+a^2)/Sigma > 0 and lam2 = -b. */
#define TEUK_NCOEF 10

typedef struct {
    int32_t abi_version;     /* must equal TEUK_ABI_VERSION                          */
    int32_t s;               /* spin weight, |s| <= 2                                 */
    int32_t m;               /* azimuthal number, |m| <= 8                            */
    int32_t chart;           /* TEUK_CHART_*                                          */
    int32_t nr;              /* radial points, 7 <= nr <= 2^24                         */
    int32_t ntheta;          /* polar points, 2 <= ntheta <= 65536                     */
    int32_t weight_prec;     /* TEUK_W_*                                              */
    int32_t extract_every;   /* steps between waveform samples (0: no waveform)        */
    int32_t max_samples;     /* waveform ring-buffer capacity (samples)                */
    int32_t workgroups;      /* stage-kernel workgroups; 0 = all the GPU holds at once */
    int32_t state_prec;      /* TEUK_S_*                                              */
    int32_t integrator;      /* TEUK_RK_*                                             */
    int32_t scheme;          /* TEUK_SCHEME_*                                         */
    int32_t theta_order;     /* order of the centred theta differences (Sec. 3.1):
                                0 or 2: D1 = (u+ - u-)/(2 dth), D2 = (u+ - 2u + u-)/dth^2;
                                4: D1 = (-u++ + 8u+ - 8u- + u--)/(12 dth),
                                   D2 = (-u++ + 16u+ - 30u + 16u- - u--)/(12 dth^2)
                                (tortoise chart, FP64 state, WENO5, TEUK_RK_SSP33 or
                                TEUK_RK_SSP104; any weight precision; groups and graph
                                mode too; else UNSUPPORTED)                             */
    double M;                /* black-hole mass (> 0)                                  */
    double a;                /* spin, 0 <= a <= M                                      */
    double x_min, x_max;     /* radial range of x (r_* or rho; x_min < x_max)          */
    double dt;               /* > 0: time step used as given; <= 0: cfl * C * stability bound,
                                C the integrator's SSP coefficient (1 or 6)            */
    double cfl;              /* used when dt <= 0 (e.g. 0.5)                           */
    double weno_eps;         /* epsilon of the WENO weights (e.g. 1e-6), in [1e-30, 1e30]
                                (normal in FP32, so reduced-precision weights stay finite) */
    double x_extract;        /* waveform radius; the nearest grid node is sampled       */
    double S;                /* hyperboloidal chart parameter (Sec. 2.2; e.g. 20); the
                                grid needs 0 < x_min, x_max < S and the horizon
                                rho_H = S r+/(r+ + S) on it (at most half a step
                                outside); for a = M start it on the horizon, where
                                the pi-row speed vanishes (no incoming data) */
    double ko_sigma;         /* Kreiss-Oliger sigma of TEUK_SCHEME_FD6KO8, in [0, 1] (e.g. 0.01) */
} teuk_config;

typedef struct {
    void* stream;            /* hipStream_t to enqueue on; NULL = null stream          */
    void* workspace;         /* caller-owned device memory for every device buffer of
                                the solver, or NULL to let the library allocate        */
    size_t workspace_bytes;  /* size of workspace; must be >= teuk_footprint_bytes     */
} teuk_device_ctx;

typedef struct {
    double dt;               /* time step in use                                       */
    double t;                /* current time (steps * dt)                              */
    int64_t steps;           /* steps taken since teuk_set_initial                     */
    int64_t samples;         /* waveform samples recorded (may exceed max_samples)     */
    int32_t j_extract;       /* radial index sampled for the waveform                  */
    int32_t workgroups;      /* stage-kernel workgroups in use (stages 2-3)             */
    double dt_bound;         /* stability bound (cfl = 1), from the device reduction   */
} teuk_info_t;

/* Fill cfg with defaults: ABI version, M = 1, chart T, FP64 state and weights,
 * SSP-RK(3,3), WENO5 (ko_sigma 0.01 for FD6), second-order theta differences, cfl 0.5,
 * eps 1e-6, dt from the bound, no waveform.  Sizes and ranges must still be set. */
void teuk_default_config(teuk_config* cfg);

/* Device bytes one solver needs (three state buffers, coefficient tables,
 * waveform ring, reduction cells), each carved at 256-byte alignment.  Returns
 * 0 if cfg is invalid.  Used for admission by HBM footprint. */
size_t teuk_footprint_bytes(const teuk_config* cfg);

/* Create a solver on the current HIP device: validate cfg, build the chart-T
 * background r(x), Delta(x) and the radial / polar coefficient tables on the
 * host in FP64 (Sec. 2.1-2.3), upload them, and compute the stability bound by
 * a device max-reduction over every grid point (Sec. 3.2, dt <= C dt_FE):
 *     dt_bound = 1 / max( b/dx + sqrt(c2 A~thth/dtheta^2 + c1 |B~th|/dtheta + |C~|) ),
 * c2 and c1 the largest moduli of the Fourier symbols of dtheta^2 D2 and
 * dtheta D1: (4, 1) at second order, (16/3, 1.3722...) at fourth, the latter
 * sin(xi) (4 - cos xi)/3 at cos xi = 1 - sqrt(3/2).
 * If cfg->dt <= 0 the step is cfl * C * dt_bound (C = 1 for SSP-RK(3,3), 6 for
 * SSP-RK(10,4)).  ctx may be NULL.  On success
 * *out owns its device buffers (or lives in ctx->workspace, which the caller
 * keeps alive until teuk_destroy and which the library never frees).
 * Errors: INVALID_ARG, OUT_OF_MEMORY (allocation, or workspace too small),
 * DEVICE.  On error *out is NULL and teuk_last_error(NULL) says why. */
teuk_status teuk_create(const teuk_config* cfg, const teuk_device_ctx* ctx, teuk_solver** out);

/* Set the state u^n = {Phi_R, Phi_I, pi_R, pi_I} of the first-order system
 * (eq. evln; pi = d_t Phi + b d_x Phi, Sec. 2.3) -- the initial data of the
 * evolution, e.g. the real Gaussian packets times an angular profile of the
 * runs of Sec. 4 (layout above; on_device != 0 means u is a device pointer
 * with that dense layout, else a host pointer), reset t and the step and
 * sample counters, and record the first waveform sample (t = 0).  The data
 * are copied; u is not retained.  Host input is checked for NaN/Inf
 * (NONFINITE); device input is checked by the device guard.  Double-double
 * pairs are stored normalised (TwoSum of hi and lo: same value, |lo| at most
 * half an ulp of hi).
 * Errors: INVALID_ARG (NULL), NONFINITE, DEVICE. */
teuk_status teuk_set_initial(teuk_solver* h, const double* u, int32_t on_device);

/* Advance nsteps steps of the configured integrator (Sec. 3.2).  SSP-RK(3,3)
 * is three fused stage kernels
 *     u1 = u + dt F(u);  u2 = 3/4 u + 1/4 (u1 + dt F(u1));  u = 1/3 u + 2/3 (u2 + dt F(u2)),
 * SSP-RK(10,4) ten (see TEUK_RK_SSP104),
 * with F(u) = -(M d_x u + L u + A u) of eq. evln and WENO5 radial derivatives
 * (Sec. 3.1.2).  A waveform sample is taken after every extract_every-th step.
 * Asynchronous on the solver's stream.  nsteps = 0 is a no-op.
 * Errors: STATE (no initial data), INVALID_ARG (nsteps < 0), DEVICE. */
teuk_status teuk_step(teuk_solver* h, int64_t nsteps);

/* Graph mode (HIP graphs).  With chunk_steps > 0, teuk_step runs its steps as
 * replays of one graph that holds chunk_steps steps -- every stage launch and
 * waveform sample of them, exactly the launches of stepping one call at a
 * time -- captured on first use, so that the host enqueues one graph launch
 * per chunk instead of three or more kernel launches per step: nsteps / chunk
 * replays, then the remaining nsteps % chunk steps launch by launch.  Results
 * are bitwise those of graph mode off.  Samples reach the right ring slots on
 * every replay because the sample kernel takes its slot from a device copy of
 * the sample count.  The graph is recaptured only when the sampling phase
 * (steps % extract_every) at the start of a replay run differs from the one
 * it was captured at, so stepping in multiples of chunk_steps captures once.
 * The captured work is kernel launches only (no memset or copy nodes).  A
 * solver that has initial data captures its graph in this call, at its current
 * sampling phase (otherwise at its first teuk_step of at least chunk_steps).
 * chunk_steps = 0 turns graph mode off (the default); at most 4096.
 * Errors: INVALID_ARG (NULL, chunk out of range, chunk not a multiple of
 * extract_every, odd chunk with TEUK_RK_SSP33_BLOCKED), UNSUPPORTED
 * (double-double state).  teuk_step may then also return DEVICE from the
 * capture or a replay. */
teuk_status teuk_set_graph(teuk_solver* h, int32_t chunk_steps);

/* Copy results to the host array out (capacity in doubles); *written receives
 * the number of doubles written (may be NULL).  The waveform is the field Phi
 * at a fixed radius sampled in time, the series whose late-time decay (local
 * power-law index t dPhi/dt / Phi) Sec. 4 studies; the horizon samples are Phi
 * and d_rho Phi on the extremal horizon, the quantities of the horizon laws of
 * Sec. 4 (Phi_H decaying as 1/tau while d_rho Phi_H tends to a constant, the
 * Aretakis behaviour).  Synchronises the stream and
 * runs the non-finite guard on the state first (NONFINITE if it trips; the
 * data are still copied for inspection).
 *   TEUK_X_STATE     4*ntheta*nr doubles (twice that in double-double)
 *   TEUK_X_WAVEFORM  min(samples, max_samples)*ntheta*2 doubles, oldest first
 *                    (twice that in double-double)
 *   TEUK_X_TIMES     min(samples, max_samples) doubles
 *   TEUK_X_HORIZON   min(samples, max_samples)*ntheta*4 doubles, oldest first
 *                    (hyperboloidal chart; UNSUPPORTED in the tortoise chart)
 *   TEUK_X_COEFFS    TEUK_NCOEF*ntheta*nr doubles (twice that in double-double)
 *   TEUK_X_RHS       4*ntheta*nr doubles (uses the stage scratch buffer; the
 *                    state is unchanged; twice that in double-double)
 * Errors: INVALID_ARG, CAPACITY (out too small; nothing written), NONFINITE,
 * DEVICE. */
teuk_status teuk_extract(teuk_solver* h, int32_t what, double* out, size_t capacity, size_t* written);

/* Solver information (synchronises the stream).  Errors: INVALID_ARG, DEVICE. */
teuk_status teuk_info(teuk_solver* h, teuk_info_t* info);

/* Run the device non-finite guard on the current state: a max-reduction that
 * flags any NaN/Inf.  Synchronises.  Errors: NONFINITE, STATE, DEVICE. */
teuk_status teuk_check_finite(teuk_solver* h);

/* Release the solver and the device memory it allocated.  NULL-safe. */
void teuk_destroy(teuk_solver* h);

/* Last error message of h, or of the calling thread's last failed
 * teuk_create / teuk_host_coefficients when h is NULL.  Never NULL. */
const char* teuk_last_error(const teuk_solver* h);

/* Host-only evaluation, in FP64, of the per-point coefficients (TEUK_X_COEFFS
 * layout) from the same tables and the same formula the device uses.  Needs no
 * GPU.  out holds capacity doubles (>= TEUK_NCOEF*ntheta*nr).  For a
 * TEUK_S_DD configuration: the double-double table the device streams, as
 * pairs (>= 2*TEUK_NCOEF*ntheta*nr doubles).
 * Errors: INVALID_ARG, CAPACITY. */
teuk_status teuk_host_coefficients(const teuk_config* cfg, double* out, size_t capacity);

/* ------------------------------------------------------------------------
 * Launch-shape autotuner.
 *
 * A stage launch of a single solve runs nstrips x segs workgroups (radial
 * strips of 63 points, 114 for the blocked step, each cut into segs theta
 * segments that its workgroups march), with segs derived from a workgroup
 * budget: cfg->workgroups, or by default the number of stage workgroups the
 * GPU holds at once.  teuk_tune times the stage kernels of cfg for a set of
 * budgets from 1/4 to 4 times that default and those giving segments of 2, 4
 * and 8 rows (one per distinct segs), each the
 * best of three runs of `steps` steps (0: chosen to take about 2 ms) on a
 * scratch solver of the same grid, chart, precisions and integrator with a
 * smooth synthetic state of order one, and remembers the fastest budget for that launch class (device, chart
 * and theta order, weight and state precision, integrator, scheme, nr, ntheta) for the rest of
 * the process: a later teuk_create of that class with workgroups = 0 uses it
 * (teuk_info reports the workgroups in use).  The tiling does not change any
 * point's arithmetic, so results are bitwise independent of the choice.  The
 * scratch solver is allocated and freed inside the call; the stream is a
 * private one.  Errors: INVALID_ARG, UNSUPPORTED (double-double state), the
 * errors of teuk_create and teuk_step, DEVICE; teuk_tune_last_error() says why. */
typedef struct {
    int32_t workgroups;          /* fastest budget (the value teuk_create will use)  */
    int32_t segs;                /* theta segments per strip it gives               */
    int32_t default_workgroups;  /* the untuned default budget                      */
    int32_t default_segs;
    int32_t candidates;          /* budgets timed                                   */
    int32_t steps;               /* steps per timed run                             */
    double us_per_step;          /* fastest, microseconds per step                   */
    double us_per_step_default;  /* the default budget, microseconds per step        */
} teuk_tune_info_t;
teuk_status teuk_tune(const teuk_config* cfg, int32_t steps, teuk_tune_info_t* info);

/* Forget every tuned budget of the process (later solvers use the defaults). */
void teuk_tune_forget(void);

/* Message of the calling thread's last failed teuk_tune.  Never NULL. */
const char* teuk_tune_last_error(void);

/* Allocation-free stepping, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Advances the caller's device state u ([4][ntheta][nr] FP64
 * planes, the layout above; read and written in place, not retained) by
 * nsteps SSP-RK(3,3) steps of cfg, enqueued on `stream` (a hipStream_t, NULL
 * for the null stream), with the same stage kernels and launch shapes as
 * teuk_step: the result is bitwise that of teuk_create + teuk_set_initial +
 * teuk_step with the same cfg.  It allocates nothing: the two stage buffers
 * and the coefficient tables live in a fixed device array of the library
 * (about 67 MiB, held by every GPU the library runs on until the process
 * ends), so the grid is limited to nr <= 32768, ntheta <= 4096 and
 * nr * ntheta <= 2^20 points.  The array keeps the last call's contents: the
 * tables are rebuilt on the host and uploaded (a synchronising copy) only
 * when s, m, M, a, nr, ntheta, x_min or x_max differ from the previous call
 * on the device.  Under stream capture the tables of cfg must already be
 * resident (an earlier call with the same cfg), else the call fails with
 * STATE and enqueues nothing; the captured work is kernel launches only.
 * Calls that overlap on one GPU (other threads or streams) share the array
 * and race.  Tortoise chart, FP64 state, WENO5, FP64/FP32/FP16/BF16 weights;
 * cfg->dt must be > 0 (no stability-bound reduction) and
 * cfg->extract_every 0 (no waveform ring).
 * Errors: INVALID_ARG (bad cfg, NULL u, nsteps < 0, dt <= 0, extract_every
 * != 0, grid beyond the limits), UNSUPPORTED (other chart, state, integrator
 * or scheme), STATE (capture without resident tables), DEVICE;
 * teuk_last_error(NULL) says why. */
teuk_status teuk_step_noalloc(const teuk_config* cfg, double* u, int64_t nsteps, void* stream);

/* ------------------------------------------------------------------------
 * Group extension: many independent solves advanced together.
 *
 * Separating exp(i m phi~) (Sec. 3) leaves one 2+1D problem per (s, m) mode
 * and per background; such solves share nothing, so a group advances all of
 * its members in one stage-kernel launch per SSP-RK stage (one per weight
 * precision present and per cache block of members) instead of three
 * launches per member per step.  A cache block whose every member fills the
 * GPU by itself (63-point strips x theta rows at least the stage kernel's
 * resident workgroups) has no launches to save: with workgroups = 0 it runs
 * its members' own single-solve stage launches, member after member within
 * each stage, which are faster on such grids.  Each
 * member keeps its own grid, coefficients, dt, waveform ring and counters, and
 * its results are bitwise those of teuk_step on the member alone: the tiles
 * of a member run the single-solve stage arithmetic unchanged.
 *
 * Members are created with teuk_create as usual and must use the group's
 * stream.  The group does not own its members; teuk_destroy of a member
 * removes it from its group first.  A solver belongs to at most one group.
 * Device memory: the group allocates one small descriptor block at creation
 * (about 3 * max_members * 160 bytes) and nothing per step.
 */
typedef struct teuk_group teuk_group;   /* opaque; owned by the library */

typedef struct {
    int32_t members;         /* solvers in the group                                 */
    int32_t classes;         /* (weight precision, chart) classes present            */
    int64_t workgroups;      /* workgroups per stage (stages 2-3), summed over the launches */
    int64_t tiles;           /* tiles (one strip x one theta segment) per stage        */
    int64_t units;           /* strip-rows per stage (63 radial points x 1 theta row)  */
    int64_t points;          /* grid points over all members                          */
} teuk_group_info_t;

/* Create an empty group on the current HIP device, enqueuing on ctx->stream
 * (ctx may be NULL: null stream; ctx->workspace is not used).  max_members in
 * [1, 65536].  Each member is cut into tiles of one 63-point radial strip by
 * one theta segment of about rows_per_tile rows (0: 8); the tiles are
 * numbered segment by segment with the strip index fastest, so that the
 * workgroups in flight march neighbouring strips over the same rows.  Each
 * stage launch runs one workgroup per tile (workgroups = 0) or `workgroups`
 * workgroups that take the tiles round-robin.  Members of one weight precision
 * and chart are launched together in cache blocks of consecutive members whose
 * footprints (teuk_footprint_bytes) sum to at most 256 MiB; teuk_group_step
 * runs all its steps on one block before the next, so that a block's state
 * stays largely in the GPU's last-level cache between stages.
 * Errors: INVALID_ARG, OUT_OF_MEMORY, DEVICE; teuk_group_last_error(NULL)
 * says why. */
teuk_status teuk_group_create(const teuk_device_ctx* ctx, int32_t max_members, int32_t workgroups,
                              int32_t rows_per_tile, teuk_group** out);

/* Add a solver (after teuk_set_initial) to the group.  Synchronises the group's
 * stream and uploads the members' descriptors.  Members step with SSP-RK(3,3),
 * three-launch (TEUK_RK_SSP33) or temporally blocked (TEUK_RK_SSP33_BLOCKED),
 * and WENO5.  Errors: INVALID_ARG (NULL, other stream, already in a group),
 * CAPACITY (group full), STATE (no initial data), UNSUPPORTED (double-double
 * state, another integrator or scheme), DEVICE. */
teuk_status teuk_group_add(teuk_group* g, teuk_solver* h);

/* Remove a member (synchronises the group's stream).  The solver stays valid
 * and can be stepped alone.  Errors: INVALID_ARG (NULL, not a member), DEVICE. */
teuk_status teuk_group_remove(teuk_group* g, teuk_solver* h);

/* Advance every member nsteps SSP-RK(3,3) steps with its own dt, sampling each
 * member's waveform as teuk_step does.  Asynchronous on the group's stream.
 * The steps run block by block (all nsteps on one cache block of members,
 * then the next), so on an error some members may have advanced and others
 * not; each member's step and sample counters stay consistent with its own
 * state.  An empty group or nsteps = 0 is a no-op.  Errors: INVALID_ARG,
 * DEVICE. */
teuk_status teuk_group_step(teuk_group* g, int64_t nsteps);

/* Graph mode for the group (see teuk_set_graph): teuk_group_step runs, cache
 * block by cache block, nsteps / chunk_steps replays of that block's graph of
 * chunk_steps steps (its stage launches and its members' samples), then the
 * remainder launch by launch.  Each block keeps its own graph, so a block still
 * runs all of a call's steps before the next block starts.  Adding or removing
 * a member drops the graphs; they are recaptured on the next step.  This
 * call captures every block's graph at once.  Every
 * member's extract_every must divide chunk_steps, and chunk_steps must be even
 * when a member takes the blocked step (else this call and teuk_group_step
 * return INVALID_ARG).  chunk_steps = 0 turns it off; at most 4096.
 * Errors: INVALID_ARG, DEVICE (capture). */
teuk_status teuk_group_set_graph(teuk_group* g, int32_t chunk_steps);

/* Tune the group's tile height and cache-block size on its current members.
 * Times rows_per_tile in {4, 8, 16, 32, 64} by cache blocks of
 * {32, 64, 128, 256, 384, 512} MiB of member footprint (and the group's current
 * shape), each the best of two runs of `steps` steps (0: chosen to take about
 * 20 ms) on clones of the members -- same grids, classes and step sizes,
 * starting from the members' current states, no waveform rings -- so the
 * members themselves do not advance; then applies the fastest shape to the
 * group.  Results do not depend on the shape (bitwise).  The clones double
 * the group's device footprint during the call.  Synchronises the group's
 * stream.  Errors: INVALID_ARG, STATE (no members), OUT_OF_MEMORY, DEVICE. */
typedef struct {
    int32_t rows_per_tile, block_mib;                  /* the shape applied            */
    int32_t default_rows_per_tile, default_block_mib;  /* the shape before the call    */
    int32_t candidates, steps;                         /* shapes timed, steps per run  */
    double us_per_step, us_per_step_default;           /* microseconds per group step  */
} teuk_group_tune_info_t;
teuk_status teuk_group_tune(teuk_group* g, int32_t steps, teuk_group_tune_info_t* info);

/* Group information (no synchronisation).  Errors: INVALID_ARG. */
teuk_status teuk_group_info(const teuk_group* g, teuk_group_info_t* info);

/* Release the group (members are detached, not destroyed).  NULL-safe. */
void teuk_group_destroy(teuk_group* g);

/* Last error message of g (or of the thread's last failed teuk_group_create
 * when g is NULL).  Never NULL. */
const char* teuk_group_last_error(const teuk_group* g);

#ifdef __cplusplus
}
#endif

#endif /* TEUK_H */
