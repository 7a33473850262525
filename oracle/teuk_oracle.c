/*
 * Oracle: plain, scalar solver for the first-order Teukolsky system.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline of the benchmark load this library; the product path never does.
 * It is built with -O2 -fno-fast-math -ffp-contract=off so that every
 * operation is rounded exactly as written.
 *
 * The same source is built twice: with `real` = double (FP64, the default
 * build) and, with -DORACLE_QUAD, with `real` = __float128 (IEEE binary128,
 * the "quad precision" of Sec. 3.1.3; every name then carries the suffix _q).
 * Scalars that must be exact in either precision are passed as (hi, lo)
 * pairs of doubles and formed as (real)hi + (real)lo.
 *
 * What it computes, step by step, in the paper's order:
 *   - WENO5 smoothness indicators IS_k, weights alpha_k / omega_k and the
 *     interface fluxes f^+_{j+1/2}, f^-_{j+1/2} of Jiang and Shu (Sec. 3.1.2),
 *     with the f^- flux pairing its first candidate with omega^-_0 (the printed
 *     omega^+_0 there is read as a typo);
 *   - the flux differences (f_{j+1/2} - f_{j-1/2}) / dx (Sec. 3.1.2);
 *   - each real plane of u = {Phi_R, Phi_I, pi_R, pi_I} differentiated by the
 *     WENO side that matches the sign of its wave speed (Sec. 3.1.2: positive
 *     speed -> f^+ treatment, negative -> f^-);
 *   - centred differences in theta (Sec. 3.1; the paper does not state their
 *     order): second order by default,
 *       D1 u = (u_{k+1} - u_{k-1}) / (2 dth),
 *       D2 u = (u_{k+1} - 2 u_k + u_{k-1}) / dth^2,
 *     or, with theta_order = 4, the fourth-order centred stencils
 *       D1 u = (-u_{k+2} + 8 u_{k+1} - 8 u_{k-1} + u_{k-2}) / (12 dth),
 *       D2 u = (-u_{k+2} + 16 u_{k+1} - 30 u_k + 16 u_{k-1} - u_{k-2}) / (12 dth^2);
 *   - the right-hand side of eq. evln, -(M d_x u + L u + A u), written with
 *     complex 2x2 blocks;
 *   - SSP-RK(3,3) in the Shu-Osher form of Sec. 3.2.
 * Ghost values: three cells per radial side copied from the end point, and in
 * theta (-1)^(m+s) times the cell mirrored across the pole: on the
 * cell-centred grid theta_k = (k + 1/2) dth, row -1 - g mirrors row g and row
 * nth + g mirrors row nth - 1 - g (one such row per pole at second order, two
 * at fourth).
 *
 * Radial schemes (Sec. 3.1): WENO5 (scheme 0, above), the third-order WENO of
 * Sec. 3.1.2 (scheme 1: two candidate stencils, IS_1 = (f_j - f_{j-1})^2,
 * IS_2 = (f_{j+1} - f_j)^2, linear weights 1/3, 2/3; the printed f^- flux is
 * read as the mirror image of f^+ about j + 1/2, i.e. built from
 * f_j, f_{j+1}, f_{j+2}), and the sixth-order centred difference with
 * eighth-order Kreiss-Oliger dissipation of Sec. 3.1.1 (scheme 2:
 * D u = (u_{j+3} - 9 u_{j+2} + 45 u_{j+1} - 45 u_{j-1} + 9 u_{j-2} - u_{j-3})/(60 dx),
 * and every plane's right-hand side receives -Q u with
 * Q = sigma dx^7 (D_+ D_-)^4 / 256 = sigma delta^8 / (256 dx), the sign that
 * makes it dissipative; four ghost cells per side).
 *
 * Weight precision (Sec. 3.1.3).  wmode 0 forms IS_k, alpha_k and omega_k in
 * `real` exactly as printed.  wmode 1 is the paper's mixed variant: the five
 * stencil values are rounded to double, IS_k, alpha_k, omega_0 and omega_1 are
 * formed from them in double arithmetic as printed, and omega_2 is the
 * complement 1 - omega_0 - omega_1 taken in `real`; the candidate fluxes and
 * their combination stay in `real`.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifdef ORACLE_QUAD
typedef __float128 real;
#define FN(name) name##_q
#else
typedef double real;
#define FN(name) name
#endif
#define R(v) ((real)(v))

static real sq(real v) { return v * v; }
static double sqd(double v) { return v * v; }
static real pair(double hi, double lo) { return R(hi) + R(lo); }

/* ---------------------------------------------------------------- WENO5 (Sec. 3.1.2) */

/* f points at f_{j-2}; f[0..4] = f_{j-2..j+2}.  Weights of f^+_{j+1/2}. */
void FN(oracle_weno5_weights_plus)(const real* f, double eps, real w[3])
{
    const real e = R(eps);
    real IS0 = R(13) / R(12) * sq(f[0] - R(2) * f[1] + f[2]) + R(1) / R(4) * sq(f[0] - R(4) * f[1] + R(3) * f[2]);
    real IS1 = R(13) / R(12) * sq(f[1] - R(2) * f[2] + f[3]) + R(1) / R(4) * sq(f[1] - f[3]);
    real IS2 = R(13) / R(12) * sq(f[2] - R(2) * f[3] + f[4]) + R(1) / R(4) * sq(R(3) * f[2] - R(4) * f[3] + f[4]);
    real a0 = R(1) / R(10) * sq(R(1) / (e + IS0));
    real a1 = R(6) / R(10) * sq(R(1) / (e + IS1));
    real a2 = R(3) / R(10) * sq(R(1) / (e + IS2));
    real sum = a0 + a1 + a2;
    w[0] = a0 / sum;
    w[1] = a1 / sum;
    w[2] = a2 / sum;
}

/* The same weights, mixed variant: f rounded to double, IS/alpha/omega_0,1 in
 * double, omega_2 = 1 - omega_0 - omega_1 in real. */
void FN(oracle_weno5_weights_plus_w64)(const real* f, double eps, real w[3])
{
    double g[5];
    for (int i = 0; i < 5; ++i) g[i] = (double)f[i];
    double IS0 = 13.0 / 12.0 * sqd(g[0] - 2.0 * g[1] + g[2]) + 0.25 * sqd(g[0] - 4.0 * g[1] + 3.0 * g[2]);
    double IS1 = 13.0 / 12.0 * sqd(g[1] - 2.0 * g[2] + g[3]) + 0.25 * sqd(g[1] - g[3]);
    double IS2 = 13.0 / 12.0 * sqd(g[2] - 2.0 * g[3] + g[4]) + 0.25 * sqd(3.0 * g[2] - 4.0 * g[3] + g[4]);
    double a0 = (1.0 / 10.0) * sqd(1.0 / (eps + IS0));
    double a1 = (6.0 / 10.0) * sqd(1.0 / (eps + IS1));
    double a2 = (3.0 / 10.0) * sqd(1.0 / (eps + IS2));
    double sum = a0 + a1 + a2;
    w[0] = R(a0 / sum);
    w[1] = R(a1 / sum);
    w[2] = R(1) - w[0] - w[1];
}

/* f^+_{j+1/2} from f_{j-2..j+2} with given weights. */
real FN(oracle_weno5_combine_plus)(const real* f, const real w[3])
{
    return w[0] * (R(2) / R(6) * f[0] - R(7) / R(6) * f[1] + R(11) / R(6) * f[2])
         + w[1] * (-(R(1) / R(6)) * f[1] + R(5) / R(6) * f[2] + R(2) / R(6) * f[3])
         + w[2] * (R(2) / R(6) * f[2] + R(5) / R(6) * f[3] - R(1) / R(6) * f[4]);
}

static real flux_plus(const real* f, double eps, int wmode)
{
    real w[3];
    if (wmode) FN(oracle_weno5_weights_plus_w64)(f, eps, w);
    else FN(oracle_weno5_weights_plus)(f, eps, w);
    return FN(oracle_weno5_combine_plus)(f, w);
}

real FN(oracle_weno5_flux_plus)(const real* f, double eps) { return flux_plus(f, eps, 0); }

/* g points at f_{j-1}; g[0..4] = f_{j-1..j+3}.  Weights of f^-_{j+1/2}. */
void FN(oracle_weno5_weights_minus)(const real* g, double eps, real w[3])
{
    const real e = R(eps);
    real IS0 = R(13) / R(12) * sq(g[2] - R(2) * g[3] + g[4]) + R(1) / R(4) * sq(R(3) * g[2] - R(4) * g[3] + g[4]);
    real IS1 = R(13) / R(12) * sq(g[1] - R(2) * g[2] + g[3]) + R(1) / R(4) * sq(g[1] - g[3]);
    real IS2 = R(13) / R(12) * sq(g[0] - R(2) * g[1] + g[2]) + R(1) / R(4) * sq(g[0] - R(4) * g[1] + R(3) * g[2]);
    real a0 = R(1) / R(10) * sq(R(1) / (e + IS0));
    real a1 = R(6) / R(10) * sq(R(1) / (e + IS1));
    real a2 = R(3) / R(10) * sq(R(1) / (e + IS2));
    real sum = a0 + a1 + a2;
    w[0] = a0 / sum;
    w[1] = a1 / sum;
    w[2] = a2 / sum;
}

void FN(oracle_weno5_weights_minus_w64)(const real* g, double eps, real w[3])
{
    double h[5];
    for (int i = 0; i < 5; ++i) h[i] = (double)g[i];
    double IS0 = 13.0 / 12.0 * sqd(h[2] - 2.0 * h[3] + h[4]) + 0.25 * sqd(3.0 * h[2] - 4.0 * h[3] + h[4]);
    double IS1 = 13.0 / 12.0 * sqd(h[1] - 2.0 * h[2] + h[3]) + 0.25 * sqd(h[1] - h[3]);
    double IS2 = 13.0 / 12.0 * sqd(h[0] - 2.0 * h[1] + h[2]) + 0.25 * sqd(h[0] - 4.0 * h[1] + 3.0 * h[2]);
    double a0 = (1.0 / 10.0) * sqd(1.0 / (eps + IS0));
    double a1 = (6.0 / 10.0) * sqd(1.0 / (eps + IS1));
    double a2 = (3.0 / 10.0) * sqd(1.0 / (eps + IS2));
    double sum = a0 + a1 + a2;
    w[0] = R(a0 / sum);
    w[1] = R(a1 / sum);
    w[2] = R(1) - w[0] - w[1];
}

real FN(oracle_weno5_combine_minus)(const real* g, const real w[3])
{
    return w[2] * (-(R(1) / R(6)) * g[0] + R(5) / R(6) * g[1] + R(2) / R(6) * g[2])
         + w[1] * (R(2) / R(6) * g[1] + R(5) / R(6) * g[2] - R(1) / R(6) * g[3])
         + w[0] * (R(11) / R(6) * g[2] - R(7) / R(6) * g[3] + R(2) / R(6) * g[4]);
}

static real flux_minus(const real* g, double eps, int wmode)
{
    real w[3];
    if (wmode) FN(oracle_weno5_weights_minus_w64)(g, eps, w);
    else FN(oracle_weno5_weights_minus)(g, eps, w);
    return FN(oracle_weno5_combine_minus)(g, w);
}

real FN(oracle_weno5_flux_minus)(const real* g, double eps) { return flux_minus(g, eps, 0); }

/* Flux-difference derivatives at point j of a padded row p (p[j] is point j,
 * valid for j-3 .. j+3). */
static real dplus(const real* p, long j, real dx, double eps, int wmode)
{
    return (flux_plus(p + j - 2, eps, wmode) - flux_plus(p + j - 3, eps, wmode)) / dx;
}

static real dminus(const real* p, long j, real dx, double eps, int wmode)
{
    return (flux_minus(p + j - 1, eps, wmode) - flux_minus(p + j - 2, eps, wmode)) / dx;
}

real FN(oracle_dplus)(const real* p, long j, double dx, double dx_lo, double eps, int wmode)
{
    return dplus(p, j, pair(dx, dx_lo), eps, wmode);
}

real FN(oracle_dminus)(const real* p, long j, double dx, double dx_lo, double eps, int wmode)
{
    return dminus(p, j, pair(dx, dx_lo), eps, wmode);
}

/* Upwinded derivative: speed >= 0 -> f^+ treatment, speed < 0 -> f^-. */
static real upwind_d(const real* p, long j, real speed, real dx, double eps, int wmode)
{
    return speed < R(0) ? dminus(p, j, dx, eps, wmode) : dplus(p, j, dx, eps, wmode);
}

/* ---------------------------------------------------------------- WENO3 (Sec. 3.1.2) */

/* f = f_{j-1..j+1}: weights of f^+_{j+1/2}. */
void FN(oracle_weno3_weights_plus)(const real* f, double eps, real w[2])
{
    const real e = R(eps);
    real IS1 = sq(f[1] - f[0]);
    real IS2 = sq(f[2] - f[1]);
    real a1 = R(1) / R(3) * sq(R(1) / (e + IS1));
    real a2 = R(2) / R(3) * sq(R(1) / (e + IS2));
    w[0] = a1 / (a1 + a2);
    w[1] = a2 / (a1 + a2);
}

real FN(oracle_weno3_flux_plus)(const real* f, double eps)
{
    real w[2];
    FN(oracle_weno3_weights_plus)(f, eps, w);
    return w[0] * (R(3) / R(2) * f[1] - R(1) / R(2) * f[0]) + w[1] * (R(1) / R(2) * f[1] + R(1) / R(2) * f[2]);
}

/* g = f_{j..j+2}: weights of f^-_{j+1/2}, the mirror image of f^+. */
void FN(oracle_weno3_weights_minus)(const real* g, double eps, real w[2])
{
    const real e = R(eps);
    real IS1 = sq(g[2] - g[1]);
    real IS2 = sq(g[1] - g[0]);
    real a1 = R(1) / R(3) * sq(R(1) / (e + IS1));
    real a2 = R(2) / R(3) * sq(R(1) / (e + IS2));
    w[0] = a1 / (a1 + a2);
    w[1] = a2 / (a1 + a2);
}

real FN(oracle_weno3_flux_minus)(const real* g, double eps)
{
    real w[2];
    FN(oracle_weno3_weights_minus)(g, eps, w);
    return w[0] * (R(3) / R(2) * g[1] - R(1) / R(2) * g[2]) + w[1] * (R(1) / R(2) * g[1] + R(1) / R(2) * g[0]);
}

/* ---------------------------------------------------------------- FD6 + KO8 (Sec. 3.1.1) */

static real fd6(const real* p, long j, real dx)
{
    return (p[j + 3] - R(9) * p[j + 2] + R(45) * p[j + 1] - R(45) * p[j - 1] + R(9) * p[j - 2] - p[j - 3]) /
           (R(60) * dx);
}

/* Q u at j = sigma dx^7 (D_+ D_-)^4 u / 256 = sigma delta^8 u / (256 dx). */
static real ko8(const real* p, long j, real dx, real sigma)
{
    const real d8 = p[j - 4] - R(8) * p[j - 3] + R(28) * p[j - 2] - R(56) * p[j - 1] + R(70) * p[j] -
                    R(56) * p[j + 1] + R(28) * p[j + 2] - R(8) * p[j + 3] + p[j + 4];
    return sigma * d8 / (R(256) * dx);
}

/* Radial derivative of a padded row at j by the chosen scheme; speed picks
 * the upwind side of the WENO schemes. */
static real radial_d(const real* p, long j, real speed, real dx, double eps, int wmode, int scheme)
{
    if (scheme == 2) return fd6(p, j, dx);
    if (scheme == 1) {
        if (speed < R(0))
            return (FN(oracle_weno3_flux_minus)(p + j, eps) - FN(oracle_weno3_flux_minus)(p + j - 1, eps)) / dx;
        return (FN(oracle_weno3_flux_plus)(p + j - 1, eps) - FN(oracle_weno3_flux_plus)(p + j - 2, eps)) / dx;
    }
    return upwind_d(p, j, speed, dx, eps, wmode);
}

/* The radial derivative at point j of a row padded by four cells per side
 * (pairs for dx), for tests of the schemes. */
real FN(oracle_radial_d)(const real* p, long j, double speed, double dx, double dx_lo, double eps, int scheme)
{
    return radial_d(p, j, R(speed), pair(dx, dx_lo), eps, 0, scheme);
}

/* ---------------------------------------------------------------- SSP-RK(3,3) (Sec. 3.2) */

typedef void (*oracle_rhs_fn)(const real* u, real* F, void* ctx);

/* One step of SSP-RK(3,3):
 *   u1 = u + dt F(u)
 *   u2 = 3/4 u + 1/4 (u1 + dt F(u1))
 *   u  = 1/3 u + 2/3 (u2 + dt F(u2))
 * work holds 3n values. */
static void ssprk3_step(real* u, long n, real dt, oracle_rhs_fn rhs, void* ctx, real* work)
{
    real* F = work;
    real* u1 = work + n;
    real* u2 = work + 2 * n;
    rhs(u, F, ctx);
    for (long i = 0; i < n; ++i) u1[i] = u[i] + dt * F[i];
    rhs(u1, F, ctx);
    for (long i = 0; i < n; ++i) u2[i] = R(3) / R(4) * u[i] + R(1) / R(4) * (u1[i] + dt * F[i]);
    rhs(u2, F, ctx);
    for (long i = 0; i < n; ++i) u[i] = R(1) / R(3) * u[i] + R(2) / R(3) * (u2[i] + dt * F[i]);
}

void FN(oracle_ssprk3_step)(real* u, long n, double dt, oracle_rhs_fn rhs, void* ctx, real* work)
{
    ssprk3_step(u, n, R(dt), rhs, ctx, work);
}

/* One step of the low-storage ten-stage, fourth-order SSP-RK(10,4) as the
 * paper writes it (Sec. 3.2):
 *   u(1)    = u^n + dt/6 F(u^n),  u(i) = u(i-1) + dt/6 F(u(i-1)), i = 2..4,
 *   u(5)    = 3/5 u^n + 2/5 u(4) + 1/15 dt F(u(4)),
 *   u(i)    = u(i-1) + dt/6 F(u(i-1)), i = 6..9,
 *   u^{n+1} = 1/25 u^n + 9/25 u(4) + 3/5 u(9) + 3/50 dt F(u(4)) + 1/10 dt F(u(9)).
 * work holds 5n values (u^n, u(4), F(u(4)), the current stage, F). */
static void ssprk104_step(real* u, long n, real dt, oracle_rhs_fn rhs, void* ctx, real* work)
{
    real* un = work;
    real* u4 = work + n;
    real* F4 = work + 2 * n;
    real* cur = work + 3 * n;
    real* F = work + 4 * n;
    const real h6 = dt / R(6);
    memcpy(un, u, (size_t)n * sizeof(real));
    memcpy(cur, u, (size_t)n * sizeof(real));
    for (int st = 1; st <= 4; ++st) {
        rhs(cur, F, ctx);
        for (long i = 0; i < n; ++i) cur[i] = cur[i] + h6 * F[i];
    }
    memcpy(u4, cur, (size_t)n * sizeof(real));
    rhs(u4, F4, ctx);
    for (long i = 0; i < n; ++i)
        cur[i] = R(3) / R(5) * un[i] + R(2) / R(5) * u4[i] + R(1) / R(15) * dt * F4[i];
    for (int st = 6; st <= 9; ++st) {
        rhs(cur, F, ctx);
        for (long i = 0; i < n; ++i) cur[i] = cur[i] + h6 * F[i];
    }
    rhs(cur, F, ctx);
    for (long i = 0; i < n; ++i)
        u[i] = R(1) / R(25) * un[i] + R(9) / R(25) * u4[i] + R(3) / R(5) * cur[i] + R(3) / R(50) * dt * F4[i] +
               R(1) / R(10) * dt * F[i];
}

void FN(oracle_ssprk104_step)(real* u, long n, double dt, oracle_rhs_fn rhs, void* ctx, real* work)
{
    ssprk104_step(u, n, R(dt), rhs, ctx, work);
}

/* ---------------------------------------------------------------- 1D advection (tests) */

typedef struct {
    long n;
    real dx, speed;
    double eps;
    int wmode, scheme;
    real sigma;
} oracle_advect;

/* u_t + speed u_x = 0 on a periodic grid: F = -speed * D u. */
static void advect_rhs(const real* u, real* F, void* vctx)
{
    const oracle_advect* A = (const oracle_advect*)vctx;
    long n = A->n;
    real* p = (real*)malloc((size_t)(n + 8) * sizeof(real));
    for (long i = 0; i < n + 8; ++i) p[i] = u[((i - 4) % n + n) % n];
    for (long j = 0; j < n; ++j) {
        F[j] = -A->speed * radial_d(p + 4, j, A->speed, A->dx, A->eps, A->wmode, A->scheme);
        if (A->scheme == 2) F[j] -= ko8(p + 4, j, A->dx, A->sigma);
    }
    free(p);
}

void FN(oracle_advect1d)(real* u, long n, double dx, double dx_lo, double speed, double dt, double dt_lo,
                         long nsteps, double eps, int wmode)
{
    oracle_advect A = {n, pair(dx, dx_lo), R(speed), eps, wmode, 0, R(0)};
    real* work = (real*)malloc((size_t)(3 * n) * sizeof(real));
    for (long s = 0; s < nsteps; ++s) ssprk3_step(u, n, pair(dt, dt_lo), advect_rhs, &A, work);
    free(work);
}

/* The same with a radial scheme (0 WENO5, 1 WENO3, 2 FD6 + KO8 with sigma). */
void FN(oracle_advect1d_scheme)(real* u, long n, double dx, double speed, double dt, long nsteps, double eps,
                                int scheme, double sigma)
{
    oracle_advect A = {n, R(dx), R(speed), eps, 0, scheme, R(sigma)};
    real* work = (real*)malloc((size_t)(3 * n) * sizeof(real));
    for (long s = 0; s < nsteps; ++s) ssprk3_step(u, n, R(dt), advect_rhs, &A, work);
    free(work);
}

/* ---------------------------------------------------------------- Teukolsky system (eq. evln) */

typedef struct {
    long nr, nth;
    double dx, dx_lo, dth, dth_lo;   /* grid steps as (hi, lo) pairs */
    double eps;
    double parity;                   /* (-1)^(m+s) for the pole ghosts */
    int wmode;                       /* 0: weights in real; 1: mixed (double) */
    int scheme;                      /* 0 WENO5, 1 WENO3, 2 FD6 + KO8 */
    double ko_sigma;                 /* sigma of the Kreiss-Oliger term (scheme 2) */
    /* per point, [nth][nr], radial index fastest */
    const real *lam1, *lam2;         /* speeds of the Phi rows and the pi rows */
    const real *m3r, *m3i;           /* m3 = m31 - i m32 */
    const real *btr, *bti;           /* B~t */
    const real *cr, *ci;             /* C~ */
    const real *ath, *bth;           /* A~thth, B~th */
    int theta_order;                 /* 4: fourth-order theta differences; else second */
} oracle_teuk;

/* Copy row k of a plane into p[0 .. nr+7] with four end-point copies per side
 * (WENO5 reads three of them, KO8 four). */
static void pad_row(const real* plane, long nr, long k, real* p)
{
    const real* row = plane + k * nr;
    for (long g = 0; g < 4; ++g) {
        p[g] = row[0];
        p[nr + 4 + g] = row[nr - 1];
    }
    memcpy(p + 4, row, (size_t)nr * sizeof(real));
}

/* Row k (possibly a ghost row beyond a pole) of a plane at radial index j:
 * rows -1, -2 mirror rows 0, 1 and rows nth, nth + 1 mirror rows nth - 1,
 * nth - 2, each times the parity (-1)^(m+s). */
static real theta_nb(const real* plane, long nr, long nth, long k, long j, real parity)
{
    if (k < 0) return parity * plane[(-1 - k) * nr + j];
    if (k >= nth) return parity * plane[(2 * nth - 1 - k) * nr + j];
    return plane[k * nr + j];
}

/* F = -(M d_x u + L u + A u) at every point; u and F are [4][nth][nr]. */
void FN(oracle_teuk_rhs)(const oracle_teuk* P, const real* u, real* F)
{
    const long nr = P->nr, nth = P->nth, N = nr * nth;
    const real *PhR = u, *PhI = u + N, *PiR = u + 2 * N, *PiI = u + 3 * N;
    const real dx = pair(P->dx, P->dx_lo), dth = pair(P->dth, P->dth_lo), par = R(P->parity);
    const int th4 = P->theta_order == 4;
    const real ih1 = R(1) / (R(2) * dth), ih2 = R(1) / (dth * dth);
    const real ih1_4 = R(1) / (R(12) * dth), ih2_4 = R(1) / (R(12) * dth * dth);
    const double eps = P->eps;
    const int wm = P->wmode, sc = P->scheme;
    const real sig = R(P->ko_sigma);
#pragma omp parallel for schedule(static)
    for (long k = 0; k < nth; ++k) {
        real* buf = (real*)malloc((size_t)(4 * (nr + 8)) * sizeof(real));
        real *pPhR = buf + 4, *pPhI = buf + (nr + 8) + 4, *pPiR = buf + 2 * (nr + 8) + 4,
             *pPiI = buf + 3 * (nr + 8) + 4;
        pad_row(PhR, nr, k, pPhR - 4);
        pad_row(PhI, nr, k, pPhI - 4);
        pad_row(PiR, nr, k, pPiR - 4);
        pad_row(PiI, nr, k, pPiI - 4);
        for (long j = 0; j < nr; ++j) {
            const long i = k * nr + j;
            const real l1 = P->lam1[i], l2 = P->lam2[i];
            /* d_x u, each plane upwinded by its row's speed */
            const real dPhR = radial_d(pPhR, j, l1, dx, eps, wm, sc);
            const real dPhI = radial_d(pPhI, j, l1, dx, eps, wm, sc);
            const real dPiR = radial_d(pPiR, j, l2, dx, eps, wm, sc);
            const real dPiI = radial_d(pPiI, j, l2, dx, eps, wm, sc);
            /* theta derivatives of Phi (centred, second or fourth order) */
            const real phRm = theta_nb(PhR, nr, nth, k - 1, j, par);
            const real phRp = theta_nb(PhR, nr, nth, k + 1, j, par);
            const real phIm = theta_nb(PhI, nr, nth, k - 1, j, par);
            const real phIp = theta_nb(PhI, nr, nth, k + 1, j, par);
            const real phR = PhR[i], phI = PhI[i], piR = PiR[i], piI = PiI[i];
            real d1R, d1I, d2R, d2I;
            if (th4) {
                const real phRmm = theta_nb(PhR, nr, nth, k - 2, j, par);
                const real phRpp = theta_nb(PhR, nr, nth, k + 2, j, par);
                const real phImm = theta_nb(PhI, nr, nth, k - 2, j, par);
                const real phIpp = theta_nb(PhI, nr, nth, k + 2, j, par);
                d1R = (-phRpp + R(8) * phRp - R(8) * phRm + phRmm) * ih1_4;
                d1I = (-phIpp + R(8) * phIp - R(8) * phIm + phImm) * ih1_4;
                d2R = (-phRpp + R(16) * phRp - R(30) * phR + R(16) * phRm - phRmm) * ih2_4;
                d2I = (-phIpp + R(16) * phIp - R(30) * phI + R(16) * phIm - phImm) * ih2_4;
            } else {
                d1R = (phRp - phRm) * ih1;
                d1I = (phIp - phIm) * ih1;
                d2R = (phRp - R(2) * phR + phRm) * ih2;
                d2I = (phIp - R(2) * phI + phIm) * ih2;
            }
            /* complex products m3 dPhi, B~t pi, C~ Phi */
            const real mdR = P->m3r[i] * dPhR - P->m3i[i] * dPhI;
            const real mdI = P->m3r[i] * dPhI + P->m3i[i] * dPhR;
            const real bpR = P->btr[i] * piR - P->bti[i] * piI;
            const real bpI = P->btr[i] * piI + P->bti[i] * piR;
            const real cpR = P->cr[i] * phR - P->ci[i] * phI;
            const real cpI = P->cr[i] * phI + P->ci[i] * phR;
            /* rows 1-2: d_t Phi = pi - lam1 d_x Phi */
            F[i] = piR - l1 * dPhR;
            F[N + i] = piI - l1 * dPhI;
            /* rows 3-4: d_t pi = -lam2 d_x pi - m3 d_x Phi + B~t pi + A~thth Phi_thth + B~th Phi_th + C~ Phi */
            F[2 * N + i] = -l2 * dPiR - mdR + bpR + P->ath[i] * d2R + P->bth[i] * d1R + cpR;
            F[3 * N + i] = -l2 * dPiI - mdI + bpI + P->ath[i] * d2I + P->bth[i] * d1I + cpI;
            if (sc == 2) {
                /* Kreiss-Oliger dissipation on every plane (radial only) */
                F[i] -= ko8(pPhR, j, dx, sig);
                F[N + i] -= ko8(pPhI, j, dx, sig);
                F[2 * N + i] -= ko8(pPiR, j, dx, sig);
                F[3 * N + i] -= ko8(pPiI, j, dx, sig);
            }
        }
        free(buf);
    }
}

static void teuk_rhs_cb(const real* u, real* F, void* ctx)
{
    FN(oracle_teuk_rhs)((const oracle_teuk*)ctx, u, F);
}

/* Evolve u in place for nsteps steps of size dt = dt_hi + dt_lo of SSP-RK(3,3)
 * (integrator 0) or SSP-RK(10,4) (integrator 1).  If
 * wave != NULL, (Phi_R, Phi_I) at radial index j_e is recorded for every theta
 * row at the initial state and after every `every`-th step, as
 * wave[n][nth][2], up to max_samples samples.  Returns the number of samples
 * written. */
long FN(oracle_teuk_evolve_rk)(const oracle_teuk* P, real* u, double dt, double dt_lo, long nsteps,
                               long j_e, long every, real* wave, long max_samples, int integrator)
{
    const long N = P->nr * P->nth, n = 4 * N;
    const real h = pair(dt, dt_lo);
    real* work = (real*)malloc((size_t)(5 * n) * sizeof(real));
    long ns = 0;
    for (long s = 0; s <= nsteps; ++s) {
        if (s > 0) {
            if (integrator == 1) ssprk104_step(u, n, h, teuk_rhs_cb, (void*)P, work);
            else ssprk3_step(u, n, h, teuk_rhs_cb, (void*)P, work);
        }
        if (wave && every > 0 && s % every == 0 && ns < max_samples) {
            for (long k = 0; k < P->nth; ++k) {
                wave[(ns * P->nth + k) * 2 + 0] = u[k * P->nr + j_e];
                wave[(ns * P->nth + k) * 2 + 1] = u[N + k * P->nr + j_e];
            }
            ++ns;
        }
    }
    free(work);
    return ns;
}

/* SSP-RK(3,3) (integrator 0) as above. */
long FN(oracle_teuk_evolve)(const oracle_teuk* P, real* u, double dt, double dt_lo, long nsteps,
                            long j_e, long every, real* wave, long max_samples)
{
    return FN(oracle_teuk_evolve_rk)(P, u, dt, dt_lo, nsteps, j_e, every, wave, max_samples, 0);
}

/* u' = lam u, u(0) = 1: nsteps SSP-RK3 steps of size dt; returns u as a
 * (hi, lo) pair (tests of the integrator's order at this precision). */
static void ode_rhs(const real* u, real* F, void* ctx)
{
    F[0] = *(const real*)ctx * u[0];
}

void FN(oracle_ode_rk3)(double lam, double dt, double dt_lo, long nsteps, double out[2])
{
    real l = R(lam), u = R(1), work[3];
    const real h = pair(dt, dt_lo);
    for (long s = 0; s < nsteps; ++s) ssprk3_step(&u, 1, h, ode_rhs, &l, work);
    out[0] = (double)u;
    out[1] = (double)(u - R(out[0]));
}

#ifdef ORACLE_QUAD
/* Conversions between (hi, lo) pairs of doubles and binary128 values. */
void oracle_q_from_pairs(const double* p, real* q, long n)
{
    for (long i = 0; i < n; ++i) q[i] = pair(p[2 * i], p[2 * i + 1]);
}

void oracle_q_to_pairs(const real* q, double* p, long n)
{
    for (long i = 0; i < n; ++i) {
        const double hi = (double)q[i];
        p[2 * i] = hi;
        p[2 * i + 1] = (double)(q[i] - R(hi));
    }
}

/* f^+_{j+1/2} (side > 0, f = f_{j-2..j+2}) or f^-_{j+1/2} (side < 0,
 * f = f_{j-1..j+3}) as a pair. */
void oracle_weno5_flux_pair_q(const real* f, double eps, int side, int wmode, double out[2])
{
    const real v = side > 0 ? flux_plus(f, eps, wmode) : flux_minus(f, eps, wmode);
    oracle_q_to_pairs(&v, out, 1);
}

/* D^+ (side > 0) or D^- (side < 0) at point j of a padded row, as a pair. */
void oracle_dside_pair_q(const real* p, long j, double dx, double dx_lo, double eps, int side, int wmode,
                         double out[2])
{
    const real d = side > 0 ? dplus(p, j, pair(dx, dx_lo), eps, wmode) : dminus(p, j, pair(dx, dx_lo), eps, wmode);
    oracle_q_to_pairs(&d, out, 1);
}
#endif

int FN(oracle_num_threads)(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void FN(oracle_set_threads)(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
