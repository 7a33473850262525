/*
 * Oracle: plain, scalar FP64 solver for the first-order Teukolsky system.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline of the benchmark load this library; the product path never does.
 * It is built with -O2 -fno-fast-math -ffp-contract=off so that every
 * operation is rounded exactly as written.
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
 *   - second-order centred differences in theta (Sec. 3.1);
 *   - the right-hand side of eq. evln, -(M d_x u + L u + A u), written with
 *     complex 2x2 blocks;
 *   - SSP-RK(3,3) in the Shu-Osher form of Sec. 3.2.
 * Ghost values: three cells per radial side copied from the end point, and in
 * theta one cell per pole equal to (-1)^(m+s) times the mirrored cell.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static double sq(double v) { return v * v; }

/* ---------------------------------------------------------------- WENO5 (Sec. 3.1.2) */

/* f points at f_{j-2}; f[0..4] = f_{j-2..j+2}.  Weights of f^+_{j+1/2}. */
void oracle_weno5_weights_plus(const double* f, double eps, double w[3])
{
    double IS0 = 13.0 / 12.0 * sq(f[0] - 2.0 * f[1] + f[2]) + 0.25 * sq(f[0] - 4.0 * f[1] + 3.0 * f[2]);
    double IS1 = 13.0 / 12.0 * sq(f[1] - 2.0 * f[2] + f[3]) + 0.25 * sq(f[1] - f[3]);
    double IS2 = 13.0 / 12.0 * sq(f[2] - 2.0 * f[3] + f[4]) + 0.25 * sq(3.0 * f[2] - 4.0 * f[3] + f[4]);
    double a0 = (1.0 / 10.0) * sq(1.0 / (eps + IS0));
    double a1 = (6.0 / 10.0) * sq(1.0 / (eps + IS1));
    double a2 = (3.0 / 10.0) * sq(1.0 / (eps + IS2));
    double sum = a0 + a1 + a2;
    w[0] = a0 / sum;
    w[1] = a1 / sum;
    w[2] = a2 / sum;
}

/* f^+_{j+1/2} from f_{j-2..j+2} with given weights. */
double oracle_weno5_combine_plus(const double* f, const double w[3])
{
    return w[0] * ((2.0 / 6.0) * f[0] - (7.0 / 6.0) * f[1] + (11.0 / 6.0) * f[2])
         + w[1] * (-(1.0 / 6.0) * f[1] + (5.0 / 6.0) * f[2] + (2.0 / 6.0) * f[3])
         + w[2] * ((2.0 / 6.0) * f[2] + (5.0 / 6.0) * f[3] - (1.0 / 6.0) * f[4]);
}

double oracle_weno5_flux_plus(const double* f, double eps)
{
    double w[3];
    oracle_weno5_weights_plus(f, eps, w);
    return oracle_weno5_combine_plus(f, w);
}

/* g points at f_{j-1}; g[0..4] = f_{j-1..j+3}.  Weights of f^-_{j+1/2}. */
void oracle_weno5_weights_minus(const double* g, double eps, double w[3])
{
    double IS0 = 13.0 / 12.0 * sq(g[2] - 2.0 * g[3] + g[4]) + 0.25 * sq(3.0 * g[2] - 4.0 * g[3] + g[4]);
    double IS1 = 13.0 / 12.0 * sq(g[1] - 2.0 * g[2] + g[3]) + 0.25 * sq(g[1] - g[3]);
    double IS2 = 13.0 / 12.0 * sq(g[0] - 2.0 * g[1] + g[2]) + 0.25 * sq(g[0] - 4.0 * g[1] + 3.0 * g[2]);
    double a0 = (1.0 / 10.0) * sq(1.0 / (eps + IS0));
    double a1 = (6.0 / 10.0) * sq(1.0 / (eps + IS1));
    double a2 = (3.0 / 10.0) * sq(1.0 / (eps + IS2));
    double sum = a0 + a1 + a2;
    w[0] = a0 / sum;
    w[1] = a1 / sum;
    w[2] = a2 / sum;
}

double oracle_weno5_combine_minus(const double* g, const double w[3])
{
    return w[2] * (-(1.0 / 6.0) * g[0] + (5.0 / 6.0) * g[1] + (2.0 / 6.0) * g[2])
         + w[1] * ((2.0 / 6.0) * g[1] + (5.0 / 6.0) * g[2] - (1.0 / 6.0) * g[3])
         + w[0] * ((11.0 / 6.0) * g[2] - (7.0 / 6.0) * g[3] + (2.0 / 6.0) * g[4]);
}

double oracle_weno5_flux_minus(const double* g, double eps)
{
    double w[3];
    oracle_weno5_weights_minus(g, eps, w);
    return oracle_weno5_combine_minus(g, w);
}

/* Flux-difference derivatives at point j of a padded row p (p[j] is point j,
 * valid for j-3 .. j+3). */
double oracle_dplus(const double* p, long j, double dx, double eps)
{
    return (oracle_weno5_flux_plus(p + j - 2, eps) - oracle_weno5_flux_plus(p + j - 3, eps)) / dx;
}

double oracle_dminus(const double* p, long j, double dx, double eps)
{
    return (oracle_weno5_flux_minus(p + j - 1, eps) - oracle_weno5_flux_minus(p + j - 2, eps)) / dx;
}

/* Upwinded derivative: speed >= 0 -> f^+ treatment, speed < 0 -> f^-. */
static double upwind_d(const double* p, long j, double speed, double dx, double eps)
{
    return speed < 0.0 ? oracle_dminus(p, j, dx, eps) : oracle_dplus(p, j, dx, eps);
}

/* ---------------------------------------------------------------- SSP-RK(3,3) (Sec. 3.2) */

typedef void (*oracle_rhs_fn)(const double* u, double* F, void* ctx);

/* One step of SSP-RK(3,3):
 *   u1 = u + dt F(u)
 *   u2 = 3/4 u + 1/4 (u1 + dt F(u1))
 *   u  = 1/3 u + 2/3 (u2 + dt F(u2))
 * work holds 3n doubles. */
void oracle_ssprk3_step(double* u, long n, double dt, oracle_rhs_fn rhs, void* ctx, double* work)
{
    double* F = work;
    double* u1 = work + n;
    double* u2 = work + 2 * n;
    rhs(u, F, ctx);
    for (long i = 0; i < n; ++i) u1[i] = u[i] + dt * F[i];
    rhs(u1, F, ctx);
    for (long i = 0; i < n; ++i) u2[i] = (3.0 / 4.0) * u[i] + (1.0 / 4.0) * (u1[i] + dt * F[i]);
    rhs(u2, F, ctx);
    for (long i = 0; i < n; ++i) u[i] = (1.0 / 3.0) * u[i] + (2.0 / 3.0) * (u2[i] + dt * F[i]);
}

/* ---------------------------------------------------------------- 1D advection (tests) */

typedef struct {
    long n;
    double dx, speed, eps;
} oracle_advect;

/* u_t + speed u_x = 0 on a periodic grid: F = -speed * D u. */
static void advect_rhs(const double* u, double* F, void* vctx)
{
    const oracle_advect* A = (const oracle_advect*)vctx;
    long n = A->n;
    double* p = (double*)malloc((size_t)(n + 6) * sizeof(double));
    for (long i = 0; i < n + 6; ++i) p[i] = u[((i - 3) % n + n) % n];
    for (long j = 0; j < n; ++j) F[j] = -A->speed * upwind_d(p + 3, j, A->speed, A->dx, A->eps);
    free(p);
}

void oracle_advect1d(double* u, long n, double dx, double speed, double dt, long nsteps, double eps)
{
    oracle_advect A = {n, dx, speed, eps};
    double* work = (double*)malloc((size_t)(3 * n) * sizeof(double));
    for (long s = 0; s < nsteps; ++s) oracle_ssprk3_step(u, n, dt, advect_rhs, &A, work);
    free(work);
}

/* ---------------------------------------------------------------- Teukolsky system (eq. evln) */

typedef struct {
    long nr, nth;
    double dx, dth, eps;
    double parity;                   /* (-1)^(m+s) for the pole ghosts */
    /* per point, [nth][nr], radial index fastest */
    const double *lam1, *lam2;       /* speeds of the Phi rows and the pi rows */
    const double *m3r, *m3i;         /* m3 = m31 - i m32 */
    const double *btr, *bti;         /* B~t */
    const double *cr, *ci;           /* C~ */
    const double *ath, *bth;         /* A~thth, B~th */
} oracle_teuk;

/* Copy row k of a plane into p[0 .. nr+5] with three end-point copies per side. */
static void pad_row(const double* plane, long nr, long k, double* p)
{
    const double* row = plane + k * nr;
    for (long g = 0; g < 3; ++g) {
        p[g] = row[0];
        p[nr + 3 + g] = row[nr - 1];
    }
    memcpy(p + 3, row, (size_t)nr * sizeof(double));
}

/* theta neighbour of (k, j) in a plane, with the pole ghosts. */
static double theta_nb(const double* plane, long nr, long nth, long k, long j, double parity)
{
    if (k < 0) return parity * plane[0 * nr + j];
    if (k >= nth) return parity * plane[(nth - 1) * nr + j];
    return plane[k * nr + j];
}

/* F = -(M d_x u + L u + A u) at every point; u and F are [4][nth][nr]. */
void oracle_teuk_rhs(const oracle_teuk* P, const double* u, double* F)
{
    const long nr = P->nr, nth = P->nth, N = nr * nth;
    const double *PhR = u, *PhI = u + N, *PiR = u + 2 * N, *PiI = u + 3 * N;
    const double ih1 = 1.0 / (2.0 * P->dth), ih2 = 1.0 / (P->dth * P->dth);
#pragma omp parallel for schedule(static)
    for (long k = 0; k < nth; ++k) {
        double* buf = (double*)malloc((size_t)(4 * (nr + 6)) * sizeof(double));
        double *pPhR = buf + 3, *pPhI = buf + (nr + 6) + 3, *pPiR = buf + 2 * (nr + 6) + 3,
               *pPiI = buf + 3 * (nr + 6) + 3;
        pad_row(PhR, nr, k, pPhR - 3);
        pad_row(PhI, nr, k, pPhI - 3);
        pad_row(PiR, nr, k, pPiR - 3);
        pad_row(PiI, nr, k, pPiI - 3);
        for (long j = 0; j < nr; ++j) {
            const long i = k * nr + j;
            const double l1 = P->lam1[i], l2 = P->lam2[i];
            /* d_x u, each plane upwinded by its row's speed */
            const double dPhR = upwind_d(pPhR, j, l1, P->dx, P->eps);
            const double dPhI = upwind_d(pPhI, j, l1, P->dx, P->eps);
            const double dPiR = upwind_d(pPiR, j, l2, P->dx, P->eps);
            const double dPiI = upwind_d(pPiI, j, l2, P->dx, P->eps);
            /* theta derivatives of Phi (second-order centred) */
            const double phRm = theta_nb(PhR, nr, nth, k - 1, j, P->parity);
            const double phRp = theta_nb(PhR, nr, nth, k + 1, j, P->parity);
            const double phIm = theta_nb(PhI, nr, nth, k - 1, j, P->parity);
            const double phIp = theta_nb(PhI, nr, nth, k + 1, j, P->parity);
            const double phR = PhR[i], phI = PhI[i], piR = PiR[i], piI = PiI[i];
            const double d1R = (phRp - phRm) * ih1, d1I = (phIp - phIm) * ih1;
            const double d2R = (phRp - 2.0 * phR + phRm) * ih2, d2I = (phIp - 2.0 * phI + phIm) * ih2;
            /* complex products m3 dPhi, B~t pi, C~ Phi */
            const double mdR = P->m3r[i] * dPhR - P->m3i[i] * dPhI;
            const double mdI = P->m3r[i] * dPhI + P->m3i[i] * dPhR;
            const double bpR = P->btr[i] * piR - P->bti[i] * piI;
            const double bpI = P->btr[i] * piI + P->bti[i] * piR;
            const double cpR = P->cr[i] * phR - P->ci[i] * phI;
            const double cpI = P->cr[i] * phI + P->ci[i] * phR;
            /* rows 1-2: d_t Phi = pi - lam1 d_x Phi */
            F[i] = piR - l1 * dPhR;
            F[N + i] = piI - l1 * dPhI;
            /* rows 3-4: d_t pi = -lam2 d_x pi - m3 d_x Phi + B~t pi + A~thth Phi_thth + B~th Phi_th + C~ Phi */
            F[2 * N + i] = -l2 * dPiR - mdR + bpR + P->ath[i] * d2R + P->bth[i] * d1R + cpR;
            F[3 * N + i] = -l2 * dPiI - mdI + bpI + P->ath[i] * d2I + P->bth[i] * d1I + cpI;
        }
        free(buf);
    }
}

static void teuk_rhs_cb(const double* u, double* F, void* ctx)
{
    oracle_teuk_rhs((const oracle_teuk*)ctx, u, F);
}

/* Evolve u in place for nsteps SSP-RK3 steps of size dt.  If wave != NULL,
 * (Phi_R, Phi_I) at radial index j_e is recorded for every theta row at the
 * initial state and after every `every`-th step, as wave[n][nth][2], up to
 * max_samples samples.  Returns the number of samples written. */
long oracle_teuk_evolve(const oracle_teuk* P, double* u, double dt, long nsteps,
                        long j_e, long every, double* wave, long max_samples)
{
    const long N = P->nr * P->nth, n = 4 * N;
    double* work = (double*)malloc((size_t)(3 * n) * sizeof(double));
    long ns = 0;
    for (long s = 0; s <= nsteps; ++s) {
        if (s > 0) oracle_ssprk3_step(u, n, dt, teuk_rhs_cb, (void*)P, work);
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

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
