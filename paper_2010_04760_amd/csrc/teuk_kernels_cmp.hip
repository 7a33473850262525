// Stage kernel of the comparison schemes of Sec. 3.1 (FP64): third-order WENO
// (two candidate stencils, IS_1 = (f_j - f_{j-1})^2, IS_2 = (f_{j+1} - f_j)^2,
// linear weights 1/3 and 2/3; the f^- flux is the mirror image of f^+ about
// j + 1/2), and the sixth-order centred difference with eighth-order
// Kreiss-Oliger dissipation (every plane's right-hand side receives
// -sigma delta^8 u / (256 dx), the dissipative sign of sigma dx^7 (D+ D-)^4 / 256).
// Everything else -- theta differences with the pole ghosts, the coefficients
// of either chart, the assembly of F and the RK stage combinations -- is as in
// the WENO5 stage kernel.
//
// Work layout: one wave per (63-point radial strip, theta row), four rows per
// workgroup, no march.  Lane l owns point j = 63 strip + l and loads the nine
// radial values j-4 .. j+4 of each plane (ghosts by clamped index: the end
// value); for WENO3 it computes both interface fluxes f^+ and f^- at j - 1/2
// and takes those at j + 1/2 from lane l + 1, then differences the side of
// the row's speed at the point (speed >= 0: f^+).
#include <hip/hip_runtime.h>

#include "teuk_coef.h"
#include "teuk_internal.h"

namespace teuk {

namespace {

constexpr int kModeFirst = 0, kModeLater = 1, kModeRhs = 2, kModeDual = 3;

__device__ __forceinline__ double sq(double v) { return v * v; }

// f^+_{j+1/2} from a = f_{j-1}, b = f_j, c = f_{j+1}
__device__ __forceinline__ double weno3_plus(double a, double b, double c, double eps)
{
    const double a1 = (1.0 / 3.0) * sq(1.0 / (eps + sq(b - a)));
    const double a2 = (2.0 / 3.0) * sq(1.0 / (eps + sq(c - b)));
    return (a1 * (1.5 * b - 0.5 * a) + a2 * (0.5 * b + 0.5 * c)) / (a1 + a2);
}

// f^-_{j+1/2} from b = f_j, c = f_{j+1}, d = f_{j+2}: the mirror image
__device__ __forceinline__ double weno3_minus(double b, double c, double d, double eps)
{
    return weno3_plus(d, c, b, eps);
}

template <int kScheme, int kMode, int kChart>
__global__ __launch_bounds__(256) void cmp_stage_kernel(StageArgs A)
{
    const int lane = threadIdx.x & 63;
    const int k = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (k >= A.nth) return;                       // whole wave
    const int nr = A.nr;
    const int j = blockIdx.x * kStripPoints + lane;
    const long long P = A.plane;
    const long long row = (long long)k * nr;
    const bool own = lane < kStripPoints && j < nr;
    const int jc = j < nr ? j : nr - 1;
    const long long i = row + jc;

    // speeds of the Phi rows and the pi rows at the point
    double lam1, lam2;
    double rt[kNRT];
    double sn2 = 0.0, cs = 0.0, cot = 0.0, th = 0.0;
    if constexpr (kChart == 0) {
#pragma unroll
        for (int q = 0; q < kNRT; ++q) rt[q] = A.rtab[(size_t)q * nr + jc];
        sn2 = A.ttab[kSn2 * A.nth + k];
        cs = A.ttab[kCs * A.nth + k];
        cot = A.ttab[kCot * A.nth + k];
        th = A.ttab[kTh * A.nth + k];
        lam1 = rt[kRa2] / sqrt(sigma2(rt, sn2));
        lam2 = -lam1;
    } else {
        lam1 = A.ctab[kHLam1 * P + i];
        lam2 = A.ctab[kHLam2 * P + i];
    }

    double D[4], KO[4], u0[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const double* U = A.uk + p * P + row;
        double w[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            int jj = j - 4 + t;
            jj = jj < 0 ? 0 : (jj > nr - 1 ? nr - 1 : jj);
            w[t] = U[jj];
        }
        u0[p] = w[4];
        const double speed = p < 2 ? lam1 : lam2;
        if constexpr (kScheme == TEUK_SCHEME_WENO3) {
            // interface j - 1/2
            const double fp = weno3_plus(w[2], w[3], w[4], A.eps);    // f_{j-2}, f_{j-1}, f_j
            const double fm = weno3_minus(w[3], w[4], w[5], A.eps);   // f_{j-1}, f_j, f_{j+1}
            const double fp1 = __shfl_down(fp, 1, 64);
            const double fm1 = __shfl_down(fm, 1, 64);
            D[p] = (speed < 0.0 ? fm1 - fm : fp1 - fp) * A.inv_dx;
            KO[p] = 0.0;
        } else {
            D[p] = (w[7] - 9.0 * w[6] + 45.0 * w[5] - 45.0 * w[3] + 9.0 * w[2] - w[1]) * (A.inv_dx / 60.0);
            const double d8 = w[0] - 8.0 * w[1] + 28.0 * w[2] - 56.0 * w[3] + 70.0 * w[4] - 56.0 * w[5] +
                              28.0 * w[6] - 8.0 * w[7] + w[8];
            KO[p] = A.ko_sigma * d8 * (A.inv_dx / 256.0);
        }
    }
    if (!own) return;

    // theta differences of Phi with the pole ghosts
    double d1[2], d2[2];
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const double* U = A.uk + p * P;
        const double c = u0[p];
        const double m = k > 0 ? U[i - nr] : A.parity * c;
        const double pp = k < A.nth - 1 ? U[i + nr] : A.parity * c;
        d1[p] = (pp - m) * A.ih1;
        d2[p] = (pp - 2.0 * c + m) * A.ih2;
    }
    double m3r, m3i, btr, bti, cr, ci, ath, bth;
    if constexpr (kChart == 0) {
        const PointCoef c = point_coef(rt, sn2, cs, cot, th, 1.0 / sqrt(sigma2(rt, sn2)));
        m3r = c.m3r; m3i = c.m3i; btr = c.btr; bti = c.bti; cr = c.cr; ci = c.ci; ath = c.ath; bth = c.bth;
    } else {
        m3r = A.ctab[kHM3r * P + i]; m3i = A.ctab[kHM3i * P + i];
        btr = A.ctab[kHBtr * P + i]; bti = A.ctab[kHBti * P + i];
        cr = A.ctab[kHCr * P + i]; ci = A.ctab[kHCi * P + i];
        ath = A.ctab[kHAth * P + i]; bth = A.ctab[kHBth * P + i];
    }
    const double phR = u0[0], phI = u0[1], piR = u0[2], piI = u0[3];
    double F[4];
    F[0] = piR - lam1 * D[0];
    F[1] = piI - lam1 * D[1];
    F[2] = -lam2 * D[2] - (m3r * D[0] - m3i * D[1]) + (btr * piR - bti * piI) + ath * d2[0] + bth * d1[0] +
           (cr * phR - ci * phI);
    F[3] = -lam2 * D[3] - (m3r * D[1] + m3i * D[0]) + (btr * piI + bti * piR) + ath * d2[1] + bth * d1[1] +
           (cr * phI + ci * phR);
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        F[p] -= KO[p];
        const double v = u0[p] + A.dt * F[p];
        double out;
        if (kMode == kModeRhs) out = F[p];
        else if (kMode == kModeFirst) out = v;
        else out = A.ca * A.un[p * P + i] + A.cb * v;
        if (kMode == kModeDual) A.out2[p * P + i] = A.ca2 * A.un[p * P + i] + A.cb2 * v;
        A.out[p * P + i] = out;
    }
}

}  // namespace

int launch_cmp_stage(const StageArgs& a, int stage, int scheme, int chart, void* stream)
{
    if (a.nr < 1 || a.nth < 1 || a.nstrips < 1) return (int)hipErrorInvalidValue;
    const dim3 grid((unsigned)a.nstrips, (unsigned)((a.nth + 3) / 4)), block(256);
    hipStream_t st = (hipStream_t)stream;
    (void)hipGetLastError();
    const int mode = stage == 0 ? kModeRhs : stage == 1 ? kModeFirst : stage == 4 ? kModeDual : kModeLater;
    bool done = false;
#define TEUK_CMP(S, M, C)                                                                 \
    if (scheme == S && mode == M && chart == C) {                                          \
        hipLaunchKernelGGL((cmp_stage_kernel<S, M, C>), grid, block, 0, st, a);            \
        done = true;                                                                       \
    }
#define TEUK_CMP_MODES(S, C) TEUK_CMP(S, kModeFirst, C) TEUK_CMP(S, kModeLater, C) TEUK_CMP(S, kModeRhs, C) TEUK_CMP(S, kModeDual, C)
    TEUK_CMP_MODES(TEUK_SCHEME_WENO3, 0)
    TEUK_CMP_MODES(TEUK_SCHEME_WENO3, 1)
    TEUK_CMP_MODES(TEUK_SCHEME_FD6KO8, 0)
    TEUK_CMP_MODES(TEUK_SCHEME_FD6KO8, 1)
#undef TEUK_CMP_MODES
#undef TEUK_CMP
    if (!done) return (int)hipErrorInvalidValue;
    return (int)hipGetLastError();
}

}  // namespace teuk
