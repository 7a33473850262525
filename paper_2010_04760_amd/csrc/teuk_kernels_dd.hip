// Double-double stage kernel (tortoise chart): the paper's quad-precision
// baseline of Sec. 3.1.3, with every state value carried as an unevaluated sum
// hi + lo of two doubles (106 significant bits) and the WENO weights either in
// double-double or, as in the paper's mixed variant, in double.
//
// Arithmetic (all of it in this file is rounded exactly as written: the
// pragma below turns off multiply-add contraction; fused operations are
// spelled out as fma):
//   - error-free transformations: TwoSum (Knuth), FastTwoSum (Dekker), TwoProd
//     by one FMA;
//   - double-word sum, products and reciprocal after Joldes, Muller and
//     Popescu, "Tight and rigorous error bounds for basic building blocks of
//     double-word arithmetic" (ACM TOMS 2017): AccurateDWPlusDW (relative error
//     <= 3u^2), DWPlusFP (2u^2), DWTimesFP3 (2u^2), DWTimesDW3 (4u^2), u = 2^-53;
//     the reciprocal is the double reciprocal corrected by one Newton step
//     carried to second order in the residual.
// Work layout: one wave per (63-point radial strip, theta row), four rows per
// workgroup.  Lane l of a strip owns point j = 63 strip + l and computes the
// four interface fluxes at j - 1/2; the flux at j + 1/2 comes from lane l + 1.
// Values are (hi, lo) pairs stored as double2, [4][ntheta][nr], radial index
// fastest.  The kernel is bound by FP64 VALU issue: a double-double operation
// costs 3-20 FP64 instructions.
#include <hip/hip_runtime.h>

#include "teuk_dd_tables.h"
#include "teuk_internal.h"

#pragma clang fp contract(off)

namespace teuk {

namespace {

struct dd {
    double hi, lo;
};

__device__ __forceinline__ dd two_sum(double a, double b)
{
    const double s = a + b;
    const double bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}

// |a| >= |b| (or a = 0)
__device__ __forceinline__ dd fast_two_sum(double a, double b)
{
    const double s = a + b;
    return {s, b - (s - a)};
}

__device__ __forceinline__ dd two_prod(double a, double b)
{
    const double p = a * b;
    return {p, fma(a, b, -p)};
}

__device__ __forceinline__ dd dd_add(dd x, dd y)
{
    const dd s = two_sum(x.hi, y.hi);
    const dd t = two_sum(x.lo, y.lo);
    const dd v = fast_two_sum(s.hi, s.lo + t.hi);
    return fast_two_sum(v.hi, t.lo + v.lo);
}

__device__ __forceinline__ dd dd_neg(dd x) { return {-x.hi, -x.lo}; }
__device__ __forceinline__ dd dd_sub(dd x, dd y) { return dd_add(x, dd_neg(y)); }
// exact scaling by a power of two
__device__ __forceinline__ dd dd_scale(dd x, double p2) { return {x.hi * p2, x.lo * p2}; }

__device__ __forceinline__ dd dd_add_d(dd x, double y)
{
    const dd s = two_sum(x.hi, y);
    return fast_two_sum(s.hi, x.lo + s.lo);
}

__device__ __forceinline__ dd dd_mul_d(dd x, double y)
{
    const dd c = two_prod(x.hi, y);
    return fast_two_sum(c.hi, fma(x.lo, y, c.lo));
}

__device__ __forceinline__ dd dd_mul(dd x, dd y)
{
    const dd c = two_prod(x.hi, y.hi);
    const double tl1 = fma(x.hi, y.lo, x.lo * y.lo);
    const double cl2 = fma(x.lo, y.hi, tl1);
    return fast_two_sum(c.hi, c.lo + cl2);
}

// 1/y: t = fl(1/y.hi), e = 1 - y t (exact up to 2u^2), 1/y = t (1 + e + e^2 + ...)
__device__ __forceinline__ dd dd_recip(dd y)
{
    const double t = 1.0 / y.hi;
    const dd p = dd_mul_d(y, t);
    const double e = (1.0 - p.hi) - p.lo;
    return fast_two_sum(t, t * fma(e, e, e));
}

__device__ __forceinline__ double sqd(double v) { return v * v; }

__device__ __forceinline__ dd ld(const double2* p, long long i)
{
    const double2 v = p[i];
    return {v.x, v.y};
}

__device__ __forceinline__ void st(double2* p, long long i, dd v) { p[i] = make_double2(v.hi, v.lo); }

__device__ __forceinline__ dd shfl_down1(dd v)
{
    return {__shfl_down(v.hi, 1, 64), __shfl_down(v.lo, 1, 64)};
}

struct DDK {
    dd inv_dx, ih1, ih2, ca, cb, sixth, c13_3, d[3];
};

// Mixed weights (Sec. 3.1.3): the stencil rounded to double, IS_k, alpha_k,
// omega_0 and omega_1 in double exactly as printed (f^+_{j+1/2} from
// g = f_{j-2..j+2}).
__device__ __forceinline__ void w64_plus(const double g[5], double eps, double& w0, double& w1)
{
    const double IS0 = 13.0 / 12.0 * sqd(g[0] - 2.0 * g[1] + g[2]) + 0.25 * sqd(g[0] - 4.0 * g[1] + 3.0 * g[2]);
    const double IS1 = 13.0 / 12.0 * sqd(g[1] - 2.0 * g[2] + g[3]) + 0.25 * sqd(g[1] - g[3]);
    const double IS2 = 13.0 / 12.0 * sqd(g[2] - 2.0 * g[3] + g[4]) + 0.25 * sqd(3.0 * g[2] - 4.0 * g[3] + g[4]);
    const double a0 = (1.0 / 10.0) * sqd(1.0 / (eps + IS0));
    const double a1 = (6.0 / 10.0) * sqd(1.0 / (eps + IS1));
    const double a2 = (3.0 / 10.0) * sqd(1.0 / (eps + IS2));
    const double sum = a0 + a1 + a2;
    w0 = a0 / sum;
    w1 = a1 / sum;
}

// The same for f^-_{j+1/2} from g = f_{j-1..j+3} (omega_0 pairs with the
// right-most stencil g_2..g_4).
__device__ __forceinline__ void w64_minus(const double g[5], double eps, double& w0, double& w1)
{
    const double IS0 = 13.0 / 12.0 * sqd(g[2] - 2.0 * g[3] + g[4]) + 0.25 * sqd(3.0 * g[2] - 4.0 * g[3] + g[4]);
    const double IS1 = 13.0 / 12.0 * sqd(g[1] - 2.0 * g[2] + g[3]) + 0.25 * sqd(g[1] - g[3]);
    const double IS2 = 13.0 / 12.0 * sqd(g[0] - 2.0 * g[1] + g[2]) + 0.25 * sqd(g[0] - 4.0 * g[1] + 3.0 * g[2]);
    const double a0 = (1.0 / 10.0) * sqd(1.0 / (eps + IS0));
    const double a1 = (6.0 / 10.0) * sqd(1.0 / (eps + IS1));
    const double a2 = (3.0 / 10.0) * sqd(1.0 / (eps + IS2));
    const double sum = a0 + a1 + a2;
    w0 = a0 / sum;
    w1 = a1 / sum;
}

// f^+_{j+1/2} from f = f_{j-2..j+2} (the f^- flux is this on the mirrored
// stencil).  With first differences g_i = f_{i+1} - f_i the candidates are
//     6 (q_0 - f_2) = 5 g_1 - 2 g_0,  6 (q_1 - f_2) = g_1 + 2 g_2,  6 (q_2 - f_2) = 4 g_2 - g_3,
// and the smoothness indicators 4 IS_k = (13/3) d_k^2 + e_k^2 with
//     d_0 = g_1 - g_0, d_1 = g_2 - g_1, d_2 = g_3 - g_2,
//     e_0 = 3 g_1 - g_0, e_1 = -(g_1 + g_2), e_2 = g_3 - 3 g_2
// (identities of the printed formulas).  WM = 1: omega_0, omega_1 given in
// double, omega_2 = 1 - omega_0 - omega_1 in double-double.
template <int WM>
__device__ __forceinline__ dd weno(dd f0, dd f1, dd f2, dd f3, dd f4, const DDK& K, double eps, double w0d,
                                   double w1d)
{
    const dd g0 = dd_sub(f1, f0), g1 = dd_sub(f2, f1);
    const dd g2 = dd_sub(f3, f2), g3 = dd_sub(f4, f3);
    const dd A = dd_sub(dd_mul_d(g1, 5.0), dd_scale(g0, 2.0));
    const dd B = dd_add(g1, dd_scale(g2, 2.0));
    const dd C = dd_sub(dd_scale(g2, 4.0), g3);
    dd s6;
    if constexpr (WM == 1) {
        // 6 (f - f_2) = C + omega_0 (A - C) + omega_1 (B - C)
        s6 = dd_add(C, dd_add(dd_mul_d(dd_sub(A, C), w0d), dd_mul_d(dd_sub(B, C), w1d)));
    } else {
        const dd d0 = dd_sub(g1, g0), d1 = dd_sub(g2, g1), d2 = dd_sub(g3, g2);
        const dd e0 = dd_sub(dd_mul_d(g1, 3.0), g0);
        const dd e1 = dd_add(g1, g2);
        const dd e2 = dd_sub(g3, dd_mul_d(g2, 3.0));
        // IS_k = ((13/3) d^2 + e^2) / 4; alpha_k = d_k / (eps + IS_k)^2
        const dd is0 = dd_scale(dd_add(dd_mul(K.c13_3, dd_mul(d0, d0)), dd_mul(e0, e0)), 0.25);
        const dd is1 = dd_scale(dd_add(dd_mul(K.c13_3, dd_mul(d1, d1)), dd_mul(e1, e1)), 0.25);
        const dd is2 = dd_scale(dd_add(dd_mul(K.c13_3, dd_mul(d2, d2)), dd_mul(e2, e2)), 0.25);
        const dd r0 = dd_recip(dd_add_d(is0, eps)), r1 = dd_recip(dd_add_d(is1, eps)), r2 = dd_recip(dd_add_d(is2, eps));
        const dd a0 = dd_mul(K.d[0], dd_mul(r0, r0));
        const dd a1 = dd_mul(K.d[1], dd_mul(r1, r1));
        const dd a2 = dd_mul(K.d[2], dd_mul(r2, r2));
        const dd inv = dd_recip(dd_add(dd_add(a0, a1), a2));
        s6 = dd_add(dd_add(dd_mul(dd_mul(a0, inv), A), dd_mul(dd_mul(a1, inv), B)), dd_mul(dd_mul(a2, inv), C));
    }
    return dd_add(f2, dd_mul(s6, K.sixth));
}

template <int WM>
__global__ __launch_bounds__(256) void dd_stage_kernel(DDStageArgs a, int stage)
{
    const int lane = threadIdx.x & 63;
    const int k = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (k >= a.nth) return;                       // whole wave
    const int nr = a.nr;
    const int j = blockIdx.x * kStripPoints + lane;
    const long long plane = a.plane;
    const long long row = (long long)k * nr;
    DDK K;
    K.inv_dx = {a.inv_dx[0], a.inv_dx[1]};
    K.ih1 = {a.ih1[0], a.ih1[1]};
    K.ih2 = {a.ih2[0], a.ih2[1]};
    K.ca = {a.ca[0], a.ca[1]};
    K.cb = {a.cb[0], a.cb[1]};
    K.sixth = {a.sixth[0], a.sixth[1]};
    K.c13_3 = {a.c13_3[0], a.c13_3[1]};
    for (int q = 0; q < 3; ++q) K.d[q] = {a.d[q][0], a.d[q][1]};

    // radial derivatives: Phi rows f^+ (speed b > 0), pi rows f^- (speed -b)
    dd D[4], own[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const double2* P = (const double2*)a.uk + p * plane + row;
        dd w[6];
#pragma unroll
        for (int t = 0; t < 6; ++t) {
            int jj = j - 3 + t;
            jj = jj < 0 ? 0 : (jj > nr - 1 ? nr - 1 : jj);
            w[t] = ld(P, jj);
        }
        own[p] = w[3];
        dd flux;
        double w0 = 0.0, w1 = 0.0;
        if (p < 2) {
            // f^+_{j-1/2} from f_{j-3..j+1}
            if constexpr (WM == 1) {
                const double g[5] = {w[0].hi, w[1].hi, w[2].hi, w[3].hi, w[4].hi};
                w64_plus(g, a.eps, w0, w1);
            }
            flux = weno<WM>(w[0], w[1], w[2], w[3], w[4], K, a.eps, w0, w1);
        } else {
            // f^-_{j-1/2} from f_{j-2..j+2}: the f^+ form on the mirrored stencil
            if constexpr (WM == 1) {
                const double g[5] = {w[1].hi, w[2].hi, w[3].hi, w[4].hi, w[5].hi};
                w64_minus(g, a.eps, w0, w1);
            }
            flux = weno<WM>(w[5], w[4], w[3], w[2], w[1], K, a.eps, w0, w1);
        }
        const dd right = shfl_down1(flux);
        D[p] = dd_mul(dd_sub(right, flux), K.inv_dx);
    }
    if (lane == 63 || j >= nr) return;

    const long long i = row + j;
    // theta differences of Phi_R, Phi_I with the pole ghosts
    dd d1[2], d2[2];
    for (int p = 0; p < 2; ++p) {
        const double2* P = (const double2*)a.uk + p * plane;
        const dd c = own[p];
        const dd m = k > 0 ? ld(P, i - nr) : (a.parity < 0 ? dd_neg(c) : c);
        const dd pp = k < a.nth - 1 ? ld(P, i + nr) : (a.parity < 0 ? dd_neg(c) : c);
        d1[p] = dd_mul(dd_sub(pp, m), K.ih1);
        d2[p] = dd_mul(dd_add(dd_sub(pp, dd_scale(c, 2.0)), m), K.ih2);
    }
    const dd b = ld((const double2*)a.ctab + kDB * plane, i);
    const dd m3r = ld((const double2*)a.ctab + kDM3r * plane, i), m3i = ld((const double2*)a.ctab + kDM3i * plane, i);
    const dd btr = ld((const double2*)a.ctab + kDBtr * plane, i), bti = ld((const double2*)a.ctab + kDBti * plane, i);
    const dd cr = ld((const double2*)a.ctab + kDCr * plane, i), ci = ld((const double2*)a.ctab + kDCi * plane, i);
    const dd ath = ld((const double2*)a.ctab + kDAth * plane, i), bth = ld((const double2*)a.ctab + kDBth * plane, i);

    const dd phR = own[0], phI = own[1], piR = own[2], piI = own[3];
    const dd mdR = dd_sub(dd_mul(m3r, D[0]), dd_mul(m3i, D[1]));
    const dd mdI = dd_add(dd_mul(m3r, D[1]), dd_mul(m3i, D[0]));
    const dd bpR = dd_sub(dd_mul(btr, piR), dd_mul(bti, piI));
    const dd bpI = dd_add(dd_mul(btr, piI), dd_mul(bti, piR));
    const dd cpR = dd_sub(dd_mul(cr, phR), dd_mul(ci, phI));
    const dd cpI = dd_add(dd_mul(cr, phI), dd_mul(ci, phR));
    dd F[4];
    F[0] = dd_sub(piR, dd_mul(b, D[0]));
    F[1] = dd_sub(piI, dd_mul(b, D[1]));
    // -lam2 d_x pi = b d_x pi in the tortoise chart
    F[2] = dd_add(dd_add(dd_add(dd_sub(dd_mul(b, D[2]), mdR), bpR), dd_add(dd_mul(ath, d2[0]), dd_mul(bth, d1[0]))), cpR);
    F[3] = dd_add(dd_add(dd_add(dd_sub(dd_mul(b, D[3]), mdI), bpI), dd_add(dd_mul(ath, d2[1]), dd_mul(bth, d1[1]))), cpI);

    for (int p = 0; p < 4; ++p) {
        dd v;
        if (stage == 0) {
            v = F[p];
        } else {
            v = dd_add(own[p], dd_mul_d(F[p], a.dt));
            if (stage > 1) v = dd_add(dd_mul(K.ca, ld((const double2*)a.un + p * plane, i)), dd_mul(K.cb, v));
        }
        st((double2*)a.out + p * plane, i, v);
    }
}

__global__ void dd_extract_kernel(const double2* u, long long plane, int nr, int nth, int j_e, double2* slot)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nth) return;
    slot[2 * k + 0] = u[(long long)k * nr + j_e];
    slot[2 * k + 1] = u[plane + (long long)k * nr + j_e];
}

// (hi, lo) -> TwoSum(hi, lo): the normalised pair of the same value.
__global__ void dd_normalise_kernel(double2* u, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double2 v = u[i];
    const dd s = two_sum(v.x, v.y);
    u[i] = make_double2(s.hi, s.lo);
}

}  // namespace

int launch_dd_stage(const DDStageArgs& a, int stage, int weight_prec, void* stream)
{
    if (a.nr < 1 || a.nth < 1 || a.nstrips < 1) return (int)hipErrorInvalidValue;
    const dim3 grid((unsigned)a.nstrips, (unsigned)((a.nth + 3) / 4));
    if (weight_prec == TEUK_W_FP64)
        hipLaunchKernelGGL(dd_stage_kernel<1>, grid, dim3(256), 0, (hipStream_t)stream, a, stage);
    else
        hipLaunchKernelGGL(dd_stage_kernel<0>, grid, dim3(256), 0, (hipStream_t)stream, a, stage);
    return (int)hipGetLastError();
}

int launch_dd_extract(const double* u, long long plane, int nr, int nth, int j_e, double* slot, void* stream)
{
    if (j_e < 0 || j_e >= nr) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(dd_extract_kernel, dim3((nth + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                       (const double2*)u, plane, nr, nth, j_e, (double2*)slot);
    return (int)hipGetLastError();
}

int launch_dd_normalise(double* u, long long n, void* stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(dd_normalise_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       (double2*)u, n);
    return (int)hipGetLastError();
}

}  // namespace teuk
