// Device kernels of libteuk for gfx950 (CDNA4, wave64).
//
// Hot path: one fused kernel per SSP-RK(3,3) stage (paper Sec. 3.2) that
// evaluates F(u) = -(M d_x u + L u + A u) of eq. evln and combines it with u^n:
//   - WENO5 interface fluxes per real plane (Sec. 3.1.2): Phi_R, Phi_I with the
//     f^+ treatment (speed +b), pi_R, pi_I with the f^- treatment (speed -b);
//   - flux differences (f_{j+1/2} - f_{j-1/2}) / dx;
//   - second-order centred theta differences of Phi (Sec. 3.1);
//   - complex 2x2 blocks of M, A, L with per-point coefficients rebuilt from
//     radial and polar tables;
//   - u^(k+1) = ca u^n + cb (u^(k) + dt F).
//
// Work decomposition.  A workgroup is one wave of 64 lanes.  It owns a radial
// strip of 63 points and marches over a chunk of theta rows.  Per row the wave
// stages the strip plus a 3/2-cell halo of the four planes in LDS (coalesced
// along the radial index), each lane computes the four fluxes of the interface
// just left of its point, and takes the flux of the interface on its right from
// the next lane, so every interface flux is computed once.  The Phi values of
// the rows above and below the own point stay in registers across the march,
// as do the thirteen radial coefficient factors; the polar factors of a row
// are uniform across the wave.  Tiles are ordered theta-chunk fastest and
// dealt to the eight XCDs in contiguous ranges, so neighbouring chunks (which
// share boundary rows) run on the same L2.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "teuk_coef.h"
#include "teuk_internal.h"

namespace teuk {

namespace {

constexpr int kWave = 64;
constexpr int kRow = kWave + 5;   // staged positions j0-3 .. j0+65

// 1/x to full FP64 precision: hardware estimate refined by two Newton steps.
__device__ __forceinline__ double rcp64(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    return r;
}

// 1/sqrt(x), x > 0, to full FP64 precision: estimate plus two Newton steps.
__device__ __forceinline__ double rsq64(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = y * __builtin_fma(-h * y, y, 1.5);
    y = y * __builtin_fma(-h * y, y, 1.5);
    return y;
}

// Six times the WENO5 flux f^+_{j+1/2} from v0..v4 = f_{j-2..j+2} (Sec. 3.1.2).
// The f^- flux f^-_{j+1/2} is the same function of the mirrored stencil
// (f_{j+3}, f_{j+2}, f_{j+1}, f_j, f_{j-1}).
//
// Weights: alpha_k = d_k / (eps + IS_k)^2, omega_k = alpha_k / sum alpha, taken
// over the common denominator (one reciprocal instead of four divisions);
// omega_2 = 1 - omega_0 - omega_1 in FP64, so the weights sum to one exactly
// in the combination whatever precision they were computed in.
template <int WP>
struct Weno;

template <>
struct Weno<TEUK_W_FP64> {
    __device__ __forceinline__ static double flux6(double v0, double v1, double v2, double v3, double v4,
                                                    double eps)
    {
        const double d0 = v0 - 2.0 * v1 + v2;
        const double d1 = v1 - 2.0 * v2 + v3;
        const double d2 = v2 - 2.0 * v3 + v4;
        const double e0 = v0 - 4.0 * v1 + 3.0 * v2;
        const double e1 = v1 - v3;
        const double e2 = 3.0 * v2 - 4.0 * v3 + v4;
        const double b0 = (13.0 / 12.0) * d0 * d0 + 0.25 * e0 * e0;
        const double b1 = (13.0 / 12.0) * d1 * d1 + 0.25 * e1 * e1;
        const double b2 = (13.0 / 12.0) * d2 * d2 + 0.25 * e2 * e2;
        double t0 = eps + b0, t1 = eps + b1, t2 = eps + b2;
        t0 *= t0;
        t1 *= t1;
        t2 *= t2;
        const double n0 = 0.1 * t1 * t2;
        const double n1 = 0.6 * t0 * t2;
        const double n2 = 0.3 * t0 * t1;
        const double inv = rcp64(n0 + n1 + n2);
        const double w0 = n0 * inv, w1 = n1 * inv;
        const double q0 = 2.0 * v0 - 7.0 * v1 + 11.0 * v2;
        const double q1 = -v1 + 5.0 * v2 + 2.0 * v3;
        const double q2 = 2.0 * v2 + 5.0 * v3 - v4;
        return q2 + w0 * (q0 - q2) + w1 * (q1 - q2);
    }
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

template <int WP, bool kFirstStage>
__global__ __launch_bounds__(kWave) void stage_kernel(StageArgs A)
{
    __shared__ double s[4][kRow];
    const int l = threadIdx.x;

    // XCD-aware tile order: block ids are dealt round-robin to the 8 XCDs, so
    // give XCD x the contiguous tile range [x q + min(x, r), ...).
    const int total = A.nstrips * A.nchunks;
    const int bid = blockIdx.x;
    const int xcd = bid & 7, loc = bid >> 3;
    const int q8 = total >> 3, r8 = total & 7;
    const int tile = xcd * q8 + (xcd < r8 ? xcd : r8) + loc;
    const int strip = tile / A.nchunks;
    const int chunk = tile - strip * A.nchunks;
    const int j0 = strip * kStripPoints;
    const int k0 = chunk * A.rows;
    const int k1 = min(k0 + A.rows, A.nth);

    const int nr = A.nr;
    const int j = j0 + l;
    const bool active = (l < kStripPoints) && (j < nr);
    const int jc = min(j, nr - 1);
    const int pa = clampi(j0 - 3 + l, 0, nr - 1);    // LDS index l
    const int pb = clampi(j0 + 61 + l, 0, nr - 1);   // LDS index 64 + l, l < 5

    double rt[kNRT];
#pragma unroll
    for (int i = 0; i < kNRT; ++i) rt[i] = A.rtab[(size_t)i * nr + jc];

    const long long P = A.plane;
    const double* __restrict__ uk = A.uk;
    const double* un = A.un;
    double* out = A.out;

    // Phi at the own point on the row below the first row of the chunk.
    double prvR, prvI;
    if (k0 > 0) {
        prvR = uk[(size_t)(k0 - 1) * nr + jc];
        prvI = uk[P + (size_t)(k0 - 1) * nr + jc];
    } else {
        prvR = A.parity * uk[jc];
        prvI = A.parity * uk[P + jc];
    }

    for (int k = k0; k < k1; ++k) {
        const size_t row = (size_t)k * nr;
#pragma unroll
        for (int p = 0; p < 4; ++p) s[p][l] = uk[p * P + row + pa];
        if (l < 5) {
#pragma unroll
            for (int p = 0; p < 4; ++p) s[p][kWave + l] = uk[p * P + row + pb];
        }
        double nxtR, nxtI;
        if (k + 1 < A.nth) {
            nxtR = uk[row + nr + jc];
            nxtI = uk[P + row + nr + jc];
        } else {
            nxtR = A.parity * uk[row + jc];
            nxtI = A.parity * uk[P + row + jc];
        }
        __syncthreads();

        const double fR = Weno<WP>::flux6(s[0][l], s[0][l + 1], s[0][l + 2], s[0][l + 3], s[0][l + 4], A.eps);
        const double fI = Weno<WP>::flux6(s[1][l], s[1][l + 1], s[1][l + 2], s[1][l + 3], s[1][l + 4], A.eps);
        const double gR = Weno<WP>::flux6(s[2][l + 5], s[2][l + 4], s[2][l + 3], s[2][l + 2], s[2][l + 1], A.eps);
        const double gI = Weno<WP>::flux6(s[3][l + 5], s[3][l + 4], s[3][l + 3], s[3][l + 2], s[3][l + 1], A.eps);
        const double phR = s[0][l + 3], phI = s[1][l + 3];
        const double piR = s[2][l + 3], piI = s[3][l + 3];
        __syncthreads();

        const double fR1 = __shfl_down(fR, 1);
        const double fI1 = __shfl_down(fI, 1);
        const double gR1 = __shfl_down(gR, 1);
        const double gI1 = __shfl_down(gI, 1);

        if (active) {
            const double dPhR = (fR1 - fR) * A.inv6dx;
            const double dPhI = (fI1 - fI) * A.inv6dx;
            const double dPiR = (gR1 - gR) * A.inv6dx;
            const double dPiI = (gI1 - gI) * A.inv6dx;

            const double sn2 = A.ttab[kSn2 * A.nth + k];
            const double cs = A.ttab[kCs * A.nth + k];
            const double cot = A.ttab[kCot * A.nth + k];
            const double th = A.ttab[kTh * A.nth + k];
            const PointCoef c = point_coef(rt, sn2, cs, cot, th, rsq64(sigma2(rt, sn2)));

            const double d1R = (nxtR - prvR) * A.ih1, d1I = (nxtI - prvI) * A.ih1;
            const double d2R = (nxtR - 2.0 * phR + prvR) * A.ih2;
            const double d2I = (nxtI - 2.0 * phI + prvI) * A.ih2;

            // d_t Phi = pi - b d_x Phi
            const double FphR = piR - c.b * dPhR;
            const double FphI = piI - c.b * dPhI;
            // d_t pi = b d_x pi - m3 d_x Phi + B~t pi + A~thth Phi_thth + B~th Phi_th + C~ Phi
            const double FpiR = c.b * dPiR - (c.m3r * dPhR - c.m3i * dPhI) + (c.btr * piR - c.bti * piI) +
                                c.ath * d2R + c.bth * d1R + (c.cr * phR - c.ci * phI);
            const double FpiI = c.b * dPiI - (c.m3r * dPhI + c.m3i * dPhR) + (c.btr * piI + c.bti * piR) +
                                c.ath * d2I + c.bth * d1I + (c.cr * phI + c.ci * phR);

            const size_t o = row + j;
            if (kFirstStage) {
                out[o] = phR + A.dt * FphR;
                out[P + o] = phI + A.dt * FphI;
                out[2 * P + o] = piR + A.dt * FpiR;
                out[3 * P + o] = piI + A.dt * FpiI;
            } else {
                const double u0 = un[o], u1 = un[P + o], u2 = un[2 * P + o], u3 = un[3 * P + o];
                out[o] = A.ca * u0 + A.cb * (phR + A.dt * FphR);
                out[P + o] = A.ca * u1 + A.cb * (phI + A.dt * FphI);
                out[2 * P + o] = A.ca * u2 + A.cb * (piR + A.dt * FpiR);
                out[3 * P + o] = A.ca * u3 + A.cb * (piI + A.dt * FpiI);
            }
        }
        prvR = phR;
        prvI = phI;
    }
}

// ---------------------------------------------------------------- stability bound
// max over points of b/dx + sqrt(4 A~thth/dtheta^2 + |B~th|/dtheta + |C~|); the
// values are >= 0, so their bit patterns order like unsigned integers and the
// reduction ends in one 64-bit atomic max per workgroup.
__global__ __launch_bounds__(256) void dt_bound_kernel(const double* __restrict__ rtab,
                                                       const double* __restrict__ ttab, int nr, int nth,
                                                       double idx, double idth, unsigned long long* cell)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double val = 0.0;
    if (i < (long long)nr * nth) {
        const int k = (int)(i / nr), j = (int)(i - (long long)k * nr);
        double rt[kNRT];
        for (int t = 0; t < kNRT; ++t) rt[t] = rtab[(size_t)t * nr + j];
        const double sn2 = ttab[kSn2 * nth + k];
        const PointCoef c = point_coef(rt, sn2, ttab[kCs * nth + k], ttab[kCot * nth + k], ttab[kTh * nth + k],
                                       rsq64(sigma2(rt, sn2)));
        val = c.b * idx + sqrt(4.0 * c.ath * idth * idth + fabs(c.bth) * idth + hypot(c.cr, c.ci));
    }
    for (int off = 32; off > 0; off >>= 1) val = fmax(val, __shfl_xor(val, off));
    __shared__ double sm[4];
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = val;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double mx = fmax(fmax(sm[0], sm[1]), fmax(sm[2], sm[3]));
        atomicMax(cell, (unsigned long long)__double_as_longlong(mx));
    }
}

// ---------------------------------------------------------------- non-finite guard
__global__ __launch_bounds__(256) void guard_kernel(const double* __restrict__ u, long long n, int* flag)
{
    bool bad = false;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        bad |= !isfinite(u[i]);
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

// ---------------------------------------------------------------- waveform sample
__global__ __launch_bounds__(256) void extract_kernel(const double* __restrict__ u, long long plane, int nr,
                                                      int nth, int j_e, double* __restrict__ slot)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nth) {
        slot[2 * k] = u[(size_t)k * nr + j_e];
        slot[2 * k + 1] = u[plane + (size_t)k * nr + j_e];
    }
}

// ---------------------------------------------------------------- coefficient dump
__global__ __launch_bounds__(256) void coef_dump_kernel(const double* __restrict__ rtab,
                                                        const double* __restrict__ ttab, int nr, int nth,
                                                        double* __restrict__ out)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long n = (long long)nr * nth;
    if (i >= n) return;
    const int k = (int)(i / nr), j = (int)(i - (long long)k * nr);
    double rt[kNRT];
    for (int t = 0; t < kNRT; ++t) rt[t] = rtab[(size_t)t * nr + j];
    const double sn2 = ttab[kSn2 * nth + k];
    const PointCoef c = point_coef(rt, sn2, ttab[kCs * nth + k], ttab[kCot * nth + k], ttab[kTh * nth + k],
                                   rsq64(sigma2(rt, sn2)));
    out[0 * n + i] = c.b;
    out[1 * n + i] = c.m3r;
    out[2 * n + i] = c.m3i;
    out[3 * n + i] = c.btr;
    out[4 * n + i] = c.bti;
    out[5 * n + i] = c.cr;
    out[6 * n + i] = c.ci;
    out[7 * n + i] = c.ath;
    out[8 * n + i] = c.bth;
}

}  // namespace

int launch_stage(const StageArgs& a, int stage, int weight_prec, void* stream)
{
    const dim3 grid((unsigned)(a.nstrips * a.nchunks)), block(kWave);
    hipStream_t st = (hipStream_t)stream;
    (void)hipGetLastError();   // report only what this launch does
    switch (weight_prec) {
    case TEUK_W_FP64:
        if (stage == 1)
            hipLaunchKernelGGL((stage_kernel<TEUK_W_FP64, true>), grid, block, 0, st, a);
        else
            hipLaunchKernelGGL((stage_kernel<TEUK_W_FP64, false>), grid, block, 0, st, a);
        break;
    default:
        return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

int launch_dt_bound(const double* rtab, const double* ttab, int nr, int nth, double dx, double dth,
                    unsigned long long* cell, void* stream)
{
    (void)hipGetLastError();
    const long long n = (long long)nr * nth;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(dt_bound_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, rtab, ttab, nr, nth,
                       1.0 / dx, 1.0 / dth, cell);
    return (int)hipGetLastError();
}

int launch_guard(const double* u, long long n, int* flag, void* stream)
{
    (void)hipGetLastError();
    long long blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(guard_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, u, n, flag);
    return (int)hipGetLastError();
}

int launch_extract(const double* u, long long plane, int nr, int nth, int j_e, double* wave_slot, void* stream)
{
    (void)hipGetLastError();
    hipLaunchKernelGGL(extract_kernel, dim3((unsigned)((nth + 255) / 256)), dim3(256), 0, (hipStream_t)stream, u,
                       plane, nr, nth, j_e, wave_slot);
    return (int)hipGetLastError();
}

int launch_coef_dump(const double* rtab, const double* ttab, int nr, int nth, double* out, void* stream)
{
    (void)hipGetLastError();
    const long long n = (long long)nr * nth;
    hipLaunchKernelGGL(coef_dump_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       rtab, ttab, nr, nth, out);
    return (int)hipGetLastError();
}

}  // namespace teuk
