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

// What a stage launch writes.
constexpr int kStageFirst = 0;    // out = u + dt F(u)
constexpr int kStageLater = 1;    // out = ca u^n + cb (u^(k) + dt F(u^(k)))
constexpr int kRhsOnly = 2;       // out = F(u)
constexpr int kStageDual = 3;     // v = u^(k) + dt F(u^(k)): out = ca u^n + cb v, out2 = ca2 u^n + cb2 v
// stage modes that read u^n at the own point
template <int kMode>
constexpr bool reads_un() { return kMode == kStageLater || kMode == kStageDual; }

// Radial chart (TEUK_CHART_*).
constexpr int kChartT = TEUK_CHART_TORTOISE;
constexpr int kChartH = TEUK_CHART_HYPERBOLOIDAL;
// The tortoise chart with fourth-order theta differences (a launch class of
// its own; the ABI's chart field stays TEUK_CHART_TORTOISE).
constexpr int kChartT4 = kChartTortoise4;

// 1/x from the hardware estimate refined by one Newton step.
__device__ __forceinline__ double rcp64(double x)
{
    const double r = __builtin_amdgcn_rcp(x);
    const double e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
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
// Arithmetic, rearranged by exact identities (only rounding differs from the
// printed formulas):
//  * with the second differences d_k and first differences e_k of IS_k,
//    4 IS_k = (13/3) d_k^2 + e_k^2; eps is scaled by 4 as well, so every
//    t_k = (eps + IS_k)^2 carries the same factor 16, which cancels in omega;
//  * omega_k = alpha_k / sum alpha with alpha_k = d_k / t_k is taken over the
//    common denominator, constants scaled by 10:
//        omega_0 = t1 t2 / D,  omega_1 = 6 t0 t2 / D,  D = t1 t2 + 6 t0 t2 + 3 t0 t1,
//    one reciprocal instead of four divisions;
//  * omega_2 = 1 - omega_0 - omega_1, i.e. the flux is
//        6 f = q2 + omega_0 (q0 - q2) + omega_1 (q1 - q2),
//    so the weights sum to one exactly in the combination;
//  * the candidates (times 6) reuse the differences:
//        q2 = 3 (v2 + v3) - d2,  q1 - q2 = d2 - d1,  q0 = 2 d0 + 9 v2 - 3 v1.
template <int WP>
struct Weno;

// Candidate part shared by every weight precision: 6 f from omega_0, omega_1.
struct Candidates {
    double q2, dq0, dq1;
    __device__ __forceinline__ Candidates(double v0, double v1, double v2, double v3, double d0, double d1,
                                          double d2)
    {
        (void)v0;
        q2 = 3.0 * (v2 + v3) - d2;
        dq1 = d2 - d1;
        dq0 = (2.0 * d0 + (9.0 * v2 - 3.0 * v1)) - q2;
    }
};

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
        constexpr double c = 13.0 / 3.0;
        const double eps4 = 4.0 * eps;
        double t0 = __builtin_fma(c * d0, d0, __builtin_fma(e0, e0, eps4));
        double t1 = __builtin_fma(c * d1, d1, __builtin_fma(e1, e1, eps4));
        double t2 = __builtin_fma(c * d2, d2, __builtin_fma(e2, e2, eps4));
        t0 *= t0;
        t1 *= t1;
        t2 *= t2;
        const double p12 = t1 * t2, p02 = t0 * t2, p01 = t0 * t1;
        const double inv = rcp64(p12 + (6.0 * p02 + 3.0 * p01));
        const Candidates q(v0, v1, v2, v3, d0, d1, d2);
        return q.q2 + inv * (p12 * q.dq0 + (6.0 * p02) * q.dq1);
    }
};

// ---------------------------------------------------------------- reduced-precision weights
// Sec. 3.1.3: the smoothness indicators and nonlinear weights are computed in a
// lower precision and the weights are made to sum to one in FP64.  Here the six
// stencil differences of IS_k are taken in FP64 (differencing first keeps the
// information the low format would lose to cancellation), converted, and
// IS_k, alpha_k and omega_0, omega_1 are formed in the low format; omega_2 is
// the FP64 complement and the candidate fluxes stay FP64.
//
// The 16-bit weights use the ratio form
//     alpha'_k = d_k (tau_min / tau_k)^2,   tau_k = eps + IS_k,
// which equals alpha_k tau_min^2 (so omega is unchanged in exact arithmetic)
// and keeps every intermediate in [0, 1] whatever the magnitude of the data.
// rho_k = 1 where tau_k equals tau_min (also when both are zero).  FP32 has
// the range for the FP64 form and takes it (Weno<TEUK_W_FP32> below).

// Arithmetic in the low format: every result rounded to it.  ratio(a, b) is
// a / b for 0 <= a < b, a true division: after the power-of-two scaling eps
// can underflow to zero, so a flat stencil gives tau_min = 0 next to a tau_k
// below 2^-16 whose reciprocal overflows, and 0 * inf would poison the weights.
struct LowF16 {
    typedef _Float16 T;
    __device__ static T cvt(float x) { return (_Float16)x; }
    __device__ static T rcp(T x) { return (_Float16)1.0 / x; }
    __device__ static T ratio(T a, T b) { return a / b; }
    __device__ static float f(T x) { return (float)x; }
};
// BF16 arithmetic: compute in FP32 and round each result to BF16 (round to
// nearest even).  FP32 carries more than 2p+2 bits for p = 8, so this equals a
// correctly rounded BF16 operation for +, -, * and /.
struct Bf16Val {
    float v;
};
__device__ __forceinline__ float bf16_round(float x)
{
    return (float)(__bf16)x;
}
__device__ __forceinline__ Bf16Val operator+(Bf16Val a, Bf16Val b) { return {bf16_round(a.v + b.v)}; }
__device__ __forceinline__ Bf16Val operator*(Bf16Val a, Bf16Val b) { return {bf16_round(a.v * b.v)}; }
__device__ __forceinline__ bool operator<(Bf16Val a, Bf16Val b) { return a.v < b.v; }
__device__ __forceinline__ bool operator==(Bf16Val a, Bf16Val b) { return a.v == b.v; }
struct LowBF16 {
    typedef Bf16Val T;
    __device__ static T cvt(float x) { return {bf16_round(x)}; }
    __device__ static T rcp(T x) { return {bf16_round(1.0f / x.v)}; }
    __device__ static T ratio(T a, T b) { return {bf16_round(a.v / b.v)}; }
    __device__ static float f(T x) { return x.v; }
};

template <class L, bool kScale>
__device__ __forceinline__ void low_weights(double d0, double d1, double d2, double e0, double e1, double e2,
                                            double eps, double* w0, double* w1)
{
    typedef typename L::T T;
    float fd0 = (float)d0, fd1 = (float)d1, fd2 = (float)d2;
    float fe0 = (float)e0, fe1 = (float)e1, fe2 = (float)e2;
    float feps = (float)eps;
    if (kScale) {
        // Scale by an exact power of two so that the largest of the differences
        // and sqrt(eps) is O(1): IS' = sigma^2 IS and eps' = sigma^2 eps leave the
        // weights unchanged and keep a 16-bit format away from overflow.
        float m = fmaxf(fmaxf(fmaxf(fabsf(fd0), fabsf(fd1)), fmaxf(fabsf(fd2), fabsf(fe0))),
                        fmaxf(fmaxf(fabsf(fe1), fabsf(fe2)), sqrtf(feps)));
        const int ex = __builtin_amdgcn_frexp_expf(m);
        fd0 = ldexpf(fd0, -ex); fd1 = ldexpf(fd1, -ex); fd2 = ldexpf(fd2, -ex);
        fe0 = ldexpf(fe0, -ex); fe1 = ldexpf(fe1, -ex); fe2 = ldexpf(fe2, -ex);
        feps = ldexpf(feps, -2 * ex);
    }
    const T c1312 = L::cvt(13.0f / 12.0f), c14 = L::cvt(0.25f);
    const T D0 = L::cvt(fd0), D1 = L::cvt(fd1), D2 = L::cvt(fd2);
    const T E0 = L::cvt(fe0), E1 = L::cvt(fe1), E2 = L::cvt(fe2);
    const T ep = L::cvt(feps);
    const T t0 = ep + (c1312 * (D0 * D0) + c14 * (E0 * E0));
    const T t1 = ep + (c1312 * (D1 * D1) + c14 * (E1 * E1));
    const T t2 = ep + (c1312 * (D2 * D2) + c14 * (E2 * E2));
    T tm = t0 < t1 ? t0 : t1;
    tm = t2 < tm ? t2 : tm;
    const T one = L::cvt(1.0f);
    const T r0 = t0 == tm ? one : L::ratio(tm, t0);
    const T r1 = t1 == tm ? one : L::ratio(tm, t1);
    const T r2 = t2 == tm ? one : L::ratio(tm, t2);
    const T a0 = L::cvt(0.1f) * (r0 * r0);
    const T a1 = L::cvt(0.6f) * (r1 * r1);
    const T a2 = L::cvt(0.3f) * (r2 * r2);
    const T inv = L::rcp(a0 + a1 + a2);
    *w0 = (double)L::f(a0 * inv);
    *w1 = (double)L::f(a1 * inv);
}

template <class L, bool kScale>
struct WenoLow {
    __device__ __forceinline__ static double flux6(double v0, double v1, double v2, double v3, double v4,
                                                    double eps)
    {
        const double d0 = v0 - 2.0 * v1 + v2;
        const double d1 = v1 - 2.0 * v2 + v3;
        const double d2 = v2 - 2.0 * v3 + v4;
        const double e0 = v0 - 4.0 * v1 + 3.0 * v2;
        const double e1 = v1 - v3;
        const double e2 = 3.0 * v2 - 4.0 * v3 + v4;
        double w0, w1;
        low_weights<L, kScale>(d0, d1, d2, e0, e1, e2, eps, &w0, &w1);
        const Candidates q(v0, v1, v2, v3, d0, d1, d2);
        return q.q2 + (w0 * q.dq0 + w1 * q.dq1);
    }
};

// FP32 weights take the FP64 form above -- common denominator, one
// reciprocal (v_rcp_f32, 1 ulp) -- evaluated in FP32 from the six FP64
// stencil differences, with omega_2 the FP64 complement.  FP32 has the range
// for it over most of the data: with t_k = (4 eps + 4 IS_k)^2 the denominator
// is at least 2560 eps^4 and stays finite for differences up to about 1e4.  It
// must also stay well above the subnormals, where the reciprocal overflows to
// inf (and 0 * inf is a NaN) or loses its precision: below 2^-100 -- every
// flat stencil once eps is under about 4e-9 -- and above 3e38 the lane takes
// the FP64 weights instead.  From 2^-100 on, a product that is subnormal or
// flushed to zero moves its weight by at most 2^-26 absolute.
template <>
struct Weno<TEUK_W_FP32> {
    __device__ __forceinline__ static double flux6(double v0, double v1, double v2, double v3, double v4,
                                                    double eps)
    {
        const double d0 = v0 - 2.0 * v1 + v2;
        const double d1 = v1 - 2.0 * v2 + v3;
        const double d2 = v2 - 2.0 * v3 + v4;
        const double e0 = v0 - 4.0 * v1 + 3.0 * v2;
        const double e1 = v1 - v3;
        const double e2 = 3.0 * v2 - 4.0 * v3 + v4;
        const float D0 = (float)d0, D1 = (float)d1, D2 = (float)d2;
        const float E0 = (float)e0, E1 = (float)e1, E2 = (float)e2;
        constexpr float c = 13.0f / 3.0f;
        const float eps4 = (float)(4.0 * eps);
        float t0 = __builtin_fmaf(c * D0, D0, __builtin_fmaf(E0, E0, eps4));
        float t1 = __builtin_fmaf(c * D1, D1, __builtin_fmaf(E1, E1, eps4));
        float t2 = __builtin_fmaf(c * D2, D2, __builtin_fmaf(E2, E2, eps4));
        t0 *= t0;
        t1 *= t1;
        t2 *= t2;
        const float p12 = t1 * t2, p02 = t0 * t2, p01 = t0 * t1;
        const float den = p12 + (6.0f * p02 + 3.0f * p01);
        const Candidates q(v0, v1, v2, v3, d0, d1, d2);
        if (!(den >= 0x1p-100f && den <= 3.0e38f)) return Weno<TEUK_W_FP64>::flux6(v0, v1, v2, v3, v4, eps);
        const float inv = __builtin_amdgcn_rcpf(den);
        const double w0 = (double)(p12 * inv), w1 = (double)((6.0f * p02) * inv);
        return q.q2 + (w0 * q.dq0 + w1 * q.dq1);
    }
};
template <>
struct Weno<TEUK_W_FP16> : WenoLow<LowF16, true> {};
template <>
struct Weno<TEUK_W_BF16> : WenoLow<LowBF16, true> {};

// x of lane l + 1 (lane 63 keeps its own), by a DPP wavefront shift: no LDS
// round trip, unlike __shfl_down.  Used wherever a lane takes the interface
// flux of the lane after it.
__device__ __forceinline__ double next_lane(double x)
{
    int lo = __double2loint(x), hi = __double2hiint(x);
    lo = __builtin_amdgcn_update_dpp(lo, lo, 0x130 /* wave_shl:1 */, 0xF, 0xF, false);
    hi = __builtin_amdgcn_update_dpp(hi, hi, 0x130 /* wave_shl:1 */, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Barrier that orders LDS only.  __syncthreads() is also a workgroup fence on
// global memory, which makes every wave drain its outstanding global loads
// (s_waitcnt vmcnt(0)) before the barrier: that would serialise the row
// prefetch below with the arithmetic it is meant to overlap.
__device__ __forceinline__ void lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Load a double at a byte offset from a uniform base: the 32-bit offset lets
// the compiler use the scalar-base addressing form (no 64-bit address math).
__device__ __forceinline__ double ldb(const double* base, unsigned off)
{
    return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(base) + off);
}
__device__ __forceinline__ void stb(double* base, unsigned off, double v)
{
    *reinterpret_cast<double*>(reinterpret_cast<char*>(base) + off) = v;
}

// ---------------------------------------------------------------- chart-T row pipeline
// The tortoise-chart stage streams each theta row of the four planes straight
// from HBM into a four-row LDS ring with LDS-DMA loads (global_load_lds: every
// lane moves one dword, no VGPRs involved), three rows ahead of the row being
// computed.  The compiler does not model these loads, so they and the u^n
// loads are issued from inline assembly and waited for with explicit vmcnt
// counts.  Each count covers only the loads issued here; any other memory
// operation the compiler places in between can only make a wait stricter.
constexpr int kRowP = 72;                                   // LDS row stride (doubles)
constexpr int kRing = 4;                                    // rows in the LDS ring
constexpr unsigned kPlaneBytes = kRowP * 8;                 // 576
constexpr unsigned kSlotBytes = 4 * kPlaneBytes;            // 2304

// One LDS-DMA dword per lane: LDS[m0 + 4 lane] = global[sbase + voff].  The
// LDS address reaches m0 through an operand constrained to that register, so
// the compiler writes m0 itself and knows the instruction reads it.
__device__ __forceinline__ void dma_dword(unsigned voff, const double* sbase, unsigned lds)
{
    asm volatile("global_load_lds_dword %0, %1" : : "v"(voff), "s"(sbase), "{m0}"(lds) : "memory");
}

// A double from global memory whose arrival is waited for explicitly: the
// register holds the value only after the vm_wait that takes it as an operand.
// Until then no instruction may read, copy or reuse it; the compiler sees the
// value as ready at once, so this is checked in the built assembly (every
// wait names its operands in a comment for that check).
__device__ __forceinline__ double ld_async(unsigned voff, const double* sbase)
{
    double v;
    asm volatile("global_load_dwordx2 %0, %1, %2 ; async-load" : "=&v"(v) : "v"(voff), "s"(sbase) : "memory");
    return v;
}

// Wait until at most N vector-memory operations are outstanding.
template <int N>
__device__ __forceinline__ void vm_wait()
{
    asm volatile("s_waitcnt vmcnt(%0)" : : "n"(N) : "memory");
}
// The same, also making four values depend on the wait (so that no use of
// them can be scheduled before it).
template <int N>
__device__ __forceinline__ void vm_wait(double& a, double& b, double& c, double& d)
{
    asm volatile("s_waitcnt vmcnt(%4) ; async-wait %0 %1 %2 %3" : "+v"(a), "+v"(b), "+v"(c), "+v"(d) : "n"(N) : "memory");
}

// Agent-coherent forms of the row traffic (the sc1 cache policy that the
// compiler gives agent-scope atomics: not served from a non-coherent cache
// line, and stores written through), for the pipelined step, whose workgroups
// on any CU or XCD exchange tiles without cache write-back or invalidation.
// With kCoh false they are the plain forms above.
template <bool kCoh>
__device__ __forceinline__ double ldb_c(const double* base, unsigned off)
{
    if constexpr (kCoh) {
        const unsigned long long* q =
            reinterpret_cast<const unsigned long long*>(reinterpret_cast<const char*>(base) + off);
        return __longlong_as_double((long long)__hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    } else {
        return ldb(base, off);
    }
}
template <bool kCoh>
__device__ __forceinline__ void stb_c(double* base, unsigned off, double v)
{
    if constexpr (kCoh) {
        unsigned long long* q = reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(base) + off);
        __hip_atomic_store(q, (unsigned long long)__double_as_longlong(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        stb(base, off, v);
    }
}
template <bool kCoh>
__device__ __forceinline__ void dma_dword_c(unsigned voff, const double* sbase, unsigned lds)
{
    if constexpr (kCoh)
        asm volatile("global_load_lds_dword %0, %1 sc1" : : "v"(voff), "s"(sbase), "{m0}"(lds) : "memory");
    else
        dma_dword(voff, sbase, lds);
}
template <bool kCoh>
__device__ __forceinline__ double ld_async_c(unsigned voff, const double* sbase)
{
    if constexpr (kCoh) {
        double v;
        asm volatile("global_load_dwordx2 %0, %1, %2 sc1 ; async-load" : "=&v"(v) : "v"(voff), "s"(sbase) : "memory");
        return v;
    } else {
        return ld_async(voff, sbase);
    }
}

// Hyperboloidal chart: one radial strip [j0, j0 + 63) marched over the theta
// rows [k0, k1), upward (dir = +1, from k0) or downward (dir = -1, from
// k1 - 1).  Rows are staged in a two-row LDS ring: while row k is computed
// from LDS, the loads of row k + 2 dir and of u^n at row k are already in
// flight and are consumed at the end of the iteration, so each wave always has
// its next rows' memory traffic overlapping its arithmetic.  The ten
// coefficients of the point are read from the per-point table, and each row
// takes the flux side of the sign of its own speed at the point (speed >= 0:
// f^+, speed < 0: f^-); a wave whose lanes disagree computes both sides and
// each lane differences its own.
template <int WP, int kMode>
__device__ __forceinline__ void march_strip_h(const StageArgs& A, double (*s)[4][kRow], int strip, int k0, int k1,
                                              int dir)
{
    const int l = threadIdx.x;
    const int nr = A.nr, nth = A.nth;
    const long long P = A.plane;
    const int j0 = strip * kStripPoints;
    const int j = j0 + l;
    const bool active = (l < kStripPoints) && (j < nr);
    const int jc = min(j, nr - 1);
    // byte offsets within a row (rows are < 2^27 doubles, so these fit in 32 bits)
    const unsigned oa = (unsigned)clampi(j0 - 3 + l, 0, nr - 1) * 8u;    // LDS index l
    const unsigned ob = (unsigned)clampi(j0 + 61 + l, 0, nr - 1) * 8u;   // LDS index 64 + l, l < 5
    const unsigned oc = (unsigned)jc * 8u;                                 // own point
    const bool halo = l < 5;
    const double* __restrict__ ukp[4] = {A.uk, A.uk + P, A.uk + 2 * P, A.uk + 3 * P};
    const double* unp[4] = {A.un, A.un + P, A.un + 2 * P, A.un + 3 * P};   // read where reads_un<kMode>()
    double* outp[4] = {A.out, A.out + P, A.out + 2 * P, A.out + 3 * P};

    const int n = k1 - k0;
    const int first = dir > 0 ? k0 : k1 - 1;
    // Phi at the own point on the row behind the first one (pole ghost past
    // either pole).
    double bhR, bhI;
    {
        const int kb = first - dir;
        if (kb >= 0 && kb < nth) {
            bhR = ldb(ukp[0] + (size_t)kb * nr, oc);
            bhI = ldb(ukp[1] + (size_t)kb * nr, oc);
        } else {
            bhR = A.parity * ldb(ukp[0] + (size_t)first * nr, oc);
            bhI = A.parity * ldb(ukp[1] + (size_t)first * nr, oc);
        }
    }

    // Rows staged: first + dir i for i = 0 .. nst-1, i.e. every computed row
    // plus the one ahead of the last (its theta neighbour) unless that is past
    // a pole.
    const int ahead_last = first + dir * n;
    const int nst = (ahead_last >= 0 && ahead_last < nth) ? n + 1 : n;
    double xa[4], xb[4];
    auto load_row = [&](int k) {
        const size_t row = (size_t)k * nr;
#pragma unroll
        for (int p = 0; p < 4; ++p) xa[p] = ldb(ukp[p] + row, oa);
        if (halo) {
#pragma unroll
            for (int p = 0; p < 4; ++p) xb[p] = ldb(ukp[p] + row, ob);
        }
    };
    auto store_row = [&](int buf) {
#pragma unroll
        for (int p = 0; p < 4; ++p) s[buf][p][l] = xa[p];
        if (halo) {
#pragma unroll
            for (int p = 0; p < 4; ++p) s[buf][p][kWave + l] = xb[p];
        }
    };
    load_row(first);
    store_row(0);
    if (nst > 1) {
        load_row(first + dir);
        store_row(1);
    }

    for (int i = 0; i < n; ++i) {
        const int k = first + dir * i;
        const int b = i & 1;
        const size_t row = (size_t)k * nr;
        // next rows' traffic, consumed at the end of this iteration
        const bool pre = i + 2 < nst;
        if (pre) load_row(k + 2 * dir);
        double n0, n1, n2, n3;
        if (reads_un<kMode>()) {
            n0 = ldb(unp[0] + row, oc);
            n1 = ldb(unp[1] + row, oc);
            n2 = ldb(unp[2] + row, oc);
            n3 = ldb(unp[3] + row, oc);
        }
        double hc[kNCH];
#pragma unroll
        for (int q = 0; q < kNCH; ++q) hc[q] = ldb(A.ctab + (size_t)q * P + row, oc);
        lds_sync();

        double dPhR, dPhI, dPiR, dPiI;
        {
            // upwind side per lane and row: speed >= 0 -> f^+, speed < 0 -> f^-
            const bool up1 = hc[kHLam1] >= 0.0, up2 = hc[kHLam2] >= 0.0;
            auto deriv = [&](int p, bool up, bool any_up, bool any_dn) {
                double fp = 0.0, fm = 0.0, d = 0.0;
                if (any_up) {
                    fp = Weno<WP>::flux6(s[b][p][l], s[b][p][l + 1], s[b][p][l + 2], s[b][p][l + 3], s[b][p][l + 4], A.eps);
                    const double dp = next_lane(fp) - fp;
                    if (up) d = dp;
                }
                if (any_dn) {
                    fm = Weno<WP>::flux6(s[b][p][l + 5], s[b][p][l + 4], s[b][p][l + 3], s[b][p][l + 2], s[b][p][l + 1], A.eps);
                    const double dm = next_lane(fm) - fm;
                    if (!up) d = dm;
                }
                return d * A.inv6dx;
            };
            const bool up1_any = __any(active && up1), dn1_any = __any(active && !up1);
            const bool up2_any = __any(active && up2), dn2_any = __any(active && !up2);
            dPhR = deriv(0, up1, up1_any, dn1_any);
            dPhI = deriv(1, up1, up1_any, dn1_any);
            dPiR = deriv(2, up2, up2_any, dn2_any);
            dPiI = deriv(3, up2, up2_any, dn2_any);
        }
        const double phR = s[b][0][l + 3], phI = s[b][1][l + 3];
        const double piR = s[b][2][l + 3], piI = s[b][3][l + 3];
        double ahR, ahI;   // Phi on the row ahead (k + dir)
        if (i + 1 < nst) {
            ahR = s[b ^ 1][0][l + 3];
            ahI = s[b ^ 1][1][l + 3];
        } else {
            ahR = A.parity * phR;
            ahI = A.parity * phI;
        }

        if (active) {
            const double lam1 = hc[kHLam1], lam2n = -hc[kHLam2], m3r = hc[kHM3r], m3i = hc[kHM3i];
            const double btr = hc[kHBtr], bti = hc[kHBti], cr = hc[kHCr], ci = hc[kHCi];
            const double ath = hc[kHAth], bth = hc[kHBth];

            // rows k+1 and k-1
            const double upR = dir > 0 ? ahR : bhR, upI = dir > 0 ? ahI : bhI;
            const double dnR = dir > 0 ? bhR : ahR, dnI = dir > 0 ? bhI : ahI;
            const double d1R = (upR - dnR) * A.ih1, d1I = (upI - dnI) * A.ih1;
            const double d2R = (upR - 2.0 * phR + dnR) * A.ih2;
            const double d2I = (upI - 2.0 * phI + dnI) * A.ih2;

            // d_t Phi = pi - lam1 d_x Phi
            const double FphR = piR - lam1 * dPhR;
            const double FphI = piI - lam1 * dPhI;
            // d_t pi = -lam2 d_x pi - m3 d_x Phi + B~t pi + A~thth Phi_thth + B~th Phi_th + C~ Phi
            const double FpiR = lam2n * dPiR - (m3r * dPhR - m3i * dPhI) + (btr * piR - bti * piI) +
                                ath * d2R + bth * d1R + (cr * phR - ci * phI);
            const double FpiI = lam2n * dPiI - (m3r * dPhI + m3i * dPhR) + (btr * piI + bti * piR) +
                                ath * d2I + bth * d1I + (cr * phI + ci * phR);

            if (kMode == kRhsOnly) {
                stb(outp[0] + row, oc, FphR);
                stb(outp[1] + row, oc, FphI);
                stb(outp[2] + row, oc, FpiR);
                stb(outp[3] + row, oc, FpiI);
            } else if (kMode == kStageFirst) {
                stb(outp[0] + row, oc, phR + A.dt * FphR);
                stb(outp[1] + row, oc, phI + A.dt * FphI);
                stb(outp[2] + row, oc, piR + A.dt * FpiR);
                stb(outp[3] + row, oc, piI + A.dt * FpiI);
            } else if (kMode == kStageLater) {
                stb(outp[0] + row, oc, A.ca * n0 + A.cb * (phR + A.dt * FphR));
                stb(outp[1] + row, oc, A.ca * n1 + A.cb * (phI + A.dt * FphI));
                stb(outp[2] + row, oc, A.ca * n2 + A.cb * (piR + A.dt * FpiR));
                stb(outp[3] + row, oc, A.ca * n3 + A.cb * (piI + A.dt * FpiI));
            } else {
                const double v0 = phR + A.dt * FphR, v1 = phI + A.dt * FphI;
                const double v2 = piR + A.dt * FpiR, v3 = piI + A.dt * FpiI;
                stb(outp[0] + row, oc, A.ca * n0 + A.cb * v0);
                stb(outp[1] + row, oc, A.ca * n1 + A.cb * v1);
                stb(outp[2] + row, oc, A.ca * n2 + A.cb * v2);
                stb(outp[3] + row, oc, A.ca * n3 + A.cb * v3);
                stb(A.out2 + row, oc, A.ca2 * n0 + A.cb2 * v0);
                stb(A.out2 + P + row, oc, A.ca2 * n1 + A.cb2 * v1);
                stb(A.out2 + 2 * P + row, oc, A.ca2 * n2 + A.cb2 * v2);
                stb(A.out2 + 3 * P + row, oc, A.ca2 * n3 + A.cb2 * v3);
            }
        }
        bhR = phR;
        bhI = phI;
        lds_sync();               // every lane is done reading s[b] (row k)
        if (pre) store_row(b);    // row k + 2 dir takes its place
    }
}

// Chart-T march of one strip over rows [k0, k1) with the LDS-DMA row pipeline.
// Row i of the march (k = first + dir i) lives in ring slot i mod 4; the
// rows first, first + dir, first + 2 dir are issued before the loop and row
// i + 3 at the top of iteration i.  Where the march has no such row, one
// cache line is loaded into the free slot instead, so that every iteration
// issues the same operations and the wait counts are constants:
//     per iteration: [u^n of row i: 4 loads (later stages)] [row i + 3: 12 DMA];
//     before reading rows i and i + 1: everything up to row i + 1 has landed,
//         i.e. vmcnt <= (12 + it) at i = 0 and vmcnt <= 2 it for i >= 1,
//         it = loads per iteration (16 later stages, 12 otherwise);
//     before the stores: u^n of row i has landed, vmcnt <= 12.
// kTh4 (fourth-order theta differences) also reads Phi on row i + 2, so it
// waits for everything up to row i + 2 (vmcnt <= it at every i), keeps the
// two rows behind in registers, and stages up to two rows past the segment.
// Beyond a pole, ghost row -1 - g is parity x row g (and row nth + g is
// parity x row nth - 1 - g): the ahead rows then come from the rows already
// at hand (row k + 2 dir mirrors k + dir when only it is a ghost, and k - dir
// when both are).
template <int WP, int kMode, bool kLevel, bool kCoh = false, bool kTh4 = false>
__device__ __forceinline__ void march_strip_t(const StageArgs& A, char* ring, int strip, int k0, int k1, int dir)
{
    const int l = threadIdx.x;
    const int nr = A.nr, nth = A.nth;
    const long long P = A.plane;
    const int j0 = strip * kStripPoints;
    const int j = j0 + l;
    const bool active = (l < kStripPoints) && (j < nr);
    const int jc = min(j, nr - 1);
    const unsigned oc = (unsigned)jc * 8u;                                 // own point
    // staged dword d = 64 c + l of a row holds half (d & 1) of position j0 - 3 + d/2
    unsigned od[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int d = 64 * c + l;
        od[c] = (unsigned)clampi(j0 - 3 + (d >> 1), 0, nr - 1) * 8u + (unsigned)(d & 1) * 4u;
    }
    const unsigned lds0 = (unsigned)(size_t)ring;          // LDS byte address of the ring
    const double* ukp[4] = {A.uk, A.uk + P, A.uk + 2 * P, A.uk + 3 * P};
    const double* unp[4] = {A.un, A.un + P, A.un + 2 * P, A.un + 3 * P};
    double* outp[4] = {A.out, A.out + P, A.out + 2 * P, A.out + 3 * P};

    double rt[kNRT];
#pragma unroll
    for (int i = 0; i < kNRT; ++i) rt[i] = ldb(A.rtab + (size_t)i * nr, oc);
    const __attribute__((address_space(4))) double* tt =
        (const __attribute__((address_space(4))) double*)A.ttab;

    const int n = k1 - k0;
    const int first = dir > 0 ? k0 : k1 - 1;
    // Phi on the rows behind (k - dir, and k - 2 dir for kTh4), pole ghosts mirrored
    auto behind = [&](int kb, double& vR, double& vI) {
        const bool ghost = kb < 0 || kb >= nth;
        const int km = kb < 0 ? -1 - kb : (kb >= nth ? 2 * nth - 1 - kb : kb);
        vR = ldb_c<kCoh>(ukp[0] + (size_t)km * nr, oc);
        vI = ldb_c<kCoh>(ukp[1] + (size_t)km * nr, oc);
        if (ghost) {
            vR *= A.parity;
            vI *= A.parity;
        }
    };
    double bhR, bhI, bh2R = 0.0, bh2I = 0.0;
    behind(first - dir, bhR, bhI);
    if constexpr (kTh4) behind(first - 2 * dir, bh2R, bh2I);
    // rows staged: the segment's n rows and the rows past it that lie in the grid
    const int ahead_last = first + dir * n;
    int nst = (ahead_last >= 0 && ahead_last < nth) ? n + 1 : n;
    if constexpr (kTh4) {
        const int ahead2 = ahead_last + dir;
        if (nst > n && ahead2 >= 0 && ahead2 < nth) ++nst;
    }

    // 12 DMA operations: march row i into its slot, or, where the march has no
    // row i, the first dword of each plane (one cache line, read by every lane)
    // into the free slot
    auto issue_row = [&](int i) {
        const bool real = i < nst;
        const size_t row = real ? (size_t)(first + dir * i) * nr : 0;
        const unsigned slot = lds0 + (unsigned)(i & (kRing - 1)) * kSlotBytes;
        const unsigned o0 = real ? od[0] : 0u, o1 = real ? od[1] : 0u, o2 = real ? od[2] : 0u;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const double* base = ukp[p] + row;
            dma_dword_c<kCoh>(o0, base, slot + p * kPlaneBytes);
            dma_dword_c<kCoh>(o1, base, slot + p * kPlaneBytes + 256u);
            if (l < 10) dma_dword_c<kCoh>(o2, base, slot + p * kPlaneBytes + 512u);
        }
    };
    issue_row(0);
    issue_row(1);
    issue_row(2);

    const double (*sr)[4][kRowP] = reinterpret_cast<const double (*)[4][kRowP]>(ring);
    for (int i = 0; i < n; ++i) {
        // Waves of one SIMD issue oldest first.  When every workgroup of the
        // launch is resident from the start (kLevel: the single-solve launch),
        // the oldest wave of a SIMD would end its segment long before the
        // youngest (measured: 15 us against 30 us), leaving the SIMD with one
        // or two waves for the last third of the launch.  Lowering a wave's
        // priority as it advances lets the younger waves keep up, and the
        // segments end closer together.  A launch whose tiles are dispatched
        // as slots free up (the batched launch) measured slower with it.
        if constexpr (kLevel) {
            if (i == 0) __builtin_amdgcn_s_setprio(3);
            else if (i == 2) __builtin_amdgcn_s_setprio(2);
            else if (i == 4) __builtin_amdgcn_s_setprio(1);
            else if (i == 6) __builtin_amdgcn_s_setprio(0);
        }
        const int k = first + dir * i;
        const size_t row = (size_t)k * nr;
        const double sn2 = tt[kSn2 * nth + k];
        const double cs = tt[kCs * nth + k];
        const double cot = tt[kCot * nth + k];
        const double th = tt[kTh * nth + k];
        double n0 = 0.0, n1 = 0.0, n2 = 0.0, n3 = 0.0;
        if (reads_un<kMode>()) {
            n0 = ld_async_c<kCoh>(oc, unp[0] + row);
            n1 = ld_async_c<kCoh>(oc, unp[1] + row);
            n2 = ld_async_c<kCoh>(oc, unp[2] + row);
            n3 = ld_async_c<kCoh>(oc, unp[3] + row);
        }
        // 1/Sigma of the point.  In the single-solve launch its dependent chain
        // (reciprocal square root and two Newton steps) is started here, where
        // it overlaps the row's loads (the empty asm keeps the compiler from
        // sinking it to its use); the batched launch, whose tiles start as
        // slots free up, measured 0.7 % slower on C4 with that, and leaves the
        // placement to the compiler.
        const double vsig = rsq64(sigma2(rt, sn2));
        if constexpr (kLevel) asm volatile("" : : "v"(vsig));
        issue_row(i + 3);
        constexpr int it = reads_un<kMode>() ? 16 : 12;
        if constexpr (kTh4) vm_wait<it>();
        else if (i == 0) vm_wait<12 + it>();
        else vm_wait<2 * it>();
        const int b = i & (kRing - 1), bn = (i + 1) & (kRing - 1);

        const double fR = Weno<WP>::flux6(sr[b][0][l], sr[b][0][l + 1], sr[b][0][l + 2], sr[b][0][l + 3], sr[b][0][l + 4], A.eps);
        const double fI = Weno<WP>::flux6(sr[b][1][l], sr[b][1][l + 1], sr[b][1][l + 2], sr[b][1][l + 3], sr[b][1][l + 4], A.eps);
        const double gR = Weno<WP>::flux6(sr[b][2][l + 5], sr[b][2][l + 4], sr[b][2][l + 3], sr[b][2][l + 2], sr[b][2][l + 1], A.eps);
        const double gI = Weno<WP>::flux6(sr[b][3][l + 5], sr[b][3][l + 4], sr[b][3][l + 3], sr[b][3][l + 2], sr[b][3][l + 1], A.eps);
        const double phR = sr[b][0][l + 3], phI = sr[b][1][l + 3];
        const double piR = sr[b][2][l + 3], piI = sr[b][3][l + 3];
        double ahR, ahI;   // Phi on the row ahead (k + dir)
        if (i + 1 < nst) {
            ahR = sr[bn][0][l + 3];
            ahI = sr[bn][1][l + 3];
        } else {
            ahR = A.parity * phR;
            ahI = A.parity * phI;
        }
        double ah2R = 0.0, ah2I = 0.0;   // Phi on row k + 2 dir (kTh4)
        if constexpr (kTh4) {
            if (i + 2 < nst) {
                const int bn2 = (i + 2) & (kRing - 1);
                ah2R = sr[bn2][0][l + 3];
                ah2I = sr[bn2][1][l + 3];
            } else if (i + 1 < nst) {
                ah2R = A.parity * ahR;
                ah2I = A.parity * ahI;
            } else {
                ah2R = A.parity * bhR;
                ah2I = A.parity * bhI;
            }
        }
        // the interface flux of the next lane: by DPP in the single-solve
        // launch; the batched launch measured 1.2 % slower on C4 with the DPP
        // moves (VALU work) than with ds_bpermute (LDS work)
        const double fR1 = kLevel ? next_lane(fR) : __shfl_down(fR, 1);
        const double fI1 = kLevel ? next_lane(fI) : __shfl_down(fI, 1);
        const double gR1 = kLevel ? next_lane(gR) : __shfl_down(gR, 1);
        const double gI1 = kLevel ? next_lane(gI) : __shfl_down(gI, 1);

        if (reads_un<kMode>()) vm_wait<12>(n0, n1, n2, n3);
        if (active) {
            const double dPhR = (fR1 - fR) * A.inv6dx;
            const double dPhI = (fI1 - fI) * A.inv6dx;
            const double dPiR = (gR1 - gR) * A.inv6dx;
            const double dPiI = (gI1 - gI) * A.inv6dx;
            const PointCoef c = point_coef(rt, sn2, cs, cot, th, vsig);
            const double upR = dir > 0 ? ahR : bhR, upI = dir > 0 ? ahI : bhI;
            const double dnR = dir > 0 ? bhR : ahR, dnI = dir > 0 ? bhI : ahI;
            double d1R, d1I, d2R, d2I;
            if constexpr (kTh4) {
                // ih1 = 1/(12 dtheta), ih2 = 1/(12 dtheta^2)
                const double up2R = dir > 0 ? ah2R : bh2R, up2I = dir > 0 ? ah2I : bh2I;
                const double dn2R = dir > 0 ? bh2R : ah2R, dn2I = dir > 0 ? bh2I : ah2I;
                d1R = (8.0 * (upR - dnR) - (up2R - dn2R)) * A.ih1;
                d1I = (8.0 * (upI - dnI) - (up2I - dn2I)) * A.ih1;
                d2R = (16.0 * (upR + dnR) - 30.0 * phR - (up2R + dn2R)) * A.ih2;
                d2I = (16.0 * (upI + dnI) - 30.0 * phI - (up2I + dn2I)) * A.ih2;
            } else {
                d1R = (upR - dnR) * A.ih1;
                d1I = (upI - dnI) * A.ih1;
                d2R = (upR - 2.0 * phR + dnR) * A.ih2;
                d2I = (upI - 2.0 * phI + dnI) * A.ih2;
            }
            const double FphR = piR - c.b * dPhR;
            const double FphI = piI - c.b * dPhI;
            const double FpiR = c.b * dPiR - (c.m3r * dPhR - c.m3i * dPhI) + (c.btr * piR - c.bti * piI) +
                                c.ath * d2R + c.bth * d1R + (c.cr * phR - c.ci * phI);
            const double FpiI = c.b * dPiI - (c.m3r * dPhI + c.m3i * dPhR) + (c.btr * piI + c.bti * piR) +
                                c.ath * d2I + c.bth * d1I + (c.cr * phI + c.ci * phR);
            if (kMode == kRhsOnly) {
                stb_c<kCoh>(outp[0] + row, oc, FphR);
                stb_c<kCoh>(outp[1] + row, oc, FphI);
                stb_c<kCoh>(outp[2] + row, oc, FpiR);
                stb_c<kCoh>(outp[3] + row, oc, FpiI);
            } else if (kMode == kStageFirst) {
                stb_c<kCoh>(outp[0] + row, oc, phR + A.dt * FphR);
                stb_c<kCoh>(outp[1] + row, oc, phI + A.dt * FphI);
                stb_c<kCoh>(outp[2] + row, oc, piR + A.dt * FpiR);
                stb_c<kCoh>(outp[3] + row, oc, piI + A.dt * FpiI);
            } else if (kMode == kStageLater) {
                stb_c<kCoh>(outp[0] + row, oc, A.ca * n0 + A.cb * (phR + A.dt * FphR));
                stb_c<kCoh>(outp[1] + row, oc, A.ca * n1 + A.cb * (phI + A.dt * FphI));
                stb_c<kCoh>(outp[2] + row, oc, A.ca * n2 + A.cb * (piR + A.dt * FpiR));
                stb_c<kCoh>(outp[3] + row, oc, A.ca * n3 + A.cb * (piI + A.dt * FpiI));
            } else {
                const double v0 = phR + A.dt * FphR, v1 = phI + A.dt * FphI;
                const double v2 = piR + A.dt * FpiR, v3 = piI + A.dt * FpiI;
                stb_c<kCoh>(outp[0] + row, oc, A.ca * n0 + A.cb * v0);
                stb_c<kCoh>(outp[1] + row, oc, A.ca * n1 + A.cb * v1);
                stb_c<kCoh>(outp[2] + row, oc, A.ca * n2 + A.cb * v2);
                stb_c<kCoh>(outp[3] + row, oc, A.ca * n3 + A.cb * v3);
                stb_c<kCoh>(A.out2 + row, oc, A.ca2 * n0 + A.cb2 * v0);
                stb_c<kCoh>(A.out2 + P + row, oc, A.ca2 * n1 + A.cb2 * v1);
                stb_c<kCoh>(A.out2 + 2 * P + row, oc, A.ca2 * n2 + A.cb2 * v2);
                stb_c<kCoh>(A.out2 + 3 * P + row, oc, A.ca2 * n3 + A.cb2 * v3);
            }
        }
        if constexpr (kTh4) {
            bh2R = bhR;
            bh2I = bhI;
        }
        bhR = phR;
        bhI = phI;
    }
    vm_wait<0>();   // nothing of this strip may still be landing in the ring
}

// Launch layout: every radial strip is cut into the same number `segs` of theta
// segments (an even number when there is more than one), workgroup
// rank = strip * segs + i owns segment i of its strip, and even segments march
// upward, odd ones downward.  Two segments that share a boundary row then read
// it at the same moment (both start there, or both end there), and segment i
// of neighbouring strips -- which share the radial halo -- march the same rows
// in step, so the shared lines are read from HBM once and hit in L2 for the
// second reader.
// LDS of one stage workgroup: the four-row DMA ring (chart T) or the two-row
// staging ring (chart H).
constexpr unsigned kLdsBytes = kRing * kSlotBytes;   // 9216 >= 2 * 4 * kRow * 8

template <int WP, int kMode, int kChart, bool kLevel = false, bool kCoh = false>
__device__ __forceinline__ void march(const StageArgs& A, char* lds, int strip, int k0, int k1, int dir)
{
    if constexpr (kChart == kChartT || kChart == kChartT4)
        march_strip_t<WP, kMode, kLevel, kCoh, kChart == kChartT4>(A, lds, strip, k0, k1, dir);
    else
        march_strip_h<WP, kMode>(A, reinterpret_cast<double (*)[4][kRow]>(lds), strip, k0, k1, dir);
}

template <int WP, int kMode, int kChart>
__device__ __forceinline__ void run_tile(const StageArgs& A, char* lds, int rank)
{
    const int strip = rank / A.segs;
    const int seg = rank - strip * A.segs;
    const int k0 = (int)((long long)A.nth * seg / A.segs);
    const int k1 = (int)((long long)A.nth * (seg + 1) / A.segs);
    if (k1 > k0) march<WP, kMode, kChart, true>(A, lds, strip, k0, k1, ((seg ^ A.flip) & 1) ? -1 : 1);
}

// Ranks are dealt so that each XCD (which receives every eighth workgroup id)
// owns a contiguous block of ranks, i.e. whole strips and their neighbours.
__device__ __forceinline__ int xcd_rank(int bid, int G)
{
    const int xcd = bid & 7, loc = bid >> 3;
    const int q8 = G >> 3, r8 = G & 7;
    return xcd * q8 + (xcd < r8 ? xcd : r8) + loc;
}

template <int WP, int kMode, int kChart>
__global__ __launch_bounds__(kWave) void stage_kernel(StageArgs A)
{
    __shared__ __attribute__((aligned(16))) char lds[kLdsBytes];
    run_tile<WP, kMode, kChart>(A, lds, xcd_rank((int)blockIdx.x, (int)gridDim.x));
}

// One stage of several independent solves in one launch.  Member m is cut
// into tiles of one radial strip by one theta segment (args[m].segs segments
// per strip) and owns the tile numbers [start[m], start[m+1]), numbered
// segment by segment with the strip index fastest; args[m] holds its buffers,
// tables, grid and dt.  Workgroup `rank` takes the tiles rank, rank + G,
// rank + 2G, ...: at any moment the workgroups in flight hold consecutive
// tiles, i.e. neighbouring strips of the same theta segment, which march the
// same rows together -- their reads of a row are one contiguous stretch of
// each plane, and the radial halo they share is read once into L2.  Even
// segments march upward and odd ones downward, so the two tiles that share a
// boundary row meet there at the end of their march.  By default G equals the
// tile count (one tile per workgroup, dispatched in tile order by the
// hardware as slots free up), which measured faster than fewer workgroups
// looping over tiles.  A tile runs exactly the single-solve code.
template <int WP, int kMode, int kChart>
__global__ __launch_bounds__(kWave) void group_stage_kernel(const StageArgs* __restrict__ args,
                                                            const long long* __restrict__ start, int nmem,
                                                            long long tiles)
{
    __shared__ __attribute__((aligned(16))) char lds[kLdsBytes];
    const int G = (int)gridDim.x;
    for (long long t = xcd_rank((int)blockIdx.x, G); t < tiles; t += G) {
        int lo = 0, hi = nmem - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (start[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        const StageArgs A = args[lo];
        const int local = (int)(t - start[lo]);
        const int seg = local / A.nstrips;
        const int strip = local - seg * A.nstrips;
        const int k0 = (int)((long long)A.nth * seg / A.segs);
        const int k1 = (int)((long long)A.nth * (seg + 1) / A.segs);
        if (k1 > k0) march<WP, kMode, kChart>(A, lds, strip, k0, k1, ((seg ^ A.flip) & 1) ? -1 : 1);
    }
}

// ---------------------------------------------------------------- pipelined steps
// Several SSP-RK(3,3) steps in one cooperative launch (tortoise chart).  The
// work items are the tiles of every stage of every step -- tile (strip,
// segment) of stage S, the tiles of the single-solve stage launch -- numbered
// stage by stage, and workgroup w takes items w, w + G, w + 2G, ... in order.
// A tile's stage S reads the stage S-1 results of its own tile and of the
// tiles around it (the radial halo from the neighbouring strips, the theta row
// across a segment boundary, and the corners of both), so it waits for those
// nine tiles only, not for the whole grid: waves drift apart, and the memory
// traffic of some overlaps the arithmetic of others across stage boundaries,
// where stage-by-stage launches drain and refill the GPU three times a step.
// Every other hazard (a stage overwriting values that a neighbour's earlier
// stage still reads: u(1) by the next step's stage 1, u^n by stage 3 in place)
// is ordered through these waits by induction, because a neighbour's stage
// S-1 itself waited for the stage S-2 of its own neighbours.
// Progress: the earliest unfinished item waits only on earlier items, which
// have finished, and its workgroup has finished its own earlier items, so it is
// working on that item; this needs every workgroup resident at once, which the
// cooperative launch guarantees.
// Counters: done[tile] = stages the tile has completed since the state was set
// (absolute, so launches need no reset).  The tiles' rows are read and written
// with agent-coherent accesses (the sc1 forms of the row loads, LDS-DMA loads
// and stores), so no cache needs writing back or invalidating: a workgroup
// waits for its stores to complete and then writes its tile's count; a reader
// polls the neighbours' counts with agent-scope loads and issues its coherent
// loads only after seeing them.
// A wait longer than spin_ticks of the 100 MHz real-time counter sets *err and
// goes on, so a fault of this scheme shows up as an error, never as a hang.
struct PipeArgs {
    StageArgs st[3];       // stage 1, 2, 3 arguments (segs, nstrips equal in all three)
    long long* done;       // [nstrips * segs] stages completed per tile
    int* err;              // set to 1 by a wait that timed out
    long long s0;          // stages completed before this launch (3 x steps)
    int nsteps;            // steps in this launch
    int tiles;             // nstrips * segs
    long long spin_ticks;  // wait limit
};

__device__ __forceinline__ void pipe_wait(const PipeArgs& P, int strip, int seg, long long need)
{
    const int l = threadIdx.x;
    const int nstrips = P.st[0].nstrips, segs = P.st[0].segs;
    const long long* c = nullptr;
    if (l < 9) {
        const int s2 = strip + l / 3 - 1, g2 = seg + l % 3 - 1;
        if (s2 >= 0 && s2 < nstrips && g2 >= 0 && g2 < segs) c = P.done + (size_t)s2 * segs + g2;
    }
    const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
    for (;;) {
        const bool ok = !c || __hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need;
        if (__all(ok)) break;
        // after one timed-out wait anywhere, no wait blocks any more
        const int failed = __hip_atomic_load(P.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (failed) break;
        if ((long long)(__builtin_amdgcn_s_memrealtime() - t0) > P.spin_ticks) {
            if (l == 0) __hip_atomic_store(P.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
        __builtin_amdgcn_s_sleep(2);
    }
    // the tile's loads are issued after the counts were seen (the loop exit
    // depends on them) and are coherent loads, so they see the neighbours'
    // completed stores; this keeps the compiler from hoisting them
    asm volatile("" ::: "memory");
}

template <int WP>
__global__ __launch_bounds__(kWave) void pipe_kernel(PipeArgs P)
{
    __shared__ __attribute__((aligned(16))) char lds[kLdsBytes];
    const long long items = 3LL * P.nsteps * P.tiles;
    const int segs = P.st[0].segs;
    for (long long it = blockIdx.x; it < items; it += gridDim.x) {
        const long long S = it / P.tiles;
        const int r = (int)(it - S * P.tiles);
        const int strip = r / segs, seg = r - strip * segs;
        const long long need = P.s0 + S;
        if (need > 0) pipe_wait(P, strip, seg, need);
        const int stage = (int)(S % 3);
        StageArgs A = P.st[stage];
        A.flip = (int)(need & 1);
        const int k0 = (int)((long long)A.nth * seg / segs);
        const int k1 = (int)((long long)A.nth * (seg + 1) / segs);
        const int dir = ((seg ^ A.flip) & 1) ? -1 : 1;
        if (k1 > k0) {
            if (stage == 0) march<WP, kStageFirst, kChartT, false, true>(A, lds, strip, k0, k1, dir);
            else march<WP, kStageLater, kChartT, false, true>(A, lds, strip, k0, k1, dir);
        }
        // publish: every coherent store of the tile has completed before the count is written
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        if (threadIdx.x == 0)
            __hip_atomic_store(P.done + r, need + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ---------------------------------------------------------------- temporal blocking
// One whole SSP-RK(3,3) step per launch (tortoise chart): the three stages of a
// tile are computed in one workgroup of two waves, the intermediate states u(1)
// and u(2) never leave LDS, and HBM sees one read of u^n and one write of
// u^{n+1} per point (64 B instead of 256 B per point-step).  The price is
// recomputation at the tile edges: a stage needs three radial neighbours and one
// theta neighbour of its input on each side, so
//   - a tile spans 127 radial points q = 0 .. 126, point q standing for
//     j = 114 strip - 6 + q in all three stages.  Wave 0 holds points 0..63 and
//     wave 1 points 63..126: the two overlap by one point so that every point
//     but the last of each wave finds its j + 1/2 flux in the next lane of its
//     own wave.  Point 63 is computed by wave 1 (wave 0's copy, lacking that
//     flux, is never stored);
//   - stage 1 is valid on points 0..125, stage 2 on 3..122 and stage 3 (the
//     output) on 6..119: 114 outputs per 128 lanes;
//   - a tile of final rows [k0, k1) computes stage 1 on [k0-2, k1+2) and stage
//     2 on [k0-1, k1+1) (clipped to the grid; a pole takes the parity ghost of
//     the stage's own input, as in the three-launch step).
// The workgroup marches the rows upward: at step r it stages u^n row r+1 (LDS),
// computes u(1) at row r, u(2) at row r-1 and u^{n+1} at row r-2.  Radial
// ghosts of u(1) and u(2) are the end values, read by clamping the point index
// to the points inside the grid.  The arithmetic of each point and stage is
// the three-launch stage kernel's, term for term, except that the per-point
// coefficients of a row are built once, by stage 1, and reused by stages 2
// and 3 when the march reaches that row for them (a lane keeps its radial
// point through all three stages).
constexpr int kBW = 114;                 // output points per tile
constexpr int kBLead = 6;                // first output point of a tile
constexpr int kBThreads = 2 * kWave;     // two waves
constexpr int kBPts = 2 * kWave - 1;     // points of a tile (the waves share one)
constexpr int kBStage = kBPts + 6;       // staged u^n positions: q - 3 .. q + 3 of every point
static_assert(kBLead + kBW + kBLead + 1 == kBPts, "tile geometry");

template <int WP>
__global__ __launch_bounds__(kBThreads) void blocked_step_kernel(StageArgs A)
{
    __shared__ double sn[3][4][kBStage];   // u^n rows (three-slot ring), position s = point p0 - 3 + s
    __shared__ double s1[2][4][kBPts];     // u(1) rows, one value per point
    __shared__ double s2[2][4][kBPts];     // u(2) rows
    const int tid = threadIdx.x;
    const int l = tid - (tid >= kWave ? 1 : 0);          // point of this lane in the tile
    const bool dup = tid == kWave - 1;                    // wave 0's copy of point 63
    const int nr = A.nr, nth = A.nth;
    const long long P = A.plane;
    const int rank = xcd_rank((int)blockIdx.x, (int)gridDim.x);
    const int strip = rank / A.segs;
    const int seg = rank - strip * A.segs;
    const int k0 = (int)((long long)nth * seg / A.segs);
    const int k1 = (int)((long long)nth * (seg + 1) / A.segs);
    if (k1 <= k0) return;                                 // uniform over the workgroup
    const int p0 = strip * kBW - kBLead;                  // grid point of tile point 0
    const int j = p0 + l;
    const int jc = clampi(j, 0, nr - 1);
    const unsigned oc = (unsigned)jc * 8u;
    const unsigned oa = (unsigned)clampi(p0 - 3 + tid, 0, nr - 1) * 8u;               // staged position tid
    const unsigned ob = (unsigned)clampi(p0 - 3 + kBThreads + tid, 0, nr - 1) * 8u;   // position 128 + tid
    const bool halo = tid < kBStage - kBThreads;
    const int lo = clampi(-p0, 0, kBPts - 1), hi = clampi(nr - 1 - p0, 0, kBPts - 1);   // points inside the grid
    const bool out_lane = !dup && l >= kBLead && l < kBLead + kBW && j < nr;
    const double* ukp[4] = {A.uk, A.uk + P, A.uk + 2 * P, A.uk + 3 * P};
    double* outp[4] = {A.out, A.out + P, A.out + 2 * P, A.out + 3 * P};
    double rt[kNRT];
#pragma unroll
    for (int i = 0; i < kNRT; ++i) rt[i] = ldb(A.rtab + (size_t)i * nr, oc);
    const __attribute__((address_space(4))) double* tt =
        (const __attribute__((address_space(4))) double*)A.ttab;

    const int r1lo = max(k0 - 2, 0), r1hi = min(k1 + 2, nth);   // stage-1 rows
    const int r2lo = max(k0 - 1, 0), r2hi = min(k1 + 1, nth);   // stage-2 rows
    const int nstage = min(r1hi + 1, nth);                       // u^n rows staged: [r1lo, nstage)

    double xa[4], xb[4];
    auto load_row = [&](int k) {
        const size_t row = (size_t)k * nr;
#pragma unroll
        for (int p = 0; p < 4; ++p) xa[p] = ldb(ukp[p] + row, oa);
        if (halo) {
#pragma unroll
            for (int p = 0; p < 4; ++p) xb[p] = ldb(ukp[p] + row, ob);
        }
    };
    auto store_row = [&](int b) {
#pragma unroll
        for (int p = 0; p < 4; ++p) sn[b][p][tid] = xa[p];
        if (halo) {
#pragma unroll
            for (int p = 0; p < 4; ++p) sn[b][p][kBThreads + tid] = xb[p];
        }
    };
    auto cl = [&](int q) { return clampi(q, lo, hi); };

    // one stage at one row for this lane: w[p][t] = input of plane p at j - 3 + t,
    // dn / up = input Phi at the own point on rows k - 1 / k + 1
    struct Out { double v[4]; };
    auto stage = [&](const double (&w)[4][6], double dnR, double dnI, double upR, double upI, const PointCoef& c,
                     double ca, double cb, const double (&un)[4], bool first) {
        const double fR = Weno<WP>::flux6(w[0][0], w[0][1], w[0][2], w[0][3], w[0][4], A.eps);
        const double fI = Weno<WP>::flux6(w[1][0], w[1][1], w[1][2], w[1][3], w[1][4], A.eps);
        const double gR = Weno<WP>::flux6(w[2][5], w[2][4], w[2][3], w[2][2], w[2][1], A.eps);
        const double gI = Weno<WP>::flux6(w[3][5], w[3][4], w[3][3], w[3][2], w[3][1], A.eps);
        const double fR1 = next_lane(fR), fI1 = next_lane(fI);
        const double gR1 = next_lane(gR), gI1 = next_lane(gI);
        const double phR = w[0][3], phI = w[1][3], piR = w[2][3], piI = w[3][3];
        const double dPhR = (fR1 - fR) * A.inv6dx;
        const double dPhI = (fI1 - fI) * A.inv6dx;
        const double dPiR = (gR1 - gR) * A.inv6dx;
        const double dPiI = (gI1 - gI) * A.inv6dx;
        const double d1R = (upR - dnR) * A.ih1, d1I = (upI - dnI) * A.ih1;
        const double d2R = (upR - 2.0 * phR + dnR) * A.ih2;
        const double d2I = (upI - 2.0 * phI + dnI) * A.ih2;
        const double FphR = piR - c.b * dPhR;
        const double FphI = piI - c.b * dPhI;
        const double FpiR = c.b * dPiR - (c.m3r * dPhR - c.m3i * dPhI) + (c.btr * piR - c.bti * piI) +
                            c.ath * d2R + c.bth * d1R + (c.cr * phR - c.ci * phI);
        const double FpiI = c.b * dPiI - (c.m3r * dPhI + c.m3i * dPhR) + (c.btr * piI + c.bti * piR) +
                            c.ath * d2I + c.bth * d1I + (c.cr * phI + c.ci * phR);
        Out o;
        if (first) {
            o.v[0] = phR + A.dt * FphR;
            o.v[1] = phI + A.dt * FphI;
            o.v[2] = piR + A.dt * FpiR;
            o.v[3] = piI + A.dt * FpiI;
        } else {
            o.v[0] = ca * un[0] + cb * (phR + A.dt * FphR);
            o.v[1] = ca * un[1] + cb * (phI + A.dt * FphI);
            o.v[2] = ca * un[2] + cb * (piR + A.dt * FpiR);
            o.v[3] = ca * un[3] + cb * (piI + A.dt * FpiI);
        }
        return o;
    };

    // rolling own-point values: u^n (4 planes) at rows r, r-1, r-2; Phi of
    // u^n at r-1; Phi of u(1) at r-2, r-1, r; Phi of u(2) at r-3, r-2, r-1
    double un0[4] = {0, 0, 0, 0}, un1[4] = {0, 0, 0, 0}, un2[4] = {0, 0, 0, 0};
    double nbR = 0, nbI = 0;                 // u^n Phi on row r - 1
    double a2R = 0, a2I = 0, a1R = 0, a1I = 0, a0R = 0, a0I = 0;   // u(1) Phi on r-2, r-1, r
    double c3R = 0, c3I = 0, c2R = 0, c2I = 0, c1R = 0, c1I = 0;   // u(2) Phi on r-3, r-2, r-1
    // per-point coefficients of rows r, r - 1, r - 2, built by stage 1 and
    // reused by stages 2 and 3 (the same point and row one and two steps of
    // the march later)
    PointCoef pc0{}, pc1{}, pc2{};
    {
        const int kb = r1lo - 1;
        if (kb >= 0) {
            nbR = ldb(ukp[0] + (size_t)kb * nr, oc);
            nbI = ldb(ukp[1] + (size_t)kb * nr, oc);
        } else {
            nbR = A.parity * ldb(ukp[0] + (size_t)r1lo * nr, oc);
            nbI = A.parity * ldb(ukp[1] + (size_t)r1lo * nr, oc);
        }
    }
    // u^n row k sits in ring slot k mod 3: row r + 2 is stored during step r
    // into the slot of row r - 1, which every wave finished reading before
    // the barrier that opens step r, so one barrier per row orders all LDS
    // traffic (u(1) and u(2) rows are likewise read one step after they are
    // written, into slots last read one step before).
    int sc = r1lo % 3;                            // slot of row r
    load_row(r1lo);
    store_row(sc);
    if (r1lo + 1 < nstage) {
        load_row(r1lo + 1);
        store_row(sc == 2 ? 0 : sc + 1);
    }
    if (r1lo + 2 < nstage) load_row(r1lo + 2);

    // Issue priority steps down from 3 to 0 at 1/2, 3/4 and 7/8 of the march,
    // so that waves which started later keep pace with the older waves of
    // their SIMD (see march_strip_t).  On C2 the steps took the blocked step
    // from 0.97x to above 1.02x of the three-launch step; with two-wave tiles
    // these late steps measured 0.8 % faster than steps at the quarters, and
    // steps at the thirds (never reaching 0) 1.3 % slower.
    const int nit = k1 + 2 - r1lo;
    const int q1 = (nit + 1) / 2, q2 = (3 * nit + 3) / 4, q3 = (7 * nit + 7) / 8;
    for (int r = r1lo; r < k1 + 2; ++r) {
        const int it = r - r1lo;
        if (it == 0) __builtin_amdgcn_s_setprio(3);
        else if (it == q1) __builtin_amdgcn_s_setprio(2);
        else if (it == q2) __builtin_amdgcn_s_setprio(1);
        else if (it == q3) __builtin_amdgcn_s_setprio(0);
        lds_sync();                                   // u^n rows r, r+1 staged; u(1) row r-1, u(2) row r-2
        const int su = sc == 2 ? 0 : sc + 1;          // slot of row r + 1
        const int r2 = r - 1, r3 = r - 2;
        if (r < r1hi) {
            // ---- stage 1 at row r: u(1) = u^n + dt F(u^n)
            const int b = r & 1;
            double w[4][6];
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int t = 0; t < 6; ++t) w[p][t] = sn[sc][p][l + t];
            double upR, upI;
            if (r + 1 < nth) {
                upR = sn[su][0][l + 3];
                upI = sn[su][1][l + 3];
            } else {
                upR = A.parity * w[0][3];
                upI = A.parity * w[1][3];
            }
            const double none[4] = {0, 0, 0, 0};
            const double sn2 = tt[kSn2 * nth + r], cs = tt[kCs * nth + r];
            const double cot = tt[kCot * nth + r], th = tt[kTh * nth + r];
            pc2 = pc1;
            pc1 = pc0;
            pc0 = point_coef(rt, sn2, cs, cot, th, rsq64(sigma2(rt, sn2)));
            const Out o = stage(w, nbR, nbI, upR, upI, pc0, 0.0, 1.0, none, true);
            if (!dup) {
#pragma unroll
                for (int p = 0; p < 4; ++p) s1[b][p][l] = o.v[p];
            }
            un2[0] = un1[0]; un2[1] = un1[1]; un2[2] = un1[2]; un2[3] = un1[3];
            un1[0] = un0[0]; un1[1] = un0[1]; un1[2] = un0[2]; un1[3] = un0[3];
#pragma unroll
            for (int p = 0; p < 4; ++p) un0[p] = w[p][3];
            nbR = w[0][3];
            nbI = w[1][3];
            a2R = a1R; a2I = a1I; a1R = a0R; a1I = a0I;
            a0R = o.v[0]; a0I = o.v[1];
        } else {
            un2[0] = un1[0]; un2[1] = un1[1]; un2[2] = un1[2]; un2[3] = un1[3];
            un1[0] = un0[0]; un1[1] = un0[1]; un1[2] = un0[2]; un1[3] = un0[3];
            a2R = a1R; a2I = a1I; a1R = a0R; a1I = a0I;
            pc2 = pc1;
            pc1 = pc0;
        }
        if (r2 >= r2lo && r2 < r2hi) {
            // ---- stage 2 at row r - 1: u(2) = 3/4 u^n + 1/4 (u(1) + dt F(u(1)))
            const int b = r2 & 1;
            double w[4][6];
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int t = 0; t < 6; ++t) w[p][t] = s1[b][p][cl(l - 3 + t)];
            const double dnR = r2 - 1 >= 0 ? a2R : A.parity * a1R, dnI = r2 - 1 >= 0 ? a2I : A.parity * a1I;
            const double upR = r2 + 1 < nth ? a0R : A.parity * a1R, upI = r2 + 1 < nth ? a0I : A.parity * a1I;
            const Out o = stage(w, dnR, dnI, upR, upI, pc1, 0.75, 0.25, un1, false);
            if (!dup) {
#pragma unroll
                for (int p = 0; p < 4; ++p) s2[b][p][l] = o.v[p];
            }
            c3R = c2R; c3I = c2I; c2R = c1R; c2I = c1I;
            c1R = o.v[0]; c1I = o.v[1];
        } else {
            c3R = c2R; c3I = c2I; c2R = c1R; c2I = c1I;
        }
        if (r3 >= k0 && r3 < k1) {
            // ---- stage 3 at row r - 2: u^{n+1} = 1/3 u^n + 2/3 (u(2) + dt F(u(2)))
            const int b = r3 & 1;
            double w[4][6];
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int t = 0; t < 6; ++t) w[p][t] = s2[b][p][cl(l - 3 + t)];
            const double dnR = r3 - 1 >= 0 ? c3R : A.parity * c2R, dnI = r3 - 1 >= 0 ? c3I : A.parity * c2I;
            const double upR = r3 + 1 < nth ? c1R : A.parity * c2R, upI = r3 + 1 < nth ? c1I : A.parity * c2I;
            const Out o = stage(w, dnR, dnI, upR, upI, pc2, 1.0 / 3.0, 2.0 / 3.0, un2, false);
            if (out_lane) {
                const size_t row = (size_t)r3 * nr;
#pragma unroll
                for (int p = 0; p < 4; ++p) stb(outp[p] + row, oc, o.v[p]);
            }
        }
        // row r + 2 into the slot of row r - 1
        if (r + 2 < nstage) {
            store_row(sc == 0 ? 2 : sc - 1);
            if (r + 3 < nstage) load_row(r + 3);
        }
        sc = su;
    }
}

// ---------------------------------------------------------------- stability bound
// max over points of max(|lam1|, |lam2|)/dx + sqrt(4 A~thth/dtheta^2 + |B~th|/dtheta + |C~|);
// the values are >= 0, so their bit patterns order like unsigned integers and
// the reduction ends in one 64-bit atomic max per workgroup.  Chart T takes the
// coefficients from the radial / polar tables (|lam1| = |lam2| = b), chart H
// from the per-point table (ctab != nullptr).
__global__ __launch_bounds__(256) void dt_bound_kernel(const double* __restrict__ rtab,
                                                       const double* __restrict__ ttab,
                                                       const double* __restrict__ ctab, int nr, int nth,
                                                       double idx, double idth, double c2, double c1,
                                                       unsigned long long* cell)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long n = (long long)nr * nth;
    double val = 0.0;
    if (i < n) {
        double lam, ath, bth, cr, ci;
        if (ctab) {
            lam = fmax(fabs(ctab[kHLam1 * n + i]), fabs(ctab[kHLam2 * n + i]));
            ath = ctab[kHAth * n + i];
            bth = ctab[kHBth * n + i];
            cr = ctab[kHCr * n + i];
            ci = ctab[kHCi * n + i];
        } else {
            const int k = (int)(i / nr), j = (int)(i - (long long)k * nr);
            double rt[kNRT];
            for (int t = 0; t < kNRT; ++t) rt[t] = rtab[(size_t)t * nr + j];
            const double sn2 = ttab[kSn2 * nth + k];
            const PointCoef c = point_coef(rt, sn2, ttab[kCs * nth + k], ttab[kCot * nth + k], ttab[kTh * nth + k],
                                           rsq64(sigma2(rt, sn2)));
            lam = c.b;
            ath = c.ath;
            bth = c.bth;
            cr = c.cr;
            ci = c.ci;
        }
        val = lam * idx + sqrt(c2 * ath * idth * idth + c1 * fabs(bth) * idth + hypot(cr, ci));
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

// ---------------------------------------------------------------- horizon weights
// Weights of the four nodes j0 .. j0 + 3 for the value (w) and the
// rho-derivative (dw, already divided by dx) on the horizon.
struct HorizonWeights {
    double w[4], dw[4];
};

// ---------------------------------------------------------------- ring sample
// One waveform sample (and, in the hyperboloidal chart, one horizon sample)
// into ring slot counter % ring, then counter + 1.  The count lives in device
// memory, so the same launch recorded once into a graph writes each replay's
// samples to the slots that stepping launch by launch would.  One workgroup
// walks the theta rows.
__global__ __launch_bounds__(256) void sample_kernel(const double* __restrict__ u, long long plane, int nr, int nth,
                                                     int j_e, double* __restrict__ wave, double* __restrict__ hwave,
                                                     int j0, HorizonWeights W, long long ring,
                                                     unsigned long long* counter)
{
    __shared__ unsigned long long c;
    if (threadIdx.x == 0) c = *counter;
    __syncthreads();
    const long long slot = (long long)(c % (unsigned long long)ring);
    double* w = wave + (size_t)slot * nth * 2;
    double* hw = hwave ? hwave + (size_t)slot * nth * 4 : nullptr;
    for (int k = threadIdx.x; k < nth; k += blockDim.x) {
        const double* pr = u + (size_t)k * nr;
        const double* pi = pr + plane;
        w[2 * k] = pr[j_e];
        w[2 * k + 1] = pi[j_e];
        if (hw) {
            double vr = 0.0, vi = 0.0, dr = 0.0, di = 0.0;
            for (int q = 0; q < 4; ++q) {
                vr += W.w[q] * pr[j0 + q];
                vi += W.w[q] * pi[j0 + q];
                dr += W.dw[q] * pr[j0 + q];
                di += W.dw[q] * pi[j0 + q];
            }
            hw[4 * k] = vr;
            hw[4 * k + 1] = vi;
            hw[4 * k + 2] = dr;
            hw[4 * k + 3] = di;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) *counter = c + 1;
}

// ---------------------------------------------------------------- coefficient dump
// TEUK_X_COEFFS order: lam1, Re m3, Im m3, Re B~t, Im B~t, Re C~, Im C~, A~thth, B~th, lam2.
__global__ __launch_bounds__(256) void coef_dump_kernel(const double* __restrict__ rtab,
                                                        const double* __restrict__ ttab,
                                                        const double* __restrict__ ctab, int nr, int nth,
                                                        double* __restrict__ out)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long n = (long long)nr * nth;
    if (i >= n) return;
    if (ctab) {
        const int order[TEUK_NCOEF] = {kHLam1, kHM3r, kHM3i, kHBtr, kHBti, kHCr, kHCi, kHAth, kHBth, kHLam2};
        for (int q = 0; q < TEUK_NCOEF; ++q) out[q * n + i] = ctab[order[q] * n + i];
        return;
    }
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
    out[9 * n + i] = -c.b;
}

}  // namespace

int stage_grid(int weight_prec, bool first, int chart)
{
    // resident workgroups of one stage-kernel instantiation on the current device
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    hipError_t e = hipErrorInvalidValue;
#define TEUK_OCC(W, C)                                                                                            \
    if (weight_prec == W && chart == C)                                                                          \
        e = first ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, stage_kernel<W, kStageFirst, C>, kWave, 0) \
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, stage_kernel<W, kStageLater, C>, kWave, 0);
    TEUK_OCC(TEUK_W_FP64, kChartT)
    TEUK_OCC(TEUK_W_FP32, kChartT)
    TEUK_OCC(TEUK_W_FP16, kChartT)
    TEUK_OCC(TEUK_W_BF16, kChartT)
    TEUK_OCC(TEUK_W_FP64, kChartH)
    TEUK_OCC(TEUK_W_FP32, kChartH)
    TEUK_OCC(TEUK_W_FP16, kChartH)
    TEUK_OCC(TEUK_W_BF16, kChartH)
    TEUK_OCC(TEUK_W_FP64, kChartT4)
    TEUK_OCC(TEUK_W_FP32, kChartT4)
    TEUK_OCC(TEUK_W_FP16, kChartT4)
    TEUK_OCC(TEUK_W_BF16, kChartT4)
#undef TEUK_OCC
    if (e != hipSuccess || per_cu < 1) return 0;
    return cus * per_cu;
}

int pipe_grid(int weight_prec)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    hipError_t e = hipErrorInvalidValue;
    if (weight_prec == TEUK_W_FP64) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pipe_kernel<TEUK_W_FP64>, kWave, 0);
    if (weight_prec == TEUK_W_FP32) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pipe_kernel<TEUK_W_FP32>, kWave, 0);
    if (weight_prec == TEUK_W_FP16) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pipe_kernel<TEUK_W_FP16>, kWave, 0);
    if (weight_prec == TEUK_W_BF16) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pipe_kernel<TEUK_W_BF16>, kWave, 0);
    if (e != hipSuccess || per_cu < 1) return 0;
    return cus * per_cu;
}

int launch_pipe(const StageArgs st[3], long long* done, int* err, long long s0, int nsteps, int grid,
                long long spin_ticks, int weight_prec, void* stream)
{
    PipeArgs P;
    for (int i = 0; i < 3; ++i) P.st[i] = st[i];
    P.done = done;
    P.err = err;
    P.s0 = s0;
    P.nsteps = nsteps;
    P.tiles = st[0].nstrips * st[0].segs;
    P.spin_ticks = spin_ticks;
    if (grid < 1 || grid > P.tiles || nsteps < 1) return (int)hipErrorInvalidValue;
    void* args[] = {&P};
    const void* fn = nullptr;
    if (weight_prec == TEUK_W_FP64) fn = (const void*)pipe_kernel<TEUK_W_FP64>;
    if (weight_prec == TEUK_W_FP32) fn = (const void*)pipe_kernel<TEUK_W_FP32>;
    if (weight_prec == TEUK_W_FP16) fn = (const void*)pipe_kernel<TEUK_W_FP16>;
    if (weight_prec == TEUK_W_BF16) fn = (const void*)pipe_kernel<TEUK_W_BF16>;
    if (!fn) return (int)hipErrorInvalidValue;
    (void)hipGetLastError();
    const hipError_t e = hipLaunchCooperativeKernel(fn, dim3((unsigned)grid), dim3(kWave), args, 0, (hipStream_t)stream);
    if (e != hipSuccess) return (int)e;
    return (int)hipGetLastError();
}

int launch_stage(const StageArgs& a, int stage, int weight_prec, int chart, void* stream)
{
    const dim3 grid((unsigned)a.grid), block(kWave);
    hipStream_t st = (hipStream_t)stream;
    (void)hipGetLastError();   // report only what this launch does
    bool done = false;
#define TEUK_LAUNCH(W, C)                                                                      \
    if (weight_prec == W && chart == C) {                                                     \
        if (stage == 1)                                                                       \
            hipLaunchKernelGGL((stage_kernel<W, kStageFirst, C>), grid, block, 0, st, a);     \
        else if (stage == 0)                                                                  \
            hipLaunchKernelGGL((stage_kernel<W, kRhsOnly, C>), grid, block, 0, st, a);        \
        else if (stage == 4)                                                                  \
            hipLaunchKernelGGL((stage_kernel<W, kStageDual, C>), grid, block, 0, st, a);      \
        else                                                                                  \
            hipLaunchKernelGGL((stage_kernel<W, kStageLater, C>), grid, block, 0, st, a);     \
        done = true;                                                                          \
    }
    TEUK_LAUNCH(TEUK_W_FP64, kChartT)
    TEUK_LAUNCH(TEUK_W_FP32, kChartT)
    TEUK_LAUNCH(TEUK_W_FP16, kChartT)
    TEUK_LAUNCH(TEUK_W_BF16, kChartT)
    TEUK_LAUNCH(TEUK_W_FP64, kChartH)
    TEUK_LAUNCH(TEUK_W_FP32, kChartH)
    TEUK_LAUNCH(TEUK_W_FP16, kChartH)
    TEUK_LAUNCH(TEUK_W_BF16, kChartH)
    TEUK_LAUNCH(TEUK_W_FP64, kChartT4)
    TEUK_LAUNCH(TEUK_W_FP32, kChartT4)
    TEUK_LAUNCH(TEUK_W_FP16, kChartT4)
    TEUK_LAUNCH(TEUK_W_BF16, kChartT4)
#undef TEUK_LAUNCH
    if (!done) return (int)hipErrorInvalidValue;
    return (int)hipGetLastError();
}

int blocked_grid(int weight_prec)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    hipError_t e = hipErrorInvalidValue;
    if (weight_prec == TEUK_W_FP64)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, blocked_step_kernel<TEUK_W_FP64>, kBThreads, 0);
    else if (weight_prec == TEUK_W_FP32)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, blocked_step_kernel<TEUK_W_FP32>, kBThreads, 0);
    if (e != hipSuccess || per_cu < 1) return 0;
    return cus * per_cu;
}

int launch_blocked_step(const StageArgs& a, int weight_prec, void* stream)
{
    if (a.nr < 1 || a.nth < 1 || a.nstrips < 1 || a.segs < 1 || a.grid != a.nstrips * a.segs ||
        (long long)a.nstrips * kBW < a.nr || a.uk == a.out)
        return (int)hipErrorInvalidValue;
    (void)hipGetLastError();
    const dim3 grid((unsigned)a.grid), block(kBThreads);
    hipStream_t st = (hipStream_t)stream;
    if (weight_prec == TEUK_W_FP64)
        hipLaunchKernelGGL(blocked_step_kernel<TEUK_W_FP64>, grid, block, 0, st, a);
    else if (weight_prec == TEUK_W_FP32)
        hipLaunchKernelGGL(blocked_step_kernel<TEUK_W_FP32>, grid, block, 0, st, a);
    else
        return (int)hipErrorInvalidValue;
    return (int)hipGetLastError();
}

int launch_group_stage(const StageArgs* args, const long long* start, int nmem, long long tiles, int grid,
                       int stage, int weight_prec, int chart, void* stream)
{
    if (nmem < 1 || tiles < 1 || grid < 1 || stage < 1 || stage > 3) return (int)hipErrorInvalidValue;
    const dim3 g((unsigned)grid), block(kWave);
    hipStream_t st = (hipStream_t)stream;
    (void)hipGetLastError();
    bool done = false;
#define TEUK_GLAUNCH(W, C)                                                                                      \
    if (weight_prec == W && chart == C) {                                                                      \
        if (stage == 1)                                                                                        \
            hipLaunchKernelGGL((group_stage_kernel<W, kStageFirst, C>), g, block, 0, st, args, start, nmem, tiles); \
        else                                                                                                   \
            hipLaunchKernelGGL((group_stage_kernel<W, kStageLater, C>), g, block, 0, st, args, start, nmem, tiles); \
        done = true;                                                                                           \
    }
    TEUK_GLAUNCH(TEUK_W_FP64, kChartT)
    TEUK_GLAUNCH(TEUK_W_FP32, kChartT)
    TEUK_GLAUNCH(TEUK_W_FP16, kChartT)
    TEUK_GLAUNCH(TEUK_W_BF16, kChartT)
    TEUK_GLAUNCH(TEUK_W_FP64, kChartH)
    TEUK_GLAUNCH(TEUK_W_FP32, kChartH)
    TEUK_GLAUNCH(TEUK_W_FP16, kChartH)
    TEUK_GLAUNCH(TEUK_W_BF16, kChartH)
    TEUK_GLAUNCH(TEUK_W_FP64, kChartT4)
    TEUK_GLAUNCH(TEUK_W_FP32, kChartT4)
    TEUK_GLAUNCH(TEUK_W_FP16, kChartT4)
    TEUK_GLAUNCH(TEUK_W_BF16, kChartT4)
#undef TEUK_GLAUNCH
    if (!done) return (int)hipErrorInvalidValue;
    return (int)hipGetLastError();
}

int launch_dt_bound(const double* rtab, const double* ttab, const double* ctab, int nr, int nth, double dx,
                    double dth, int theta_order, unsigned long long* cell, void* stream)
{
    // Largest moduli of the Fourier symbols of dth^2 D2 and dth D1.  Second
    // order: |2 cos xi - 2| <= 4 and |sin xi| <= 1.  Fourth order:
    // |(32 cos xi - 2 cos 2xi - 30)/12| <= 16/3 (at xi = pi), and
    // (8 sin xi - sin 2xi)/6 peaks where 8 cos xi = 2 cos 2xi, i.e. at
    // cos xi = 1 - sqrt(3/2), with the value sin xi (4 - cos xi)/3.
    double c2 = 4.0, c1 = 1.0;
    if (theta_order == 4) {
        const double cx = 1.0 - std::sqrt(1.5);
        c2 = 16.0 / 3.0;
        c1 = std::sqrt(1.0 - cx * cx) * (4.0 - cx) / 3.0;
    }
    (void)hipGetLastError();
    const long long n = (long long)nr * nth;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(dt_bound_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, rtab, ttab, ctab, nr, nth,
                       1.0 / dx, 1.0 / dth, c2, c1, cell);
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

int launch_sample(const double* u, long long plane, int nr, int nth, int j_e, double* wave, double* hwave, int j0,
                  const double* w, const double* dw, long long ring, unsigned long long* counter, void* stream)
{
    if (j_e < 0 || j_e >= nr || ring < 1) return (int)hipErrorInvalidValue;
    HorizonWeights W{};
    if (hwave) {
        if (j0 < 0 || j0 + 3 > nr - 1) return (int)hipErrorInvalidValue;
        for (int q = 0; q < 4; ++q) {
            W.w[q] = w[q];
            W.dw[q] = dw[q];
        }
    }
    (void)hipGetLastError();
    hipLaunchKernelGGL(sample_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream, u, plane, nr, nth, j_e, wave,
                       hwave, j0, W, ring, counter);
    return (int)hipGetLastError();
}

int launch_coef_dump(const double* rtab, const double* ttab, const double* ctab, int nr, int nth, double* out,
                     void* stream)
{
    (void)hipGetLastError();
    const long long n = (long long)nr * nth;
    hipLaunchKernelGGL(coef_dump_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       rtab, ttab, ctab, nr, nth, out);
    return (int)hipGetLastError();
}

}  // namespace teuk
