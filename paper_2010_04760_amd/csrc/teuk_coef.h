// Chart-T coefficient tables and their per-point evaluation.
//
// The divided second-order Teukolsky equation (paper eq. final, obtained from
// eq. teuk0 with Psi = exp(i m phi~) r^-(2s+1) Phi and x = r_*, Sec. 2.1-2.3)
// has coefficients that all share the factor w = 1/Sigma^2,
//     Sigma^2 = (r^2+a^2)^2 - a^2 Delta sin^2(theta),
// times a polynomial in (cos, sin^2) with radial coefficients.  With
// q = 2s+1, ra2 = r^2+a^2 and v = 1/Sigma:
//     b       = ra2 v                                          (speed of Phi, pi: +b, -b)
//     A~thth  = Delta w,            B~th = A~thth cot(theta)
//     B~t     = w [T0 + i (T1 + T2 cos)]
//         T0 = -2s (r Delta - M (r^2 - a^2)),  T1 = -4 M a m r,  T2 = -2 s a Delta
//     C~      = w [A0 - Delta Th(theta) + i A1],  Th = (m + s cos)^2 / sin^2
//         A0 = Delta (q(q+1) Delta/r^2 - 2(s+1) q (r-M)/r + s),
//         A1 = -2 m a q Delta / r + 4 s m a (r - M)
//     B~x     = w [X0 + i X1]
//         X0 = -2 q Delta ra2 / r + 2 r Delta + 2 s (r-M) ra2,   X1 = 2 m a ra2
//     b d_x b = w [G0 - w (G1 - G2 sin^2)]
//         G0 = 2 r Delta,  G1 = 2 r Delta ra2^2,  G2 = Delta ra2 a^2 (r - M)
//     m3      = b d_x b + b B~t - B~x                          (Sec. 2.3 reduction)
//             = b B~t + w [H0 - w (G1 - G2 sin^2)] - i w X1,   H0 = G0 - X0.
// The radial factors are tabulated once per radial node on the host in FP64
// (one row per factor, radial index fastest); the polar factors once per
// theta node.  The per-point combination costs one reciprocal square root and
// about thirty multiply-adds, instead of streaming nine doubles per point.
#pragma once

#if defined(__HIPCC__)
#define TEUK_HD __host__ __device__
#else
#define TEUK_HD
#endif

namespace teuk {

// Radial table rows, [kNRT][nr].
enum RadialRow : int {
    kDl = 0,   // Delta
    kP,        // ra2^2
    kQ,        // a^2 Delta
    kRa2,      // r^2 + a^2
    kT0, kT1, kT2,
    kA0, kA1,
    kH0, kG1, kG2,
    kX1,
    kNRT
};

// Polar table rows, [kNTT][ntheta].
enum PolarRow : int {
    kSn2 = 0,  // sin^2(theta)
    kCs,       // cos(theta)
    kCot,      // cot(theta)
    kTh,       // (m + s cos)^2 / sin^2
    kNTT
};

// Chart-H per-point coefficient table, [kNCH][ntheta][nr] (streamed by the
// stage kernel: the hyperboloidal coefficients have no cheap on-chip form).
enum ChartHPlane : int {
    kHLam1 = 0,  // lam1 = b, speed of the Phi rows
    kHLam2,      // lam2, speed of the pi rows
    kHM3r, kHM3i,
    kHBtr, kHBti,
    kHCr, kHCi,
    kHAth, kHBth,
    kNCH
};

struct PointCoef {
    double b, m3r, m3i, btr, bti, cr, ci, ath, bth;
};

// Sigma^2 at one point.
TEUK_HD inline double sigma2(const double* rt, double sn2) { return rt[kP] - rt[kQ] * sn2; }

// Per-point coefficients from the radial factors rt[kNRT], the polar factors
// and v = 1/Sigma (the caller chooses how to form the reciprocal square root).
TEUK_HD inline PointCoef point_coef(const double* rt, double sn2, double cs, double cot, double th,
                                    double v)
{
    PointCoef c;
    const double w = v * v;
    c.b = rt[kRa2] * v;
    c.ath = rt[kDl] * w;
    c.bth = c.ath * cot;
    c.btr = w * rt[kT0];
    c.bti = w * (rt[kT1] + rt[kT2] * cs);
    c.cr = w * (rt[kA0] - rt[kDl] * th);
    c.ci = w * rt[kA1];
    c.m3r = c.b * c.btr + w * (rt[kH0] - w * (rt[kG1] - rt[kG2] * sn2));
    c.m3i = c.b * c.bti - w * rt[kX1];
    return c;
}

}  // namespace teuk
