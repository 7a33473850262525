// Host tables of the double-double state path (tortoise chart).  Plain C++:
// included by teuk_background_dd.cpp (host compiler, binary128) and by the
// HIP sources.
#pragma once

#include <string>
#include <vector>

#include "teuk.h"

namespace teuk {

// Per-point coefficient planes of the double-double table, [kNDD][ntheta][nr]
// (hi, lo) pairs: b, Re m3, Im m3, Re B~t, Im B~t, Re C~, Im C~, A~thth, B~th
// (lam1 = b and lam2 = -b in the tortoise chart).
enum DDPlane : int { kDB = 0, kDM3r, kDM3i, kDBtr, kDBti, kDCr, kDCi, kDAth, kDBth, kNDD };

// Double-double constants of a solve, each a (hi, lo) pair.
struct DDScalars {
    double inv_dx[2];       // 1 / dx
    double ih1[2], ih2[2];  // 1 / (2 dtheta), 1 / dtheta^2
    double third[2], two_thirds[2];
    double d[3][2];         // WENO5 linear weights 1/10, 6/10, 3/10
    double c13_3[2];        // 13 / 3
    double sixth[2];        // 1 / 6
};

// ln(r - r_+) at tortoise coordinate x, solved in FP64 (teuk_background.cpp).
double tortoise_lny(const teuk_config& c, double x);

// Build the double-double table (2 * kNDD * ntheta * nr doubles) and the
// constants for a validated chart-T configuration, in binary128.  False (with
// err) if a node lies too close to the horizon.
bool build_tables_dd(const teuk_config& c, std::vector<double>& dtab, DDScalars* sc, std::string& err);

}  // namespace teuk
