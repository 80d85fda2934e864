// Host-side entry points shared between translation units of the library.
#pragma once

#include "common.hpp"

namespace poba {

// Linearisation passes; gate (device, may be null) skips the work when 0.
// F of each problem goes to cost_out[j] and, for active problems, to st[j]
// (either may be null).
poba_status launch_linearize(Problem* p, const double* cams, const double* lms, const int32_t* gate,
                             double* cost_out, poba_lm_state* st, hipStream_t s);

// Per-camera records of cams (rotation data) into out (b.cam_rec for a trial
// state, b.lin_rec for the linearisation).
poba_status launch_cam_prep(Problem* p, const double* cams, const int32_t* gate, double* out, hipStream_t s);

// Damped inverses, reduced right-hand side, power series and
// back-substitution, each problem with the damping in its pctl[j].lambda;
// problems that are not active are skipped.  Writes dx_cams / dx_lms (active
// problems) and info[j] (device, may be null).
// rhs_p / rhs_l (device, may be null) replace b_p / b_l of the linearisation.
poba_status launch_solve(Problem* p, int m, double eps, double* dx_cams, double* dx_lms, poba_solve_info* info,
                         hipStream_t s, const double* rhs_p = nullptr, const double* rhs_l = nullptr);

// Makes every problem active with damping lam and clears the series flags.
poba_status launch_begin_solve(Problem* p, double lam, hipStream_t s);

// Building blocks of the conjugate-gradient solver (each covers the active
// problems of the handle):
//  - damped inverses and b~ (into b.bt), as a power solve computes them;
//  - orders 1..m of the power series from the current term (b.v with its
//    gather copy or folded data) into the sum b.x;
//  - v into the gather copy or folded data of the series' current term;
//  - the float64 product W V_lambda^-1 W^T x as per-piece partial sums
//    (b.part, 9 per piece, summed per camera over cam_piece);
//  - dx_l = -V^-1 (b_l + W^T b.x) and dx_cams = b.x.
poba_status launch_solve_prepare(Problem* p, hipStream_t s);
poba_status launch_series_orders(Problem* p, int m, hipStream_t s);
poba_status launch_load_v(Problem* p, const double* v, hipStream_t s);
poba_status launch_schur_part64(Problem* p, const double* x, hipStream_t s);
poba_status launch_backsub_from_x(Problem* p, double* dx_cams, double* dx_lms, hipStream_t s);

}  // namespace poba
