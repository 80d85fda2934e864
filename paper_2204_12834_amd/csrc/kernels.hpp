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

}  // namespace poba
