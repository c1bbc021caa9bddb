// Entry points of the solver driver (solver.hip) used by the C ABI.
#pragma once

#include "common.h"

namespace rhmc {

// x[r][i] (element offset r*x_sys + i*x_shift) = (A + shifts[i])^-1 b[r]
rhmc_status multishift(rhmc_gauge* g, double m, int nshift, const double* shifts, int nrhs,
                       const double2* b, double2* x, size_t x_sys, size_t x_shift,
                       const rhmc_solver_params& prm, rhmc_solver_stats* stats, hipStream_t s);

// y[r] = alpha0 b[r] + sum_i alpha_i (A + beta_i)^-1 b[r]
rhmc_status rational(rhmc_gauge* g, double m, const rhmc_rational* rat, int nrhs,
                     const double2* b, double2* y, const rhmc_solver_params& prm,
                     rhmc_solver_stats* stats, hipStream_t s);

// S[r] = Re <phi[r], r(A) phi[r]> (host array), r(A) as in rational()
rhmc_status pf_action(rhmc_gauge* g, double m, const rhmc_rational* rat, int nrhs,
                      const double2* phi, double* S, const rhmc_solver_params& prm,
                      rhmc_solver_stats* stats, hipStream_t s);

// force[lex][mu] = TA(U M) of S = sum_r phi[r]^dagger r(A) phi[r] (force.hip); with
// mom non-null, mom^a -= eps * i Tr(T^a F) instead and force is not written
rhmc_status pf_force(rhmc_gauge* g, double m, const rhmc_rational* rat, int nrhs,
                     const double2* phi, double2* force, double* mom, double eps,
                     const rhmc_solver_params& prm, rhmc_solver_stats* stats, hipStream_t s);

}  // namespace rhmc
