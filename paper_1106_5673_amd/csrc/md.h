// Molecular-dynamics driver (md.hip) used by the C ABI.
#pragma once

#include "common.h"

namespace rhmc {

rhmc_status gauge_action(rhmc_gauge* g, double beta, double* S, hipStream_t s);
rhmc_status kinetic(rhmc_gauge* g, const double* mom, double* K, hipStream_t s);
rhmc_status md_integrate(rhmc_gauge* g, const rhmc_md_params& p, int npf, const double2* phi,
                         double* mom, rhmc_md_stats* stats, hipStream_t s);
rhmc_status trajectory(rhmc_gauge* g, const rhmc_hmc_params& p, int npf, const double2* R,
                       double* mom, double u, rhmc_trajectory_stats* stats, hipStream_t s);

}  // namespace rhmc
