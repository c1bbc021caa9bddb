// Launchers of the gauge-sector kernels (gauge.hip).
//
// Momenta are FP64 arrays [8][4*V]: component a of omega (H = sum_a omega^a
// T^a, T^a = lambda^a / 2), then the link index k = (2*mu + parity)*Vh + eo
// of the link storages.
#pragma once

#include "common.h"

namespace rhmc {

// mom -= eps * c_g with c_g^a = i Tr(T^a F_g), F_g = -(beta/3) TA(U Sigma)
hipError_t launch_gauge_force_mom(const rhmc_gauge* g, double beta, double eps, double* mom,
                                  hipStream_t s);
// U -> reunitarised exp(i eps H) U in every link storage of the gauge object
hipError_t launch_update_links(rhmc_gauge* g, double eps, const double* mom, hipStream_t s);
// Block sums of sum over plaquettes of (1 - Re Tr P / 3) into partial[0 .. nblk-1]
int plaquette_blocks(const rhmc_gauge* g);
hipError_t launch_plaquette(const rhmc_gauge* g, double* partial, hipStream_t s);
// Canonical FP64 links out[lex][mu][3][3] (complex) from the FP64 storage
hipError_t launch_get_links(const rhmc_gauge* g, double2* out, hipStream_t s);

}  // namespace rhmc
