// Launch arguments of the pseudofermion-force kernel (force.hip).
#pragma once

#include "common.h"

namespace rhmc {

struct ForceArgs {
    Geom g;
    const double2* x;        // shifted solutions, even sites: [nrhs][npole][3][Vh]
    const double2* y;        // D_oe x, odd sites: [nrhs][npole][3][Vh]
    int nrhs, npole;
    double alpha[kMaxShift];
    double2* out;            // F, [Lt][Lz][Ly][Lx][4][3][3] complex (lexicographic sites)
    int accumulate;          // add to out instead of overwriting it
    double* mom;             // if non-null: mom^a -= eps * i Tr(T^a F) ([8][4*V], link
    double eps;              // index (2*mu + parity)*Vh + eo) and out is not written
};

hipError_t launch_force(const rhmc_gauge* g, const ForceArgs& a, hipStream_t s);

}  // namespace rhmc
