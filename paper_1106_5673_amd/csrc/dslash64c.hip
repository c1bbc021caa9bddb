// Hopping-term launches for FP64-12 links (rows 1-2 in FP64, row 3 rebuilt).
#include "dslash_kernel.h"

namespace rhmc {

hipError_t launch_dslash64c(const Fp64x12Link* u, int nlinks, const DslashArgs<double2>& a,
                            int mode, hipStream_t s) {
    switch (mode) {
        case kModeD: return dispatch<double2, Fp64x12Link, kModeD>(u, nlinks, a, s);
        case kModeA: return dispatch<double2, Fp64x12Link, kModeA>(u, nlinks, a, s);
        default: return dispatch<double2, Fp64x12Link, kModeResid>(u, nlinks, a, s);
    }
}

}  // namespace rhmc
