// Hopping-term launches for FP64-18 links (the reference FP64 operator).
#include "dslash_kernel.h"

namespace rhmc {

hipError_t launch_dslash64(const double2* u64, int nlinks, const DslashArgs<double2>& a, int mode,
                           hipStream_t s) {
    switch (mode) {
        case kModeD: return dispatch<double2, double2, kModeD>(u64, nlinks, a, s);
        case kModeA: return dispatch<double2, double2, kModeA>(u64, nlinks, a, s);
        default: return dispatch<double2, double2, kModeResid>(u64, nlinks, a, s);
    }
}

}  // namespace rhmc
