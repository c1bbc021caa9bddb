// Hopping-term launches for the FP64 operator rebuilt from hi/lo FP32-12 planes.
#include "dslash_kernel.h"

namespace rhmc {

hipError_t launch_dslash64hl(const HiLoLink* u, int nlinks, const DslashArgs<double2>& a,
                             int mode, hipStream_t s) {
    switch (mode) {
        case kModeD: return dispatch<double2, HiLoLink, kModeD>(u, nlinks, a, s);
        case kModeA: return dispatch<double2, HiLoLink, kModeA>(u, nlinks, a, s);
        default: return dispatch<double2, HiLoLink, kModeResid>(u, nlinks, a, s);
    }
}

}  // namespace rhmc
