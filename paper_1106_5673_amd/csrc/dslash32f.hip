// Hopping-term launches for FP32-18 links (all 18 reals stored, no reconstruction).
#include "dslash_kernel.h"

namespace rhmc {

hipError_t launch_dslash32f(const Fp32x18Link* u, int nlinks, const DslashArgs<float2>& a,
                            int mode, hipStream_t s) {
    switch (mode) {
        case kModeD: return dispatch<float2, Fp32x18Link, kModeD>(u, nlinks, a, s);
        default: return dispatch<float2, Fp32x18Link, kModeA>(u, nlinks, a, s);
    }
}

}  // namespace rhmc
