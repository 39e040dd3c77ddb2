// Bottom-of-hierarchy kernel (k_bottom): every level up to a cap in one
// work-group, resident in LDS.  This file is compiled once per P
// (-DTMG_BOTTOM_P=1..6) so that the instantiations build in parallel.
#include <hip/hip_runtime.h>

#include "tmg_kernels.h"

#ifndef TMG_BOTTOM_P
#error "compile once per P with -DTMG_BOTTOM_P=<1..6>"
#endif

namespace tmg {

template <typename TIO, int PP>
hipError_t launch_bottom_p(bool backward, const BottomArgsT<TIO> &a, int ninst, hipStream_t s)
{
    const dim3 grid(ninst), block(a.small ? 64 : bottom_threads(PP));
#define TMG_BOTTOM(NT)                                                                            \
    if (a.lbs) {                                                                                  \
        if (backward) hipLaunchKernelGGL((k_bottom<PP, true, TIO, true, NT>), grid, block, 0, s, a); \
        else hipLaunchKernelGGL((k_bottom<PP, false, TIO, true, NT>), grid, block, 0, s, a);      \
    } else {                                                                                      \
        if (backward) hipLaunchKernelGGL((k_bottom<PP, true, TIO, false, NT>), grid, block, 0, s, a); \
        else hipLaunchKernelGGL((k_bottom<PP, false, TIO, false, NT>), grid, block, 0, s, a);     \
    }
    if (a.small) {
        TMG_BOTTOM(64)
    } else {
        TMG_BOTTOM(bottom_threads(PP))
    }
#undef TMG_BOTTOM
    return hipGetLastError();
}

template hipError_t launch_bottom_p<double, TMG_BOTTOM_P>(bool, const BottomArgsT<double> &, int,
                                                          hipStream_t);
template hipError_t launch_bottom_p<float, TMG_BOTTOM_P>(bool, const BottomArgsT<float> &, int,
                                                         hipStream_t);

}  // namespace tmg
