// Level-0 pass of the FP32-inner defect correction (k_mix).
#include <hip/hip_runtime.h>

#include "tmg_kernels.h"

namespace tmg {

hipError_t launch_mix(int P, bool backward, const MixArgs &a, int64_t ntiles, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    TMG_DISPATCH_P(P, {
        if (backward) hipLaunchKernelGGL((k_mix<PP, true>), dim3((unsigned)ntiles), dim3(kLegThreads), 0, s, a);
        else hipLaunchKernelGGL((k_mix<PP, false>), dim3((unsigned)ntiles), dim3(kLegThreads), 0, s, a);
    })
    return hipGetLastError();
}

}  // namespace tmg
