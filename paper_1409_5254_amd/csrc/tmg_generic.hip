// Generic kernels (tmg_generic.h) for one P = TMG_GEN_P: this file is
// compiled once per P (-DTMG_GEN_P=1..kMaxP) so that the instantiations
// build in parallel.
#include <hip/hip_runtime.h>

#include "tmg_generic.h"

#ifndef TMG_GEN_P
#error "compile once per P with -DTMG_GEN_P=<1..21>"
#endif

namespace tmg {

template <int PP>
hipError_t launch_gleg_p(bool backward, const LegArgsT<double> &a, int64_t ntiles, hipStream_t s)
{
    const dim3 grid((unsigned)ntiles), block(kGenThreads);
    if (backward) hipLaunchKernelGGL((k_gleg<PP, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_gleg<PP, false>), grid, block, 0, s, a);
    return hipGetLastError();
}

template <int PP>
hipError_t launch_gbottom_p(bool backward, const BottomArgsT<double> &a, int ninst, hipStream_t s)
{
    const dim3 grid(ninst), block(kGenThreads);
    if (a.visit) {
        if (backward) hipLaunchKernelGGL((k_gvisit<PP, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_gvisit<PP, false>), grid, block, 0, s, a);
    } else {
        if (backward) hipLaunchKernelGGL((k_gbottom<PP, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_gbottom<PP, false>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

template <int PP>
hipError_t launch_gdense_cols_p(const DenseColArgs &a, hipStream_t s)
{
    if (a.N < 1 || a.N > gbottom_max(PP) || a.Lc <= a.level || a.N * PP > kDenseMaxN)
        return hipErrorInvalidValue;
    if (a.backward)
        hipLaunchKernelGGL((k_gdense_cols<PP, true>), dim3((unsigned)(a.N * PP)), dim3(kGenThreads), 0, s, a);
    else
        hipLaunchKernelGGL((k_gdense_cols<PP, false>), dim3((unsigned)(a.N * PP)), dim3(kGenThreads), 0, s, a);
    return hipGetLastError();
}

template <int PP>
hipError_t launch_gcoarse_p(bool backward, const CoarseArgs &a, int periodic, int ninst,
                            hipStream_t s)
{
    const dim3 grid(ninst), block(kGenThreads);
    if (backward) hipLaunchKernelGGL((k_gcoarse<PP, true>), grid, block, 0, s, a, periodic);
    else hipLaunchKernelGGL((k_gcoarse<PP, false>), grid, block, 0, s, a, periodic);
    return hipGetLastError();
}

template hipError_t launch_gleg_p<TMG_GEN_P>(bool, const LegArgsT<double> &, int64_t, hipStream_t);
template hipError_t launch_gbottom_p<TMG_GEN_P>(bool, const BottomArgsT<double> &, int,
                                                hipStream_t);
template hipError_t launch_gcoarse_p<TMG_GEN_P>(bool, const CoarseArgs &, int, int, hipStream_t);
template hipError_t launch_gdense_cols_p<TMG_GEN_P>(const DenseColArgs &, hipStream_t);

}  // namespace tmg
