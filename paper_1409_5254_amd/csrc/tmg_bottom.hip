// Bottom-of-hierarchy kernel (k_bottom): every level up to a cap in one
// work-group, resident in LDS; and the columns of the dense operator of a
// W-cycle's bottom visits (k_dense_cols), which run the same visits.  This
// file is compiled once per P (-DTMG_BOTTOM_P=1..6) so that the
// instantiations build in parallel.
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

// Column `col` of the dense bottom operator, one work-group per column: the
// level's right-hand side is the unit load e_col, and gamma visits of the
// level run from zero in LDS exactly as k_bottom's launches run them (the
// iterate kept between visits, the right-hand side of the level untouched
// by them).  The column goes to row-major D.
template <int P, int NT, bool BW>
__global__ __launch_bounds__(NT) void k_dense_cols(DenseColArgs a)
{
    // the levels sit in LDS in physical slab order (BW: Bottom's steps map
    // logical slabs onto it), so the unit load and the column are physical
    using B = Bottom<P, BW, NT>;
    constexpr int STRIDE = B::STRIDE;
    __shared__ BottomLds<P, NT> sm;
    const int64_t col = blockIdx.x;
    const int64_t N = a.N, n = N * P;
    const int lb = a.level;
    const int ntab = (a.Lc - lb + 1) * STRIDE;
    for (int i = threadIdx.x; i < ntab + 2 * P * P; i += NT) {
        if (i < ntab) sm.tab[i] = a.tab[(int64_t)(lb + i / STRIDE) * a.tab_level + i % STRIDE];
        else sm.R[i - ntab] = a.R[i - ntab];
    }
    for (int64_t i = threadIdx.x; i < n; i += NT) {
        sm.f[i] = i == col ? 1.0 : 0.0;
        sm.x[i] = 0.0;
    }
    __syncthreads();
    int lw = lb;
    while ((N >> (lw - lb)) > B::WAVE_SLABS) ++lw;
    const B b{sm, lb, N, a.Lc, lw, a.nu1, a.nu2, a.gamma};
    for (int g = 0; g < a.gamma; ++g) {
        if (lb >= lw) {
            if (threadIdx.x < 64) b.template visit<1>(lb, g == 0);
        } else {
            b.template visit<B::NW>(lb, g == 0);
        }
        __syncthreads();
    }
    for (int64_t i = threadIdx.x; i < n; i += NT) a.D[i * n + col] = sm.x[i];
}

template <int PP>
hipError_t launch_dense_cols_p(const DenseColArgs &a, hipStream_t s)
{
    constexpr int NT = bottom_threads(PP);
    if (a.N < 1 || a.N > NT * bottom_slabs(PP) || a.Lc <= a.level ||
        a.Lc - a.level + 1 > kBottomMaxLevels)
        return hipErrorInvalidValue;
    if (a.backward)
        hipLaunchKernelGGL((k_dense_cols<PP, NT, true>), dim3((unsigned)(a.N * PP)), dim3(NT), 0, s, a);
    else
        hipLaunchKernelGGL((k_dense_cols<PP, NT, false>), dim3((unsigned)(a.N * PP)), dim3(NT), 0, s, a);
    return hipGetLastError();
}

template hipError_t launch_bottom_p<double, TMG_BOTTOM_P>(bool, const BottomArgsT<double> &, int,
                                                          hipStream_t);
template hipError_t launch_bottom_p<float, TMG_BOTTOM_P>(bool, const BottomArgsT<float> &, int,
                                                         hipStream_t);

template hipError_t launch_dense_cols_p<TMG_BOTTOM_P>(const DenseColArgs &, hipStream_t);

}  // namespace tmg
