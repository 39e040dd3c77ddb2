// The dense operator of a W-cycle's bottom visits: its rows' lengths and
// its application (the columns are built in tmg_bottom.hip).
#include <hip/hip_runtime.h>

#include "tmg_kernels.h"

namespace tmg {

namespace {

constexpr int kDenseThreads = 256;          // four wavefronts
constexpr int kDenseWaves = kDenseThreads / 64;
constexpr int kDenseRows = 4;               // rows per work-group (one load of r feeds them)
// column pairs per thread that cover the largest operator's rows
constexpr int kDensePasses = (int)(kDenseMaxN / (2 * kDenseThreads));

// len[row] = 1 + the last column with a nonzero entry: one wavefront per row.
__global__ __launch_bounds__(kDenseThreads) void k_dense_len(const double *__restrict__ D, int64_t n,
                                                          int *__restrict__ len)
{
    const int64_t row = (int64_t)blockIdx.x * kDenseWaves + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    const double *d = D + row * n;
    int last = -1;
    for (int64_t c = lane; c < n; c += 64)
        if (d[c] != 0.0) last = (int)c;
    for (int o = 32; o > 0; o >>= 1) last = max(last, __shfl_xor(last, o));
    if (lane == 0) len[row] = last + 1;
}

// x = D r: kDenseRows rows per work-group.  Thread t takes the column pairs
// (c, c + 1), c = 2 t + 2 kDenseThreads i, of every row: every load is
// issued first (16-byte loads; VEC = false: one column at a time, for an odd
// n or unaligned arrays), then the thread sums its products in column
// order, and the threads' sums of a row are combined in a fixed order
// (butterfly within each wavefront, the wavefronts in turn), so every run
// gives the same bits.  Pairs at or past a row's length are not read (the
// entries there are zero; a pair that straddles the length adds 0 r_c).
template <bool VEC>
__global__ __launch_bounds__(kDenseThreads) void k_dense_apply(const double *__restrict__ D,
                                                            const int *__restrict__ len,
                                                            const double *__restrict__ r,
                                                            double *__restrict__ x, int64_t n,
                                                            const InstState *__restrict__ st)
{
    if (st && st->done) return;
    __shared__ double red[kDenseRows][kDenseWaves];
    const int64_t row0 = (int64_t)blockIdx.x * kDenseRows;
    const int t = threadIdx.x;
    int m[kDenseRows];
    int mm = 0;
#pragma unroll
    for (int q = 0; q < kDenseRows; ++q) {
        m[q] = row0 + q < n ? len[row0 + q] : 0;
        mm = max(mm, m[q]);
    }
    double rv[kDensePasses][2], dv[kDenseRows][kDensePasses][2];
#pragma unroll
    for (int i = 0; i < kDensePasses; ++i) {
        const int64_t c = 2 * t + 2 * kDenseThreads * i;
        if (VEC) {
            double2 a = make_double2(0.0, 0.0);
            if (c < mm) a = *reinterpret_cast<const double2 *>(r + c);
            rv[i][0] = a.x;
            rv[i][1] = a.y;
#pragma unroll
            for (int q = 0; q < kDenseRows; ++q) {
                double2 d = make_double2(0.0, 0.0);
                if (c < m[q]) d = *reinterpret_cast<const double2 *>(D + (row0 + q) * n + c);
                dv[q][i][0] = d.x;
                dv[q][i][1] = d.y;
            }
        } else {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                rv[i][h] = c + h < mm ? r[c + h] : 0.0;
#pragma unroll
                for (int q = 0; q < kDenseRows; ++q)
                    dv[q][i][h] = c + h < m[q] ? D[(row0 + q) * n + c + h] : 0.0;
            }
        }
    }
    double acc[kDenseRows];
#pragma unroll
    for (int q = 0; q < kDenseRows; ++q) {
        acc[q] = 0.0;
#pragma unroll
        for (int i = 0; i < kDensePasses; ++i) {
            acc[q] = fma(dv[q][i][0], rv[i][0], acc[q]);
            acc[q] = fma(dv[q][i][1], rv[i][1], acc[q]);
        }
    }
    const int lane = t & 63, w = t >> 6;
#pragma unroll
    for (int q = 0; q < kDenseRows; ++q) {
        double v = acc[q];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0) red[q][w] = v;
    }
    __syncthreads();
    if (t < kDenseRows && row0 + t < n) {
        double v = red[t][0];
#pragma unroll
        for (int k = 1; k < kDenseWaves; ++k) v += red[t][k];
        x[row0 + t] = v;
    }
}

}  // namespace

hipError_t launch_dense_cols(int P, const DenseColArgs &a, hipStream_t s)
{
    TMG_DISPATCH_P(P, { return launch_dense_cols_p<PP>(a, s); })
    return hipErrorInvalidValue;
}

hipError_t launch_dense_len(const double *D, int64_t n, int *len, hipStream_t s)
{
    if (n < 1 || n > kDenseMaxN) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_dense_len, dim3((unsigned)((n + kDenseWaves - 1) / kDenseWaves)),
                       dim3(kDenseThreads), 0, s, D, n, len);
    return hipGetLastError();
}

hipError_t launch_dense_apply(const double *D, const int *len, const double *r, double *x,
                              int64_t n, const InstState *st, hipStream_t s)
{
    if (n < 1 || n > kDenseMaxN) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((n + kDenseRows - 1) / kDenseRows)), block(kDenseThreads);
    const bool vec = n % 2 == 0 && ((reinterpret_cast<uintptr_t>(D) | reinterpret_cast<uintptr_t>(r)) & 15) == 0;
    if (vec) hipLaunchKernelGGL(k_dense_apply<true>, grid, block, 0, s, D, len, r, x, n, st);
    else hipLaunchKernelGGL(k_dense_apply<false>, grid, block, 0, s, D, len, r, x, n, st);
    return hipGetLastError();
}

}  // namespace tmg
