// The dense operator of a W-cycle's bottom visits: its rows' windows and
// its application (the columns are built in tmg_bottom.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>

#include "tmg_kernels.h"

namespace tmg {

namespace {

constexpr int kDenseThreads = 256;          // four wavefronts
constexpr int kDenseWaves = kDenseThreads / 64;
// rows per work-group of the product's wide form (one load of r feeds
// them); spans of up to kDenseWaveSpan columns take one row per wavefront
constexpr int kDenseRows = 4;
constexpr int kDenseWaveSpan = 4 * 2 * 64;
// column pairs per thread that cover the largest operator's rows
constexpr int kDensePasses = (int)(kDenseMaxN / (2 * kDenseThreads));
// passes that cover n columns (1, 2, 4 or 8: fewer registers, more
// work-groups resident for the short operators)
inline int dense_passes(int64_t n)
{
    const int64_t q = (n + 2 * kDenseThreads - 1) / (2 * kDenseThreads);
    return q <= 1 ? 1 : q <= 2 ? 2 : q <= 4 ? 4 : kDensePasses;
}

// Stands in for a missing state (never finished), so that the flag's load
// needs no branch.
__device__ InstState g_no_state{};

// Row windows (see launch_dense_window): one wavefront per row, a pass for
// the row's largest magnitude, a pass for the first and last column above
// the drop threshold.
__global__ __launch_bounds__(kDenseThreads) void k_dense_window(const double *__restrict__ D,
                                                             int64_t n, int *__restrict__ win)
{
    const int64_t row = (int64_t)blockIdx.x * kDenseWaves + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    const double *d = D + row * n;
    double M = 0.0;
    int bad = 0;
    for (int64_t c = lane; c < n; c += 64) {
        if (!isfinite(d[c])) bad = 1;
        else M = fmax(M, fabs(d[c]));
    }
    for (int o = 32; o > 0; o >>= 1) {
        M = fmax(M, __shfl_xor(M, o));
        bad |= __shfl_xor(bad, o);
    }
    const double thr = ldexp(M, kDenseDropExp);
    int first = (int)n, last = -1;
    for (int64_t c = lane; c < n; c += 64)
        if (fabs(d[c]) > thr) {
            first = min(first, (int)c);
            last = (int)c;
        }
    for (int o = 32; o > 0; o >>= 1) {
        first = min(first, __shfl_xor(first, o));
        last = max(last, __shfl_xor(last, o));
    }
    if (lane == 0) {
        int s = 0, e = 0;
        if (bad) {
            e = (int)n;
        } else if (last >= 0) {
            s = first & ~1;
            e = last + 1;
        }
        win[2 * row] = s;
        win[2 * row + 1] = e;
    }
}

// x = D r: ROWS rows per work-group of THREADS threads.  Thread t takes
// the column pairs (c, c + 1), c = c0 + 2 t + 2 THREADS i, from the smallest window
// start c0 of the group's rows, and of each row the pairs inside its window:
// every load is issued first (16-byte loads; VEC = false: one column at a
// time, for an odd n or unaligned arrays), then the thread sums its
// products in column order, and the threads' sums of a row are combined in
// a fixed order (butterfly within each wavefront, the wavefronts in turn),
// so every run gives the same bits.  (A pair that ends one past a window
// adds one more small product.)  A single wavefront (THREADS = 64) needs
// no exchange between wavefronts: its butterfly leaves the row's sum in
// every lane.
template <bool VEC, int PASSES, int ROWS, int THREADS>
__global__ __launch_bounds__(THREADS) void k_dense_apply(const double *__restrict__ D,
                                                            const int *__restrict__ win,
                                                            const double *__restrict__ r,
                                                            double *__restrict__ x, int64_t n,
                                                            const InstState *__restrict__ st)
{
    constexpr int WAVES = THREADS / 64;
    __shared__ double red[ROWS][WAVES];
    const int64_t row0 = (int64_t)blockIdx.x * ROWS;
    const int t = threadIdx.x;
    // a batch of operators (the heat equation's sine modes): operator y
    {
        const int64_t y = blockIdx.y;
        D += y * n * n;
        win += y * 2 * n;
        r += y * n;
        x += y * n;
    }
    // the windows and the state flag in one round trip
    const InstState *sp = st ? st : &g_no_state;
    int ws[ROWS], we[ROWS];
#pragma unroll
    for (int q = 0; q < ROWS; ++q) {
        const int64_t rq = min(row0 + q, n - 1);   // clamped: loads without branches
        ws[q] = win[2 * rq];
        we[q] = win[2 * rq + 1];
    }
    const int done = sp->done;
    // the windows are inputs of these (empty) statements, so their loads are
    // issued with the flag's, ahead of the exit test, and one wait covers all
#pragma unroll
    for (int q = 0; q < ROWS; ++q) __asm__ volatile("" ::"s"(ws[q]), "s"(we[q]));
    __asm__ volatile("" ::"s"(done));
    if (done) return;
#pragma unroll
    for (int q = 0; q < ROWS; ++q)
        if (row0 + q >= n) we[q] = ws[q];   // a row past the end: an empty window
    int c0 = (int)n, c1 = 0;
#pragma unroll
    for (int q = 0; q < ROWS; ++q) {
        if (we[q] > ws[q]) {
            c0 = min(c0, ws[q]);
            c1 = max(c1, we[q]);
        }
    }
    double rv[PASSES][2], dv[ROWS][PASSES][2];
#pragma unroll
    for (int i = 0; i < PASSES; ++i) {
        const int64_t c = c0 + 2 * t + 2 * THREADS * i;
        if (VEC) {
            double2 a = make_double2(0.0, 0.0);
            if (c < c1) a = *reinterpret_cast<const double2 *>(r + c);
            rv[i][0] = a.x;
            rv[i][1] = a.y;
#pragma unroll
            for (int q = 0; q < ROWS; ++q) {
                double2 d = make_double2(0.0, 0.0);
                if (c >= ws[q] && c < we[q])
                    d = *reinterpret_cast<const double2 *>(D + (row0 + q) * n + c);
                dv[q][i][0] = d.x;
                dv[q][i][1] = d.y;
            }
        } else {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int64_t cc = c + h;
                rv[i][h] = cc < c1 ? r[cc] : 0.0;
#pragma unroll
                for (int q = 0; q < ROWS; ++q)
                    dv[q][i][h] = cc >= ws[q] && cc < we[q] ? D[(row0 + q) * n + cc] : 0.0;
            }
        }
    }
    double acc[ROWS];
#pragma unroll
    for (int q = 0; q < ROWS; ++q) {
        acc[q] = 0.0;
#pragma unroll
        for (int i = 0; i < PASSES; ++i) {
            acc[q] = fma(dv[q][i][0], rv[i][0], acc[q]);
            acc[q] = fma(dv[q][i][1], rv[i][1], acc[q]);
        }
    }
    const int lane = t & 63, w = t >> 6;
#pragma unroll
    for (int q = 0; q < ROWS; ++q) {
        double v = acc[q];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (WAVES == 1) {
            if (lane == 0 && row0 + q < n) x[row0 + q] = v;
        } else if (lane == 0) {
            red[q][w] = v;
        }
    }
    if (WAVES == 1) return;
    __syncthreads();
    if (t < ROWS && row0 + t < n) {
        double v = red[t][0];
#pragma unroll
        for (int k = 1; k < WAVES; ++k) v += red[t][k];
        x[row0 + t] = v;
    }
}

// *wmax = the widest span a work-group of k_dense_apply loads: over the
// groups of kDenseRows consecutive rows of each of nop operators of n rows
// (win: 2 ints per row), the largest end minus the smallest start of the
// group's nonempty windows.  One work-group, a fixed reduction.
__global__ __launch_bounds__(kDenseThreads) void k_dense_wmax(const int *__restrict__ win, int64_t n,
                                                           int nop, int *__restrict__ wmax)
{
    __shared__ int red[kDenseWaves];
    const int64_t groups = (n + kDenseRows - 1) / kDenseRows;
    int w = 0;
    for (int64_t i = threadIdx.x; i < groups * nop; i += kDenseThreads) {
        const int64_t y = i / groups, r0 = (i - y * groups) * kDenseRows;
        int c0 = INT_MAX, c1 = 0;
        for (int q = 0; q < kDenseRows && r0 + q < n; ++q) {
            const int *p = win + 2 * (y * n + r0 + q);
            if (p[1] > p[0]) {
                c0 = min(c0, p[0]);
                c1 = max(c1, p[1]);
            }
        }
        if (c1 > c0) w = max(w, c1 - c0);
    }
    for (int o = 32; o > 0; o >>= 1) w = max(w, __shfl_xor(w, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < kDenseWaves; ++k) w = max(w, red[k]);
        *wmax = w;
    }
}

// out[a][j] = sum_b Q[a][b] in[b][j] over a, b < nx, j < n: one thread per
// output, the b in order.
__global__ __launch_bounds__(kDenseThreads) void k_mode_transform(const double *__restrict__ Q,
                                                               const double *__restrict__ in,
                                                               double *__restrict__ out, int nx,
                                                               int64_t n)
{
    const int64_t j = (int64_t)blockIdx.x * kDenseThreads + threadIdx.x;
    const int a = blockIdx.y;
    if (j >= n) return;
    const double *q = Q + (int64_t)a * nx;
    double acc = 0.0;
#pragma unroll 8
    for (int b = 0; b < nx; ++b) acc = fma(q[b], in[(int64_t)b * n + j], acc);
    out[(int64_t)a * n + j] = acc;
}

// k_dense_apply with 16-byte loads where n is even and D, r are 16-byte
// aligned.
template <int PASSES, int ROWS, int THREADS>
void launch_apply_p(const double *D, const int *win, const double *r, double *x, int64_t n,
                    const InstState *st, dim3 grid, hipStream_t s)
{
    const bool vec = n % 2 == 0 && ((reinterpret_cast<uintptr_t>(D) | reinterpret_cast<uintptr_t>(r)) & 15) == 0;
    if (vec)
        hipLaunchKernelGGL((k_dense_apply<true, PASSES, ROWS, THREADS>), grid, dim3(THREADS), 0, s,
                           D, win, r, x, n, st);
    else
        hipLaunchKernelGGL((k_dense_apply<false, PASSES, ROWS, THREADS>), grid, dim3(THREADS), 0,
                           s, D, win, r, x, n, st);
}

// The passes cover the widest span a group of kDenseRows rows loads (at
// most n), which bounds a single row's.  Up to kDenseWaveSpan columns: one
// row per work-group of a single wavefront (a work-group's chain after its
// loads is then one butterfly, with no exchange between wavefronts);
// wider: kDenseRows rows per work-group of kDenseThreads threads.
void launch_apply(const double *D, const int *win, const double *r, double *x, int64_t n,
                  const InstState *st, unsigned nop, hipStream_t s, int64_t width)
{
    const int64_t span = std::min<int64_t>(n, width);
    if (span <= kDenseWaveSpan) {
        const dim3 grid((unsigned)n, nop);
        if (span <= 2 * 64) launch_apply_p<1, 1, 64>(D, win, r, x, n, st, grid, s);
        else if (span <= 2 * 2 * 64) launch_apply_p<2, 1, 64>(D, win, r, x, n, st, grid, s);
        else launch_apply_p<4, 1, 64>(D, win, r, x, n, st, grid, s);
        return;
    }
    const dim3 grid((unsigned)((n + kDenseRows - 1) / kDenseRows), nop);
    switch (dense_passes(span)) {   // at least 2 here
    case 2: launch_apply_p<2, kDenseRows, kDenseThreads>(D, win, r, x, n, st, grid, s); break;
    case 4: launch_apply_p<4, kDenseRows, kDenseThreads>(D, win, r, x, n, st, grid, s); break;
    default:
        launch_apply_p<kDensePasses, kDenseRows, kDenseThreads>(D, win, r, x, n, st, grid, s);
        break;
    }
}

}  // namespace

hipError_t launch_mode_transform(const double *Q, const double *in, double *out, int nx,
                                 int64_t n, hipStream_t s)
{
    if (nx < 1 || nx > 65535 || n < 1) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((n + kDenseThreads - 1) / kDenseThreads), (unsigned)nx);
    hipLaunchKernelGGL(k_mode_transform, grid, dim3(kDenseThreads), 0, s, Q, in, out, nx, n);
    return hipGetLastError();
}

hipError_t launch_dense_window_max(const int *win, int64_t n, int nop, int *wmax, hipStream_t s)
{
    if (n < 1 || nop < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_dense_wmax, dim3(1), dim3(kDenseThreads), 0, s, win, n, nop, wmax);
    return hipGetLastError();
}

hipError_t launch_dense_apply_batch(const double *D, const int *win, const double *r, double *x,
                                    int64_t n, int nop, hipStream_t s, int64_t width)
{
    if (n < 1 || n > kDenseMaxN || nop < 1 || nop > 65535) return hipErrorInvalidValue;
    launch_apply(D, win, r, x, n, nullptr, (unsigned)nop, s, width);
    return hipGetLastError();
}

hipError_t launch_dense_cols(int P, const DenseColArgs &a, hipStream_t s)
{
    TMG_DISPATCH_P(P, { return launch_dense_cols_p<PP>(a, s); })
    return hipErrorInvalidValue;
}

hipError_t launch_gdense_cols(int P, const DenseColArgs &a, hipStream_t s)
{
    TMG_DISPATCH_PALL(P, { return launch_gdense_cols_p<PP>(a, s); })
    return hipErrorInvalidValue;
}

hipError_t launch_dense_window(const double *D, int64_t n, int *win, hipStream_t s)
{
    if (n < 1 || n > kDenseMaxN) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_dense_window, dim3((unsigned)((n + kDenseWaves - 1) / kDenseWaves)),
                       dim3(kDenseThreads), 0, s, D, n, win);
    return hipGetLastError();
}

hipError_t launch_dense_apply(const double *D, const int *win, const double *r, double *x,
                              int64_t n, const InstState *st, hipStream_t s, int64_t width)
{
    if (n < 1 || n > kDenseMaxN) return hipErrorInvalidValue;
    launch_apply(D, win, r, x, n, st, 1u, s, width);
    return hipGetLastError();
}

}  // namespace tmg
