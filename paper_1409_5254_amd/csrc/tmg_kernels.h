// HIP kernels (gfx950) of the time-multigrid cycle for DG-in-time
// discretisations of u' + lambda u = f: the kernel templates and the
// templated launchers, included by the translation units that instantiate
// them (tmg_leg64.hip, tmg_leg32.hip, tmg_span.hip, tmg_mix.hip,
// tmg_bottom.hip, tmg_kernels.hip), which compile in parallel.
//
// All cycle kernels are HBM-bound streaming kernels (well under 1 flop/byte;
// no MFMA).  A work-group of 256 threads owns a tile of consecutive slabs of
// one instance, each thread S consecutive slabs (S*P doubles per array in
// registers), and runs several steps on the tile without leaving registers:
//
//   k_down : nsweep damped block Jacobi sweeps (eq. chap4_ODESmoother), the
//            residual r = f - L u and its factor-2 restriction
//            (eq. chap4_restrictionTime);
//   k_up   : prolongation and correction (eq. chap4_prolongationTime),
//            nsweep sweeps, optionally the squared residual norm.
//
// A Jacobi sweep of slab n needs only the end value w_{n-1} = c^T u_{n-1} of
// the *old* left neighbour: one double per slab, passed thread to thread
// with a wavefront shuffle and wave to wave through LDS.  Dependencies run
// one way in time, so a tile carries a left halo of `halo` slabs (>= sweeps
// + 1) that is recomputed and discarded (temporal blocking); tiles write to
// a buffer other than the one they read (ping-pong), so no tile can see a
// neighbour's new values.
//
//   k_coarse : exact solve on the coarsest level as a parallel prefix scan
//              over the per-slab affine maps w_n = alpha w_{n-1} + c^T A^{-1} r_n;
//   k_norm_f, k_finalize : deterministic per-instance norms and the device
//              side convergence state;
//   k_grad   : adjoint gradient reductions.
//
// The transposed (adjoint) system runs the same kernels backward in time:
// logical slab m is physical slab N-1-m, with A^T, c = v, v = 1 and R_1 / R_2
// swapped in the tables passed by the host.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "tmg_internal.h"

namespace tmg {
namespace {

constexpr int kWaves = kThreads / 64;
constexpr int kLegWaves = kLegThreads / 64;


// Instance owning a tile: largest j with off[j] <= tile (off[0] = 0).
__device__ __forceinline__ int find_instance(const int64_t *__restrict__ off, int batch,
                                             int64_t tile)
{
    int lo = 0, hi = batch;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (off[mid] <= tile) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Value of lane - 1 (lane 0 receives 0): a DPP whole-wavefront shift by one
// lane, which stays in the VALU (no LDS round trip).
__device__ __forceinline__ float lane_shr1(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ double lane_shr1(double x)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0x138, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0x138, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// End value of the left neighbour of this thread's first slab, for the
// current sweep.  Double-buffered LDS slots (phase) need one barrier per call.
template <int NW, typename T>
__device__ __forceinline__ T left_value(T mine_last, double (*xchg)[NW], int &phase)
{
    if constexpr (NW == 1) return lane_shr1(mine_last);  // one wavefront: no LDS, no barrier
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    T v = lane_shr1(mine_last);
    if (lane == 63) xchg[phase][wave] = (double)mine_last;
    __syncthreads();
    if (lane == 0) v = wave ? (T)xchg[phase][wave - 1] : (T)0;
    phase ^= 1;
    return v;
}

// Sum over the work-group (fixed reduction tree); the result is valid in
// thread 0.  Ends with a barrier, so `red` may be reused right away.
template <int NW>
__device__ __forceinline__ double block_sum(double x, double *red)
{
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    if constexpr (NW == 1) return x;
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < NW; ++w) s += red[w];
    __syncthreads();
    return s;
}

// Orders LDS accesses of one wavefront that exchange data between its lanes
// (the LDS executes a wavefront's operations in order; the fences only keep
// the compiler from moving them).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Barrier over the NW wavefronts taking part (NW = 1: the first wavefront).
template <int NW>
__device__ __forceinline__ void group_sync()
{
    if constexpr (NW == 1) wave_sync();
    else __syncthreads();
}

// 16-byte vector of T
template <typename T> struct Vec16;
template <> struct Vec16<double> { typedef double type __attribute__((ext_vector_type(2))); static constexpr int n = 2; };
template <> struct Vec16<float> { typedef float type __attribute__((ext_vector_type(4))); static constexpr int n = 4; };

// Load logical slabs [m0, m0+S) of an instance level with N slabs (zeros
// outside [0, N)).  Backward: logical m is physical N-1-m.
template <int P, int S, bool BW, typename T>
__device__ __forceinline__ void load_chunk(const T *__restrict__ base, int64_t m0, int64_t N,
                                           T (&x)[S][P])
{
    constexpr int VN = Vec16<T>::n;
    if (m0 >= 0 && m0 + S <= N) {
        const int64_t plo = BW ? (N - m0 - S) : m0;
        const T *src = base + plo * P;
        T tmp[S * P];
        if constexpr ((S * P) % VN == 0) {
            if ((reinterpret_cast<uintptr_t>(src) & 15) == 0) {
                typedef typename Vec16<T>::type V;
                const V *vs = reinterpret_cast<const V *>(src);
#pragma unroll
                for (int i = 0; i < S * P / VN; ++i) {
                    V t = vs[i];
#pragma unroll
                    for (int q = 0; q < VN; ++q) tmp[VN * i + q] = t[q];
                }
            } else {
#pragma unroll
                for (int i = 0; i < S * P; ++i) tmp[i] = src[i];
            }
        } else {
#pragma unroll
            for (int i = 0; i < S * P; ++i) tmp[i] = src[i];
        }
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int k = 0; k < P; ++k) x[s][k] = tmp[(BW ? S - 1 - s : s) * P + k];
    } else {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int64_t m = m0 + s;
            const bool ok = m >= 0 && m < N;
            const int64_t pm = BW ? N - 1 - m : m;
#pragma unroll
            for (int k = 0; k < P; ++k) x[s][k] = ok ? base[pm * P + k] : (T)0;
        }
    }
}

// Store logical slabs [m0, m0+S) whose tile-local index (li0 + s) is >= lo
// and whose logical index is < N.
template <int P, int S, bool BW, typename T>
__device__ __forceinline__ void store_chunk(T *__restrict__ base, int64_t m0, int64_t N,
                                            const T (&x)[S][P], int li0, int lo)
{
    constexpr int VN = Vec16<T>::n;
    if (li0 >= lo && m0 >= 0 && m0 + S <= N) {
        const int64_t plo = BW ? (N - m0 - S) : m0;
        T *dst = base + plo * P;
        T tmp[S * P];
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int k = 0; k < P; ++k) tmp[(BW ? S - 1 - s : s) * P + k] = x[s][k];
        if constexpr ((S * P) % VN == 0) {
            if ((reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
                typedef typename Vec16<T>::type V;
                V *vd = reinterpret_cast<V *>(dst);
#pragma unroll
                for (int i = 0; i < S * P / VN; ++i) {
                    V t;
#pragma unroll
                    for (int q = 0; q < VN; ++q) t[q] = tmp[VN * i + q];
                    vd[i] = t;
                }
                return;
            }
        }
#pragma unroll
        for (int i = 0; i < S * P; ++i) dst[i] = tmp[i];
    } else {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int64_t m = m0 + s;
            if (li0 + s >= lo && m >= 0 && m < N) {
                const int64_t pm = BW ? N - 1 - m : m;
#pragma unroll
                for (int k = 0; k < P; ++k) base[pm * P + k] = x[s][k];
            }
        }
    }
}

// The pointer as a value the compiler cannot see through: loads through it
// are issued where they are written and not merged with, or hoisted to, the
// same loads elsewhere.  The level tables are uniform, so they live in scalar
// registers; loading each group where it is used (from the scalar cache)
// keeps a few dozen of them live instead of all of them, which would spill
// into vector-register lanes.
// The tables are read-only for the whole launch, so they are read through
// the constant address space (scalar loads).
template <typename X>
using ConstPtr = const __attribute__((address_space(4))) X *;

template <typename X>
__device__ __forceinline__ ConstPtr<X> opaque(const X *p)
{
    // uniform by construction (one instance per work-group); say so
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    ConstPtr<X> q = (ConstPtr<X>)(((uint64_t)hi << 32) | lo);
    asm volatile("" : "+s"(q));
    return q;
}

// Brings `bytes` of a read-only table into the scalar cache: one load per
// 64-byte line, all issued at once and their values dropped.  A small
// (latency-bound) launch calls it for every table it will read, before the
// wait for its state flag, so that the first use of each table hits the
// cache instead of waiting for memory in turn; in a launch that streams HBM
// the extra wait at entry costs more than it saves.
__device__ __forceinline__ void touch_table(const void *p, int bytes)
{
    if (!p) return;
    const auto q = opaque(reinterpret_cast<const uint32_t *>(p));
    // dwords 64 bytes apart from the start, then the last dword (the region
    // need not start on a line); nothing outside [p, p + bytes) is read
    constexpr int kMaxLines = 12;
    uint32_t v[kMaxLines + 1];
#pragma unroll
    for (int i = 0; i < kMaxLines; ++i)
        if (i * 64 < bytes) v[i] = q[i * 16];
    v[kMaxLines] = q[bytes / 4 - 1];
#pragma unroll
    for (int i = 0; i < kMaxLines; ++i)
        if (i * 64 < bytes) asm volatile("" ::"s"(v[i]));
    asm volatile("" ::"s"(v[kMaxLines]));
}

// N entries of a read-only table, stride `stride`, loaded at the point of use.
template <int N, typename X>
struct Vals {
    X v[N];
};
template <int N, int STRIDE = 1, typename X>
__device__ __forceinline__ Vals<N, X> load_vals(const X *p, int off)
{
    const auto q = opaque(p);
    Vals<N, X> r;
#pragma unroll
    for (int i = 0; i < N; ++i) r.v[i] = q[off + i * STRIDE];
    return r;
}

// Groups of a level's operator table.  Smoothing runs in T (tables rounded
// to T); the residual always runs in FP64 arithmetic (A, v, c from the FP64
// table).
template <int P, typename T>
struct SweepTab {
    T h[P], c[P], omc;
};
template <int P>
struct ResidTab {
    double A[P * P], v[P], cd[P];
};
template <int P, typename T>
struct GTab {
    T G[P * P];
};

// Level tables read where they are used (streaming kernels: the tables of
// two levels and the transfer matrices would not fit the scalar registers).
template <int P, typename T = double>
struct LazyOps {
    const double *tab;
    const T *tabT;
    __device__ __forceinline__ void load(const double *t, const T *tT)
    {
        tab = t;
        tabT = tT;
    }
    __device__ __forceinline__ SweepTab<P, T> sw() const
    {
        constexpr TabLayout L(P);
        const auto q = opaque(tabT);
        SweepTab<P, T> r;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            r.h[k] = q[L.H() + k];
            r.c[k] = q[L.C() + k];
        }
        r.omc = q[L.OMC()];
        return r;
    }
    __device__ __forceinline__ ResidTab<P> res() const
    {
        constexpr TabLayout L(P);
        const auto q = opaque(tab);
        ResidTab<P> r;
#pragma unroll
        for (int i = 0; i < P * P; ++i) r.A[i] = q[L.A() + i];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            r.v[k] = q[L.V() + k];
            r.cd[k] = q[L.C() + k];
        }
        return r;
    }
    __device__ __forceinline__ GTab<P, T> gm() const
    {
        constexpr TabLayout L(P);
        const auto q = opaque(tabT);
        GTab<P, T> r;
#pragma unroll
        for (int i = 0; i < P * P; ++i) r.G[i] = q[L.G() + i];
        return r;
    }
    // single rows, for steps that use one row at a time
    __device__ __forceinline__ Vals<P, T> g_row(int k) const
    {
        return load_vals<P>(tabT, TabLayout(P).G() + k * P);
    }
    __device__ __forceinline__ Vals<P, double> a_row(int k) const
    {
        return load_vals<P>(tab, TabLayout(P).A() + k * P);
    }
    __device__ __forceinline__ Vals<P, double> cd() const { return load_vals<P>(tab, TabLayout(P).C()); }
    __device__ __forceinline__ Vals<P, double> v() const { return load_vals<P>(tab, TabLayout(P).V()); }
    static constexpr bool kRows = true;
};

// Level tables held in registers (the bottom kernel: tables in LDS, one
// level at a time).
template <int P, typename T = double>
struct Ops {
    SweepTab<P, T> s;
    ResidTab<P> r;
    GTab<P, T> g;
    __device__ __forceinline__ void load(const double *__restrict__ tab, const T *__restrict__ tabT)
    {
        constexpr TabLayout L(P);
#pragma unroll
        for (int i = 0; i < P * P; ++i) {
            r.A[i] = tab[L.A() + i];
            g.G[i] = tabT[L.G() + i];
        }
#pragma unroll
        for (int k = 0; k < P; ++k) {
            s.h[k] = tabT[L.H() + k];
            s.c[k] = tabT[L.C() + k];
            r.v[k] = tab[L.V() + k];
            r.cd[k] = tab[L.C() + k];
        }
        s.omc = tabT[L.OMC()];
    }
    __device__ __forceinline__ void load(const double *__restrict__ tab) { load(tab, tab); }
    __device__ __forceinline__ const SweepTab<P, T> &sw() const { return s; }
    __device__ __forceinline__ const ResidTab<P> &res() const { return r; }
    __device__ __forceinline__ const GTab<P, T> &gm() const { return g; }
    static constexpr bool kRows = false;
};

// Fold the initial value into logical slab 0 (forward system, level 0):
// f_1 += u0 v.
template <int P, int S, typename T, class OP>
__device__ __forceinline__ void fold_u0(T (&f)[S][P], int64_t m0, double u0, const OP &op)
{
    double v[P];
    if constexpr (OP::kRows) {
        const auto t = op.v();
#pragma unroll
        for (int k = 0; k < P; ++k) v[k] = t.v[k];
    } else {
#pragma unroll
        for (int k = 0; k < P; ++k) v[k] = op.res().v[k];
    }
    // branch-free select keeps f in registers (no dynamic indexing)
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const double a = (m0 + s == 0) ? u0 : 0.0;
#pragma unroll
        for (int k = 0; k < P; ++k) f[s][k] += (T)(a * v[k]);
    }
}

// nsweep damped block Jacobi sweeps in registers (arithmetic in T):
//   u_n <- (1 - omega) u_n + omega A^{-1} f_n + omega A^{-1} v w_{n-1},
// the same update as u + omega D^{-1} (f - L u), with g = omega A^{-1} f
// precomputed.
template <int P, int S, int NW, typename T, class OP>
__device__ __forceinline__ void sweeps(T (&u)[S][P], const T (&g)[S][P], const OP &op,
                                       int nsweep, double (*xchg)[NW], int &phase)
{
    if (nsweep <= 0) return;
    const auto &tb = op.sw();
    for (int sw = 0; sw < nsweep; ++sw) {
        T w[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            T t = 0;
#pragma unroll
            for (int k = 0; k < P; ++k) t += tb.c[k] * u[s][k];
            w[s] = t;
        }
        const T wl = left_value<NW, T>(w[S - 1], xchg, phase);
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const T wn = s == 0 ? wl : w[s - 1];
#pragma unroll
            for (int k = 0; k < P; ++k) u[s][k] = tb.omc * u[s][k] + g[s][k] + tb.h[k] * wn;
        }
    }
}

// r_n = f_n + v w_{n-1} - A u_n in FP64 arithmetic (operands of type TU, TF).
template <int P, int S, int NW, typename TU, typename TF, class OP>
__device__ __forceinline__ void residual(double (&r)[S][P], const TU (&u)[S][P],
                                         const TF (&f)[S][P], const OP &op,
                                         double (*xchg)[NW], int &phase)
{
    if constexpr (OP::kRows) {
        const auto cd = op.cd();
        double w[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            double t = 0.0;
#pragma unroll
            for (int k = 0; k < P; ++k) t += cd.v[k] * (double)u[s][k];
            w[s] = t;
        }
        const double wl = left_value<NW, double>(w[S - 1], xchg, phase);
        const auto v = op.v();
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const auto a = op.a_row(k);
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const double wn = s == 0 ? wl : w[s - 1];
                double t = (double)f[s][k] + v.v[k] * wn;
#pragma unroll
                for (int l = 0; l < P; ++l) t -= a.v[l] * (double)u[s][l];
                r[s][k] = t;
            }
        }
    } else {
        const auto &tb = op.res();
        double w[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            double t = 0.0;
#pragma unroll
            for (int k = 0; k < P; ++k) t += tb.cd[k] * (double)u[s][k];
            w[s] = t;
        }
        const double wl = left_value<NW, double>(w[S - 1], xchg, phase);
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const double wn = s == 0 ? wl : w[s - 1];
#pragma unroll
            for (int k = 0; k < P; ++k) {
                double t = (double)f[s][k] + tb.v[k] * wn;
#pragma unroll
                for (int l = 0; l < P; ++l) t -= tb.A[k * P + l] * (double)u[s][l];
                r[s][k] = t;
            }
        }
    }
}

template <int P, int S, typename T, class OP>
__device__ __forceinline__ void apply_G(T (&g)[S][P], const T (&f)[S][P], const OP &op)
{
    if constexpr (OP::kRows) {
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const auto G = op.g_row(k);
#pragma unroll
            for (int s = 0; s < S; ++s) {
                T t = 0;
#pragma unroll
                for (int l = 0; l < P; ++l) t += G.v[l] * f[s][l];
                g[s][k] = t;
            }
        }
    } else {
        const auto &tb = op.gm();
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int k = 0; k < P; ++k) {
                T t = 0;
#pragma unroll
                for (int l = 0; l < P; ++l) t += tb.G[k * P + l] * f[s][l];
                g[s][k] = t;
            }
    }
}

// Rows and columns of the transfer matrices R_1^T (i = 0) and R_2^T (i = 1):
// from global memory, loaded where used (streaming kernels), or from a copy
// in LDS (bottom kernel).
template <int P, typename T>
struct RGlob {
    const T *R;
    __device__ __forceinline__ Vals<P, T> row(int i, int k) const
    {
        return load_vals<P>(R, i * P * P + k * P);
    }
    __device__ __forceinline__ Vals<P, T> col(int i, int k) const
    {
        return load_vals<P, P>(R, i * P * P + k);
    }
};
template <int P>
struct RLds {
    const double *R;
    __device__ __forceinline__ Vals<P, double> row(int i, int k) const
    {
        Vals<P, double> r;
#pragma unroll
        for (int l = 0; l < P; ++l) r.v[l] = R[i * P * P + k * P + l];
        return r;
    }
    __device__ __forceinline__ Vals<P, double> col(int i, int k) const
    {
        Vals<P, double> r;
#pragma unroll
        for (int l = 0; l < P; ++l) r.v[l] = R[i * P * P + l * P + k];
        return r;
    }
};

// u_{2i} += R_1^T e_i, u_{2i+1} += R_2^T e_i (in T); with S = 1 each lane
// adds the half that belongs to its own slab.
template <int P, int S, typename T, class RA>
__device__ __forceinline__ void prolong_add(T (&u)[S][P], const T (&e)[S >= 2 ? S / 2 : 1][P],
                                            const RA &ra, int64_t m0)
{
    // row k of R_1^T and of R_2^T, loaded per row
    if constexpr (S >= 2) {
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const auto r1 = ra.row(0, k), r2 = ra.row(1, k);
#pragma unroll
            for (int i = 0; i < S / 2; ++i) {
                T s1 = 0, s2 = 0;
#pragma unroll
                for (int l = 0; l < P; ++l) {
                    s1 += r1.v[l] * e[i][l];
                    s2 += r2.v[l] * e[i][l];
                }
                u[2 * i][k] += s1;
                u[2 * i + 1][k] += s2;
            }
        }
    } else {
        const bool second = (m0 & 1) != 0;  // second fine slab of its coarse slab
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const auto r1 = ra.row(0, k), r2 = ra.row(1, k);
            T s1 = 0, s2 = 0;
#pragma unroll
            for (int l = 0; l < P; ++l) {
                s1 += r1.v[l] * e[0][l];
                s2 += r2.v[l] * e[0][l];
            }
            u[0][k] += second ? s2 : s1;
        }
    }
}

template <int P, int S, typename T>
__device__ __forceinline__ void prolong_add(T (&u)[S][P], const T (&e)[S >= 2 ? S / 2 : 1][P],
                                            const T *__restrict__ R, int64_t m0)
{
    prolong_add<P, S, T>(u, e, RGlob<P, T>{R}, m0);
}

// Restrict the residual r (rounded to T) of this thread's slabs and store
// the coarse slabs of output pairs: rc_m = R_1 r_{2m} + R_2 r_{2m+1}.
template <int P, int S, typename T, class RA>
__device__ __forceinline__ void restrict_pairs(const double (&r)[S][P], const RA &ra,
                                               T (&rc)[S / 2][P])
{
    // column k of R_1^T and of R_2^T, loaded per column
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const auto c1 = ra.col(0, k), c2 = ra.col(1, k);
#pragma unroll
        for (int i = 0; i < S / 2; ++i) {
            T s1 = 0;
#pragma unroll
            for (int l = 0; l < P; ++l) s1 += c1.v[l] * (T)r[2 * i][l] + c2.v[l] * (T)r[2 * i + 1][l];
            rc[i][k] = s1;
        }
    }
}

template <int P, int S, typename T>
__device__ __forceinline__ void restrict_pairs(const double (&r)[S][P], const T *__restrict__ R,
                                               T (&rc)[S / 2][P])
{
    restrict_pairs<P, S, T>(r, RGlob<P, T>{R}, rc);
}

template <int P, int S, bool BW, typename T>
__device__ __forceinline__ void restrict_store(const double (&r)[S][P], const T *__restrict__ R,
                                               T *__restrict__ rc_base, int64_t m0, int64_t N,
                                               int64_t Nc, int li0, int halo)
{
    if constexpr (S >= 2) {
        T rc[S / 2][P];
        restrict_pairs<P, S, T>(r, R, rc);
        store_chunk<P, S / 2, BW, T>(rc_base, m0 / 2, Nc, rc, li0 / 2, halo / 2);
    } else {
        // the first slab of each pair takes its partner's residual from the next lane
        double rn[P];
#pragma unroll
        for (int k = 0; k < P; ++k) rn[k] = __shfl_down(r[0][k], 1, 64);
        if (!(m0 & 1) && li0 >= halo && m0 >= 0 && m0 < N) {
            T rc[1][P];
#pragma unroll
            for (int k = 0; k < P; ++k) {
                const auto c1 = load_vals<P, P>(R, k), c2 = load_vals<P, P>(R, P * P + k);
                T s1 = 0;
#pragma unroll
                for (int l = 0; l < P; ++l) s1 += c1.v[l] * (T)r[0][l] + c2.v[l] * (T)rn[l];
                rc[0][k] = s1;
            }
            store_chunk<P, 1, BW, T>(rc_base, m0 / 2, Nc, rc, 0, 0);
        }
    }
}

// Instance, tile and sizes of the work-group's tile.
struct TileRef {
    int j;
    int64_t t, off, N, coff, Nc, c2off, Nc2;   // levels l, l+1, l+2 of instance j
};

template <typename A>
__device__ __forceinline__ TileRef tile_ref(const A &a)
{
    TileRef r{0, (int64_t)blockIdx.x, 0, a.n0, 0, a.n0 / 2, 0, a.n0 / 4};
    if (a.batch > 1) {
        r.j = a.tile_inst ? a.tile_inst[r.t] : find_instance(a.tile_off, a.batch, r.t);
        r.t = (int64_t)blockIdx.x - a.tile_off[r.j];
        r.off = a.slab_off[r.j];
        r.N = a.slab_off[r.j + 1] - r.off;
        if (a.cslab_off) {
            r.coff = a.cslab_off[r.j];
            r.Nc = a.cslab_off[r.j + 1] - r.coff;
        }
        if (a.c2slab_off) {
            r.c2off = a.c2slab_off[r.j];
            r.Nc2 = a.c2slab_off[r.j + 1] - r.c2off;
        }
    }
    return r;
}

// Iterate of the tile: zero, the left halo from the previous pass's halo
// buffer, or the array itself.
template <int P, int S, bool BW, typename T>
__device__ __forceinline__ void load_iterate(T (&u)[S][P], const T *u_in, const T *halo_in,
                                             const TileRef &tr, int64_t m0, int li0, int halo)
{
    if (u_in) {
        if (halo_in && li0 < halo) {
            // left halo: the previous tile's last output slabs of the last
            // pass (the first tile of an instance starts at slab 0: zeros)
            if (tr.t > 0) {
                const T *hb =
                    halo_in + ((int64_t)blockIdx.x - 1) * (int64_t)halo * P + (int64_t)li0 * P;
#pragma unroll
                for (int s = 0; s < S; ++s)
#pragma unroll
                    for (int k = 0; k < P; ++k) u[s][k] = hb[s * P + k];
            } else {
#pragma unroll
                for (int s = 0; s < S; ++s)
#pragma unroll
                    for (int k = 0; k < P; ++k) u[s][k] = (T)0;
            }
        } else {
            load_chunk<P, S, BW, T>(u_in + tr.off * P, m0, tr.N, u);
        }
    } else {
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int k = 0; k < P; ++k) u[s][k] = (T)0;
    }
}

template <int P, int S, typename T>
__device__ __forceinline__ void store_halo(T *halo_out, const T (&u)[S][P], int li0, int halo)
{
    constexpr int TS = kLegThreads * S;
    if (halo_out && li0 >= TS - halo) {
        T *hb = halo_out + (int64_t)blockIdx.x * (int64_t)halo * P + (int64_t)(li0 - (TS - halo)) * P;
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int k = 0; k < P; ++k) hb[s * P + k] = u[s][k];
    }
}

// An instance still running after its last cycle.
__device__ __forceinline__ bool running(const InstState &s, const Control *ctl)
{
    return !s.done && s.cycles < ctl->max_cycles;
}

// Cycles to have queued for a running instance: the count at which it
// converges at the rate of its last two cycles (the first cycle, from zero,
// gives no rate), one short of it while more than three cycles are ahead (a
// later summary refines it); two past its count while it has no rate.
__device__ __forceinline__ int want_cycles(const InstState &s, const Control *ctl)
{
    if (s.prev_rsq > 0.0 && s.rsq > 0.0 && s.rsq < s.prev_rsq) {
        const double k = log(ctl->rtol2 * s.r0sq / s.rsq) / log(s.rsq / s.prev_rsq);
        const int n = (int)fmin(fmax(ceil(k), 1.0), 64.0);
        return s.cycles + (n > 3 ? n - 1 : n);
    }
    return s.cycles + 2;
}

// Writes the host copy (see HostHead) from one thread.  A system-scope
// release fence is an L2 writeback here: one pair per copy.
__device__ __forceinline__ void put_summary(HostHead *h, long long v, int nrun, int want,
                                            const InstState *one)
{
    HostSum *m = reinterpret_cast<HostSum *>(h + 1);
    __hip_atomic_store(&h->begin, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
    __hip_atomic_store(&m->running, nrun, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&m->want, want, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    if (one) {
        __hip_atomic_store(&m->cycles, one->cycles, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&m->done, one->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&m->r0sq, one->r0sq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&m->rsq, one->rsq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&m->prev_rsq, one->prev_rsq, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_SYSTEM);
    }
    __hip_atomic_store(&h->end, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Host copy for a single instance, by the thread that finished its cycle:
// its state (batches: k_publish after the cycle).
__device__ __forceinline__ void publish(HostHead *h, const InstState &s, const Control *ctl)
{
    if (!h) return;
    put_summary(h, ((long long)ctl->epoch << 32) | (unsigned)s.cycles, 0, 0, &s);
}

// Convergence state after a cycle whose squared residual norm is acc
// (relative residual criterion of section 4.2); s is st[j] before it.
__device__ __forceinline__ void finish_cycle(InstState *st, int j, InstState s, double acc,
                                             const Control *ctl, HostHead *mirror)
{
    s.prev_rsq = s.cycles >= 1 ? s.rsq : -1.0;
    s.cycles += 1;
    s.rsq = acc;
    if (!isfinite(acc)) s.done = 3;
    else if (acc <= ctl->rtol2 * s.r0sq) s.done = 1;
    else if (acc > 1e6 * s.r0sq) s.done = 4;
    else if (s.cycles >= ctl->max_cycles) s.done = 2;
    st[j] = s;
    publish(mirror, s, ctl);
}

// Squared residual of the tile's output slabs into its partial slot (summed
// per instance in a fixed order by k_finalize).
template <int P, int S, int NW>
__device__ __forceinline__ void norm_partial(const double (&r)[S][P], double *partial,
                                             const int64_t *norm_off, const TileRef &tr, int64_t m0,
                                             int li0, int halo, double *red)
{
    double acc = 0.0;
#pragma unroll
    for (int s = 0; s < S; ++s)
        if (li0 + s >= halo && m0 + s < tr.N)
#pragma unroll
            for (int k = 0; k < P; ++k) acc += r[s][k] * r[s][k];
    acc = block_sum<NW>(acc, red);
    if (threadIdx.x == 0) partial[norm_off[tr.j] + tr.t] = acc;
}

// The streaming leg (see LegArgsT), storage and smoothing in T, residual in
// FP64 arithmetic.  Every step runs on the tile in registers; the tile's
// first `halo` slabs are recomputed copies of the left neighbour's last
// output slabs and are never stored.  With one slab per thread (S = 1) the
// two fine slabs of a coarse slab sit in neighbouring lanes (tiles start at
// an even slab) and meet through a lane shuffle.
// TOUCH (a.touch): the tables are brought into the scalar cache at entry
// (small launches); a separate instantiation, as even an untaken branch
// costs the level-0 pass registers.  LEG: 0 any leg; 1 down legs and 2 up
// legs of a first visit from zero (the levels below 0 of a V-cycle), with
// the paths they do not take compiled out, which frees registers for more
// work-groups per CU; 4 the first level-0 down pass of a solve, which also
// leaves the norm partials of f (u0 folded), the initial residual.
template <int P, bool BW, typename T, bool TOUCH, int LEG>
__global__ __launch_bounds__(kLegThreads) void k_leg(LegArgsT<T> a)
{
    constexpr bool kNormF = LEG == 4;   // a down leg from zero that also folds u0
    constexpr bool kAny = LEG == 0, kDown = LEG == 1 || kNormF, kUp = LEG == 2;
    constexpr int S = slabs_per_thread(P);
    constexpr int SC = S >= 2 ? S / 2 : 1;  // coarse slabs touched per thread
    __shared__ double xchg[2][kLegWaves];
    __shared__ double red[kLegWaves];
    const TileRef tr = tile_ref(a);
    // a batch: the tiles of finished instances leave before loading anything
    // (one instance keeps its loads ahead of the flag's, for their latency)
    if (a.batch > 1 && a.st && a.st[tr.j].done) return;
    const int li0 = threadIdx.x * S;
    const int64_t m0 = tr.t * a.tile_out - a.halo + li0;
    // every load is issued before the early-exit test: data first, then the
    // state flag and the level tables
    constexpr int SC2 = SC >= 2 ? SC / 2 : 1;  // level-2 slabs touched per thread
    T f[S][P], u[S][P], g[S][P], e[SC][P];
    T f1[SC][P], e2[SC2][P];
    // coarse slab of this thread's slabs (floor division; -1 is outside)
    const int64_t cm0 = S >= 2 ? m0 / 2 : (m0 >> 1);
    const int64_t c2m0 = SC >= 2 ? cm0 / 2 : (cm0 >> 1);
    load_chunk<P, S, BW, T>(a.f + tr.off * P, m0, tr.N, f);
    if constexpr (kAny) {
        load_iterate<P, S, BW, T>(u, a.u_in, a.halo_in, tr, m0, li0, a.halo);
    } else {
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int k = 0; k < P; ++k) u[s][k] = (T)0;
    }
    if constexpr (!kDown) {
        if (a.e2) {
            load_chunk<P, SC, BW, T>(a.f1 + tr.coff * P, cm0, tr.Nc, f1);
            load_chunk<P, SC2, BW, T>(a.e2 + tr.c2off * P, c2m0, tr.Nc2, e2);
        } else if (a.e) {
            load_chunk<P, SC, BW, T>(a.e + tr.coff * P, cm0, tr.Nc, e);
        }
    }
    const int done = (a.batch == 1 && a.st) ? a.st[tr.j].done : 0;
    LazyOps<P, T> op;
    op.load(a.tab + (int64_t)tr.j * a.tab_stride, a.tabT + (int64_t)tr.j * a.tab_stride);
    if constexpr (TOUCH) {
        const int tb = TabLayout(P).stride() * 8, tbT = TabLayout(P).stride() * (int)sizeof(T);
        touch_table(op.tab, tb);
        if ((const void *)op.tabT != (const void *)op.tab) touch_table(op.tabT, tbT);
        if (a.tab1) {
            touch_table(a.tab1 + (int64_t)tr.j * a.tab_stride, tb);
            if ((const void *)a.tab1T != (const void *)a.tab1)
                touch_table(a.tab1T + (int64_t)tr.j * a.tab_stride, tbT);
        }
        touch_table(a.R, 2 * P * P * (int)sizeof(T));
    }
    if (done) return;
    int phase = 0;
    LazyOps<P, T> op1;   // the next level (two-level launches)
    op1.load(a.tab1 + (int64_t)tr.j * a.tab_stride, a.tab1T + (int64_t)tr.j * a.tab_stride);
    if (!kDown && a.e2) {
        // the next level's up leg on the tile's coarse slabs: its first slabs
        // (pre + post - 1 of them) see a zero left neighbour and are wrong,
        // which the halo absorbs
        T g1[SC][P];
        apply_G<P, SC, T>(g1, f1, op1);
#pragma unroll
        for (int s = 0; s < SC; ++s)
#pragma unroll
            for (int k = 0; k < P; ++k) e[s][k] = (T)0;
        sweeps<P, SC, kLegWaves, T>(e, g1, op1, a.pre, xchg, phase);
        prolong_add<P, SC, T>(e, e2, a.R, cm0);
        sweeps<P, SC, kLegWaves, T>(e, g1, op1, a.post, xchg, phase);
    }
    if ((kAny || kNormF) && a.u0) fold_u0<P, S, T>(f, m0, a.u0[tr.j], op);
    apply_G<P, S, T>(g, f, op);
    sweeps<P, S, kLegWaves, T>(u, g, op, a.pre, xchg, phase);
    if (!kDown && (a.e || a.e2)) prolong_add<P, S, T>(u, e, a.R, m0);
    if constexpr (!kDown) sweeps<P, S, kLegWaves, T>(u, g, op, a.post, xchg, phase);
    if (!kDown && a.u_out) store_chunk<P, S, BW, T>(a.u_out + tr.off * P, m0, tr.N, u, li0, a.halo);
    if constexpr (kAny) store_halo<P, S, T>(a.halo_out, u, li0, a.halo);
    double r[S][P];
    if constexpr (kNormF)   // after the sweeps: its barrier waits on nothing then
        norm_partial<P, S, kLegWaves>(f, a.partial, a.norm_off, tr, m0, li0, a.halo, red);
    if (kAny && a.partial) {
        residual<P, S, kLegWaves>(r, u, f, op, xchg, phase);
        norm_partial<P, S, kLegWaves>(r, a.partial, a.norm_off, tr, m0, li0, a.halo, red);
    }
    if (!kUp && a.rc) {
        static_assert(S >= 2, "streaming tiles hold whole coarse slabs per thread");
        sweeps<P, S, kLegWaves, T>(u, g, op, a.next, xchg, phase);
        residual<P, S, kLegWaves>(r, u, f, op, xchg, phase);
        T rc1[SC][P];
        restrict_pairs<P, S, T>(r, a.R, rc1);
        store_chunk<P, SC, BW, T>(a.rc + tr.coff * P, cm0, tr.Nc, rc1, li0 / 2, a.halo / 2);
        if (a.f2) {
            // the next level's down leg of a first visit on the restricted
            // residual: sweeps from zero, residual, restriction (its first
            // coarse slabs are wrong; the halo absorbs them)
            T g1[SC][P], x1[SC][P];
            apply_G<P, SC, T>(g1, rc1, op1);
#pragma unroll
            for (int s = 0; s < SC; ++s)
#pragma unroll
                for (int k = 0; k < P; ++k) x1[s][k] = (T)0;
            sweeps<P, SC, kLegWaves, T>(x1, g1, op1, a.pre, xchg, phase);
            double r1[SC][P];
            residual<P, SC, kLegWaves>(r1, x1, rc1, op1, xchg, phase);
            restrict_store<P, SC, BW, T>(r1, a.R, a.f2 + tr.c2off * P, cm0, tr.Nc, tr.Nc2, li0 / 2,
                                         a.halo / 2);
        }
    }
}

// ---- spans: several small levels per launch ------------------------------
//
// The small streaming levels are latency-bound: a launch spends most of its
// time starting up, waiting for data the previous launch wrote and draining,
// not computing.  A span runs the legs of up to four consecutive levels of a
// V-cycle's first visits in one launch.  Every thread holds one slab of the
// top level l; at level l+k the tile's slabs are 2^k times fewer and each is
// held (and computed, identically) by the 2^k neighbouring lanes that held
// its fine slabs.  The left neighbour is then 2^k lanes back, and the two
// fine slabs of a coarse slab are 2^k lanes apart.  Each step computes what
// the pair and single launches compute, in the same order, so a span gives
// the same iterate to the last bit; its tile's left halo is sized for the
// wrong leading slabs of all its levels.

// Value of lane `lane - d` (d < 64; lanes below d receive their own value).
__device__ __forceinline__ double lane_back(double x, int d)
{
    const int lane = threadIdx.x & 63;
    const int src = (lane >= d ? lane - d : lane) << 2;
    const int lo = __builtin_amdgcn_ds_bpermute(src, __double2loint(x));
    const int hi = __builtin_amdgcn_ds_bpermute(src, __double2hiint(x));
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane_back(float x, int d)
{
    const int lane = threadIdx.x & 63;
    const int src = (lane >= d ? lane - d : lane) << 2;
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(x)));
}
// Value of lane `lane ^ d` (d a power of two below 64).
__device__ __forceinline__ double lane_xor(double x, int d)
{
    const int src = ((threadIdx.x & 63) ^ d) << 2;
    const int lo = __builtin_amdgcn_ds_bpermute(src, __double2loint(x));
    const int hi = __builtin_amdgcn_ds_bpermute(src, __double2hiint(x));
    return __hiloint2double(hi, lo);
}

// End value of the left neighbour of this lane's slab when each slab is held
// by d neighbouring lanes (the tile's first slab sees zero); one barrier.
template <int NW, typename T>
__device__ __forceinline__ T left_value_d(T mine, int d, double (*xchg)[NW], int &phase)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    T v = lane_back(mine, d);
    if (lane == 63) xchg[phase][wave] = (double)mine;
    __syncthreads();
    if (lane < d) v = wave ? (T)xchg[phase][wave - 1] : (T)0;
    phase ^= 1;
    return v;
}

// Sweeps and residual of one slab per lane (as sweeps / residual with S = 1).
template <int P, int NW, typename T, class OP>
__device__ __forceinline__ void sweeps_d(T (&u)[P], const T (&g)[P], const OP &op, int nsweep,
                                         int d, double (*xchg)[NW], int &phase)
{
    if (nsweep <= 0) return;
    const auto &tb = op.sw();
    for (int sw = 0; sw < nsweep; ++sw) {
        T w = 0;
#pragma unroll
        for (int k = 0; k < P; ++k) w += tb.c[k] * u[k];
        const T wn = left_value_d<NW, T>(w, d, xchg, phase);
#pragma unroll
        for (int k = 0; k < P; ++k) u[k] = tb.omc * u[k] + g[k] + tb.h[k] * wn;
    }
}

template <int P, int NW, typename T, class OP>
__device__ __forceinline__ void residual_d(double (&r)[P], const T (&u)[P], const T (&f)[P],
                                           const OP &op, int d, double (*xchg)[NW], int &phase)
{
    const auto cd = op.cd();
    double w = 0.0;
#pragma unroll
    for (int k = 0; k < P; ++k) w += cd.v[k] * (double)u[k];
    const double wn = left_value_d<NW, double>(w, d, xchg, phase);
    const auto v = op.v();
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const auto a = op.a_row(k);
        double t = (double)f[k] + v.v[k] * wn;
#pragma unroll
        for (int l = 0; l < P; ++l) t -= a.v[l] * (double)u[l];
        r[k] = t;
    }
}

template <int P, typename T, class OP>
__device__ __forceinline__ void apply_G1(T (&g)[P], const T (&f)[P], const OP &op)
{
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const auto G = op.g_row(k);
        T t = 0;
#pragma unroll
        for (int l = 0; l < P; ++l) t += G.v[l] * f[l];
        g[k] = t;
    }
}

// Restriction of a pair of slabs held d lanes apart: every lane of the pair
// gets the coarse slab rc_m = R_1 r_{2m} + R_2 r_{2m+1}.
template <int P, typename T>
__device__ __forceinline__ void restrict_d(const double (&r)[P], bool second, int d,
                                           const T *R, T (&rc)[P])
{
    double rp[P];
#pragma unroll
    for (int k = 0; k < P; ++k) rp[k] = lane_xor(r[k], d);
    const RGlob<P, T> ra{R};
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const auto c1 = ra.col(0, k), c2 = ra.col(1, k);
        T s1 = 0;
#pragma unroll
        for (int l = 0; l < P; ++l) {
            const double r0 = second ? rp[l] : r[l], r1 = second ? r[l] : rp[l];
            s1 += c1.v[l] * (T)r0 + c2.v[l] * (T)r1;
        }
        rc[k] = s1;
    }
}

// u += R_1^T e or R_2^T e (the half for this slab's position in its pair).
template <int P, typename T>
__device__ __forceinline__ void prolong_d(T (&u)[P], const T (&e)[P], bool second, const T *R)
{
    const RGlob<P, T> ra{R};
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const auto r1 = ra.row(0, k), r2 = ra.row(1, k);
        T s1 = 0, s2 = 0;
#pragma unroll
        for (int l = 0; l < P; ++l) {
            s1 += r1.v[l] * e[l];
            s2 += r2.v[l] * e[l];
        }
        u[k] += second ? s2 : s1;
    }
}

template <int P, bool BW, typename T>
__global__ __launch_bounds__(kSpanThreads) void k_span(SpanArgsT<T> a)
{
    constexpr int NW = kSpanThreads / 64;
    __shared__ double xchg[2][NW];
    const int t = threadIdx.x;
    int j = 0;
    int64_t tile = blockIdx.x;
    if (a.batch > 1) {
        j = a.tile_inst ? a.tile_inst[tile] : find_instance(a.tile_off, a.batch, tile);
        tile -= a.tile_off[j];
    }
    if (a.batch > 1 && a.st && a.st[j].done) return;   // as in k_leg
    const int K = min(a.K, a.lb[j] - a.level);
    // first slab of the tile at level l (a multiple of 2^K: no coarse slab
    // of the span straddles two tiles)
    const int64_t s0 = tile * a.tile_out - a.halo;
    int64_t off[kMaxSpan + 1], N[kMaxSpan + 1];
#pragma unroll
    for (int k = 0; k <= kMaxSpan; ++k) {
        if (k > K) break;
        if (a.batch > 1) {
            off[k] = a.slab_off[k][j];
            N[k] = a.slab_off[k][j + 1] - off[k];
        } else {
            off[k] = 0;
            N[k] = a.n0 >> k;
        }
    }
    // every load is issued before the wait for the state flag and the tables
    T f[kMaxSpan][P], e[P];
    if (a.up) {
#pragma unroll
        for (int k = 0; k < kMaxSpan; ++k) {
            if (k >= K) break;
            T tmp[1][P];
            load_chunk<P, 1, BW, T>(a.f[k] + off[k] * P, (s0 >> k) + (t >> k), N[k], tmp);
#pragma unroll
            for (int q = 0; q < P; ++q) f[k][q] = tmp[0][q];
        }
        // the correction of level l+K (K is per instance: read its arrays
        // from the argument block, not from the per-level copies above)
        const int64_t offK = a.batch > 1 ? a.slab_off[K][j] : 0;
        const int64_t NK = a.batch > 1 ? a.slab_off[K][j + 1] - offK : a.n0 >> K;
        T tmp[1][P];
        load_chunk<P, 1, BW, T>(a.x[K] + offK * P, (s0 >> K) + (t >> K), NK, tmp);
#pragma unroll
        for (int q = 0; q < P; ++q) e[q] = tmp[0][q];
    } else {
        T tmp[1][P];
        load_chunk<P, 1, BW, T>(a.f[0] + off[0] * P, s0 + t, N[0], tmp);
#pragma unroll
        for (int q = 0; q < P; ++q) f[0][q] = tmp[0][q];
    }
    const int done = (a.batch == 1 && a.st) ? a.st[j].done : 0;
    const int tb = TabLayout(P).stride() * 8, tbT = TabLayout(P).stride() * (int)sizeof(T);
    for (int k = 0; k < K; ++k) {
        const double *tk = a.tab + k * a.tab_level + (int64_t)j * a.tab_stride;
        const T *tkT = a.tabT + k * a.tab_level + (int64_t)j * a.tab_stride;
        touch_table(tk, tb);
        if ((const void *)tkT != (const void *)tk) touch_table(tkT, tbT);
    }
    touch_table(a.R, 2 * P * P * (int)sizeof(T));
    if (done) return;
    int phase = 0;
    if (!a.up) {
        // down legs from the top: sweeps from zero, residual, restriction
#pragma unroll
        for (int k = 0; k < kMaxSpan; ++k) {
            if (k >= K) break;
            LazyOps<P, T> op;
            op.load(a.tab + k * a.tab_level + (int64_t)j * a.tab_stride,
                    a.tabT + k * a.tab_level + (int64_t)j * a.tab_stride);
            const int d = 1 << k;
            const int64_t m = (s0 >> k) + (t >> k);
            T g[P], x[P];
            apply_G1<P, T>(g, f[k], op);
#pragma unroll
            for (int q = 0; q < P; ++q) x[q] = (T)0;
            sweeps_d<P, NW, T>(x, g, op, a.nu1, d, xchg, phase);
            double r[P];
            residual_d<P, NW, T>(r, x, f[k], op, d, xchg, phase);
            T rc[P];
            restrict_d<P, T>(r, (m & 1) != 0, d, a.R, rc);
            // one lane per coarse slab stores it, outside the halo
            const int lc = t >> (k + 1);
            if ((t & (2 * d - 1)) == 0) {
                T tmp[1][P];
#pragma unroll
                for (int q = 0; q < P; ++q) tmp[0][q] = rc[q];
                store_chunk<P, 1, BW, T>(a.f[k + 1] + off[k + 1] * P, (s0 >> (k + 1)) + lc,
                                         N[k + 1], tmp, lc, a.halo >> (k + 1));
            }
            if (k + 1 < kMaxSpan) {
#pragma unroll
                for (int q = 0; q < P; ++q) f[k + 1][q] = rc[q];
            }
        }
    } else {
        // up legs from the bottom: pre sweeps from zero recomputed,
        // correction from the level below, post sweeps
#pragma unroll
        for (int k = kMaxSpan - 1; k >= 0; --k) {
            if (k >= K) continue;
            LazyOps<P, T> op;
            op.load(a.tab + k * a.tab_level + (int64_t)j * a.tab_stride,
                    a.tabT + k * a.tab_level + (int64_t)j * a.tab_stride);
            const int d = 1 << k;
            const int64_t m = (s0 >> k) + (t >> k);
            T g[P], x[P];
            apply_G1<P, T>(g, f[k], op);
#pragma unroll
            for (int q = 0; q < P; ++q) x[q] = (T)0;
            sweeps_d<P, NW, T>(x, g, op, a.nu1, d, xchg, phase);
            prolong_d<P, T>(x, e, (m & 1) != 0, a.R);
            sweeps_d<P, NW, T>(x, g, op, a.nu2, d, xchg, phase);
#pragma unroll
            for (int q = 0; q < P; ++q) e[q] = x[q];
        }
        T tmp[1][P];
#pragma unroll
        for (int q = 0; q < P; ++q) tmp[0][q] = e[q];
        store_chunk<P, 1, BW, T>(a.x[0] + off[0] * P, s0 + t, N[0], tmp, t, a.halo);
    }
}

// Fused level-0 pass of the FP32-inner defect correction (see MixArgs).
// With u_k the FP64 iterate (in place):
//   up:   r_k = f - L u_k (FP64) -> FP32; the inner level-0 up leg on
//         L e = r_k: pre sweeps from e = 0 recomputed, prolongation of the
//         level-1 correction, post sweeps (FP32); u_{k+1} = u_k + e (FP64);
//   norm: ||f - L u_{k+1}||^2 (FP64);
//   next: the next inner down leg: r_{k+1} -> FP32, next sweeps from zero
//         (FP32), inner residual in FP64 arithmetic, restriction (FP32).
template <int P, bool BW>
__global__ __launch_bounds__(kLegThreads) void k_mix(MixArgs a)
{
    constexpr int S = slabs_per_thread(P);
    constexpr int SC = S >= 2 ? S / 2 : 1;
    __shared__ double xchg[2][kLegWaves];
    __shared__ double red[kLegWaves];
    const TileRef tr = tile_ref(a);
    // a batch: the tiles of finished instances leave before loading anything
    // (one instance keeps its loads ahead of the flag's, for their latency)
    if (a.batch > 1 && a.st && a.st[tr.j].done) return;
    const int li0 = threadIdx.x * S;
    const int64_t m0 = tr.t * a.tile_out - a.halo + li0;
    constexpr int SC2 = SC >= 2 ? SC / 2 : 1;
    double f[S][P], u[S][P], r[S][P];
    float e[SC][P], f1[SC][P], e2[SC2][P];
    const int64_t cm0 = S >= 2 ? m0 / 2 : (m0 >> 1);
    const int64_t c2m0 = SC >= 2 ? cm0 / 2 : (cm0 >> 1);
    load_chunk<P, S, BW, double>(a.f + tr.off * P, m0, tr.N, f);
    load_iterate<P, S, BW, double>(u, a.u_in, a.halo_in, tr, m0, li0, a.halo);
    if (a.up && a.e2) {
        load_chunk<P, SC, BW, float>(a.f1 + tr.coff * P, cm0, tr.Nc, f1);
        load_chunk<P, SC2, BW, float>(a.e2 + tr.c2off * P, c2m0, tr.Nc2, e2);
    } else if (a.up) {
        load_chunk<P, SC, BW, float>(a.e + tr.coff * P, cm0, tr.Nc, e);
    }
    const int done = (a.batch == 1 && a.st) ? a.st[tr.j].done : 0;
    LazyOps<P, float> op;
    op.load(a.tab + (int64_t)tr.j * a.tab_stride, a.tab32 + (int64_t)tr.j * a.tab_stride);
    LazyOps<P, float> op1;   // level 1 (two-level pass)
    op1.load(a.tab1 + (int64_t)tr.j * a.tab_stride, a.tab1_32 + (int64_t)tr.j * a.tab_stride);
    if (done) return;
    if (a.u0) fold_u0<P, S, double>(f, m0, a.u0[tr.j], op);   // in FP64
    int phase = 0;
    float rf[S][P], g[S][P], ei[S][P];
    if (a.up && a.e2) {
        // level 1's inner up leg on the tile's coarse slabs (FP32; its first
        // slabs see a zero left neighbour, the halo absorbs them)
        float g1[SC][P];
        apply_G<P, SC, float>(g1, f1, op1);
#pragma unroll
        for (int s = 0; s < SC; ++s)
#pragma unroll
            for (int k = 0; k < P; ++k) e[s][k] = 0.0f;
        sweeps<P, SC, kLegWaves, float>(e, g1, op1, a.pre, xchg, phase);
        prolong_add<P, SC, float>(e, e2, a.R32, cm0);
        sweeps<P, SC, kLegWaves, float>(e, g1, op1, a.post, xchg, phase);
    }
    if (a.up) {
        residual<P, S, kLegWaves>(r, u, f, op, xchg, phase);
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int k = 0; k < P; ++k) {
                rf[s][k] = (float)r[s][k];
                ei[s][k] = 0.0f;
            }
        apply_G<P, S, float>(g, rf, op);
        sweeps<P, S, kLegWaves, float>(ei, g, op, a.pre, xchg, phase);
        prolong_add<P, S, float>(ei, e, a.R32, m0);
        sweeps<P, S, kLegWaves, float>(ei, g, op, a.post, xchg, phase);
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int k = 0; k < P; ++k) u[s][k] += (double)ei[s][k];
        if (a.u_out) store_chunk<P, S, BW, double>(a.u_out + tr.off * P, m0, tr.N, u, li0, a.halo);
        store_halo<P, S, double>(a.halo_out, u, li0, a.halo);
    }
    residual<P, S, kLegWaves>(r, u, f, op, xchg, phase);
    if (a.partial)
        norm_partial<P, S, kLegWaves>(r, a.partial, a.norm_off, tr, m0, li0, a.halo, red);
    if (a.rc) {
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int k = 0; k < P; ++k) {
                rf[s][k] = (float)r[s][k];
                ei[s][k] = 0.0f;
            }
        apply_G<P, S, float>(g, rf, op);
        sweeps<P, S, kLegWaves, float>(ei, g, op, a.next, xchg, phase);
        residual<P, S, kLegWaves>(r, ei, rf, op, xchg, phase);
        static_assert(S >= 2, "streaming tiles hold whole coarse slabs per thread");
        float rc1[SC][P];
        restrict_pairs<P, S, float>(r, a.R32, rc1);
        store_chunk<P, SC, BW, float>(a.rc + tr.coff * P, cm0, tr.Nc, rc1, li0 / 2, a.halo / 2);
        if (a.f2) {
            // level 1's next inner down leg (FP32 sweeps from zero, residual
            // in FP64 arithmetic) restricted into f2
            float g1[SC][P], x1[SC][P];
            apply_G<P, SC, float>(g1, rc1, op1);
#pragma unroll
            for (int s = 0; s < SC; ++s)
#pragma unroll
                for (int k = 0; k < P; ++k) x1[s][k] = 0.0f;
            sweeps<P, SC, kLegWaves, float>(x1, g1, op1, a.pre, xchg, phase);
            double r1[SC][P];
            residual<P, SC, kLegWaves>(r1, x1, rc1, op1, xchg, phase);
            restrict_store<P, SC, BW, float>(r1, a.R32, a.f2 + tr.c2off * P, cm0, tr.Nc, tr.Nc2,
                                             li0 / 2, a.halo / 2);
        }
    }
}

// Exact solve of L e = r for one instance by the whole work-group (NT
// threads).  With d_n = A^{-1} r_n and b_n = c^T d_n the end values obey the
// affine recurrence w_n = alpha w_{n-1} + b_n (alpha = c^T A^{-1} v,
// w_{-1} = 0); the maps x -> alpha x + b_n are composed by a work-group
// prefix scan (wavefront shuffles, then LDS across waves), NT slabs per pass
// with the last end value carried, and e_n = d_n + A^{-1} v w_{n-1}.
// u0 != 0 folds the initial value into slab 0 (forward system, level 0).
template <int NT>
struct ScanSmem {
    double wa[NT / 64], wb[NT / 64];
    double wend[NT];
};

// NT = 64 runs in one wavefront with shuffles only (sm unused, may be null).
template <int P, bool BW, int NT, typename TR, typename TE>
__device__ __forceinline__ void coarse_scan(const TR *__restrict__ r_base, double u0,
                                            TE *__restrict__ e_base, int64_t N,
                                            const double *__restrict__ tab, ScanSmem<NT> *sm)
{
    constexpr TabLayout L(P);
    double AI[P * P], q[P], c[P], v[P];
#pragma unroll
    for (int i = 0; i < P * P; ++i) AI[i] = tab[L.AI() + i];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        q[k] = tab[L.Q() + k];
        c[k] = tab[L.C() + k];
        v[k] = tab[L.V() + k];
    }
    const double alpha = tab[L.ALPHA()];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double carry = 0.0;
    for (int64_t base = 0; base < N; base += NT) {
        const int64_t m = base + threadIdx.x;
        const bool ok = m < N;
        const int64_t pm = BW ? N - 1 - m : m;
        double r[P], d[P];
#pragma unroll
        for (int k = 0; k < P; ++k) r[k] = ok ? (double)r_base[pm * P + k] : 0.0;
        const double a0 = (m == 0) ? u0 : 0.0;
#pragma unroll
        for (int k = 0; k < P; ++k) r[k] += a0 * v[k];
        double b = 0.0;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            double t = 0.0;
#pragma unroll
            for (int l = 0; l < P; ++l) t += AI[k * P + l] * r[l];
            d[k] = t;
            b += c[k] * t;
        }
        // inclusive scan of (A, B) ~ x -> A x + B in slab order
        double A = ok ? alpha : 1.0, B = ok ? b : 0.0;
        for (int o = 1; o < 64; o <<= 1) {
            const double Ao = __shfl_up(A, o, 64), Bo = __shfl_up(B, o, 64);
            if (lane >= o) {
                B = A * Bo + B;
                A = A * Ao;
            }
        }
        const int64_t nlast = (N - base < NT) ? (N - base) : NT;
        if constexpr (NT == 64) {
            const double wm = A * carry + B;   // end value of slab m
            const double wl = __shfl_up(wm, 1, 64);
            const double wprev = lane == 0 ? carry : wl;
            if (ok)
#pragma unroll
                for (int k = 0; k < P; ++k) e_base[pm * P + k] = (TE)(d[k] + q[k] * wprev);
            carry = __shfl(wm, (int)nlast - 1, 64);
        } else {
            if (lane == 63) {
                sm->wa[wave] = A;
                sm->wb[wave] = B;
            }
            __syncthreads();
            // compose the totals of the earlier waves and the carried end value
            double Bp = carry;
            for (int w = 0; w < wave; ++w) Bp = sm->wa[w] * Bp + sm->wb[w];
            const double wm = A * Bp + B;   // end value of slab m
            sm->wend[threadIdx.x] = wm;
            __syncthreads();
            const double wprev = threadIdx.x == 0 ? carry : sm->wend[threadIdx.x - 1];
            if (ok)
#pragma unroll
                for (int k = 0; k < P; ++k) e_base[pm * P + k] = (TE)(d[k] + q[k] * wprev);
            carry = sm->wend[nlast - 1];
            __syncthreads();
        }
    }
}

template <int P, bool BW>
__global__ __launch_bounds__(kThreads) void k_coarse(CoarseArgs a)
{
    __shared__ ScanSmem<kThreads> sm;
    const int j = a.inst[blockIdx.x];
    if (a.st && a.st[j].done) return;
    const int64_t off = a.slab_off[j];
    const int64_t N = a.slab_off[j + 1] - off;
    coarse_scan<P, BW, kThreads, double, double>(a.r + off * P, a.u0 ? a.u0[j] : 0.0, a.e + off * P,
                                                 N, a.tab + (int64_t)j * a.tab_stride, &sm);
}

// ---------------------------------------------------------------------------
// Bottom of the hierarchy: one work-group of kBottomThreads runs a whole
// multigrid visit of levels `level` .. L_j - 1 of instance j (V or W, gamma
// visits of each coarser level, exact scan on the coarsest), with every
// level's right-hand side and iterate resident in LDS and every level held
// in registers (S slabs per thread, so no halo).  The pre-smoothed iterate
// of the down leg is recomputed in the up leg instead of stored.
// ---------------------------------------------------------------------------

// NT threads (kBottomThreads, or 64 for bottoms one wavefront holds).
template <int P, int NT>
struct BottomLds {
    static constexpr int BMAX = NT * bottom_slabs(P);
    static constexpr int STRIDE = TabLayout(P).stride();
    double f[2 * BMAX * P];
    double x[2 * BMAX * P];
    double tab[kBottomMaxLevels * STRIDE];
    double R[2 * P * P];     // R_1^T, R_2^T
    double xchg[2][NT / 64];
    double red[NT / 64];
    ScanSmem<NT> scan;
};

template <int P, bool BW, int NT_ = kBottomThreads>
struct Bottom {
    static constexpr int NT = NT_;
    static constexpr int NW = NT / 64;
    static constexpr int S = bottom_slabs(P);
    static constexpr int STRIDE = TabLayout(P).stride();
    static constexpr int WAVE_SLABS = 64 * S;   // largest level one wavefront holds
    BottomLds<P, NT> &sm;
    int lb;        // first level of this visit
    int64_t Nlb;   // its slab count
    int Lc;        // coarsest level
    int lw;        // first level with at most WAVE_SLABS slabs
    int nu1, nu2, gamma;

    __device__ int64_t nslab(int l) const { return Nlb >> (l - lb); }
    // offset (doubles) of level l in the f / x regions
    __device__ int64_t loff(int l) const { return (2 * Nlb - 2 * nslab(l)) * P; }
    __device__ const double *tab(int l) const { return sm.tab + (l - lb) * STRIDE; }

    __device__ void load_ops(Ops<P> &op, int l) const { op.load(tab(l)); }
    // exchange slots for G wavefronts (unused by a single wavefront)
    template <int G>
    __device__ double (*xchg() const)[G] { return reinterpret_cast<double (*)[G]>(sm.xchg); }

    // nu1 sweeps from x_l (zero if `zero`), residual, restriction into
    // f_{l+1}; run by the first G wavefronts (G = NW or 1)
    template <int G>
    __device__ __forceinline__ void down(int l, bool zero) const
    {
        Ops<P> op;
        load_ops(op, l);
        const int64_t N = nslab(l), m0 = (int64_t)threadIdx.x * S;
        double f[S][P], u[S][P], g[S][P], r[S][P];
        load_chunk<P, S, BW>(sm.f + loff(l), m0, N, f);
        if (zero) {
#pragma unroll
            for (int s = 0; s < S; ++s)
#pragma unroll
                for (int k = 0; k < P; ++k) u[s][k] = 0.0;
        } else {
            load_chunk<P, S, BW>(sm.x + loff(l), m0, N, u);
        }
        apply_G<P, S>(g, f, op);
        int phase = 0;
        sweeps<P, S, G>(u, g, op, nu1, xchg<G>(), phase);
        residual<P, S, G>(r, u, f, op, xchg<G>(), phase);
        double rc[S / 2][P];
        restrict_pairs<P, S, double>(r, RLds<P>{sm.R}, rc);
        store_chunk<P, S / 2, BW>(sm.f + loff(l + 1), m0 / 2, nslab(l + 1), rc, 0, 0);
        group_sync<G>();
    }

    // x_l <- S^nu2 (S^nu1 x_l + P x_{l+1}), the pre-smoothing recomputed
    // from x_l (or zero) exactly as in the down leg.
    template <int G>
    __device__ __forceinline__ void up(int l, bool zero) const
    {
        Ops<P> op;
        load_ops(op, l);
        const int64_t N = nslab(l), m0 = (int64_t)threadIdx.x * S;
        double f[S][P], u[S][P], g[S][P], e[S / 2][P];
        load_chunk<P, S, BW>(sm.f + loff(l), m0, N, f);
        if (zero) {
#pragma unroll
            for (int s = 0; s < S; ++s)
#pragma unroll
                for (int k = 0; k < P; ++k) u[s][k] = 0.0;
        } else {
            load_chunk<P, S, BW>(sm.x + loff(l), m0, N, u);
        }
        load_chunk<P, S / 2, BW>(sm.x + loff(l + 1), m0 / 2, nslab(l + 1), e);
        apply_G<P, S>(g, f, op);
        int phase = 0;
        sweeps<P, S, G>(u, g, op, nu1, xchg<G>(), phase);
        prolong_add<P, S, double>(u, e, RLds<P>{sm.R}, m0);
        sweeps<P, S, G>(u, g, op, nu2, xchg<G>(), phase);
        // every thread owns the slabs it writes, so the update is in place
        store_chunk<P, S, BW>(sm.x + loff(l), m0, N, u, 0, 0);
        group_sync<G>();
    }

    template <int G>
    __device__ __forceinline__ void coarse(int l) const
    {
        if constexpr (G == 1)
            coarse_scan<P, BW, 64, double, double>(sm.f + loff(l), 0.0, sm.x + loff(l), nslab(l),
                                                   tab(l), (ScanSmem<64> *)nullptr);
        else
            coarse_scan<P, BW, NT, double, double>(sm.f + loff(l), 0.0, sm.x + loff(l), nslab(l),
                                                   tab(l), &sm.scan);
        group_sync<G>();
    }

    // One visit of level `top` (top < Lc): down(top); then, until the
    // coarsest level, gamma visits of each coarser level (the exact scan on
    // the coarsest); up(top).  `zero`: the iterate of `top` starts at zero.
    // Bit l of `again` marks the second visit of level l.  With G = NW, the
    // levels from lw on are handed to the first wavefront as whole visits.
    template <int G>
    __device__ __forceinline__ void visit(int top, bool zero) const
    {
        uint64_t again = 0;
        int l = top;
        down<G>(l, zero);
        while (true) {
            bool descend = false;
            if (l + 1 == Lc) {
                coarse<G>(l + 1);
            } else if constexpr (G > 1) {
                if (l + 1 >= lw) {
                    if (threadIdx.x < 64)
                        for (int rep = 0; rep < gamma; ++rep) visit<1>(l + 1, rep == 0);
                    __syncthreads();
                } else {
                    descend = true;
                }
            } else {
                descend = true;
            }
            if (descend) {
                ++l;
                down<G>(l, true);
                continue;
            }
            // the coarser levels of l are done: climb
            bool finished = false;
            while (true) {
                up<G>(l, l == top ? zero : !((again >> l) & 1));
                if (l == top) {
                    finished = true;
                    break;
                }
                if (gamma > 1 && !((again >> l) & 1)) {
                    again |= (uint64_t)1 << l;
                    down<G>(l, false);
                    break;
                }
                again &= ~((uint64_t)1 << l);
                --l;
            }
            if (finished) break;
        }
    }
};

// NT = 64 (one wavefront per instance) where every level of the launch's
// instances fits one wavefront: a fraction of the registers and LDS, so many
// instances share a CU.
template <int P, bool BW, typename TIO, bool MULTI, int NT_>
__global__ __launch_bounds__(NT_) void k_bottom(BottomArgsT<TIO> a)
{
    using B = Bottom<P, BW, NT_>;
    constexpr int NT = B::NT, S = B::S, STRIDE = B::STRIDE;
    __shared__ BottomLds<P, NT> sm;
    const int j = a.inst[blockIdx.x];
    if (a.st && a.st[j].done) return;
    // MULTI: the instances' own first bottom levels (V-cycle first visits)
    const int lb = MULTI ? a.lbs[j] : a.level, Lc = a.nlev[j] - 1;
    const TIO *const fl = MULTI ? a.f_lv[lb] : a.f;
    TIO *const xl = MULTI ? a.x_lv[lb] : a.x_out;
    const int64_t *const so = MULTI ? a.soff_lv[lb] : a.slab_off;
    const int64_t off = so[j];
    const int64_t N = so[j + 1] - off;
    if (lb == Lc) {
        // a single level (any size up to the largest coarsest level): the
        // exact solve, directly in global memory
        const double *tab = a.tab + ((int64_t)lb * a.batch + j) * a.tab_stride;
        const double u0 = (lb == 0 && a.u0) ? a.u0[j] : 0.0;
        coarse_scan<P, BW, NT, TIO, TIO>(fl + off * P, u0, xl + off * P, N, tab, &sm.scan);
        if (lb == 0 && a.st) {
            // squared residual of the result, one slab per thread and pass
            constexpr TabLayout L(P);
            const TIO *x = xl + off * P, *f = fl + off * P;
            double acc = 0.0;
            for (int64_t m = threadIdx.x; m < N; m += NT) {
                const int64_t pm = BW ? N - 1 - m : m;
                double w = 0.0;
                if (m > 0) {
                    const int64_t pl = BW ? pm + 1 : pm - 1;
#pragma unroll
                    for (int k = 0; k < P; ++k) w += tab[L.C() + k] * x[pl * P + k];
                }
#pragma unroll
                for (int k = 0; k < P; ++k) {
                    double r = f[pm * P + k] + tab[L.V() + k] * (w + (m == 0 ? u0 : 0.0));
#pragma unroll
                    for (int q = 0; q < P; ++q) r -= tab[L.A() + k * P + q] * x[pm * P + q];
                    acc += r * r;
                }
            }
            acc = block_sum<B::NW>(acc, sm.red);
            if (threadIdx.x == 0) finish_cycle(a.st, j, a.st[j], acc, a.ctl, a.mirror);
        }
        return;
    }
    int lw = lb;
    while ((N >> (lw - lb)) > B::WAVE_SLABS) ++lw;
    const B b{sm, lb, N, Lc, lw, a.nu1, a.nu2, a.gamma};
    {
        // tables of levels lb .. Lc and the transfer matrices into LDS, and
        // the right-hand side and initial guess of level lb (S slabs per
        // thread, physical order): every load issued before any LDS store
        constexpr int NTAB = kBottomMaxLevels * STRIDE + 2 * P * P;
        constexpr int TPT = (NTAB + NT - 1) / NT;
        const int ntab = (Lc - lb + 1) * STRIDE;
        double tv[TPT];
#pragma unroll
        for (int q = 0; q < TPT; ++q) {
            const int i = threadIdx.x + q * NT;
            tv[q] = 0.0;
            if (i < ntab)
                tv[q] = a.tab[((int64_t)(lb + i / STRIDE) * a.batch + j) * a.tab_stride + i % STRIDE];
            else if (i < ntab + 2 * P * P)
                tv[q] = a.R[i - ntab];
        }
        const int64_t m0 = (int64_t)threadIdx.x * S;
        TIO fv[S][P], xv[S][P];
        load_chunk<P, S, false, TIO>(fl + off * P, m0, N, fv);
        if (a.x_in) {
            load_chunk<P, S, false, TIO>(a.x_in + off * P, m0, N, xv);
        } else {
#pragma unroll
            for (int s = 0; s < S; ++s)
#pragma unroll
                for (int k = 0; k < P; ++k) xv[s][k] = (TIO)0;
        }
#pragma unroll
        for (int q = 0; q < TPT; ++q) {
            const int i = threadIdx.x + q * NT;
            if (i < ntab) sm.tab[i] = tv[q];
            else if (i < ntab + 2 * P * P) sm.R[i - ntab] = tv[q];
        }
        double fd[S][P], xd[S][P];
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int k = 0; k < P; ++k) {
                fd[s][k] = (double)fv[s][k];
                xd[s][k] = (double)xv[s][k];
            }
        store_chunk<P, S, false, double>(sm.f, m0, N, fd, 0, 0);
        store_chunk<P, S, false, double>(sm.x, m0, N, xd, 0, 0);
    }
    __syncthreads();
    if (a.u0 && threadIdx.x < P) {
        // fold u0 into the first slab in time (physical slab 0, forward only)
        constexpr TabLayout L(P);
        sm.f[threadIdx.x] += a.u0[j] * sm.tab[L.V() + threadIdx.x];
    }
    __syncthreads();
    const bool zero = a.x_in == nullptr;
    if (lb >= lw) {
        // the whole visit fits one wavefront
        if (threadIdx.x < 64) b.template visit<1>(lb, zero);
        __syncthreads();
    } else {
        b.template visit<B::NW>(lb, zero);
    }
    {
        // result of level lb back to global memory
        const int64_t m0 = (int64_t)threadIdx.x * S;
        double xd[S][P];
        TIO xo[S][P];
        load_chunk<P, S, false, double>(sm.x, m0, N, xd);
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int k = 0; k < P; ++k) xo[s][k] = (TIO)xd[s][k];
        store_chunk<P, S, false, TIO>(xl + off * P, m0, N, xo, 0, 0);
    }
    if (lb == 0 && a.st) {
        // squared residual of the result (level 0 of this instance): the
        // work-group finishes the cycle of its instance itself
        Ops<P> op;
        b.load_ops(op, 0);
        const int64_t m0 = (int64_t)threadIdx.x * S;
        double f[S][P], u[S][P], r[S][P];
        load_chunk<P, S, BW>(sm.f, m0, N, f);
        load_chunk<P, S, BW>(sm.x, m0, N, u);
        int phase = 0;
        residual<P, S, B::NW>(r, u, f, op, sm.xchg, phase);
        double acc = 0.0;
#pragma unroll
        for (int s = 0; s < S; ++s)
            if (m0 + s < N)   // slabs past the end see a nonzero left neighbour
#pragma unroll
                for (int k = 0; k < P; ++k) acc += r[s][k] * r[s][k];
        acc = block_sum<B::NW>(acc, sm.red);
        if (threadIdx.x == 0) finish_cycle(a.st, j, a.st[j], acc, a.ctl, a.mirror);
    }
}

// Per-tile sum of squares of the folded load vector (the initial residual).
template <int P>
__global__ __launch_bounds__(kLegThreads) void k_norm_f(const double *__restrict__ f,
                                                     const double *__restrict__ u0,
                                                     const double *__restrict__ tab, int tab_stride,
                                                     const int64_t *__restrict__ slab_off,
                                                     const int64_t *__restrict__ tile_off,
                                                     const int *__restrict__ tile_inst, int batch,
                                                     double *__restrict__ partial)
{
    constexpr int S = slabs_per_thread(P);
    constexpr TabLayout L(P);
    __shared__ double red[kLegWaves];
    const int64_t tile = blockIdx.x;
    const int j = batch == 1 ? 0 : tile_inst ? tile_inst[tile] : find_instance(tile_off, batch, tile);
    const int64_t t = tile - tile_off[j];
    const int64_t off = slab_off[j];
    const int64_t N = slab_off[j + 1] - off;
    const int64_t m0 = t * tile_slabs(P) + threadIdx.x * S;
    double x[S][P];
    load_chunk<P, S, false>(f + off * P, m0, N, x);
    double acc = 0.0;
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
        for (int k = 0; k < P; ++k) {
            double y = x[s][k];
            if (u0 && m0 + s == 0) y += u0[j] * tab[(int64_t)j * tab_stride + L.V() + k];
            acc += y * y;
        }
    acc = block_sum<kLegWaves>(acc, red);
    if (threadIdx.x == 0) partial[tile] = acc;
}

// One work-group per instance: sum its partials in a fixed order and update
// the convergence state (relative residual criterion of section 4.2).  After
// a cycle, instances without partials (no tile in the level-0 pass: their
// whole hierarchy ran in the bottom kernel, which updated their state) are
// left alone.  A solve's first launch (is_r0 with ctl_set) also installs
// the solve's control block `val` at ctl_set for the kernels after it (one
// launch instead of a host-to-device copy).
constexpr int kFinThreads = 1024;
__global__ __launch_bounds__(kFinThreads) void k_finalize(const double *__restrict__ partial,
                                                          const int64_t *__restrict__ norm_off,
                                                          InstState *__restrict__ st,
                                                          const Control *__restrict__ ctl,
                                                          HostHead *__restrict__ mirror, int is_r0,
                                                          Control *__restrict__ ctl_set,
                                                          Control val)
{
    __shared__ double red[kFinThreads / 64];
    const int j = blockIdx.x;
    if (ctl_set) {
        if (j == 0 && threadIdx.x == 0) *ctl_set = val;
        ctl = &val;
    }
    const int64_t lo = norm_off[j], hi = norm_off[j + 1];
    // the state is read once, here, so that its load overlaps the partials'
    const InstState s0 = st[j];
    // an instance outside the launch's tile list (lo == hi) is left alone
    if (lo == hi || (!is_r0 && s0.done)) return;
    // eight independent loads in flight per thread, summed in a fixed order
    double acc = 0.0;
    for (int64_t b = lo; b < hi; b += 8 * kFinThreads) {
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t i = b + q * kFinThreads + threadIdx.x;
            v[q] = i < hi ? partial[i] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) acc += v[q];
    }
    acc = block_sum<kFinThreads / 64>(acc, red);
    if (threadIdx.x != 0) return;
    if (!is_r0) {
        finish_cycle(st, j, s0, acc, ctl, mirror);
        return;
    }
    InstState s = s0;
    s.r0sq = acc;
    s.rsq = acc;
    s.prev_rsq = -1.0;
    s.cycles = 0;
    s.done = !isfinite(acc) ? 3 : (acc == 0.0 ? 1 : 0);
    st[j] = s;
    publish(mirror, s, ctl);
}

// Host copy for a batch (see HostHead): the number of running instances,
// the most cycles any of them wants queued and the most cycles run, reduced
// over the batch by one work-group, and (batches of at most kRunBits) which
// instances run, as bits.
__global__ __launch_bounds__(kFinThreads) void k_publish(const InstState *__restrict__ st,
                                                         int batch,
                                                         const Control *__restrict__ ctl,
                                                         HostHead *__restrict__ h,
                                                         unsigned *__restrict__ count)
{
    constexpr int NW = kFinThreads / 64;
    __shared__ int rn[NW], rw[NW], rc[NW];
    __shared__ unsigned bits[kRunBits / 32];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nwords = run_words(batch);
    int nrun = 0, want = 0, cyc = 0;
    // every lane of a wave takes part in each round (ballot)
    for (int j0 = 0; j0 < batch; j0 += kFinThreads) {
        const int j = j0 + threadIdx.x;
        bool run = false;
        if (j < batch) {
            const InstState s = st[j];
            cyc = max(cyc, s.cycles);
            run = running(s, ctl);
            if (run) {
                ++nrun;
                want = max(want, want_cycles(s, ctl));
            }
        }
        const unsigned long long m = __ballot(run);
        const int w = (j0 + wave * 64) / 32;
        if (lane == 0 && w < nwords) bits[w] = (unsigned)m;
        if (lane == 1 && w + 1 < nwords) bits[w + 1] = (unsigned)(m >> 32);
    }
    for (int off = 32; off > 0; off >>= 1) {
        nrun += __shfl_down(nrun, off, 64);
        want = max(want, __shfl_down(want, off, 64));
        cyc = max(cyc, __shfl_down(cyc, off, 64));
    }
    if (lane == 0) {
        rn[wave] = nrun;
        rw[wave] = want;
        rc[wave] = cyc;
    }
    __syncthreads();
    if (wave != 0) return;
    for (int w = 1; w < NW; ++w) {
        nrun += rn[w];
        want = max(want, rw[w]);
        cyc = max(cyc, rc[w]);
    }
    // the first wave writes the copy: begin, the bits (all lanes) and the
    // counts, then end after a release fence that orders every lane's stores
    unsigned n = 0;
    if (lane == 0) {
        n = *count + 1;
        *count = n;
    }
    n = __shfl(n, 0, 64);
    const long long v = ((long long)ctl->epoch << 32) | n;
    HostSum *m = reinterpret_cast<HostSum *>(h + 1);
    unsigned *hb = reinterpret_cast<unsigned *>(m + 1);
    if (lane == 0) __hip_atomic_store(&h->begin, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
    for (int w = lane; w < nwords; w += 64)
        __hip_atomic_store(&hb[w], bits[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    if (lane == 0) {
        __hip_atomic_store(&m->running, nrun, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&m->want, want, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&m->cycles, cyc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
    if (lane == 0) __hip_atomic_store(&h->end, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Left halos for the in-place level-0 pass, taken from the iterate: slot g
// of a tile list holds the last `halo` output slabs of tile g, which is
// what the pass before wrote there when it stored them to u.  Used where a
// batch's tile list changes between two cycles (the slots are numbered by
// the list).  One thread per slab of a slot; slabs past the end of an
// instance (never read) are zero.
template <int P, bool BW>
__global__ __launch_bounds__(kThreads) void k_seed(const double *__restrict__ u,
                                                   double *__restrict__ hb,
                                                   const int64_t *__restrict__ tile_off,
                                                   const int *__restrict__ tile_inst,
                                                   const int64_t *__restrict__ slab_off, int batch,
                                                   int64_t n0, int tile_out, int halo,
                                                   int64_t nslabs)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= nslabs) return;
    const int64_t g = i / halo;
    const int q = (int)(i - g * halo);
    int j = 0;
    int64_t t = g, off = 0, N = n0;
    if (batch > 1) {
        j = tile_inst[g];
        t = g - tile_off[j];
        off = slab_off[j];
        N = slab_off[j + 1] - off;
    }
    const int64_t m = (t + 1) * tile_out - halo + q;   // logical slab
    double v[P];
#pragma unroll
    for (int k = 0; k < P; ++k) v[k] = 0.0;
    if (m >= 0 && m < N) {
        const double *src = u + (off + (BW ? N - 1 - m : m)) * P;
#pragma unroll
        for (int k = 0; k < P; ++k) v[k] = src[k];
    }
#pragma unroll
    for (int k = 0; k < P; ++k) hb[i * P + k] = v[k];
}

// dlambda_j = -tau_j sum_n z_n^T diag(1/(2k+1)) u_n, in two deterministic
// stages: k_grad_partial leaves one partial sum per tile of S slabs per
// thread (all CUs stream u and z), k_grad_finish sums an instance's
// partials in a fixed order and adds du0_j = v^T z_1 (v[k] = (-1)^k).
template <int P>
__global__ __launch_bounds__(kLegThreads) void k_grad_partial(const double *__restrict__ u,
                                                          const double *__restrict__ z,
                                                          const int64_t *__restrict__ slab_off,
                                                          const int64_t *__restrict__ tile_off,
                                                          const int *__restrict__ tile_inst,
                                                          int batch, double *__restrict__ partial)
{
    constexpr int S = slabs_per_thread(P);
    __shared__ double red[kLegWaves];
    const int64_t tile = blockIdx.x;
    const int j = batch == 1 ? 0 : tile_inst[tile];
    const int64_t off = slab_off[j], N = slab_off[j + 1] - off;
    const int64_t m0 = (tile - tile_off[j]) * (int64_t)(kLegThreads * S) + threadIdx.x * S;
    double acc = 0.0;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int64_t m = m0 + s;
        if (m < N) {
            const double *zz = z + (off + m) * P, *uu = u + (off + m) * P;
#pragma unroll
            for (int k = 0; k < P; ++k) acc += zz[k] * uu[k] * (1.0 / (2.0 * k + 1.0));
        }
    }
    acc = block_sum<kLegWaves>(acc, red);
    if (threadIdx.x == 0) partial[tile] = acc;
}

template <int P>
__global__ __launch_bounds__(kThreads) void k_grad_finish(const double *__restrict__ partial,
                                                      const int64_t *__restrict__ tile_off,
                                                      const double *__restrict__ z,
                                                      const double *__restrict__ tau,
                                                      const int64_t *__restrict__ slab_off,
                                                      double *__restrict__ out)
{
    __shared__ double red[kWaves];
    const int j = blockIdx.x;
    const int64_t t0 = tile_off[j], t1 = tile_off[j + 1];
    double acc = 0.0;
    for (int64_t t = t0 + threadIdx.x; t < t1; t += kThreads) acc += partial[t];
    acc = block_sum<kWaves>(acc, red);
    if (threadIdx.x == 0) {
        const double *z1 = z + slab_off[j] * P;
        double d = 0.0;
        for (int k = 0; k < P; ++k) d += ((k & 1) ? -1.0 : 1.0) * z1[k];
        out[2 * j] = -tau[j] * acc;
        out[2 * j + 1] = d;
    }
}

}  // namespace

#define TMG_DISPATCH_P(P, ...)                        \
    switch (P) {                                      \
    case 1: { constexpr int PP = 1; __VA_ARGS__; } break; \
    case 2: { constexpr int PP = 2; __VA_ARGS__; } break; \
    case 3: { constexpr int PP = 3; __VA_ARGS__; } break; \
    case 4: { constexpr int PP = 4; __VA_ARGS__; } break; \
    case 5: { constexpr int PP = 5; __VA_ARGS__; } break; \
    case 6: { constexpr int PP = 6; __VA_ARGS__; } break; \
    default: return hipErrorInvalidValue;             \
    }

// Every P of the generic kernels (1 .. kMaxP).
#define TMG_PCASE(n, ...) case n: { constexpr int PP = n; __VA_ARGS__; } break;
#define TMG_DISPATCH_PALL(P, ...)                                                              \
    switch (P) {                                                                               \
    TMG_PCASE(1, __VA_ARGS__) TMG_PCASE(2, __VA_ARGS__) TMG_PCASE(3, __VA_ARGS__)              \
    TMG_PCASE(4, __VA_ARGS__) TMG_PCASE(5, __VA_ARGS__) TMG_PCASE(6, __VA_ARGS__)              \
    TMG_PCASE(7, __VA_ARGS__) TMG_PCASE(8, __VA_ARGS__) TMG_PCASE(9, __VA_ARGS__)              \
    TMG_PCASE(10, __VA_ARGS__) TMG_PCASE(11, __VA_ARGS__) TMG_PCASE(12, __VA_ARGS__)           \
    TMG_PCASE(13, __VA_ARGS__) TMG_PCASE(14, __VA_ARGS__) TMG_PCASE(15, __VA_ARGS__)           \
    TMG_PCASE(16, __VA_ARGS__) TMG_PCASE(17, __VA_ARGS__) TMG_PCASE(18, __VA_ARGS__)           \
    TMG_PCASE(19, __VA_ARGS__) TMG_PCASE(20, __VA_ARGS__) TMG_PCASE(21, __VA_ARGS__)           \
    default: return hipErrorInvalidValue;                                                      \
    }

// The generic kernels' launchers for one P, instantiated in tmg_generic.hip
// (compiled once per P).
template <int P>
hipError_t launch_gleg_p(bool backward, const LegArgsT<double> &a, int64_t ntiles, hipStream_t s);
template <int P>
hipError_t launch_gbottom_p(bool backward, const BottomArgsT<double> &a, int ninst, hipStream_t s);
template <int P>
hipError_t launch_gcoarse_p(bool backward, const CoarseArgs &a, int periodic, int ninst,
                            hipStream_t s);

template <typename T>
hipError_t launch_leg(int P, bool backward, const LegArgsT<T> &a, int64_t ntiles, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    if (a.generic) {
        if constexpr (std::is_same<T, double>::value) return launch_gleg(P, backward, a, ntiles, s);
        else return hipErrorInvalidValue;   // the FP32-inner cycle has no generic form
    }
    TMG_DISPATCH_P(P, {
        const dim3 grid((unsigned)ntiles), block(kLegThreads);
        // legs of a first visit from zero below level 0: the pruned forms
        const bool plain = a.touch && !a.u_in && !a.halo_in && !a.halo_out && !a.partial &&
                           !a.u0 && a.next == 0;
        const int leg = !plain ? 0
                        : (a.rc && !a.e && !a.e2 && !a.u_out && a.post == 0) ? 1
                        : (!a.rc && (a.e || a.e2)) ? 2 : 0;
        if (!a.touch && a.norm_f) {
            if constexpr (std::is_same<T, double>::value) {
                if (backward) hipLaunchKernelGGL((k_leg<PP, true, T, false, 4>), grid, block, 0, s, a);
                else hipLaunchKernelGGL((k_leg<PP, false, T, false, 4>), grid, block, 0, s, a);
            } else {
                return hipErrorInvalidValue;
            }
        } else if (!a.touch) {
            if (backward) hipLaunchKernelGGL((k_leg<PP, true, T, false, 0>), grid, block, 0, s, a);
            else hipLaunchKernelGGL((k_leg<PP, false, T, false, 0>), grid, block, 0, s, a);
        } else if (leg == 1) {
            if (backward) hipLaunchKernelGGL((k_leg<PP, true, T, true, 1>), grid, block, 0, s, a);
            else hipLaunchKernelGGL((k_leg<PP, false, T, true, 1>), grid, block, 0, s, a);
        } else if (leg == 2) {
            if (backward) hipLaunchKernelGGL((k_leg<PP, true, T, true, 2>), grid, block, 0, s, a);
            else hipLaunchKernelGGL((k_leg<PP, false, T, true, 2>), grid, block, 0, s, a);
        } else {
            if (backward) hipLaunchKernelGGL((k_leg<PP, true, T, true, 0>), grid, block, 0, s, a);
            else hipLaunchKernelGGL((k_leg<PP, false, T, true, 0>), grid, block, 0, s, a);
        }
    })
    return hipGetLastError();
}

template <typename T>
hipError_t launch_span(int P, bool backward, const SpanArgsT<T> &a, int64_t ntiles, hipStream_t s)
{
    TMG_DISPATCH_P(P, {
        const dim3 grid((unsigned)ntiles), block(kSpanThreads);
        if (backward) hipLaunchKernelGGL((k_span<PP, true, T>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_span<PP, false, T>), grid, block, 0, s, a);
    })
    return hipGetLastError();
}

// The bottom kernel's launcher for one P: instantiated in tmg_bottom.hip,
// which is compiled once per P (TMG_BOTTOM_P); launch_bottom dispatches.
template <typename TIO, int P>
hipError_t launch_bottom_p(bool backward, const BottomArgsT<TIO> &a, int ninst, hipStream_t s);

}  // namespace tmg
