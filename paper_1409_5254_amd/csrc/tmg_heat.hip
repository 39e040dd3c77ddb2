// Kernels of the space-time heat equation u_t - u_xx = f on (0,1), u = 0 at
// both ends (section 6: the time multigrid with a spatial solve inside each
// block Jacobi step): second-order finite differences on nx interior
// points, the DG-in-time discretisation at every point.  Arrays are
// [point][slab][k].  The block of one slab couples all its points,
//     A_h = I (x) K + L_h (x) M,   L_h = tridiag(-1, 2, -1) / h^2,
// a block-tridiagonal matrix in space with P x P blocks D = K + (2/h^2) M on
// the diagonal and E = -M / h^2 (diagonal) beside it; every block Jacobi
// step solves it exactly by block elimination over the points (factors
// C_i^{-1} and C_i^{-1} E per level, C_0 = D, C_i = D - E C_{i-1}^{-1} E).
//
// A work-group is one wavefront owning a tile of 64 consecutive slabs, one
// per lane: the end values of the left slab (time) come by a lane shift at
// every point, so the lanes walk the points in lock step without barriers.
// A tile keeps its slabs' iterate and the forward-elimination values in a
// workspace of its own ([point][lane][k], coalesced); its first `halo`
// slabs are recomputed copies of the left neighbour's and never stored.
#include <hip/hip_runtime.h>

#include "tmg_heat.h"

namespace tmg {
namespace {

constexpr int kHT = kHeatThreads;   // one wavefront

__device__ __forceinline__ double shr1(double x)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0x138, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0x138, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum(double x)
{
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    return x;
}

template <int P>
struct HLeg {
    const HeatArgs &a;
    int li;
    int64_t m;
    bool valid, out;
    double *wu, *wy;
    __device__ HLeg(const HeatArgs &a_) : a(a_)
    {
        li = threadIdx.x;
        m = (int64_t)blockIdx.x * a.tile_out - a.halo + li;
        valid = m >= 0 && m < a.N;
        out = li >= a.halo && valid;
        wu = a.ws + (int64_t)blockIdx.x * 2 * a.nx * kHT * P;
        wy = wu + (int64_t)a.nx * kHT * P;
    }
    __device__ double *U(int i) const { return wu + ((int64_t)i * kHT + li) * P; }
    __device__ double *Y(int i) const { return wy + ((int64_t)i * kHT + li) * P; }
    // right-hand side at point i (u0 folded into slab 0 at level 0)
    __device__ void rhs(int i, double (&x)[P]) const
    {
#pragma unroll
        for (int k = 0; k < P; ++k) x[k] = valid ? a.f[((int64_t)i * a.N + m) * P + k] : 0.0;
        if (a.u0 && m == 0)
#pragma unroll
            for (int k = 0; k < P; ++k) x[k] += a.u0[i] * ((k & 1) ? -1.0 : 1.0);
    }
    __device__ void ld(const double *p, double (&x)[P]) const
    {
#pragma unroll
        for (int k = 0; k < P; ++k) x[k] = p[k];
    }
    __device__ void st(double *p, const double (&x)[P]) const
    {
#pragma unroll
        for (int k = 0; k < P; ++k) p[k] = x[k];
    }
    // end value c^T u of the left slab (c = 1): lane 0 sees zero
    __device__ double wl(const double (&u)[P]) const
    {
        double w = 0.0;
#pragma unroll
        for (int k = 0; k < P; ++k) w += u[k];
        return shr1(w);
    }
    // u <- (1 - omega) u + omega A_h^{-1} (f + v w_left), nsweep times
    __device__ void sweeps(int nsweep) const
    {
        for (int s = 0; s < nsweep; ++s) {
            double y[P];
#pragma unroll
            for (int k = 0; k < P; ++k) y[k] = 0.0;
            for (int i = 0; i < a.nx; ++i) {
                double u[P], z[P];
                ld(U(i), u);
                const double w = wl(u);
                rhs(i, z);
#pragma unroll
                for (int k = 0; k < P; ++k)
                    z[k] += ((k & 1) ? -w : w) + a.Md[k] * a.ih2 * y[k];   // - E y_{i-1}
                const double *Ci = a.Cinv + (int64_t)i * P * P;
#pragma unroll
                for (int k = 0; k < P; ++k) {
                    double t = 0.0;
#pragma unroll
                    for (int l = 0; l < P; ++l) t += Ci[k * P + l] * z[l];
                    y[k] = t;
                }
                st(Y(i), y);
            }
            double x[P];
#pragma unroll
            for (int k = 0; k < P; ++k) x[k] = 0.0;
            for (int i = a.nx - 1; i >= 0; --i) {
                double yi[P], u[P];
                ld(Y(i), yi);
                const double *Gi = a.G + (int64_t)i * P * P;
                double xn[P];
#pragma unroll
                for (int k = 0; k < P; ++k) {
                    double t = yi[k];
#pragma unroll
                    for (int l = 0; l < P; ++l) t -= Gi[k * P + l] * x[l];
                    xn[k] = t;
                }
#pragma unroll
                for (int k = 0; k < P; ++k) x[k] = xn[k];
                ld(U(i), u);
#pragma unroll
                for (int k = 0; k < P; ++k) u[k] = a.omc * u[k] + a.om * x[k];
                st(U(i), u);
            }
        }
    }
    // residual at point i: f + v w_left - (K u_i + M (L_h u)_i); um, up the
    // neighbouring points' iterates (zero beyond the ends)
    __device__ void residual(int i, const double (&um)[P], const double (&u)[P],
                             const double (&up)[P], double (&r)[P]) const
    {
        const double w = wl(u);
        rhs(i, r);
#pragma unroll
        for (int k = 0; k < P; ++k) {
            double s = r[k] + ((k & 1) ? -w : w);
#pragma unroll
            for (int l = 0; l < P; ++l) s -= a.K[k * P + l] * u[l];
            s -= a.Md[k] * (2.0 * u[k] - um[k] - up[k]) * a.ih2;
            r[k] = s;
        }
    }
};

template <int P>
__global__ __launch_bounds__(kHT) void k_hleg(HeatArgs a)
{
    const HLeg<P> g(a);
    // the initial iterate of the tile's slabs into the workspace
    for (int i = 0; i < a.nx; ++i) {
        double u[P];
#pragma unroll
        for (int k = 0; k < P; ++k)
            u[k] = (a.u_in && g.valid) ? a.u_in[((int64_t)i * a.N + g.m) * P + k] : 0.0;
        g.st(g.U(i), u);
    }
    if (a.norm_f) {
        double acc = 0.0;
        for (int i = 0; i < a.nx; ++i) {
            double x[P];
            g.rhs(i, x);
#pragma unroll
            for (int k = 0; k < P; ++k) acc += g.out ? x[k] * x[k] : 0.0;
        }
        acc = wave_sum(acc);
        if (g.li == 0) a.partial[blockIdx.x] = acc;
    }
    g.sweeps(a.pre);
    if (a.e) {
        // u_m += R_i^T e_{m/2} at every point (i the parity of m)
        const int par = (int)(g.m & 1);
        const double *R = a.R + par * P * P;
        for (int i = 0; i < a.nx; ++i) {
            double u[P], e[P];
            g.ld(g.U(i), u);
#pragma unroll
            for (int k = 0; k < P; ++k)
                e[k] = g.valid ? a.e[((int64_t)i * a.Nc + g.m / 2) * P + k] : 0.0;
#pragma unroll
            for (int k = 0; k < P; ++k) {
                double t = 0.0;
#pragma unroll
                for (int l = 0; l < P; ++l) t += R[k * P + l] * e[l];
                u[k] += t;
            }
            g.st(g.U(i), u);
        }
    }
    g.sweeps(a.post);
    if (a.u_out && g.out)
        for (int i = 0; i < a.nx; ++i) {
            double u[P];
            g.ld(g.U(i), u);
            g.st(a.u_out + ((int64_t)i * a.N + g.m) * P, u);
        }
    const bool norm = a.partial && !a.norm_f;
    if (!norm && !a.rc) return;
    g.sweeps(a.next);
    double acc = 0.0;
    double um[P], u[P], up[P];
#pragma unroll
    for (int k = 0; k < P; ++k) um[k] = 0.0;
    g.ld(g.U(0), u);
    for (int i = 0; i < a.nx; ++i) {
        if (i + 1 < a.nx) g.ld(g.U(i + 1), up);
        else
#pragma unroll
            for (int k = 0; k < P; ++k) up[k] = 0.0;
        double r[P];
        g.residual(i, um, u, up, r);
        if (norm)
#pragma unroll
            for (int k = 0; k < P; ++k) acc += g.out ? r[k] * r[k] : 0.0;
        if (a.rc) {
            // rc_{m/2} = R_1 r_m + R_2 r_{m+1}: the even slab's lane takes
            // its partner's residual from the next lane
            double rn[P];
#pragma unroll
            for (int k = 0; k < P; ++k) rn[k] = __shfl_down(r[k], 1, 64);
            if (g.out && !(g.m & 1)) {
                double rc[P];
#pragma unroll
                for (int k = 0; k < P; ++k) {
                    double t = 0.0;
#pragma unroll
                    for (int l = 0; l < P; ++l)
                        t += a.R[l * P + k] * r[l] + a.R[P * P + l * P + k] * rn[l];
                    rc[k] = t;
                }
                g.st(a.rc + ((int64_t)i * a.Nc + g.m / 2) * P, rc);
            }
        }
#pragma unroll
        for (int k = 0; k < P; ++k) {
            um[k] = u[k];
            u[k] = up[k];
        }
    }
    if (norm) {
        acc = wave_sum(acc);
        if (g.li == 0) a.partial[blockIdx.x] = acc;
    }
}

// Exact solve on the coarsest level: forward substitution over its slabs,
// each slab block solved by the elimination over the points (one lane).
template <int P>
__global__ __launch_bounds__(kHT) void k_hcoarse(HeatArgs a)
{
    if (threadIdx.x != 0) return;
    double *y = a.ws;
    for (int64_t n = 0; n < a.N; ++n) {
        double yp[P];
#pragma unroll
        for (int k = 0; k < P; ++k) yp[k] = 0.0;
        for (int i = 0; i < a.nx; ++i) {
            double z[P];
            double w = 0.0;
            if (n > 0)
#pragma unroll
                for (int k = 0; k < P; ++k) w += a.u_out[((int64_t)i * a.N + n - 1) * P + k];
#pragma unroll
            for (int k = 0; k < P; ++k) {
                z[k] = a.f[((int64_t)i * a.N + n) * P + k] + ((k & 1) ? -w : w) +
                       a.Md[k] * a.ih2 * yp[k];
                if (a.u0 && n == 0) z[k] += a.u0[i] * ((k & 1) ? -1.0 : 1.0);
            }
            const double *Ci = a.Cinv + (int64_t)i * P * P;
#pragma unroll
            for (int k = 0; k < P; ++k) {
                double t = 0.0;
#pragma unroll
                for (int l = 0; l < P; ++l) t += Ci[k * P + l] * z[l];
                yp[k] = t;
                y[i * P + k] = t;
            }
        }
        double x[P];
#pragma unroll
        for (int k = 0; k < P; ++k) x[k] = 0.0;
        for (int i = a.nx - 1; i >= 0; --i) {
            const double *Gi = a.G + (int64_t)i * P * P;
            double xn[P];
#pragma unroll
            for (int k = 0; k < P; ++k) {
                double t = y[i * P + k];
#pragma unroll
                for (int l = 0; l < P; ++l) t -= Gi[k * P + l] * x[l];
                xn[k] = t;
            }
#pragma unroll
            for (int k = 0; k < P; ++k) {
                x[k] = xn[k];
                a.u_out[((int64_t)i * a.N + n) * P + k] = xn[k];
            }
        }
    }
}

// Sum of the tile partials in a fixed order (one work-group).
__global__ __launch_bounds__(256) void k_hsum(const double *partial, int64_t n, double *out)
{
    __shared__ double red[4];
    double acc = 0.0;
    for (int64_t t = threadIdx.x; t < n; t += 256) acc += partial[t];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) *out = red[0] + red[1] + red[2] + red[3];
}

}  // namespace

#define TMG_HEAT_P(P, ...)                                    \
    switch (P) {                                              \
    case 1: { constexpr int PP = 1; __VA_ARGS__; } break;     \
    case 2: { constexpr int PP = 2; __VA_ARGS__; } break;     \
    case 3: { constexpr int PP = 3; __VA_ARGS__; } break;     \
    case 4: { constexpr int PP = 4; __VA_ARGS__; } break;     \
    case 5: { constexpr int PP = 5; __VA_ARGS__; } break;     \
    case 6: { constexpr int PP = 6; __VA_ARGS__; } break;     \
    default: return hipErrorInvalidValue;                     \
    }

hipError_t launch_hleg(int P, const HeatArgs &a, int64_t ntiles, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    TMG_HEAT_P(P, { hipLaunchKernelGGL((k_hleg<PP>), dim3((unsigned)ntiles), dim3(kHT), 0, s, a); })
    return hipGetLastError();
}

hipError_t launch_hcoarse(int P, const HeatArgs &a, hipStream_t s)
{
    TMG_HEAT_P(P, { hipLaunchKernelGGL((k_hcoarse<PP>), dim3(1), dim3(kHT), 0, s, a); })
    return hipGetLastError();
}

hipError_t launch_hsum(const double *partial, int64_t n, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_hsum, dim3(1), dim3(256), 0, s, partial, n, out);
    return hipGetLastError();
}

}  // namespace tmg
