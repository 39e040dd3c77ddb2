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
//
// The walks over the points are sequential (the elimination carries a value
// from point to point), so they are pipelined: points are loaded in blocks,
// a block's loads issued before the previous block's arithmetic runs.  The
// first sweep of a leg reads the caller's iterate (and adds the prolongated
// correction) on its way, and the last back substitution writes the result
// and the residual, so a leg makes 2 walks per sweep and no other pass.
#include <hip/hip_runtime.h>

#include "tmg_heat.h"

namespace tmg {
namespace {

constexpr int kHT = kHeatThreads;   // one wavefront

// The tables of a launch (elimination factors, K, M, transfer, u0) are not
// written while it runs: they are read through the constant address space,
// as scalar loads of uniform addresses, whose waits do not hold up the
// vector loads in flight.
typedef __attribute__((address_space(4))) const double cdouble;
__device__ __forceinline__ const cdouble *ro(const double *p) { return (const cdouble *)p; }

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

// Points per block of the pipelined walks (two register buffers of up to
// four B x P arrays): about 8 coefficients per array, or 4 in the lean
// variant, whose fewer registers fit 3 wavefronts per SIMD (launches with
// more tiles than 2 wavefronts per SIMD would run in two rounds).
template <int P>
constexpr int kHB = P > 3 ? 1 : ((8 / P) < 2 ? 2 : 8 / P);
template <int P>
constexpr int kHBLean = (4 / P) < 1 ? 1 : 4 / P;
// partitioned legs with their tables in LDS (wider work-groups, at most 256
// registers); with the tables in global memory, kHBLean
template <int P>
constexpr int kHBPart = P == 1 ? 4 : kHB<P>;

// Walks blocks 0 .. nb-1 (or nb-1 .. 0 when rev): load(b, buf) issues the
// loads of block b into a register buffer, run(b, buf) consumes it.  The
// next block's loads are issued before a block runs (past the last block
// they fetch the last block again), and an empty asm with a memory clobber
// keeps the compiler from moving them down to their uses.
template <class Buf, class Load, class Run>
__device__ __forceinline__ void pipe2(int nb, bool rev, Load &&load, Run &&run)
{
    if (nb <= 0) return;
    Buf A, Q;
    const int st = rev ? -1 : 1;
    auto clampb = [&](int x) { return x < 0 ? 0 : (x >= nb ? nb - 1 : x); };
    int b = rev ? nb - 1 : 0;
    load(b, A);
    for (int t = 0; t < nb; t += 2, b += 2 * st) {
        load(clampb(b + st), Q);
        __asm__ volatile("" ::: "memory");
        run(b, A);
        if (t + 1 >= nb) break;
        load(clampb(b + 2 * st), A);
        __asm__ volatile("" ::: "memory");
        run(b + st, Q);
    }
}

// Where a walk takes the iterate from: the tile's workspace, the caller's
// u_in, or zero (u_in null).
enum HSrc { kFromWs = 0, kFromIn = 1, kFromZero = 2 };

template <int P, int B, bool TL = false>
struct HLeg {
    // up to P = 3 the per-point factors travel with the prefetched data and
    // the small slab tables stay in registers; above, both are read per
    // point through the constant address space.  TL: the per-point tables
    // are in LDS (copied there by the kernel) and read where they are used.
    static constexpr bool kRegTab = P <= 3;
    static constexpr bool kPre = kRegTab && !TL;
    const HeatArgs &a;
    int li, nb;
    int i0, i1;                 // the points this wavefront walks
    const double *tC, *tG;      // its elimination factors C_i^{-1}, C_i^{-1} E
    const double *tSL, *tSR;    // partitioned sweeps: the spikes
    int64_t m, mc;   // the lane's slab, and that slab clamped into the level
    bool valid, out, resid, norm, odd;
    double *wu, *wy;
    double mdh[P];                          // diag(M) / h^2
    double Kt[kRegTab ? P * P : 1];         // K
    double Rt[kRegTab ? 2 * P * P : 1];     // R_1^T, R_2^T
    __device__ __forceinline__ HLeg(const HeatArgs &a_, int i0_, int i1_, const double *tC_,
                                    const double *tG_, const double *tSL_ = nullptr,
                                    const double *tSR_ = nullptr)
        : a(a_), i0(i0_), i1(i1_), tC(tC_), tG(tG_), tSL(tSL_), tSR(tSR_)
    {
        li = threadIdx.x & (kHT - 1);
        m = (int64_t)blockIdx.x * a.tile_out - a.halo + li;
        valid = m >= 0 && m < a.N;
        mc = m < 0 ? 0 : (m >= a.N ? a.N - 1 : m);
        odd = m & 1;
        out = li >= a.halo && valid;
        nb = (i1 - i0 + B - 1) / B;
        norm = a.partial && !a.norm_f;
        resid = norm || a.rc;
        wu = a.ws + (int64_t)blockIdx.x * 2 * a.nx * kHT * P;
        wy = wu + (int64_t)a.nx * kHT * P;
#pragma unroll
        for (int k = 0; k < P; ++k) mdh[k] = ro(a.Md)[k] * a.ih2;
        if constexpr (kRegTab) {
#pragma unroll
            for (int q = 0; q < P * P; ++q) Kt[q] = ro(a.K)[q];
#pragma unroll
            for (int q = 0; q < 2 * P * P; ++q) Rt[q] = ro(a.R)[q];
        }
    }
    // entry idx of a per-point table
    __device__ __forceinline__ double tab(const double *T, int64_t idx) const
    {
        if constexpr (TL) return T[idx];
        else return ro(T)[idx];
    }
    __device__ __forceinline__ double Kc(int q) const
    {
        if constexpr (kRegTab) return Kt[q];
        else return ro(a.K)[q];
    }
    __device__ __forceinline__ double Rc(int q) const
    {
        if constexpr (kRegTab) return Rt[q];
        else return ro(a.R)[q];
    }
    // Loads are issued without branches: a lane outside the level loads its
    // clamped slab, a point past the walk's last loads the last point.  A lane
    // outside the level computes on that copy, and no slab of the level
    // reads it: a lane takes the end value of the lane on its left, and
    // slab 0 takes u0 instead (lanes past the last slab are on the right);
    // outputs are written, and residuals summed, for the tile's own slabs
    // only.
    __device__ __forceinline__ int row(int i) const { return i < i1 ? i : i1 - 1; }
    __device__ __forceinline__ double *U(int i) const { return wu + ((int64_t)i * kHT + li) * P; }
    __device__ __forceinline__ double *Y(int i) const { return wy + ((int64_t)i * kHT + li) * P; }
    template <int n>
    __device__ __forceinline__ void ldn(const double *p, double (&x)[n]) const
    {
#pragma unroll
        for (int k = 0; k < n; ++k) x[k] = p[k];
    }
    __device__ __forceinline__ void ld(const double *p, double (&x)[P]) const { ldn<P>(p, x); }
    __device__ __forceinline__ void st(double *p, const double (&x)[P]) const
    {
#pragma unroll
        for (int k = 0; k < P; ++k) p[k] = x[k];
    }
    // the lane's slab of a [point][slab][k] array at point i
    __device__ __forceinline__ const double *at(const double *v, int i) const
    {
        return v + ((int64_t)row(i) * a.N + mc) * P;
    }
    // right-hand side f at point i and u0 at the point (zero above level
    // 0), which enters slab 0 as its left end value
    __device__ __forceinline__ void ld_rhs(int i, double (&x)[P], double &g) const
    {
        ld(at(a.f, i), x);
        g = a.u0[row(i)];
    }
    // the iterate at point i
    template <int SRC>
    __device__ __forceinline__ void ld_iter(int i, double (&u)[P]) const
    {
        if constexpr (SRC == kFromWs) ld(U(row(i)), u);
        else if constexpr (SRC == kFromIn) ld(at(a.u_in, i), u);
        else
#pragma unroll
            for (int k = 0; k < P; ++k) u[k] = 0.0;
    }
    __device__ __forceinline__ void ld_e(int i, double (&e)[P]) const
    {
        ld(a.e + ((int64_t)row(i) * a.Nc + mc / 2) * P, e);
    }
    // the per-point factor table T (C_i^{-1} or C_i^{-1} E) at point i
    __device__ __forceinline__ void ld_tab(const double *T, int i, double (&c)[P * P]) const
    {
        ldn<P * P>(T + (int64_t)row(i) * P * P, c);
    }
    // ... and at the mirrored point nx-1-i: the factors of the elimination
    // down the points (the spatial operator has the same blocks E on both
    // sides of D, so eliminating from the last point gives C'_i = C_{nx-1-i})
    __device__ __forceinline__ void ld_tab_m(const double *T, int i, double (&c)[P * P]) const
    {
        ldn<P * P>(T + (int64_t)(a.nx - 1 - row(i)) * P * P, c);
    }
    // u_m += R_i^T e_{m/2} (i the parity of m)
    __device__ __forceinline__ void add_e(const double (&e)[P], double (&u)[P]) const
    {
#pragma unroll
        for (int k = 0; k < P; ++k) {
            double t = 0.0;
#pragma unroll
            for (int l = 0; l < P; ++l) t += (odd ? Rc(P * P + k * P + l) : Rc(k * P + l)) * e[l];
            u[k] += t;
        }
    }
    // end value c^T u of the left slab (c = 1): lane 0 sees zero, slab 0
    // the initial value g
    __device__ __forceinline__ double wl(const double (&u)[P], double g) const
    {
        double w = u[0];
#pragma unroll
        for (int k = 1; k < P; ++k) w += u[k];
        w = shr1(w);
        return m == 0 ? g : w;
    }
    // residual at point i: f + v w_left - (K u_i + M (L_h u)_i), with um, up
    // the neighbouring points' iterates (zero beyond the ends), fi the f and
    // g the u0 of the point; its square into acc, its restriction into rc
    __device__ __forceinline__ void resid_point(int i, const double (&um)[P], const double (&u)[P],
                                                const double (&up)[P], const double (&fi)[P],
                                                double g, double &acc) const
    {
        const double w = wl(u, g);
        double r[P];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            double s = fi[k] + ((k & 1) ? -w : w);
#pragma unroll
            for (int l = 0; l < P; ++l) s -= Kc(k * P + l) * u[l];
            s -= ro(a.Md)[k] * (2.0 * u[k] - um[k] - up[k]) * a.ih2;
            r[k] = s;
        }
        if (norm)
#pragma unroll
            for (int k = 0; k < P; ++k) acc += out ? r[k] * r[k] : 0.0;
        if (a.rc) {
            // rc_{m/2} = R_1 r_m + R_2 r_{m+1}: the even slab's lane takes
            // its partner's residual from the next lane
            double rn[P];
#pragma unroll
            for (int k = 0; k < P; ++k) rn[k] = __shfl_down(r[k], 1, 64);
            if (out && !odd) {
                double rc[P];
#pragma unroll
                for (int k = 0; k < P; ++k) {
                    double t = 0.0;
#pragma unroll
                    for (int l = 0; l < P; ++l) t += Rc(l * P + k) * r[l] + Rc(P * P + l * P + k) * rn[l];
                    rc[k] = t;
                }
                st(a.rc + ((int64_t)i * a.Nc + m / 2) * P, rc);
            }
        }
    }
    // Forward elimination of one damped block Jacobi sweep: y_i = C_i^{-1}
    // (f_i + v w_left,i - E y_{i-1}) into the workspace.  The iterate from
    // SRC; ADDE: the prolongated correction is added first; unless it came
    // unchanged from the workspace, the iterate is stored there on the way.
    template <int SRC, bool ADDE>
    __device__ __forceinline__ void forward() const
    {
        struct Buf {
            double u[B][P], z[B][P], e[ADDE ? B : 1][P], c[kPre ? B : 1][P * P], g[B];
        };
        double y[P];
#pragma unroll
        for (int k = 0; k < P; ++k) y[k] = 0.0;
        pipe2<Buf>(
            nb, false,
            [&](int b, Buf &q) {
#pragma unroll
                for (int j = 0; j < B; ++j) {
                    ld_iter<SRC>(i0 + b * B + j, q.u[j]);
                    if constexpr (ADDE) ld_e(i0 + b * B + j, q.e[j]);
                    ld_rhs(i0 + b * B + j, q.z[j], q.g[j]);
                    if constexpr (kPre) ld_tab(tC, i0 + b * B + j, q.c[j]);
                }
            },
            [&](int b, Buf &q) {
#pragma unroll
                for (int j = 0; j < B; ++j) {
                    const int i = i0 + b * B + j;
                    if (i < i1) {
                        if constexpr (ADDE) add_e(q.e[j], q.u[j]);
                        if constexpr (SRC != kFromWs || ADDE) st(U(i), q.u[j]);
                        const double w = wl(q.u[j], q.g[j]);
                        double z[P];
#pragma unroll
                        for (int k = 0; k < P; ++k)   // - E y_{i-1} = + M y_{i-1} / h^2
                            z[k] = q.z[j][k] + ((k & 1) ? -w : w) + mdh[k] * y[k];
#pragma unroll
                        for (int k = 0; k < P; ++k) {
                            double t = 0.0;
#pragma unroll
                            for (int l = 0; l < P; ++l) {
                                double c;
                                if constexpr (kPre) c = q.c[j][k * P + l];
                                else c = tab(tC, (int64_t)i * P * P + k * P + l);
                                t += c * z[l];
                            }
                            y[k] = t;
                        }
                        st(Y(i), y);
                    }
                }
            });
    }
    // Back substitution x_i = y_i - C_i^{-1} E x_{i+1} and the damped update
    // u_i <- (1 - omega) u_i + omega x_i.  FIN (the leg's last sweep): the
    // result goes to u_out and, one point behind, into the residual, and the
    // workspace is not written.
    template <bool FIN>
    __device__ __forceinline__ void backward(double &acc) const
    {
        struct Buf {
            double y[B][P], u[B][P], f[FIN ? B : 1][P], c[kPre ? B : 1][P * P], g[FIN ? B : 1];
        };
        double x[P], u1[P], u2[P], f1[P], g1 = 0.0;   // FIN: result at i+1, i+2; f, u0 at i+1
#pragma unroll
        for (int k = 0; k < P; ++k) x[k] = u1[k] = u2[k] = f1[k] = 0.0;
        pipe2<Buf>(
            nb, true,
            [&](int b, Buf &q) {
#pragma unroll
                for (int j = 0; j < B; ++j) {
                    ld(Y(row(i0 + b * B + j)), q.y[j]);
                    ld(U(row(i0 + b * B + j)), q.u[j]);
                    if constexpr (FIN) ld_rhs(i0 + b * B + j, q.f[j], q.g[j]);
                    if constexpr (kPre) ld_tab(tG, i0 + b * B + j, q.c[j]);
                }
            },
            [&](int b, Buf &q) {
#pragma unroll
                for (int j = B - 1; j >= 0; --j) {
                    const int i = i0 + b * B + j;
                    if (i < i1) {
                        double xn[P];
#pragma unroll
                        for (int k = 0; k < P; ++k) {
                            double t = q.y[j][k];
#pragma unroll
                            for (int l = 0; l < P; ++l) {
                                double c;
                                if constexpr (kPre) c = q.c[j][k * P + l];
                                else c = tab(tG, (int64_t)i * P * P + k * P + l);
                                t -= c * x[l];
                            }
                            xn[k] = t;
                        }
                        double u[P];
#pragma unroll
                        for (int k = 0; k < P; ++k) {
                            x[k] = xn[k];
                            u[k] = a.omc * q.u[j][k] + a.om * xn[k];
                        }
                        if constexpr (!FIN) {
                            st(U(i), u);
                        } else {
                            if (a.u_out && out) st(a.u_out + ((int64_t)i * a.N + m) * P, u);
                            if (resid && i + 1 < i1) resid_point(i + 1, u, u1, u2, f1, g1, acc);
#pragma unroll
                            for (int k = 0; k < P; ++k) {
                                u2[k] = u1[k];
                                u1[k] = u[k];
                                f1[k] = q.f[j][k];
                            }
                            g1 = q.g[j];
                        }
                    }
                }
            });
        if constexpr (FIN)
            if (resid) {
                double z0[P];
#pragma unroll
                for (int k = 0; k < P; ++k) z0[k] = 0.0;
                resid_point(i0, z0, u1, u2, f1, g1, acc);
            }
    }
    // The leg's outputs from an iterate no sweep follows (from SRC), after
    // adding the correction when ADDE: u_out and, one point behind, the
    // residual.
    template <int SRC, bool ADDE>
    __device__ __forceinline__ void final_pass(double &acc) const
    {
        struct Buf {
            double u[B][P], f[B][P], e[ADDE ? B : 1][P], g[B];
        };
        double um[P], uc[P], fc[P], gc = 0.0;   // iterate at i-2, i-1; f, u0 at i-1
#pragma unroll
        for (int k = 0; k < P; ++k) um[k] = uc[k] = fc[k] = 0.0;
        pipe2<Buf>(
            nb, false,
            [&](int b, Buf &q) {
#pragma unroll
                for (int j = 0; j < B; ++j) {
                    ld_iter<SRC>(i0 + b * B + j, q.u[j]);
                    if constexpr (ADDE) ld_e(i0 + b * B + j, q.e[j]);
                    ld_rhs(i0 + b * B + j, q.f[j], q.g[j]);
                }
            },
            [&](int b, Buf &q) {
#pragma unroll
                for (int j = 0; j < B; ++j) {
                    const int i = i0 + b * B + j;
                    if (i < i1) {
                        if constexpr (ADDE) add_e(q.e[j], q.u[j]);
                        if (a.u_out && out) st(a.u_out + ((int64_t)i * a.N + m) * P, q.u[j]);
                        if (resid && i > 0) resid_point(i - 1, um, uc, q.u[j], fc, gc, acc);
#pragma unroll
                        for (int k = 0; k < P; ++k) {
                            um[k] = uc[k];
                            uc[k] = q.u[j][k];
                            fc[k] = q.f[j][k];
                        }
                        gc = q.g[j];
                    }
                }
            });
        if (resid) {
            double z0[P];
#pragma unroll
            for (int k = 0; k < P; ++k) z0[k] = 0.0;
            resid_point(i1 - 1, um, uc, z0, fc, gc, acc);
        }
    }
    // squared norm of the right-hand side (the tile's own slabs)
    __device__ __forceinline__ void norm_rhs(double &acc) const
    {
        struct Buf {
            double f[B][P], g[B];
        };
        pipe2<Buf>(
            nb, false,
            [&](int b, Buf &q) {
#pragma unroll
                for (int j = 0; j < B; ++j) ld_rhs(i0 + b * B + j, q.f[j], q.g[j]);
            },
            [&](int b, Buf &q) {
#pragma unroll
                for (int j = 0; j < B; ++j)
                    if (i0 + b * B + j < i1) {
                        // the folded f + v u0 of slab 0
                        const double g = m == 0 ? q.g[j] : 0.0;
#pragma unroll
                        for (int k = 0; k < P; ++k) {
                            const double x = q.f[j][k] + ((k & 1) ? -g : g);
                            acc += out ? x * x : 0.0;
                        }
                    }
            });
    }

    // ---- Legs of two sweeps (whole point range).  The first sweep's back
    // substitution and the second sweep's elimination run in one walk down
    // the points (the second eliminates from the last point: C'_i =
    // C_{nx-1-i}, C'^{-1}_i E = C_{nx-1-i}^{-1} E), whose back substitution
    // then runs up the points with the leg's outputs: three walks instead of
    // four.

    // x_i = y_i - C_i^{-1} E x_{i+1} and u_i <- (1 - omega) u_i + omega x_i
    // into the workspace; then y'_i = C'^{-1}_i (f_i + v w_i - E y'_{i+1}) with
    // w_i the left slab's new end value, into Y (whose y_i is consumed).
    __device__ __forceinline__ void bsub_elim_down() const
    {
        constexpr int B2 = B > 1 ? B / 2 : 1;
        const int nb2 = (i1 - i0 + B2 - 1) / B2;
        struct Buf {
            double y[B2][P], u[B2][P], f[B2][P], g[B2], cg[kPre ? B2 : 1][P * P],
                cc[kPre ? B2 : 1][P * P];
        };
        double x[P], yp[P];
#pragma unroll
        for (int k = 0; k < P; ++k) x[k] = yp[k] = 0.0;
        pipe2<Buf>(
            nb2, true,
            [&](int b, Buf &q) {
#pragma unroll
                for (int j = 0; j < B2; ++j) {
                    const int i = i0 + b * B2 + j;
                    ld(Y(row(i)), q.y[j]);
                    ld(U(row(i)), q.u[j]);
                    ld_rhs(i, q.f[j], q.g[j]);
                    if constexpr (kPre) {
                        ld_tab(tG, i, q.cg[j]);
                        ld_tab_m(tC, i, q.cc[j]);
                    }
                }
            },
            [&](int b, Buf &q) {
#pragma unroll
                for (int j = B2 - 1; j >= 0; --j) {
                    const int i = i0 + b * B2 + j;
                    if (i < i1) {
                        double un[P];
#pragma unroll
                        for (int k = 0; k < P; ++k) {
                            double t = q.y[j][k];
#pragma unroll
                            for (int l = 0; l < P; ++l) {
                                double c;
                                if constexpr (kPre) c = q.cg[j][k * P + l];
                                else c = tab(tG, (int64_t)i * P * P + k * P + l);
                                t -= c * x[l];
                            }
                            un[k] = t;
                        }
#pragma unroll
                        for (int k = 0; k < P; ++k) {
                            x[k] = un[k];
                            un[k] = a.omc * q.u[j][k] + a.om * un[k];
                        }
                        st(U(i), un);
                        const double w = wl(un, q.g[j]);
                        double z[P];
#pragma unroll
                        for (int k = 0; k < P; ++k)   // - E y'_{i+1} = + M y'_{i+1} / h^2
                            z[k] = q.f[j][k] + ((k & 1) ? -w : w) + mdh[k] * yp[k];
#pragma unroll
                        for (int k = 0; k < P; ++k) {
                            double t = 0.0;
#pragma unroll
                            for (int l = 0; l < P; ++l) {
                                double c;
                                if constexpr (kPre) c = q.cc[j][k * P + l];
                                else c = tab(tC, (int64_t)(a.nx - 1 - i) * P * P + k * P + l);
                                t += c * z[l];
                            }
                            yp[k] = t;
                        }
                        st(Y(i), yp);
                    }
                }
            });
    }
    // The back substitution of the elimination down the points, up the
    // points: x_i = y'_i - C'^{-1}_i E x_{i-1}, the damped update, the result
    // to u_out and, one point behind, into the residual.
    __device__ __forceinline__ void bsub_up_fin(double &acc) const
    {
        struct Buf {
            double y[B][P], u[B][P], f[B][P], g[B], cg[kPre ? B : 1][P * P];
        };
        double x[P], um[P], uc[P], fc[P], gc = 0.0;   // chain; iterate at i-2, i-1; f, u0 at i-1
#pragma unroll
        for (int k = 0; k < P; ++k) x[k] = um[k] = uc[k] = fc[k] = 0.0;
        pipe2<Buf>(
            nb, false,
            [&](int b, Buf &q) {
#pragma unroll
                for (int j = 0; j < B; ++j) {
                    const int i = i0 + b * B + j;
                    ld(Y(row(i)), q.y[j]);
                    ld(U(row(i)), q.u[j]);
                    ld_rhs(i, q.f[j], q.g[j]);
                    if constexpr (kPre) ld_tab_m(tG, i, q.cg[j]);
                }
            },
            [&](int b, Buf &q) {
#pragma unroll
                for (int j = 0; j < B; ++j) {
                    const int i = i0 + b * B + j;
                    if (i < i1) {
                        double un[P];
#pragma unroll
                        for (int k = 0; k < P; ++k) {
                            double t = q.y[j][k];
#pragma unroll
                            for (int l = 0; l < P; ++l) {
                                double c;
                                if constexpr (kPre) c = q.cg[j][k * P + l];
                                else c = tab(tG, (int64_t)(a.nx - 1 - i) * P * P + k * P + l);
                                t -= c * x[l];
                            }
                            un[k] = t;
                        }
#pragma unroll
                        for (int k = 0; k < P; ++k) {
                            x[k] = un[k];
                            un[k] = a.omc * q.u[j][k] + a.om * un[k];
                        }
                        if (a.u_out && out) st(a.u_out + ((int64_t)i * a.N + m) * P, un);
                        if (resid && i > i0) resid_point(i - 1, um, uc, un, fc, gc, acc);
#pragma unroll
                        for (int k = 0; k < P; ++k) {
                            um[k] = uc[k];
                            uc[k] = un[k];
                            fc[k] = q.f[j][k];
                        }
                        gc = q.g[j];
                    }
                }
            });
        if (resid) {
            double z0[P];
#pragma unroll
            for (int k = 0; k < P; ++k) z0[k] = 0.0;
            resid_point(i1 - 1, um, uc, z0, fc, gc, acc);
        }
    }

    // ---- Partitioned sweeps.  K wavefronts share the tile, wavefront c
    // walking the chunk [i0, i1) of the points with the factors of the
    // chunk's own system (the elimination restarted at i0).  With v the
    // solution of that system (zero beyond the chunk) and the spikes
    // S^L = A_c^{-1} (e_first (x) E), S^R = A_c^{-1} (e_last (x) E), the
    // block row's solution is x = v - S^L x_{i0-1} - S^R x_{i1}; the values
    // at the chunk ends solve a reduced system of 2K blocks, whose inverse
    // is a table of the level.

    // Back substitution of the chunk's system, v_i = y_i - C_i^{-1} E v_{i+1},
    // into Y; v at the chunk's first and last points into vF, vL.
    __device__ __forceinline__ void backward_local(double (&vF)[P], double (&vL)[P]) const
    {
        struct Buf {
            double y[B][P], c[kPre ? B : 1][P * P];
        };
        double x[P];
#pragma unroll
        for (int k = 0; k < P; ++k) x[k] = vF[k] = vL[k] = 0.0;
        pipe2<Buf>(
            nb, true,
            [&](int b, Buf &q) {
#pragma unroll
                for (int j = 0; j < B; ++j) {
                    ld(Y(row(i0 + b * B + j)), q.y[j]);
                    if constexpr (kPre) ld_tab(tG, i0 + b * B + j, q.c[j]);
                }
            },
            [&](int b, Buf &q) {
#pragma unroll
                for (int j = B - 1; j >= 0; --j) {
                    const int i = i0 + b * B + j;
                    if (i < i1) {
                        double xn[P];
#pragma unroll
                        for (int k = 0; k < P; ++k) {
                            double t = q.y[j][k];
#pragma unroll
                            for (int l = 0; l < P; ++l) {
                                double c;
                                if constexpr (kPre) c = q.c[j][k * P + l];
                                else c = tab(tG, (int64_t)i * P * P + k * P + l);
                                t -= c * x[l];
                            }
                            xn[k] = t;
                        }
#pragma unroll
                        for (int k = 0; k < P; ++k) x[k] = xn[k];
                        st(Y(i), xn);
                        if (i == i1 - 1)
#pragma unroll
                            for (int k = 0; k < P; ++k) vL[k] = xn[k];
                        if (i == i0)
#pragma unroll
                            for (int k = 0; k < P; ++k) vF[k] = xn[k];
                    }
                }
            });
    }
    // The neighbour chunks' end values bL = x_{i0-1}, bR = x_{i1} (zero
    // beyond the ends): every chunk's v at its ends through LDS ([2K][64][P],
    // F then L per chunk), then the two block rows of the reduced system's
    // inverse that give them.
    template <int K>
    __device__ __forceinline__ void reduce(double *lds, int c, const double (&vF)[P],
                                           const double (&vL)[P], double (&bL)[P],
                                           double (&bR)[P]) const
    {
        st(lds + ((2 * c) * kHT + li) * P, vF);
        st(lds + ((2 * c + 1) * kHT + li) * P, vL);
        __syncthreads();
        constexpr int n = 2 * K * P;
        const cdouble *Mi = ro(a.Minv);
#pragma unroll
        for (int k = 0; k < P; ++k) bL[k] = bR[k] = 0.0;
        if (c > 0) {
            const int r = (2 * (c - 1) + 1) * P;
#pragma unroll
            for (int k = 0; k < P; ++k) {
                double t = 0.0;
#pragma unroll
                for (int j = 0; j < n; ++j)
                    t += Mi[(int64_t)(r + k) * n + j] * lds[((j / P) * kHT + li) * P + j % P];
                bL[k] = t;
            }
        }
        if (c + 1 < K) {
            const int r = 2 * (c + 1) * P;
#pragma unroll
            for (int k = 0; k < P; ++k) {
                double t = 0.0;
#pragma unroll
                for (int j = 0; j < n; ++j)
                    t += Mi[(int64_t)(r + k) * n + j] * lds[((j / P) * kHT + li) * P + j % P];
                bR[k] = t;
            }
        }
        __syncthreads();
    }
    // x_i = v_i - S^L_i bL - S^R_i bR and the damped update u_i <- (1 - omega)
    // u_i + omega x_i.  FIN (the leg's last sweep): the result to u_out and,
    // one point behind, into the residual; the residual at the chunk's ends
    // takes the neighbours' results through LDS.  Otherwise the result goes
    // to the workspace, and the next sweep's forward elimination runs in the
    // same walk (it needs the point's new iterate and the chain below it).
    template <bool FIN, int K>
    __device__ __forceinline__ void correct(const double (&bL)[P], const double (&bR)[P],
                                            double *lds, int c, double &acc) const
    {
        constexpr bool FWD = !FIN;
        struct Buf {
            double v[B][P], u[B][P], sl[kPre ? B : 1][P * P], sr[kPre ? B : 1][P * P],
                f[B][P], g[B], cf[(FWD && kPre) ? B : 1][P * P];
        };
        double y[P];   // FWD: the forward elimination's chain
#pragma unroll
        for (int k = 0; k < P; ++k) y[k] = 0.0;
        // FIN: the iterate at i-2, i-1 with f, u0 at i-1; the first two
        // points' iterate with the first's f, u0
        double um[P], uc[P], fc[P], uS[P], uS1[P], fS[P], gc = 0.0, gS = 0.0;
#pragma unroll
        for (int k = 0; k < P; ++k) um[k] = uc[k] = fc[k] = uS[k] = uS1[k] = fS[k] = 0.0;
        pipe2<Buf>(
            nb, false,
            [&](int b, Buf &q) {
#pragma unroll
                for (int j = 0; j < B; ++j) {
                    const int i = i0 + b * B + j;
                    ld(Y(row(i)), q.v[j]);
                    ld(U(row(i)), q.u[j]);
                    if constexpr (kPre) {
                        ld_tab(tSL, i, q.sl[j]);
                        ld_tab(tSR, i, q.sr[j]);
                        if constexpr (FWD) ld_tab(tC, i, q.cf[j]);
                    }
                    ld_rhs(i, q.f[j], q.g[j]);
                }
            },
            [&](int b, Buf &q) {
#pragma unroll
                for (int j = 0; j < B; ++j) {
                    const int i = i0 + b * B + j;
                    if (i < i1) {
                        double un[P];
#pragma unroll
                        for (int k = 0; k < P; ++k) {
                            double t = q.v[j][k];
#pragma unroll
                            for (int l = 0; l < P; ++l) {
                                double cl, cr;
                                if constexpr (kPre) {
                                    cl = q.sl[j][k * P + l];
                                    cr = q.sr[j][k * P + l];
                                } else {
                                    cl = tab(tSL, (int64_t)i * P * P + k * P + l);
                                    cr = tab(tSR, (int64_t)i * P * P + k * P + l);
                                }
                                t -= cl * bL[l];
                                t -= cr * bR[l];
                            }
                            un[k] = a.omc * q.u[j][k] + a.om * t;
                        }
                        if constexpr (FWD) {
                            st(U(i), un);
                            const double w = wl(un, q.g[j]);
                            double z[P];
#pragma unroll
                            for (int k = 0; k < P; ++k)
                                z[k] = q.f[j][k] + ((k & 1) ? -w : w) + mdh[k] * y[k];
#pragma unroll
                            for (int k = 0; k < P; ++k) {
                                double t = 0.0;
#pragma unroll
                                for (int l = 0; l < P; ++l) {
                                    double cc;
                                    if constexpr (kPre) cc = q.cf[j][k * P + l];
                                    else cc = tab(tC, (int64_t)i * P * P + k * P + l);
                                    t += cc * z[l];
                                }
                                y[k] = t;
                            }
                            st(Y(i), y);
                        } else {
                            if (a.u_out && out) st(a.u_out + ((int64_t)i * a.N + m) * P, un);
                            if (resid && i >= i0 + 2) resid_point(i - 1, um, uc, un, fc, gc, acc);
                            if (i == i0) {
#pragma unroll
                                for (int k = 0; k < P; ++k) {
                                    uS[k] = un[k];
                                    fS[k] = q.f[j][k];
                                }
                                gS = q.g[j];
                            }
                            if (i == i0 + 1)
#pragma unroll
                                for (int k = 0; k < P; ++k) uS1[k] = un[k];
#pragma unroll
                            for (int k = 0; k < P; ++k) {
                                um[k] = uc[k];
                                uc[k] = un[k];
                                fc[k] = q.f[j][k];
                            }
                            gc = q.g[j];
                        }
                    }
                }
            });
        if constexpr (FIN) {
            st(lds + ((2 * c) * kHT + li) * P, uS);
            st(lds + ((2 * c + 1) * kHT + li) * P, uc);
            __syncthreads();
            const int cl = c > 0 ? c - 1 : 0, cr = c + 1 < K ? c + 1 : c;
            double left[P], right[P];
#pragma unroll
            for (int k = 0; k < P; ++k) {
                const double l = lds[((2 * cl + 1) * kHT + li) * P + k];
                const double r = lds[((2 * cr) * kHT + li) * P + k];
                left[k] = c > 0 ? l : 0.0;
                right[k] = c + 1 < K ? r : 0.0;
            }
            __syncthreads();
            if (resid) {
                resid_point(i0, left, uS, uS1, fS, gS, acc);
                resid_point(i1 - 1, um, uc, right, fc, gc, acc);
            }
        }
    }
};

// One leg on one level: the iterate u_in (zero when null) plus the
// prolongated correction e (when given), `sweeps` damped block Jacobi
// sweeps, then the result into u_out, and its residual restricted into rc
// and/or squared into the tile's partial.  With norm_f, only the squared
// norm of the right-hand side.  Each walk variant appears once, so that no
// loop holds the state of several.
template <int P, int B>
__global__ __launch_bounds__(kHT) void k_hleg(HeatArgs a)
{
    const HLeg<P, B> g(a, 0, a.nx, a.Cinv, a.G);
    double acc = 0.0;
    if (a.norm_f) {
        g.norm_rhs(acc);
    } else if (a.sweeps == 0) {
        if (a.u_in) {
            if (a.e) g.template final_pass<kFromIn, true>(acc);
            else g.template final_pass<kFromIn, false>(acc);
        } else {
            if (a.e) g.template final_pass<kFromZero, true>(acc);
            else g.template final_pass<kFromZero, false>(acc);
        }
    } else {
        if (a.u_in) {
            if (a.e) g.template forward<kFromIn, true>();
            else g.template forward<kFromIn, false>();
        } else {
            if (a.e) g.template forward<kFromZero, true>();
            else g.template forward<kFromZero, false>();
        }
        if (a.sweeps == 2) {
            g.bsub_elim_down();
            g.bsub_up_fin(acc);
        } else {
            for (int s = 1; s < a.sweeps; ++s) {
                g.template backward<false>(acc);
                g.template forward<kFromWs, false>();
            }
            g.template backward<true>(acc);
        }
    }
    if (a.partial) {
        acc = wave_sum(acc);
        if (g.li == 0) a.partial[blockIdx.x] = acc;
    }
}

// One leg with its spatial solves partitioned over a.chunks wavefronts (see the
// partitioned sweeps above): sweeps >= 1, otherwise as k_hleg.
template <int P, int B, int K, bool TL>
__global__ __launch_bounds__(kHT * K) void k_hlegp(HeatArgs a)
{
    // LDS: the chunk end exchange [2K][64][P], then (TL) the level's
    // per-point tables C_i^{-1}, C_i^{-1} E, S^L, S^R (nx P^2 each), copied
    // at start; without TL they are read from global memory
    extern __shared__ double lds[];
    __shared__ double red[K];
    const int c = threadIdx.x / kHT;
    const int i0 = (int)((int64_t)c * a.nx / K), i1 = (int)((int64_t)(c + 1) * a.nx / K);
    const double *tC = a.Cl, *tG = a.Gl, *tSL = a.SL, *tSR = a.SR;
    if constexpr (TL) {
        const int nt = a.nx * P * P;
        double *tl = lds + 2 * K * kHT * P;
        for (int q = threadIdx.x; q < nt; q += kHT * K) {
            tl[q] = a.Cl[q];
            tl[nt + q] = a.Gl[q];
            tl[2 * nt + q] = a.SL[q];
            tl[3 * nt + q] = a.SR[q];
        }
        __syncthreads();
        tC = tl;
        tG = tl + nt;
        tSL = tl + 2 * nt;
        tSR = tl + 3 * nt;
    }
    const HLeg<P, B, TL> g(a, i0, i1, tC, tG, tSL, tSR);
    double acc = 0.0;
    if (a.u_in) {
        if (a.e) g.template forward<kFromIn, true>();
        else g.template forward<kFromIn, false>();
    } else {
        if (a.e) g.template forward<kFromZero, true>();
        else g.template forward<kFromZero, false>();
    }
    double vF[P], vL[P], bL[P], bR[P];
    for (int s = 1; s < a.sweeps; ++s) {
        g.backward_local(vF, vL);
        g.template reduce<K>(lds, c, vF, vL, bL, bR);
        g.template correct<false, K>(bL, bR, lds, c, acc);   // with the next forward
    }
    g.backward_local(vF, vL);
    g.template reduce<K>(lds, c, vF, vL, bL, bR);
    g.template correct<true, K>(bL, bR, lds, c, acc);
    if (a.partial) {
        acc = wave_sum(acc);
        if (g.li == 0) red[c] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int q = 0; q < K; ++q) t += red[q];
            a.partial[blockIdx.x] = t;
        }
    }
}

// Exact solve on the coarsest level: forward substitution over its slabs,
// each slab block solved by the elimination over the points (one lane, the
// walks pipelined as in the legs).
template <int P>
__global__ __launch_bounds__(kHT) void k_hcoarse(HeatArgs a)
{
    if (threadIdx.x != 0) return;
    constexpr int B = kHB<P>;
    const int nb = (a.nx + B - 1) / B;
    double *y = a.ws;
    for (int64_t n = 0; n < a.N; ++n) {
        struct FB {
            double z[B][P], up[B][P], g[B];
        };
        double yp[P];
#pragma unroll
        for (int k = 0; k < P; ++k) yp[k] = 0.0;
        pipe2<FB>(
            nb, false,
            [&](int b, FB &q) {
#pragma unroll
                for (int j = 0; j < B; ++j) {
                    const int i = b * B + j;
                    if (i < a.nx) {
#pragma unroll
                        for (int k = 0; k < P; ++k) {
                            q.z[j][k] = a.f[((int64_t)i * a.N + n) * P + k];
                            q.up[j][k] = n > 0 ? a.u_out[((int64_t)i * a.N + n - 1) * P + k] : 0.0;
                        }
                        q.g[j] = n == 0 ? a.u0[i] : 0.0;
                    }
                }
            },
            [&](int b, FB &q) {
#pragma unroll
                for (int j = 0; j < B; ++j) {
                    const int i = b * B + j;
                    if (i < a.nx) {
                        double w = q.g[j];   // u0 enters slab 0 as the left end value
#pragma unroll
                        for (int k = 0; k < P; ++k) w += q.up[j][k];
                        double z[P];
#pragma unroll
                        for (int k = 0; k < P; ++k)
                            z[k] = q.z[j][k] + ((k & 1) ? -w : w) + ro(a.Md)[k] * a.ih2 * yp[k];
                        const cdouble *Ci = ro(a.Cinv) + (int64_t)i * P * P;
#pragma unroll
                        for (int k = 0; k < P; ++k) {
                            double t = 0.0;
#pragma unroll
                            for (int l = 0; l < P; ++l) t += Ci[k * P + l] * z[l];
                            yp[k] = t;
                        }
#pragma unroll
                        for (int k = 0; k < P; ++k) y[i * P + k] = yp[k];
                    }
                }
            });
        struct BB {
            double y[B][P];
        };
        double x[P];
#pragma unroll
        for (int k = 0; k < P; ++k) x[k] = 0.0;
        pipe2<BB>(
            nb, true,
            [&](int b, BB &q) {
#pragma unroll
                for (int j = 0; j < B; ++j) {
                    const int i = b * B + j;
                    if (i < a.nx)
#pragma unroll
                        for (int k = 0; k < P; ++k) q.y[j][k] = y[i * P + k];
                }
            },
            [&](int b, BB &q) {
#pragma unroll
                for (int j = B - 1; j >= 0; --j) {
                    const int i = b * B + j;
                    if (i < a.nx) {
                        const cdouble *Gi = ro(a.G) + (int64_t)i * P * P;
                        double xn[P];
#pragma unroll
                        for (int k = 0; k < P; ++k) {
                            double t = q.y[j][k];
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
            });
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

hipError_t launch_hleg(int P, const HeatArgs &a, int64_t ntiles, bool lean, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    if (lean)
        TMG_HEAT_P(P, { hipLaunchKernelGGL((k_hleg<PP, kHBLean<PP>>), dim3((unsigned)ntiles), dim3(kHT), 0, s, a); })
    else
        TMG_HEAT_P(P, { hipLaunchKernelGGL((k_hleg<PP, kHB<PP>>), dim3((unsigned)ntiles), dim3(kHT), 0, s, a); })
    return hipGetLastError();
}

hipError_t launch_hlegp(int P, const HeatArgs &a, int64_t ntiles, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    if (a.chunks < 2 || a.chunks > kHeatMaxChunks || a.sweeps < 1 || a.nx < 2 * a.chunks)
        return hipErrorInvalidValue;
    // the tables in LDS when they fit
    const size_t full = heat_part_lds_bytes(P, a.nx, a.chunks);
    const bool tl = full <= kHeatPartLdsBytes;
    const size_t lds = tl ? full : sizeof(double) * 2 * a.chunks * kHT * P;
    const dim3 grid((unsigned)ntiles), block(kHT * a.chunks);
#define TMG_HLEGP(KK)                                                                          \
    TMG_HEAT_P(P, {                                                                            \
        if (tl) hipLaunchKernelGGL((k_hlegp<PP, kHBPart<PP>, KK, true>), grid, block, lds, s, a); \
        else hipLaunchKernelGGL((k_hlegp<PP, kHBLean<PP>, KK, false>), grid, block, lds, s, a);   \
    })
    switch (a.chunks) {
    case 2: TMG_HLEGP(2) break;
    case 4: TMG_HLEGP(4) break;
    case 8: TMG_HLEGP(8) break;
    default: return hipErrorInvalidValue;
    }
#undef TMG_HLEGP
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
