// Generic kernels of the time-multigrid cycle: any P = p + 1 up to kMaxP
// coefficients per slab, and the time-periodic problem u(0) = u(T) (section
// 3, eqs. chap4_equationLinearSystemODEPeriodic and chap4_circulantMatrix).
//
// The tuned kernels hold S slabs and the block operators per thread in
// registers, which stops at P = 6, and treat the left neighbour of slab 0
// as zero.  Here a work-group of kGenThreads threads owns a tile of as many
// consecutive slabs, one per thread; the level's table block (A, omega
// A^{-1}, omega A^{-1} v, c, v, 1 - omega, ...) and the transfer matrices are
// staged in LDS and read from there by every thread (broadcast reads), so
// only the slab's own P coefficients of f, u, g = omega A^{-1} f and r live
// in registers.  A periodic instance's first tile takes its left halo from
// the instance's last slabs (slab -1 is slab N-1, coarse slab -1 is Nc-1).
// Every leg reads one array and writes another (no in-place level-0 pass).
//
//   k_gleg    : the streaming leg of LegArgs (pre sweeps, prolongation of
//               the next level's correction, post sweeps, store, residual
//               norm, next sweeps, residual, restriction), any level;
//   k_gbottom : the exact solve of a level (the coarsest) by one work-group
//               per instance: b_n = c^T A^{-1} r_n, the affine prefix scan
//               w_n = alpha w_{n-1} + b_n (periodic: closed cyclically,
//               w_{-1} = w_{N-1} = S_{N-1} / (1 - alpha^N)), then
//               e_n = A^{-1} r_n + A^{-1} v w_{n-1}; at level 0 (an
//               instance of n_coarse slabs) it also finishes the cycle.
#pragma once

#include "tmg_kernels.h"

namespace tmg {
namespace {

constexpr int kGWaves = kGenThreads / 64;
constexpr int kGMaxChunk = (int)(kMaxCoarse / kGenThreads);   // slabs per thread in the exact solve

// The level's table block and the transfer matrices in LDS.
template <int P>
struct GOps {
    double t[TabLayout(P).stride()];
    double R[2 * P * P];
    __device__ __forceinline__ double A(int k, int l) const { return t[TabLayout(P).A() + k * P + l]; }
    __device__ __forceinline__ double G(int k, int l) const { return t[TabLayout(P).G() + k * P + l]; }
    __device__ __forceinline__ double AI(int k, int l) const { return t[TabLayout(P).AI() + k * P + l]; }
    __device__ __forceinline__ double h(int k) const { return t[TabLayout(P).H() + k]; }
    __device__ __forceinline__ double c(int k) const { return t[TabLayout(P).C() + k]; }
    __device__ __forceinline__ double v(int k) const { return t[TabLayout(P).V() + k]; }
    __device__ __forceinline__ double q(int k) const { return t[TabLayout(P).Q() + k]; }
    __device__ __forceinline__ double omc() const { return t[TabLayout(P).OMC()]; }
    __device__ __forceinline__ double alpha() const { return t[TabLayout(P).ALPHA()]; }
    // R_1^T (parity 0) or R_2^T (parity 1), entry [k][l]
    __device__ __forceinline__ double RT(int par, int k, int l) const { return R[par * P * P + k * P + l]; }
    __device__ void load(const double *tab, const double *Rg)
    {
        constexpr int n = TabLayout(P).stride();
        for (int i = threadIdx.x; i < n; i += blockDim.x) t[i] = tab[i];
        if (Rg)
            for (int i = threadIdx.x; i < 2 * P * P; i += blockDim.x) R[i] = Rg[i];
    }
};

// End value c^T u of the previous thread's slab (thread 0: zero; its slab
// is a halo slab whose error the halo absorbs).  One barrier; the two LDS
// slots alternate between calls.
__device__ __forceinline__ double g_left(double mine, double (*xw)[kGWaves], int &phase)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double v = lane_shr1(mine);
    if (lane == 63) xw[phase][wave] = mine;
    __syncthreads();
    if (lane == 0) v = wave ? xw[phase][wave - 1] : 0.0;
    phase ^= 1;
    return v;
}

template <int P>
__device__ __forceinline__ double g_end(const double (&u)[P], const GOps<P> &op)
{
    double w = 0.0;
#pragma unroll
    for (int k = 0; k < P; ++k) w += op.c(k) * u[k];
    return w;
}

// nsweep damped block Jacobi sweeps: u <- (1 - omega) u + g + omega A^{-1} v w_left
template <int P>
__device__ __forceinline__ void g_sweeps(double (&u)[P], const double (&g)[P], const GOps<P> &op,
                                         int nsweep, double (*xw)[kGWaves], int &phase)
{
    for (int s = 0; s < nsweep; ++s) {
        const double wl = g_left(g_end<P>(u, op), xw, phase);
        const double om = op.omc();
#pragma unroll
        for (int k = 0; k < P; ++k) u[k] = om * u[k] + g[k] + op.h(k) * wl;
    }
}

// r = f + v w_left - A u
template <int P>
__device__ __forceinline__ void g_residual(double (&r)[P], const double (&u)[P], const double (&f)[P],
                                           const GOps<P> &op, double (*xw)[kGWaves], int &phase)
{
    const double wl = g_left(g_end<P>(u, op), xw, phase);
#pragma unroll
    for (int k = 0; k < P; ++k) {
        double s = f[k] + op.v(k) * wl;
        for (int l = 0; l < P; ++l) s -= op.A(k, l) * u[l];
        r[k] = s;
    }
}

// The logical slab a thread reads: m itself inside [0, N), the wrapped one
// left of 0 for a periodic instance; -1 when there is none (zero data).
__device__ __forceinline__ int64_t g_slab(int64_t m, int64_t N, int periodic)
{
    if (m >= 0 && m < N) return m;
    if (periodic && m < 0) return ((m % N) + N) % N;
    return -1;
}

template <int P, bool BW>
__device__ __forceinline__ void g_load(double (&x)[P], const double *base, int64_t mm, int64_t N)
{
    if (mm < 0) {
#pragma unroll
        for (int k = 0; k < P; ++k) x[k] = 0.0;
        return;
    }
    const double *p = base + (BW ? N - 1 - mm : mm) * P;
#pragma unroll
    for (int k = 0; k < P; ++k) x[k] = p[k];
}

template <int P, bool BW>
__device__ __forceinline__ void g_store(double *base, const double (&x)[P], int64_t m, int64_t N)
{
    double *p = base + (BW ? N - 1 - m : m) * P;
#pragma unroll
    for (int k = 0; k < P; ++k) p[k] = x[k];
}

// P >= 16: held to 256 registers so that two wavefronts share a SIMD (the
// legs are bound by the products with the P x P blocks, whose LDS reads one
// wavefront alone cannot hide)
template <int P, bool BW>
__global__ __launch_bounds__(kGenThreads, P >= 16 ? 2 : 1) void k_gleg(LegArgsT<double> a)
{
    __shared__ GOps<P> op;
    __shared__ double xw[2][kGWaves];
    __shared__ double red[kGWaves];
    const TileRef tr = tile_ref(a);
    if (a.batch > 1 && a.st && a.st[tr.j].done) return;
    op.load(a.tab + (int64_t)tr.j * a.tab_stride, a.R);
    const int li = threadIdx.x;
    const int64_t m = tr.t * a.tile_out - a.halo + li;
    const int64_t mm = g_slab(m, tr.N, a.periodic);
    const bool out = li >= a.halo && m >= 0 && m < tr.N;   // an output slab of the tile
    double f[P], u[P];
    g_load<P, BW>(f, a.f + tr.off * P, mm, tr.N);
    if (a.u_in) g_load<P, BW>(u, a.u_in + tr.off * P, mm, tr.N);
    else
#pragma unroll
        for (int k = 0; k < P; ++k) u[k] = 0.0;
    __syncthreads();
    if (a.batch == 1 && a.st && a.st[tr.j].done) return;   // uniform over the work-group
    if (a.u0 && mm == 0)
#pragma unroll
        for (int k = 0; k < P; ++k) f[k] += a.u0[tr.j] * op.v(k);   // u0 enters slab 0
    int phase = 0;
    if (a.norm_f) {
        // the initial residual f (u0 folded), u = 0
        double acc = 0.0;
        if (out)
#pragma unroll
            for (int k = 0; k < P; ++k) acc += f[k] * f[k];
        acc = block_sum<kGWaves>(acc, red);
        if (threadIdx.x == 0) a.partial[a.norm_off[tr.j] + tr.t] = acc;
    }
    double g[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        double s = 0.0;
        for (int l = 0; l < P; ++l) s += op.G(k, l) * f[l];
        g[k] = s;
    }
    g_sweeps<P>(u, g, op, a.pre, xw, phase);
    if (a.e) {
        // u += R_i^T e_{m/2} (i the parity of m); a periodic halo slab left of
        // 0 takes the correction of its wrapped coarse slab
        double e[P];
        const int64_t cm = mm >= 0 ? mm / 2 : -1;
        g_load<P, BW>(e, a.e + tr.coff * P, cm, tr.Nc);
        const int par = (int)(mm & 1);
#pragma unroll
        for (int k = 0; k < P; ++k) {
            double s = 0.0;
            for (int l = 0; l < P; ++l) s += op.RT(par, k, l) * e[l];
            u[k] += s;
        }
    }
    g_sweeps<P>(u, g, op, a.post, xw, phase);
    if (a.u_out && out) g_store<P, BW>(a.u_out + tr.off * P, u, m, tr.N);
    double r[P];
    if (a.partial && !a.norm_f) {
        g_residual<P>(r, u, f, op, xw, phase);
        double acc = 0.0;
        if (out)
#pragma unroll
            for (int k = 0; k < P; ++k) acc += r[k] * r[k];
        acc = block_sum<kGWaves>(acc, red);
        if (threadIdx.x == 0) a.partial[a.norm_off[tr.j] + tr.t] = acc;
    }
    if (a.rc) {
        g_sweeps<P>(u, g, op, a.next, xw, phase);
        g_residual<P>(r, u, f, op, xw, phase);
        // rc_{m/2} = R_1 r_m + R_2 r_{m+1}: the even slab's thread takes its
        // partner's residual from the next lane (pairs never straddle a
        // wavefront: tiles and halos start at even slabs)
        double rn[P];
#pragma unroll
        for (int k = 0; k < P; ++k) rn[k] = __shfl_down(r[k], 1, 64);
        if (out && !(m & 1)) {
            double rc[P];
#pragma unroll
            for (int k = 0; k < P; ++k) {
                double s = 0.0;
                for (int l = 0; l < P; ++l) s += op.RT(0, l, k) * r[l] + op.RT(1, l, k) * rn[l];
                rc[k] = s;
            }
            g_store<P, BW>(a.rc + tr.coff * P, rc, m / 2, tr.Nc);
        }
    }
}

// Exact solve L e = r of one instance's level of N <= kMaxCoarse slabs by
// the whole work-group (see the file comment); r already holds u0 folded
// where it applies.  bw: LDS for the end values.  Returns in thread 0 the
// squared residual of e when `resid` (f = r, the level-0 instance).
template <int P, bool BW>
__device__ double g_exact(const double *r, double *e, int64_t N, int periodic, const GOps<P> &op,
                          double *bw, double *scan_a, double *scan_b, double (*xw)[kGWaves],
                          double *red, bool resid, const double *u0j)
{
    const int tid = threadIdx.x;
    const int chunk = (int)((N + kGenThreads - 1) / kGenThreads);
    const int64_t n0 = (int64_t)tid * chunk;
    const double al = op.alpha();
    auto rhs = [&](int64_t n, double (&x)[P]) {
        g_load<P, BW>(x, r, n, N);
        if (u0j && n == 0)
#pragma unroll
            for (int k = 0; k < P; ++k) x[k] += *u0j * op.v(k);
    };
    // b_n = c^T A^{-1} r_n, and this thread's composed map over its chunk
    double ca = 1.0, cb = 0.0;
    for (int i = 0; i < chunk; ++i) {
        const int64_t n = n0 + i;
        if (n >= N) break;
        double x[P];
        rhs(n, x);
        double b = 0.0;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            double d = 0.0;
            for (int l = 0; l < P; ++l) d += op.AI(k, l) * x[l];
            b += op.c(k) * d;
        }
        bw[n] = b;
        ca *= al;
        cb = al * cb + b;
    }
    // inclusive scan of the maps x -> a x + b over the threads (Hillis-Steele)
    scan_a[tid] = ca;
    scan_b[tid] = cb;
    __syncthreads();
    for (int d = 1; d < kGenThreads; d <<= 1) {
        double pa = 1.0, pb = 0.0;
        if (tid >= d) {
            pa = scan_a[tid - d];
            pb = scan_b[tid - d];
        }
        __syncthreads();
        if (tid >= d) {
            // (this) o (earlier): x -> a (pa x + pb) + b
            scan_b[tid] = scan_a[tid] * pb + scan_b[tid];
            scan_a[tid] = scan_a[tid] * pa;
        }
        __syncthreads();
    }
    // w_{-1}: zero, or the periodic closure w_{N-1} = alpha^N w_{N-1} + S_{N-1}
    const double tot_a = scan_a[kGenThreads - 1], tot_b = scan_b[kGenThreads - 1];
    const double wm1 = periodic ? tot_b / (1.0 - tot_a) : 0.0;
    // exclusive prefix of this thread: the end value before its chunk
    double w = tid ? scan_a[tid - 1] * wm1 + scan_b[tid - 1] : wm1;
    __syncthreads();
    // e_n = A^{-1} r_n + A^{-1} v w_{n-1}
    double acc = 0.0;
    for (int i = 0; i < chunk; ++i) {
        const int64_t n = n0 + i;
        if (n >= N) break;
        double x[P], d[P];
        rhs(n, x);
#pragma unroll
        for (int k = 0; k < P; ++k) {
            double s = 0.0;
            for (int l = 0; l < P; ++l) s += op.AI(k, l) * x[l];
            d[k] = s + op.q(k) * w;
        }
        if (resid) {
            // r_n - (A e_n - v w_{n-1}) with the end value carried by the scan
#pragma unroll
            for (int k = 0; k < P; ++k) {
                double s = x[k] + op.v(k) * w;
                for (int l = 0; l < P; ++l) s -= op.A(k, l) * d[l];
                acc += s * s;
            }
        }
        g_store<P, BW>(e, d, n, N);
        w = al * w + bw[n];
    }
    if (resid) acc = block_sum<kGWaves>(acc, red);
    return acc;
}

template <int P, bool BW>
__global__ __launch_bounds__(kGenThreads) void k_gbottom(BottomArgsT<double> a)
{
    __shared__ GOps<P> op;
    __shared__ double bw[kMaxCoarse];
    __shared__ double sa[kGenThreads], sb[kGenThreads];
    __shared__ double xw[2][kGWaves];
    __shared__ double red[kGWaves];
    const int j = a.inst[blockIdx.x];
    const int lv = a.lbs ? a.lbs[j] : a.level;
    const double *f = a.lbs ? a.f_lv[lv] : a.f;
    double *x = a.lbs ? a.x_lv[lv] : a.x_out;
    const int64_t *soff = a.lbs ? a.soff_lv[lv] : a.slab_off;
    const int64_t off = soff[j], N = soff[j + 1] - off;
    if (a.st && a.st[j].done) return;
    op.load(a.tab + ((int64_t)lv * a.batch + j) * a.tab_stride, a.R);
    __syncthreads();
    const bool fin = lv == 0 && a.st;
    const double acc = g_exact<P, BW>(f + off * P, x + off * P, N, a.periodic, op, bw, sa, sb, xw,
                                      red, fin, (lv == 0 && a.u0) ? a.u0 + j : nullptr);
    if (fin && threadIdx.x == 0) finish_cycle(a.st, j, a.st[j], acc, a.ctl, a.mirror);
}

// A whole V/W visit of an instance's bottom levels (its first bottom level
// lb up to the coarsest, at most gbottom_max(P) slabs) by one work-group,
// one slab per thread, in place of the streaming legs and k_gbottom.  The
// levels' right-hand sides and iterates stay in LDS in logical slab order;
// the level's table block is reloaded as the visit moves between levels.
// Each step is the streaming leg's (g_sweeps, g_residual, the transfers
// in the same order of operations) on the whole level, whose slab 0 has the
// zero left neighbour, and the coarsest level's exact solve is g_exact: the
// same arithmetic as the streaming kernels.  Down legs store the restricted
// residual; up legs recompute the pre-smoothing from the visit's initial
// iterate (as the streaming legs do) and store the result.  A first bottom
// level of 0 folds u0 and finishes the instance's cycle (k_bottom's way).
template <int P>
struct GVisitLds {
    static constexpr int BMAX = gbottom_max(P);
    double f[2 * BMAX * P];
    double x[2 * BMAX * P];
};

// g_left over a whole level of nl slabs held one per thread; periodic:
// slab 0's left neighbour is slab nl-1 (through wrap[], alternating as xw).
__device__ __forceinline__ double gv_left(double mine, double (*xw)[kGWaves], double *wrap,
                                          int &phase, int nl, int periodic)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double v = lane_shr1(mine);
    if (lane == 63) xw[phase][wave] = mine;
    if (periodic && (int)threadIdx.x == nl - 1) wrap[phase] = mine;
    __syncthreads();
    if (lane == 0) v = wave ? xw[phase][wave - 1] : (periodic ? wrap[phase] : 0.0);
    phase ^= 1;
    return v;
}

// g_sweeps and g_residual on a whole level (gv_left; the same arithmetic)
template <int P>
__device__ __forceinline__ void gv_sweeps(double (&u)[P], const double (&g)[P], const GOps<P> &op,
                                          int nsweep, double (*xw)[kGWaves], double *wrap,
                                          int &phase, int nl, int periodic)
{
    for (int s = 0; s < nsweep; ++s) {
        const double wl = gv_left(g_end<P>(u, op), xw, wrap, phase, nl, periodic);
        const double om = op.omc();
#pragma unroll
        for (int k = 0; k < P; ++k) u[k] = om * u[k] + g[k] + op.h(k) * wl;
    }
}

template <int P>
__device__ __forceinline__ void gv_residual(double (&r)[P], const double (&u)[P], const double (&f)[P],
                                            const GOps<P> &op, double (*xw)[kGWaves], double *wrap,
                                            int &phase, int nl, int periodic)
{
    const double wl = gv_left(g_end<P>(u, op), xw, wrap, phase, nl, periodic);
#pragma unroll
    for (int k = 0; k < P; ++k) {
        double s = f[k] + op.v(k) * wl;
        for (int l = 0; l < P; ++l) s -= op.A(k, l) * u[l];
        r[k] = s;
    }
}

// The visit of level lb (its right-hand side and initial iterate in sm, in
// logical slab order; op holds the table block of level `cur`); periodic:
// every level wraps around (slab -1 is slab N_l - 1) and the coarsest
// level's solve closes cyclically.
template <int P>
__device__ __forceinline__ void gvisit_levels(GOps<P> &op, GVisitLds<P> &sm, double *bw, double *sa,
                                              double *sb, double (*xw)[kGWaves], double *wrap,
                                              double *red, const double *tab0, int64_t tstep, int N,
                                              int lb, int Lc, int nu1, int nu2, int gamma,
                                              int periodic, bool zero, int &cur, int &phase)
{
    const int t = threadIdx.x;
    auto use = [&](int l) {
        // the table block of level l in LDS (every thread done with the last)
        __syncthreads();
        if (l != cur) {
            op.load(tab0 + (int64_t)l * tstep, nullptr);
            __syncthreads();
            cur = l;
        }
    };
    auto nsl = [&](int l) { return N >> (l - lb); };
    auto loff = [&](int l) { return (2 * N - 2 * nsl(l)) * P; };
    auto load = [&](double (&x)[P], const double *base, int l, bool zr) {
        const bool in = !zr && t < nsl(l);
#pragma unroll
        for (int k = 0; k < P; ++k) x[k] = in ? base[loff(l) + t * P + k] : 0.0;
    };
    auto gf = [&](double (&g)[P], const double (&f)[P]) {
#pragma unroll
        for (int k = 0; k < P; ++k) {
            double s = 0.0;
            for (int l = 0; l < P; ++l) s += op.G(k, l) * f[l];
            g[k] = s;
        }
    };
    // pre-smoothing from the visit's iterate (zr: from zero), residual,
    // restriction into level l+1
    auto down = [&](int l, bool zr) {
        use(l);
        double f[P], u[P], g[P], r[P], rn[P];
        load(f, sm.f, l, false);
        load(u, sm.x, l, zr);
        gf(g, f);
        gv_sweeps<P>(u, g, op, nu1, xw, wrap, phase, nsl(l), periodic);
        gv_residual<P>(r, u, f, op, xw, wrap, phase, nsl(l), periodic);
#pragma unroll
        for (int k = 0; k < P; ++k) rn[k] = __shfl_down(r[k], 1, 64);
        if (t < nsl(l) && !(t & 1)) {
#pragma unroll
            for (int k = 0; k < P; ++k) {
                double s = 0.0;
                for (int q = 0; q < P; ++q) s += op.RT(0, q, k) * r[q] + op.RT(1, q, k) * rn[q];
                sm.f[loff(l + 1) + (t / 2) * P + k] = s;
            }
        }
    };
    // the pre-smoothing recomputed, the correction of level l+1 prolongated,
    // post-smoothing, stored
    auto up = [&](int l, bool zr) {
        use(l);
        double f[P], u[P], g[P], e[P];
        load(f, sm.f, l, false);
        load(u, sm.x, l, zr);
        gf(g, f);
        gv_sweeps<P>(u, g, op, nu1, xw, wrap, phase, nsl(l), periodic);
        const bool in = t < nsl(l);
#pragma unroll
        for (int k = 0; k < P; ++k) e[k] = in ? sm.x[loff(l + 1) + (t / 2) * P + k] : 0.0;
        const int par = t & 1;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            double s = 0.0;
            for (int q = 0; q < P; ++q) s += op.RT(par, k, q) * e[q];
            u[k] += s;
        }
        gv_sweeps<P>(u, g, op, nu2, xw, wrap, phase, nsl(l), periodic);
        __syncthreads();   // every thread has read its iterate and correction
        if (in)
#pragma unroll
            for (int k = 0; k < P; ++k) sm.x[loff(l) + t * P + k] = u[k];
    };
    auto coarse = [&](int l) {
        use(l);
        (void)g_exact<P, false>(sm.f + loff(l), sm.x + loff(l), nsl(l), periodic, op, bw, sa, sb, xw,
                                red, false, nullptr);
    };
    // bit l of `again` marks the second visit of level l
    uint64_t again = 0;
    int l = lb;
    down(l, zero);
    while (true) {
        if (l + 1 == Lc) {
            coarse(l + 1);
        } else {
            ++l;
            down(l, true);
            continue;
        }
        bool finished = false;
        while (true) {
            up(l, l == lb ? zero : !((again >> l) & 1));
            if (l == lb) {
                finished = true;
                break;
            }
            if (gamma > 1 && !((again >> l) & 1)) {
                again |= (uint64_t)1 << l;
                down(l, false);
                break;
            }
            again &= ~((uint64_t)1 << l);
            --l;
        }
        if (finished) break;
    }
    __syncthreads();
}

template <int P, bool BW>
__global__ __launch_bounds__(kGenThreads) void k_gvisit(BottomArgsT<double> a)
{
    __shared__ GOps<P> op;
    __shared__ GVisitLds<P> sm;
    __shared__ double bw[kMaxCoarse];
    __shared__ double sa[kGenThreads], sb[kGenThreads];
    __shared__ double xw[2][kGWaves];
    __shared__ double wrap[2];
    __shared__ double red[kGWaves];
    const int j = a.inst[blockIdx.x];
    if (a.st && a.st[j].done) return;
    const int lb = a.lbs ? a.lbs[j] : a.level, Lc = a.nlev[j] - 1;
    const double *fg = a.lbs ? a.f_lv[lb] : a.f;
    double *xg = a.lbs ? a.x_lv[lb] : a.x_out;
    const int64_t *soff = a.lbs ? a.soff_lv[lb] : a.slab_off;
    const int64_t off = soff[j];
    const int N = (int)(soff[j + 1] - off);
    const int t = threadIdx.x;
    const double *tab0 = a.tab + (int64_t)j * a.tab_stride;
    const int64_t tstep = (int64_t)a.batch * a.tab_stride;
    op.load(tab0 + (int64_t)lb * tstep, a.R);
    __syncthreads();
    if (lb == Lc) {
        // one level: its exact solve (k_gbottom)
        const bool fin = lb == 0 && a.st;
        const double acc = g_exact<P, BW>(fg + off * P, xg + off * P, N, a.periodic, op, bw, sa, sb,
                                          xw, red, fin, (lb == 0 && a.u0) ? a.u0 + j : nullptr);
        if (fin && t == 0) finish_cycle(a.st, j, a.st[j], acc, a.ctl, a.mirror);
        return;
    }
    if (N > GVisitLds<P>::BMAX) return;   // the host never plans such a bottom
    for (int i = t; i < N * P; i += kGenThreads) {
        const int m = i / P, k = i - m * P;
        const int64_t pm = off + (BW ? N - 1 - m : m);
        sm.f[i] = fg[pm * P + k];
        sm.x[i] = a.x_in ? a.x_in[pm * P + k] : 0.0;
    }
    __syncthreads();
    if (lb == 0 && a.u0 && t < P) sm.f[t] += a.u0[j] * op.v(t);   // u0 enters slab 0
    int phase = 0, cur = lb;
    gvisit_levels<P>(op, sm, bw, sa, sb, xw, wrap, red, tab0, tstep, N, lb, Lc, a.nu1, a.nu2, a.gamma,
                     a.periodic, a.x_in == nullptr, cur, phase);
    for (int i = t; i < N * P; i += kGenThreads) {
        const int m = i / P, k = i - m * P;
        xg[(off + (BW ? N - 1 - m : m)) * P + k] = sm.x[i];
    }
    if (lb == 0 && a.st) {
        // squared residual of the result (level 0): the work-group finishes
        // the instance's cycle
        __syncthreads();
        if (cur != 0) {
            op.load(tab0, nullptr);
            __syncthreads();
        }
        double f[P], u[P], r[P];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            f[k] = t < N ? sm.f[t * P + k] : 0.0;
            u[k] = t < N ? sm.x[t * P + k] : 0.0;
        }
        gv_residual<P>(r, u, f, op, xw, wrap, phase, N, a.periodic);
        double acc = 0.0;
        if (t < N)
#pragma unroll
            for (int k = 0; k < P; ++k) acc += r[k] * r[k];
        acc = block_sum<kGWaves>(acc, red);
        if (t == 0) finish_cycle(a.st, j, a.st[j], acc, a.ctl, a.mirror);
    }
}

// Column `col` of the dense bottom operator on the generic kernels (one
// work-group per column; see k_dense_cols): gamma visits of level a.level
// from zero on the unit load e_col, as k_gvisit runs them.  The visit
// works in logical slab order; the column and the unit load are physical
// (BW: logical slab m is physical N-1-m).
template <int P, bool BW>
__global__ __launch_bounds__(kGenThreads) void k_gdense_cols(DenseColArgs a)
{
    __shared__ GOps<P> op;
    __shared__ GVisitLds<P> sm;
    __shared__ double bw[kMaxCoarse];
    __shared__ double sa[kGenThreads], sb[kGenThreads];
    __shared__ double xw[2][kGWaves];
    __shared__ double wrap[2];
    __shared__ double red[kGWaves];
    const int64_t col = blockIdx.x;
    const int N = (int)a.N, n = N * P, lb = a.level;
    // physical index <-> logical index (an involution)
    auto phys = [&](int i) { return BW ? (N - 1 - i / P) * P + i % P : i; };
    const int lcol = phys((int)col);
    op.load(a.tab + (int64_t)lb * a.tab_level, a.R);
    for (int i = threadIdx.x; i < n; i += kGenThreads) {
        sm.f[i] = i == lcol ? 1.0 : 0.0;
        sm.x[i] = 0.0;
    }
    __syncthreads();
    int phase = 0, cur = lb;
    for (int g = 0; g < a.gamma; ++g)
        gvisit_levels<P>(op, sm, bw, sa, sb, xw, wrap, red, a.tab, a.tab_level, N, lb, a.Lc, a.nu1,
                         a.nu2, a.gamma, a.periodic, g == 0, cur, phase);
    for (int i = threadIdx.x; i < n; i += kGenThreads) a.D[(int64_t)phys(i) * n + col] = sm.x[i];
}

// tmg_op_coarse_solve on the generic path
template <int P, bool BW>
__global__ __launch_bounds__(kGenThreads) void k_gcoarse(CoarseArgs a, int periodic)
{
    __shared__ GOps<P> op;
    __shared__ double bw[kMaxCoarse];
    __shared__ double sa[kGenThreads], sb[kGenThreads];
    __shared__ double xw[2][kGWaves];
    __shared__ double red[kGWaves];
    const int j = a.inst[blockIdx.x];
    const int64_t off = a.slab_off[j], N = a.slab_off[j + 1] - off;
    op.load(a.tab + (int64_t)j * a.tab_stride, a.R);
    __syncthreads();
    (void)g_exact<P, BW>(a.r + off * P, a.e + off * P, N, periodic, op, bw, sa, sb, xw, red,
                         false, a.u0 ? a.u0 + j : nullptr);
}

}  // namespace
}  // namespace tmg
