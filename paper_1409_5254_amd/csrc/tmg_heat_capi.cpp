// Driver of the space-time heat equation (see include/tmg.h, tmg_heat_*):
// the time multigrid of section 3 with every slab block, which couples all
// spatial points of the slab, solved exactly inside the block Jacobi step.
//
// Each level l >= 1 keeps its right-hand side f_l, its result x_l and the
// pre-smoothed iterate s_l of the visit in progress; level 0 keeps s_0.  A
// visit is a down leg (pre sweeps into s_l, residual restricted into
// f_{l+1}), gamma visits of the next level (or its exact solve), and an up
// leg (correction from x_{l+1}, post sweeps) from s_l into x_l; level 0's up
// leg writes the caller's u and the residual norm.  The host reads the norm
// after every cycle.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "../../include/tmg.h"
#include "tmg_heat.h"
#include "tmg_internal.h"
#include "tmg_tables.h"

using namespace tmg;

struct tmg_heat_ctx {
    int P = 0, nx = 0, L = 0;
    int64_t N = 0;
    double T = 0.0, h = 0.0;
    tmg_options opt{};
    std::vector<int64_t> Nl;
    std::vector<double> omega;
    std::vector<double *> f, x, sx, Cinv, G, K, Md;   // per level (device)
    // per level: wavefronts sharing a tile (1: none) and the partitioned
    // solve's tables (device, null when unpartitioned)
    std::vector<int> chunks;
    std::vector<double *> Cl, Gl, SL, SR, Minv;
    double *R = nullptr, *ws = nullptr, *partial = nullptr, *sum = nullptr;
    double *zeros = nullptr;   // nx zeros: the u0 of the levels above 0
    int64_t ws_tiles = 0;
    int64_t wide_tiles = 0;   // two wavefronts per SIMD of the device
    // The coarse levels by sine modes.  The slab block, the residual and the
    // transfers in time all act on each eigenvector of L_h separately, so a
    // visit of level mode_level (its gamma visits from zero, with every
    // level below) is: the orthonormal sine transform over the points, for
    // each mode the scalar problem's visit operator (lambda = the mode's
    // eigenvalue, this cycle's damping per level; tabulated as the dense
    // bottom operator), and the inverse transform (the same matrix).
    int mode_level = -1;                  // -1: none
    bool mode_on = true;
    int64_t mode_n = 0;                   // unknowns per point of that level
    double *Q = nullptr;                  // [nx][nx], symmetric
    double *mD = nullptr;                 // [nx][n][n] per-mode operators
    int *mwin = nullptr;                  // [nx][2n] their rows' windows
    double *mt[2] = {nullptr, nullptr};   // [nx][n] the transformed f, result
    int64_t mode_w = 0;                   // the widest span a product's work-group loads
    std::vector<void *> allocs;
    int last_hip = 0;
};

namespace {

template <typename T>
int halloc(tmg_heat_ctx *c, T **p, size_t n)
{
    *p = nullptr;
    hipError_t e = hipMalloc((void **)p, (n ? n : 1) * sizeof(T));
    if (e != hipSuccess) {
        c->last_hip = (int)e;
        return TMG_ERR_OOM;
    }
    c->allocs.push_back(*p);
    return TMG_OK;
}

#define HCHK(c, expr)                                                      \
    do {                                                                   \
        hipError_t e_ = (expr);                                            \
        if (e_ != hipSuccess) {                                            \
            (c)->last_hip = (int)e_;                                       \
            return TMG_ERR_HIP;                                            \
        }                                                                  \
    } while (0)

void heat_free(tmg_heat_ctx *c)
{
    for (void *p : c->allocs) (void)hipFree(p);
    c->allocs.clear();
}

// even halos of at least 2 slabs: restriction pairs stay in a tile
int rs2(int x) { return (x + 1) & ~1; }
constexpr int64_t kLegCoarse = 32;   // coarsest levels solved by a leg (one tile)
// the sine-mode visits: a level of at most kModeSlabs slabs (and the
// per-mode operators within kModeBytes), above the coarsest
constexpr int64_t kModeSlabs = 256;
constexpr double kModeBytes = double(1u << 30);
int TO(int H) { return kHeatThreads - H; }
int64_t tiles(int64_t N, int H) { return (N + TO(H) - 1) / TO(H); }
// The largest halo of any launch (down legs nu1 + 1, up legs with the norm
// nu2 + 1, the norm pass 2): the most tiles of a level, which sizes the
// per-tile workspace and partials.
int Hmax(const tmg_options &o) { return std::max(std::max(rs2(o.nu1 + 1), rs2(o.nu2 + 1)), 2); }

// A leg's grid within the workspace it was sized for (else the launch would
// write past the per-tile buffers).
int launch_leg_checked(tmg_heat_ctx *c, const HeatArgs &a, int64_t ntiles, hipStream_t s)
{
    if (ntiles > c->ws_tiles || a.halo < 2 || a.halo >= kHeatThreads) return TMG_ERR_INTERNAL;
    if (a.chunks > 1 && a.sweeps > 0) HCHK(c, launch_hlegp(c->P, a, ntiles, s));
    else HCHK(c, launch_hleg(c->P, a, ntiles, ntiles > c->wide_tiles, s));
    return TMG_OK;
}

// Gauss-Jordan inverse with partial pivoting of an n x n matrix (row-major);
// false when singular.
bool invert_dense(int n, std::vector<double> A, std::vector<double> &Ai)
{
    Ai.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Ai[(size_t)i * n + i] = 1.0;
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (std::fabs(A[(size_t)r * n + col]) > std::fabs(A[(size_t)piv * n + col])) piv = r;
        if (!(std::fabs(A[(size_t)piv * n + col]) > 0.0)) return false;
        if (piv != col)
            for (int j = 0; j < n; ++j) {
                std::swap(A[(size_t)piv * n + j], A[(size_t)col * n + j]);
                std::swap(Ai[(size_t)piv * n + j], Ai[(size_t)col * n + j]);
            }
        const double d = 1.0 / A[(size_t)col * n + col];
        for (int j = 0; j < n; ++j) {
            A[(size_t)col * n + j] *= d;
            Ai[(size_t)col * n + j] *= d;
        }
        for (int r = 0; r < n; ++r)
            if (r != col) {
                const double fct = A[(size_t)r * n + col];
                if (fct == 0.0) continue;
                for (int j = 0; j < n; ++j) {
                    A[(size_t)r * n + j] -= fct * A[(size_t)col * n + j];
                    Ai[(size_t)r * n + j] -= fct * Ai[(size_t)col * n + j];
                }
            }
    }
    return true;
}

// Wavefronts sharing a tile at a level of `ntiles` tiles: none unless the
// level has at most a quarter wavefront per SIMD (`waves` of them; with
// more, the extra walk of the partitioned sweep costs more than the shorter
// chains save), else the largest power of two that keeps the level within
// one wavefront per SIMD, at least 2 points per chunk, and the register
// budget (P <= 4).
int pick_chunks(int P, int nx, int64_t ntiles, int64_t waves)
{
    if (P > 4 || 4 * ntiles > waves) return 1;
    const int kmax = std::min(kHeatMaxChunks, 16 / P);
    int K = 1;
    while (2 * K <= kmax && nx >= 4 * K && ntiles * 2 * K <= waves) K *= 2;
    return K;
}

// The partitioned solve's tables of one level (slab block D = K + 2 M/h^2
// on the diagonal, E = -M/h^2 beside it): per point the elimination factors
// C_i^{-1} and C_i^{-1} E restarted at every chunk's first point, the spikes
// S^L = A_c^{-1} (e_first (x) E) and S^R = A_c^{-1} (e_last (x) E) of the
// point's chunk, and the inverse of the reduced system of the chunk end
// values (block order: first, last point of chunk 0, of chunk 1, ...).
bool part_tables(int P, int nx, int K, const double *Km, const double *Md, double ih2,
                 std::vector<double> &Cl, std::vector<double> &Gl, std::vector<double> &SL,
                 std::vector<double> &SR, std::vector<double> &Minv)
{
    const int PP = P * P;
    Cl.assign((size_t)nx * PP, 0.0);
    Gl.assign((size_t)nx * PP, 0.0);
    SL.assign((size_t)nx * PP, 0.0);
    SR.assign((size_t)nx * PP, 0.0);
    std::vector<double> E(P), D(PP), C(PP), Y((size_t)nx * PP);
    for (int k = 0; k < P; ++k) E[k] = -Md[k] * ih2;
    for (int k = 0; k < P; ++k)
        for (int j = 0; j < P; ++j) D[k * P + j] = Km[k * P + j] + (k == j ? 2.0 * ih2 * Md[k] : 0.0);
    auto at = [&](std::vector<double> &v, int i) { return &v[(size_t)i * PP]; };
    for (int c = 0; c < K; ++c) {
        const int s = (int)((int64_t)c * nx / K), e = (int)((int64_t)(c + 1) * nx / K);
        for (int i = s; i < e; ++i) {
            for (int q = 0; q < PP; ++q) C[q] = D[q];
            if (i > s)
                for (int k = 0; k < P; ++k)
                    for (int j = 0; j < P; ++j) C[k * P + j] -= E[k] * at(Cl, i - 1)[k * P + j] * E[j];
            table_invert(P, C.data(), at(Cl, i));
            for (int k = 0; k < P; ++k)
                for (int j = 0; j < P; ++j) at(Gl, i)[k * P + j] = at(Cl, i)[k * P + j] * E[j];
        }
        // left spike: right-hand side E at the first point; right spike: at
        // the last point (forward elimination, then back substitution)
        for (int side = 0; side < 2; ++side) {
            std::vector<double> &S = side ? SR : SL;
            for (int i = s; i < e; ++i) {
                double *y = at(Y, i);
                const bool src = side ? i == e - 1 : i == s;
                for (int k = 0; k < P; ++k)
                    for (int j = 0; j < P; ++j) {
                        // C_i^{-1} (b_i - E y_{i-1}), b_i = E at the source point
                        double t = 0.0;
                        for (int l = 0; l < P; ++l) {
                            double r = (src && l == j) ? E[l] : 0.0;
                            if (i > s) r -= E[l] * at(Y, i - 1)[l * P + j];
                            t += at(Cl, i)[k * P + l] * r;
                        }
                        y[k * P + j] = t;
                    }
            }
            for (int i = e - 1; i >= s; --i)
                for (int k = 0; k < P; ++k)
                    for (int j = 0; j < P; ++j) {
                        double t = at(Y, i)[k * P + j];
                        if (i < e - 1)
                            for (int l = 0; l < P; ++l) t -= at(Gl, i)[k * P + l] * at(S, i + 1)[l * P + j];
                        at(S, i)[k * P + j] = t;
                    }
        }
    }
    const int n = 2 * K * P;
    std::vector<double> M((size_t)n * n, 0.0);
    for (int q = 0; q < n; ++q) M[(size_t)q * n + q] = 1.0;
    for (int c = 0; c < K; ++c) {
        const int s = (int)((int64_t)c * nx / K), e = (int)((int64_t)(c + 1) * nx / K);
        const int rows[2] = {s, e - 1};
        for (int side = 0; side < 2; ++side) {
            const int r0 = (2 * c + side) * P, i = rows[side];
            for (int k = 0; k < P; ++k)
                for (int j = 0; j < P; ++j) {
                    if (c > 0) M[(size_t)(r0 + k) * n + (2 * (c - 1) + 1) * P + j] += at(SL, i)[k * P + j];
                    if (c + 1 < K) M[(size_t)(r0 + k) * n + 2 * (c + 1) * P + j] += at(SR, i)[k * P + j];
                }
        }
    }
    return invert_dense(n, M, Minv);
}

HeatArgs base_args(const tmg_heat_ctx *c, int l)
{
    HeatArgs a{};
    a.Cinv = c->Cinv[l];
    a.G = c->G[l];
    a.K = c->K[l];
    a.Md = c->Md[l];
    a.R = c->R;
    a.u0 = c->zeros;
    a.ws = c->ws;
    a.N = c->Nl[l];
    a.Nc = l + 1 < c->L ? c->Nl[l + 1] : 0;
    a.ih2 = 1.0 / (c->h * c->h);
    a.chunks = c->chunks[l];
    a.Cl = c->Cl[l];
    a.Gl = c->Gl[l];
    a.SL = c->SL[l];
    a.SR = c->SR[l];
    a.Minv = c->Minv[l];
    a.om = c->omega[l];
    a.omc = 1.0 - c->omega[l];
    a.nx = c->nx;
    return a;
}

int visit(tmg_heat_ctx *c, int l, bool first, hipStream_t s);

// The down leg at level l (from `in`, null: zero), the coarse visits, and
// the up leg into `out`.
int level_pass(tmg_heat_ctx *c, int l, const double *f, const double *u0, const double *in,
               double *out, double *partial, hipStream_t s)
{
    const int nu1 = c->opt.nu1, nu2 = c->opt.nu2;
    int rc;
    {
        const int H = rs2(nu1 + 1);
        HeatArgs a = base_args(c, l);
        a.f = f;
        if (u0) a.u0 = u0;
        a.u_in = in;
        a.u_out = c->sx[l];
        a.rc = c->f[l + 1];
        a.halo = H;
        a.tile_out = TO(H);
        a.sweeps = nu1;
        if ((rc = launch_leg_checked(c, a, tiles(c->Nl[l], H), s))) return rc;
    }
    if (c->mode_on && c->mode_level == l + 1) {
        // the gamma visits of level l+1 by sine modes
        const int d = l + 1, nx = c->nx;
        const int64_t n = c->mode_n;
        HCHK(c, launch_mode_transform(c->Q, c->f[d], c->mt[0], nx, n, s));
        HCHK(c, launch_dense_apply_batch(c->mD, c->mwin, c->mt[0], c->mt[1], n, nx, s, c->mode_w));
        HCHK(c, launch_mode_transform(c->Q, c->mt[1], c->x[d], nx, n, s));
    } else {
        for (int g = 0; g < c->opt.gamma; ++g)
            if ((rc = visit(c, l + 1, g == 0, s))) return rc;
    }
    {
        const int H = std::max(2, rs2(nu2 + (partial ? 1 : 0)));
        HeatArgs a = base_args(c, l);
        a.f = f;
        if (u0) a.u0 = u0;
        a.u_in = c->sx[l];
        a.e = c->x[l + 1];
        a.u_out = out;
        a.partial = partial;
        a.halo = H;
        a.tile_out = TO(H);
        a.sweeps = nu2;
        if ((rc = launch_leg_checked(c, a, tiles(c->Nl[l], H), s))) return rc;
        if (partial) HCHK(c, launch_hsum(partial, tiles(c->Nl[l], H), c->sum, s));
    }
    return TMG_OK;
}

// One visit of level l >= 1 on L_l e = f_l (from zero on a first visit,
// else from the current x_l); the coarsest level is solved exactly.  With
// at most kLegCoarse slabs it is one tile's leg of as many undamped sweeps
// from zero: the system is block lower bidiagonal in time, so after k
// sweeps the first k slabs are exact.  Otherwise slab after slab on one
// lane (k_hcoarse).
int visit(tmg_heat_ctx *c, int l, bool first, hipStream_t s)
{
    if (l == c->L - 1) {
        HeatArgs a = base_args(c, l);
        a.f = c->f[l];
        a.u_out = c->x[l];
        if (c->Nl[l] <= kLegCoarse) {
            a.halo = 2;
            a.tile_out = TO(2);
            a.sweeps = (int)c->Nl[l];
            a.om = 1.0;
            a.omc = 0.0;
            return launch_leg_checked(c, a, 1, s);
        }
        HCHK(c, launch_hcoarse(c->P, a, s));
        return TMG_OK;
    }
    return level_pass(c, l, c->f[l], nullptr, first ? nullptr : c->x[l], c->x[l], nullptr, s);
}

// The sine-mode visits (see tmg_heat_ctx): the first level l >= 1 above the
// coarsest with at most kModeSlabs slabs whose per-mode operators fit
// kModeBytes; mode k (1..nx) has eigenvalue 4 sin^2(pi k h / 2) / h^2 and
// eigenvector sqrt(2h) sin(pi k i h) (i = 1..nx).  The operators' columns
// are the bottom kernel's visits of the unit loads (one launch per mode).
int build_modes(tmg_heat_ctx *c, hipStream_t s)
{
    const int P = c->P, nx = c->nx, L = c->L;
    int d = -1;
    for (int l = 1; l + 1 < L; ++l) {
        const double n = double(c->Nl[l] * P);
        if (c->Nl[l] <= kModeSlabs && nx * n * n * 8.0 <= kModeBytes) {
            d = l;
            break;
        }
    }
    if (d < 0 || L - d > kBottomMaxLevels) return TMG_OK;
    const int64_t N = c->Nl[d], n = N * P;
    const int nlv = L - d, stride = TabLayout(P).stride();
    const double h = c->h;
    std::vector<double> Q((size_t)nx * nx), tab((size_t)nx * nlv * stride);
    for (int k = 1; k <= nx; ++k) {
        const double sk = std::sin(M_PI * k * h / 2.0);
        const double mu = 4.0 * sk * sk / (h * h);
        for (int j = 0; j < nlv; ++j)
            (void)level_table(P, mu * (c->T / (double)c->Nl[d + j]), 1, c->omega[d + j], false,
                              &tab[((size_t)(k - 1) * nlv + j) * stride]);
        for (int i = 1; i <= nx; ++i)
            Q[(size_t)(k - 1) * nx + (i - 1)] = std::sqrt(2.0 * h) * std::sin(M_PI * k * i * h);
    }
    double *dtab = nullptr;
    if (halloc(c, &c->Q, Q.size()) || halloc(c, &dtab, tab.size()) ||
        halloc(c, &c->mD, (size_t)nx * n * n) || halloc(c, &c->mwin, (size_t)nx * 2 * n) ||
        halloc(c, &c->mt[0], (size_t)nx * n) || halloc(c, &c->mt[1], (size_t)nx * n)) {
        // no room for the modes' operators: every level runs its legs (the
        // buffers made so far are freed with the handle)
        c->last_hip = 0;
        (void)hipGetLastError();   // the failed allocation is no error of this call
        return TMG_OK;
    }
    HCHK(c, hipMemcpyAsync(c->Q, Q.data(), Q.size() * 8, hipMemcpyHostToDevice, s));
    HCHK(c, hipMemcpyAsync(dtab, tab.data(), tab.size() * 8, hipMemcpyHostToDevice, s));
    for (int k = 0; k < nx; ++k) {
        DenseColArgs a{};
        a.tab = dtab + (size_t)k * nlv * stride;
        a.tab_level = stride;
        a.R = c->R;
        a.D = c->mD + (size_t)k * n * n;
        a.N = N;
        a.level = 0;
        a.Lc = nlv - 1;
        a.nu1 = c->opt.nu1;
        a.nu2 = c->opt.nu2;
        a.gamma = c->opt.gamma;
        HCHK(c, launch_dense_cols(P, a, s));
        HCHK(c, launch_dense_window(a.D, n, c->mwin + (size_t)k * 2 * n, s));
    }
    // the widest span a product's work-group loads, over every mode
    int w = (int)n;
    int *wd = nullptr;
    if (halloc(c, &wd, 1) == TMG_OK) {
        HCHK(c, launch_dense_window_max(c->mwin, n, nx, wd, s));
        HCHK(c, hipMemcpyAsync(&w, wd, sizeof(int), hipMemcpyDeviceToHost, s));
    } else {
        c->last_hip = 0;
        (void)hipGetLastError();
    }
    HCHK(c, hipStreamSynchronize(s));
    c->mode_w = w;
    c->mode_level = d;
    c->mode_n = n;
    return TMG_OK;
}

// Squared residual norm of u (or of the folded f when u is null) into c->sum.
int norm2(tmg_heat_ctx *c, const double *f, const double *u0, const double *u, hipStream_t s)
{
    const int H = 2;
    HeatArgs a = base_args(c, 0);
    a.f = f;
    a.u0 = u0;
    a.u_in = u;
    a.partial = c->partial;
    a.norm_f = u ? 0 : 1;
    a.halo = H;
    a.tile_out = TO(H);
    const int rc = launch_leg_checked(c, a, tiles(c->N, H), s);
    if (rc) return rc;
    HCHK(c, launch_hsum(c->partial, tiles(c->N, H), c->sum, s));
    return TMG_OK;
}

int read_sum(tmg_heat_ctx *c, double *v, hipStream_t s)
{
    HCHK(c, hipMemcpyAsync(v, c->sum, sizeof(double), hipMemcpyDeviceToHost, s));
    HCHK(c, hipStreamSynchronize(s));
    return TMG_OK;
}

}  // namespace

extern "C" {

int tmg_heat_setup(tmg_heat_handle *hp, int64_t n_slabs, int nx, double T,
                   const tmg_options *opt, tmg_stream stream)
{
    if (!hp || !opt) return TMG_ERR_INVALID;
    *hp = nullptr;
    const tmg_options &o = *opt;
    if (o.p < 0 || o.p > TMG_MAX_TUNED_DEGREE || nx < 1 || nx > TMG_HEAT_MAX_POINTS ||
        o.nu1 < 0 || o.nu1 > kMaxSweeps || o.nu2 < 0 || o.nu2 > kMaxSweeps ||
        (o.gamma != 1 && o.gamma != 2) || o.n_coarse < 1 || o.n_coarse > kMaxCoarse ||
        (o.omega_mode != 0 && o.omega_mode != 1))
        return TMG_ERR_INVALID;
    if (o.omega_mode == 1 && !(o.omega > 0.0 && o.omega <= 1.0)) return TMG_ERR_OMEGA;
    if (o.precision != 0 || o.periodic != 0) return TMG_ERR_UNSUPPORTED;
    if (!(std::isfinite(T) && T > 0.0)) return TMG_ERR_PARAM;
    int L = 1;
    int64_t n = n_slabs;
    if (n < o.n_coarse || n > (int64_t(1) << 32)) return TMG_ERR_SIZE;
    while (n > o.n_coarse) {
        if (n & 1) return TMG_ERR_SIZE;
        n >>= 1;
        ++L;
    }
    if (n != o.n_coarse || L < 2) return TMG_ERR_SIZE;
    tmg_heat_ctx *c = new (std::nothrow) tmg_heat_ctx;
    if (!c) return TMG_ERR_OOM;
    hipStream_t s = (hipStream_t)stream;
    const int P = o.p + 1;
    c->P = P;
    c->nx = nx;
    c->L = L;
    c->N = n_slabs;
    c->T = T;
    c->h = 1.0 / (nx + 1);
    c->opt = o;
    auto fail = [&](int code) {
        heat_free(c);
        delete c;
        return code;
    };
    const double ih2 = 1.0 / (c->h * c->h);
    const double sh = std::sin(M_PI * c->h / 2.0);
    const double lam1 = 4.0 * sh * sh * ih2;   // smallest eigenvalue of L_h
    c->f.assign(L, nullptr);
    c->x.assign(L, nullptr);
    c->sx.assign(L, nullptr);
    c->Cinv.assign(L, nullptr);
    c->G.assign(L, nullptr);
    c->K.assign(L, nullptr);
    c->Md.assign(L, nullptr);
    c->omega.assign(L, 0.0);
    c->chunks.assign(L, 1);
    c->Cl.assign(L, nullptr);
    c->Gl.assign(L, nullptr);
    c->SL.assign(L, nullptr);
    c->SR.assign(L, nullptr);
    c->Minv.assign(L, nullptr);
    int64_t simds = 0;
    {
        int dev = 0, ncu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return fail(TMG_ERR_HIP);
        simds = 4 * (int64_t)ncu;
    }
    int rc;
    int64_t maxtiles = 0;
    for (int l = 0; l < L; ++l) {
        const int64_t Nl = n_slabs >> l;
        c->Nl.push_back(Nl);
        const int64_t sz = Nl * nx * P;
        if (l > 0 && ((rc = halloc(c, &c->f[l], sz)) || (rc = halloc(c, &c->x[l], sz))))
            return fail(rc);
        if (l + 1 < L && (rc = halloc(c, &c->sx[l], sz))) return fail(rc);
        maxtiles = std::max(maxtiles, tiles(Nl, Hmax(o)));
        // the slab matrices at tau_l: K, M = tau diag(1/(2k+1)); D = K + (2/h^2) M,
        // E = -M/h^2; block elimination C_0 = D, C_i = D - E C_{i-1}^{-1} E
        const double tau = T / (double)Nl;
        std::vector<double> Km(P * P), Md(P), Ci((size_t)nx * P * P), Gi((size_t)nx * P * P);
        for (int k = 0; k < P; ++k) {
            Md[k] = tau / (2.0 * k + 1.0);
            for (int j = 0; j < P; ++j) Km[k * P + j] = (j < k && ((k + j) & 1)) ? -1.0 : 1.0;
        }
        std::vector<double> C(P * P), Cprev_inv(P * P, 0.0);
        for (int i = 0; i < nx; ++i) {
            for (int k = 0; k < P; ++k)
                for (int j = 0; j < P; ++j)
                    C[k * P + j] = Km[k * P + j] + (k == j ? 2.0 * ih2 * Md[k] : 0.0);
            if (i > 0)
                // - E C_{i-1}^{-1} E with E = -diag(Md)/h^2
                for (int k = 0; k < P; ++k)
                    for (int j = 0; j < P; ++j)
                        C[k * P + j] -= Md[k] * ih2 * Cprev_inv[k * P + j] * Md[j] * ih2;
            double *inv = &Ci[(size_t)i * P * P];
            table_invert(P, C.data(), inv);
            for (int k = 0; k < P; ++k)
                for (int j = 0; j < P; ++j) Gi[(size_t)i * P * P + k * P + j] = -inv[k * P + j] * Md[j] * ih2;
            for (int q = 0; q < P * P; ++q) Cprev_inv[q] = inv[q];
        }
        std::vector<double> tab(TabLayout(P).stride());
        const double alpha = level_table(P, lam1 * tau, 0, 0.0, false, tab.data());
        c->omega[l] = o.omega_mode == 0 ? (alpha >= 0.0 ? 1.0 / (1.0 + alpha * alpha) : 1.0)
                                        : o.omega;
        if ((rc = halloc(c, &c->Cinv[l], Ci.size())) || (rc = halloc(c, &c->G[l], Gi.size())) ||
            (rc = halloc(c, &c->K[l], Km.size())) || (rc = halloc(c, &c->Md[l], Md.size())))
            return fail(rc);
        if (hipMemcpyAsync(c->Cinv[l], Ci.data(), Ci.size() * 8, hipMemcpyHostToDevice, s) ||
            hipMemcpyAsync(c->G[l], Gi.data(), Gi.size() * 8, hipMemcpyHostToDevice, s) ||
            hipMemcpyAsync(c->K[l], Km.data(), Km.size() * 8, hipMemcpyHostToDevice, s) ||
            hipMemcpyAsync(c->Md[l], Md.data(), Md.size() * 8, hipMemcpyHostToDevice, s) ||
            hipStreamSynchronize(s))
            return fail(TMG_ERR_HIP);
        // levels with few tiles (the coarsest too, when a leg solves it):
        // the spatial solves partitioned over several wavefronts per tile
        const int K = pick_chunks(P, nx, tiles(Nl, Hmax(o)), simds);
        if (K > 1) {
            std::vector<double> Cl, Gl, SL, SR, Mi;
            if (!part_tables(P, nx, K, Km.data(), Md.data(), ih2, Cl, Gl, SL, SR, Mi))
                return fail(TMG_ERR_PARAM);
            if ((rc = halloc(c, &c->Cl[l], Cl.size())) || (rc = halloc(c, &c->Gl[l], Gl.size())) ||
                (rc = halloc(c, &c->SL[l], SL.size())) || (rc = halloc(c, &c->SR[l], SR.size())) ||
                (rc = halloc(c, &c->Minv[l], Mi.size())))
                return fail(rc);
            if (hipMemcpyAsync(c->Cl[l], Cl.data(), Cl.size() * 8, hipMemcpyHostToDevice, s) ||
                hipMemcpyAsync(c->Gl[l], Gl.data(), Gl.size() * 8, hipMemcpyHostToDevice, s) ||
                hipMemcpyAsync(c->SL[l], SL.data(), SL.size() * 8, hipMemcpyHostToDevice, s) ||
                hipMemcpyAsync(c->SR[l], SR.data(), SR.size() * 8, hipMemcpyHostToDevice, s) ||
                hipMemcpyAsync(c->Minv[l], Mi.data(), Mi.size() * 8, hipMemcpyHostToDevice, s) ||
                hipStreamSynchronize(s))
                return fail(TMG_ERR_HIP);
            c->chunks[l] = K;
        }
    }
    std::vector<double> R1T(P * P), R2T(P * P), R(2 * P * P);
    build_transfer(P, R1T.data(), R2T.data());
    for (int q = 0; q < P * P; ++q) {
        R[q] = R1T[q];
        R[P * P + q] = R2T[q];
    }
    c->ws_tiles = maxtiles;
    c->wide_tiles = 2 * simds;
    if ((rc = halloc(c, &c->R, R.size())) || (rc = halloc(c, &c->zeros, nx)) ||
        (rc = halloc(c, &c->ws, (size_t)maxtiles * 2 * nx * kHeatThreads * P)) ||
        (rc = halloc(c, &c->partial, maxtiles)) || (rc = halloc(c, &c->sum, 1)))
        return fail(rc);
    if (hipMemcpyAsync(c->R, R.data(), R.size() * 8, hipMemcpyHostToDevice, s) ||
        hipMemsetAsync(c->zeros, 0, sizeof(double) * nx, s) || hipStreamSynchronize(s))
        return fail(TMG_ERR_HIP);
    if ((rc = build_modes(c, s))) return fail(rc);
    *hp = c;
    return TMG_OK;
}

int tmg_heat_vcycle(tmg_heat_handle c, const double *f, const double *u0, double *u,
                    tmg_stream stream)
{
    if (!c || !f || !u0 || !u) return TMG_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    return level_pass(c, 0, f, u0, u, u, nullptr, s);
}

int tmg_heat_solve(tmg_heat_handle c, const double *f, const double *u0, double *u, double rtol,
                   int max_cycles, int *cycles, double *relres, tmg_stream stream)
{
    if (!c || !f || !u0 || !u || !(rtol >= 0.0) || max_cycles < 0) return TMG_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    int rc;
    double r0 = 0.0, rk = 0.0;
    if ((rc = norm2(c, f, u0, nullptr, s)) || (rc = read_sum(c, &r0, s))) return rc;
    HCHK(c, hipMemsetAsync(u, 0, sizeof(double) * c->N * c->nx * c->P, s));
    rk = r0;
    int k = 0, status = TMG_OK;
    if (!std::isfinite(r0)) status = TMG_ERR_NONFINITE;
    while (status == TMG_OK && r0 > 0.0 && k < max_cycles && rk > rtol * rtol * r0) {
        if ((rc = level_pass(c, 0, f, u0, k == 0 ? nullptr : u, u, c->partial, s))) return rc;
        ++k;
        if ((rc = read_sum(c, &rk, s))) return rc;
        if (!std::isfinite(rk)) status = TMG_ERR_NONFINITE;
        else if (rk > 1e6 * r0) status = TMG_ERR_DIVERGED;
    }
    if (status == TMG_OK && r0 > 0.0 && rk > rtol * rtol * r0) status = TMG_NOT_CONVERGED;
    if (cycles) *cycles = k;
    if (relres) *relres = r0 > 0.0 ? std::sqrt(rk / r0) : 0.0;
    return status;
}

int tmg_heat_destroy(tmg_heat_handle c)
{
    if (!c) return TMG_ERR_INVALID;
    (void)hipDeviceSynchronize();
    heat_free(c);
    delete c;
    return TMG_OK;
}

int tmg_heat_last_hip_error(tmg_heat_handle c) { return c ? c->last_hip : 0; }

int tmg_heat_set_mode_solve(tmg_heat_handle c, int on)
{
    if (!c) return TMG_ERR_INVALID;
    c->mode_on = on != 0;
    return TMG_OK;
}

}  // extern "C"
