// C ABI and host driver of the time-multigrid library (see include/tmg.h).
//
// The driver owns the level hierarchy of every instance, the per-level
// tables, the tile schedules and the captured cycle graphs.  One cycle is a
// fixed sequence of kernel launches (down legs, coarsest scans, up legs,
// norm finalisation) that is recorded once into a hipGraph per
// (first-cycle, direction, user pointers) and replayed; kernels read the
// per-instance convergence state and return at once for finished
// instances, so the host only synchronises every few cycles to read it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "../../include/tmg.h"
#include "tmg_internal.h"

using namespace tmg;

namespace {

enum TileKind { kDeep = 0, kAll = 1, kHasNext = 2 };

struct TileList {
    int64_t ntiles = 0;
    int64_t *d_off = nullptr;  // [batch+1]
};

struct GraphKey {
    int first, trans;
    const void *f, *u0, *u;
    bool operator<(const GraphKey &o) const
    {
        return std::tie(first, trans, f, u0, u) < std::tie(o.first, o.trans, o.f, o.u0, o.u);
    }
};

int even_up(int x) { return (x + 1) & ~1; }

}  // namespace

struct tmg_ctx {
    int batch = 0, P = 0, Lmax = 0;
    tmg_options opt{};
    std::vector<int64_t> N;
    std::vector<double> T, lam;
    std::vector<int> L;                           // levels of each instance
    std::vector<std::vector<int64_t>> slab_off_h; // [Lmax][batch+1]
    std::vector<int64_t *> slab_off_d;
    std::vector<double *> fl, ua, ub;             // level buffers (fl[0], ua[0] are the user's)
    std::vector<int64_t> level_size;              // doubles per level
    double *tab_fwd = nullptr, *tab_adj = nullptr;
    double *R_fwd = nullptr, *R_adj = nullptr;
    int tab_stride = 0;
    InstState *st = nullptr, *st_ops = nullptr;
    InstState *st_host = nullptr;                 // pinned
    Control *ctl = nullptr, *ctl_host = nullptr;  // device / pinned
    double *partial = nullptr;
    int64_t partial_cap = 0;
    double *tau_d = nullptr, *grad_d = nullptr, *grad_host = nullptr;
    std::map<std::tuple<int, int, int>, TileList> tiles;
    std::vector<int> lb;                          // first level of the bottom kernel, per instance
    std::vector<int *> bot_visit_d, bot_coarse_d; // per level: bottom lists (visit / exact solve only)
    std::vector<int> bot_visit_n, bot_coarse_n;
    std::vector<int> deep_n;                      // per level: instances with level < lb[j]
    int *lb_d = nullptr, *nlev_d = nullptr;
    double **fl_d = nullptr, **ua_d = nullptr, **ub_d = nullptr;
    int64_t **slab_off_dd = nullptr;
    int64_t bottom_max = 0;
    std::map<std::tuple<int, int>, std::pair<int *, int>> op_coarse;  // (level, unused) -> list
    std::map<GraphKey, hipGraphExec_t> graphs;
    hipStream_t cap = nullptr;
    int last_hip = 0;
    std::vector<void *> allocs;

    int H_down() const { return even_up(opt.nu1 + 1); }
    int H_up() const { return even_up(opt.nu2 + 1); }
    int TO_down() const { return tile_slabs(P) - H_down(); }
    int TO_up() const { return tile_slabs(P) - H_up(); }
};

namespace {

#define HIPCHK(ctx, expr)                           \
    do {                                            \
        hipError_t e_ = (expr);                     \
        if (e_ != hipSuccess) {                     \
            (ctx)->last_hip = (int)e_;              \
            return e_ == hipErrorOutOfMemory ? TMG_ERR_OOM : TMG_ERR_HIP; \
        }                                           \
    } while (0)

template <typename T>
int dalloc(tmg_ctx *c, T **p, size_t n)
{
    *p = nullptr;
    if (n == 0) n = 1;
    hipError_t e = hipMalloc((void **)p, n * sizeof(T));
    if (e != hipSuccess) {
        c->last_hip = (int)e;
        return TMG_ERR_OOM;
    }
    c->allocs.push_back(*p);
    return TMG_OK;
}

bool participates(const tmg_ctx *c, int j, int level, int kind)
{
    if (level >= c->L[j]) return false;
    if (kind == kDeep) return level < c->lb[j];      // streaming kernels in the cycle
    if (kind == kHasNext) return level + 1 < c->L[j];  // level-wise entry points
    return true;
}

// Tile offsets (prefix sums of ceil(N_jl / tile_out) over participating
// instances) for one (level, kind, tile_out), cached on the device.
int get_tiles(tmg_ctx *c, int level, int kind, int tile_out, hipStream_t s, TileList **out)
{
    auto key = std::make_tuple(level, kind, tile_out);
    auto it = c->tiles.find(key);
    if (it != c->tiles.end()) {
        *out = &it->second;
        return TMG_OK;
    }
    std::vector<int64_t> off(c->batch + 1, 0);
    for (int j = 0; j < c->batch; ++j) {
        int64_t n = 0;
        if (participates(c, j, level, kind)) {
            int64_t Nl = c->N[j] >> level;
            n = (Nl + tile_out - 1) / tile_out;
        }
        off[j + 1] = off[j] + n;
    }
    TileList tl;
    tl.ntiles = off[c->batch];
    int rc = dalloc(c, &tl.d_off, off.size());
    if (rc) return rc;
    HIPCHK(c, hipMemcpyAsync(tl.d_off, off.data(), off.size() * sizeof(int64_t),
                             hipMemcpyHostToDevice, s));
    HIPCHK(c, hipStreamSynchronize(s));
    auto res = c->tiles.emplace(key, tl);
    *out = &res.first->second;
    return TMG_OK;
}

const double *tab_of(const tmg_ctx *c, int level, bool trans)
{
    return (trans ? c->tab_adj : c->tab_fwd) + (int64_t)level * c->batch * c->tab_stride;
}

LevelArgs base_args(const tmg_ctx *c, int level, bool trans)
{
    LevelArgs a{};
    a.tab = tab_of(c, level, trans);
    a.R = trans ? c->R_adj : c->R_fwd;
    a.slab_off = c->slab_off_d[level];
    a.cslab_off = level + 1 < c->Lmax ? c->slab_off_d[level + 1] : nullptr;
    a.batch = c->batch;
    a.tab_stride = c->tab_stride;
    return a;
}

// ---- one cycle ----------------------------------------------------------

struct CycleIO {
    const double *f, *u0;
    double *u;
    bool trans, first, use_state;
};

int enqueue_visit(tmg_ctx *c, const CycleIO &io, int level, bool zero_init, hipStream_t s);

int enqueue_down(tmg_ctx *c, const CycleIO &io, int level, bool zero_init, hipStream_t s)
{
    TileList *tl;
    int rc = get_tiles(c, level, kDeep, c->TO_down(), s, &tl);
    if (rc) return rc;
    LevelArgs a = base_args(c, level, io.trans);
    a.f = level == 0 ? io.f : c->fl[level];
    a.u0 = (level == 0 && !io.trans) ? io.u0 : nullptr;
    a.u_in = zero_init ? nullptr : (level == 0 ? io.u : c->ua[level]);
    a.u_out = c->ub[level];
    a.rc = c->fl[level + 1];
    a.tile_off = tl->d_off;
    a.st = io.use_state ? c->st : nullptr;
    a.nsweep = c->opt.nu1;
    a.halo = c->H_down();
    a.tile_out = c->TO_down();
    HIPCHK(c, launch_down(c->P, io.trans, a, tl->ntiles, s));
    return TMG_OK;
}

int enqueue_up(tmg_ctx *c, const CycleIO &io, int level, hipStream_t s)
{
    TileList *tl;
    int rc = get_tiles(c, level, kDeep, c->TO_up(), s, &tl);
    if (rc) return rc;
    LevelArgs a = base_args(c, level, io.trans);
    a.f = level == 0 ? io.f : c->fl[level];
    a.u0 = (level == 0 && !io.trans) ? io.u0 : nullptr;
    a.u_in = c->ub[level];
    a.e = c->ua[level + 1];
    a.u_out = level == 0 ? io.u : c->ua[level];
    a.tile_off = tl->d_off;
    a.st = io.use_state ? c->st : nullptr;
    a.nsweep = c->opt.nu2;
    a.halo = c->H_up();
    a.tile_out = c->TO_up();
    if (level == 0 && io.use_state) {
        TileList *nl;
        rc = get_tiles(c, 0, kAll, c->TO_up(), s, &nl);
        if (rc) return rc;
        a.partial = c->partial;
        a.norm_off = nl->d_off;
    }
    HIPCHK(c, launch_up(c->P, io.trans, a, tl->ntiles, s));
    return TMG_OK;
}

// Bottom kernel for the instances whose single-work-group part starts at
// `level`: exact solve only (coarse list) or a full visit (visit list).
int enqueue_bottom(tmg_ctx *c, const CycleIO &io, int level, bool visits, bool zero,
                   hipStream_t s)
{
    const int n = visits ? c->bot_visit_n[level] : c->bot_coarse_n[level];
    if (n == 0) return TMG_OK;
    BottomArgs a{};
    a.fl = c->fl_d;
    a.ua = c->ua_d;
    a.ub = c->ub_d;
    a.slab_off = c->slab_off_dd;
    a.tab = io.trans ? c->tab_adj : c->tab_fwd;
    a.R = io.trans ? c->R_adj : c->R_fwd;
    a.inst = visits ? c->bot_visit_d[level] : c->bot_coarse_d[level];
    a.lb = c->lb_d;
    a.nlev = c->nlev_d;
    a.f0 = io.f;
    a.u0 = io.trans ? nullptr : io.u0;
    a.u = io.u;
    a.st = io.use_state ? c->st : nullptr;
    if (level == 0 && io.use_state) {
        TileList *nl;
        int rc = get_tiles(c, 0, kAll, c->TO_up(), s, &nl);
        if (rc) return rc;
        a.partial = c->partial;
        a.norm_off = nl->d_off;
    }
    a.batch = c->batch;
    a.tab_stride = c->tab_stride;
    a.nu1 = c->opt.nu1;
    a.nu2 = c->opt.nu2;
    a.gamma = c->opt.gamma;
    a.zero = zero ? 1 : 0;
    HIPCHK(c, launch_bottom(c->P, io.trans, a, n, s));
    return TMG_OK;
}

// Multigrid visit of `level` for the instances that run this level with the
// streaming kernels (level < lb[j]): nu1 sweeps + residual + restriction,
// gamma visits of the next level from zero (bottom kernel or recursion; an
// exact solve once when the next level is an instance's coarsest), then
// prolongation + correction + nu2 sweeps.
int enqueue_visit(tmg_ctx *c, const CycleIO &io, int level, bool zero_init, hipStream_t s)
{
    int rc = enqueue_down(c, io, level, zero_init, s);
    if (rc) return rc;
    if ((rc = enqueue_bottom(c, io, level + 1, false, true, s))) return rc;
    for (int g = 0; g < c->opt.gamma; ++g) {
        if ((rc = enqueue_bottom(c, io, level + 1, true, g == 0, s))) return rc;
        if (level + 1 < c->Lmax && c->deep_n[level + 1] > 0)
            if ((rc = enqueue_visit(c, io, level + 1, g == 0, s))) return rc;
    }
    return enqueue_up(c, io, level, s);
}

int enqueue_cycle(tmg_ctx *c, const CycleIO &io, hipStream_t s)
{
    int rc;
    if ((rc = enqueue_bottom(c, io, 0, false, io.first, s))) return rc;
    if ((rc = enqueue_bottom(c, io, 0, true, io.first, s))) return rc;
    if (c->deep_n[0] > 0)
        if ((rc = enqueue_visit(c, io, 0, io.first, s))) return rc;
    if (io.use_state) {
        TileList *nl;
        if ((rc = get_tiles(c, 0, kAll, c->TO_up(), s, &nl))) return rc;
        HIPCHK(c, launch_finalize(c->partial, nl->d_off, c->batch, c->st, c->ctl, 0, s));
    }
    return TMG_OK;
}

int get_graph(tmg_ctx *c, const CycleIO &io, hipGraphExec_t *out)
{
    GraphKey key{io.first, io.trans, io.f, io.u0, io.u};
    auto it = c->graphs.find(key);
    if (it != c->graphs.end()) {
        *out = it->second;
        return TMG_OK;
    }
    if (c->graphs.size() >= 16) {
        for (auto &kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
        c->graphs.clear();
    }
    // make sure every tile list exists before capture (no memcpy inside)
    {
        TileList *tl;
        int rc;
        for (int l = 0; l < c->Lmax; ++l) {
            if ((rc = get_tiles(c, l, kDeep, c->TO_down(), c->cap, &tl))) return rc;
            if ((rc = get_tiles(c, l, kDeep, c->TO_up(), c->cap, &tl))) return rc;
        }
        if ((rc = get_tiles(c, 0, kAll, c->TO_up(), c->cap, &tl))) return rc;
    }
    hipGraph_t g;
    HIPCHK(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    int rc = enqueue_cycle(c, io, c->cap);
    hipError_t ee = hipStreamEndCapture(c->cap, &g);
    if (rc) return rc;
    HIPCHK(c, ee);
    hipGraphExec_t exec;
    hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCHK(c, ei);
    c->graphs[key] = exec;
    *out = exec;
    return TMG_OK;
}

int check_level_args(tmg_ctx *c, int level)
{
    if (!c || level < 0 || level >= c->Lmax) return TMG_ERR_INVALID;
    return TMG_OK;
}

void free_all(tmg_ctx *c)
{
    for (auto &kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
    for (void *p : c->allocs) (void)hipFree(p);
    c->allocs.clear();
    if (c->st_host) (void)hipHostFree(c->st_host);
    if (c->ctl_host) (void)hipHostFree(c->ctl_host);
    if (c->grad_host) (void)hipHostFree(c->grad_host);
    if (c->cap) (void)hipStreamDestroy(c->cap);
}

// Solve loop shared by tmg_solve and tmg_adjoint_solve.
int run_solve(tmg_ctx *c, const double *f, const double *u0, double *u, bool trans, double rtol,
              int max_cycles, int *cycles, double *relres, hipStream_t s)
{
    TileList *tl;
    int rc = get_tiles(c, 0, kAll, tile_slabs(c->P), s, &tl);
    if (rc) return rc;
    c->ctl_host->rtol2 = rtol * rtol;
    c->ctl_host->max_cycles = max_cycles;
    c->ctl_host->pad = 0;
    HIPCHK(c, hipMemcpyAsync(c->ctl, c->ctl_host, sizeof(Control), hipMemcpyHostToDevice, s));
    // initial residual r_0 = f (u0 folded), u = 0
    HIPCHK(c, launch_norm_f(c->P, f, trans ? nullptr : u0, tab_of(c, 0, trans), c->tab_stride,
                            c->slab_off_d[0], tl->d_off, c->batch, c->partial, tl->ntiles, s));
    HIPCHK(c, launch_finalize(c->partial, tl->d_off, c->batch, c->st, c->ctl, 1, s));

    CycleIO io{f, u0, u, trans, true, true};
    hipGraphExec_t g_first, g_next;
    if ((rc = get_graph(c, io, &g_first))) return rc;
    io.first = false;
    if ((rc = get_graph(c, io, &g_next))) return rc;

    int launched = 0;
    if (max_cycles > 0) {
        HIPCHK(c, hipGraphLaunch(g_first, s));
        launched = 1;
    }
    std::vector<double> prev_rsq(c->batch, -1.0);
    std::vector<int> prev_cyc(c->batch, 0);
    while (true) {
        HIPCHK(c, hipMemcpyAsync(c->st_host, c->st, sizeof(InstState) * c->batch,
                                 hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        bool all = true;
        int need = 1;
        for (int j = 0; j < c->batch; ++j) {
            const InstState &q = c->st_host[j];
            if (q.done) continue;
            all = false;
            // cycles still needed at the contraction rate observed since the
            // previous check (launched cycles are no-ops once converged)
            const int dc = q.cycles - prev_cyc[j];
            if (prev_rsq[j] > 0.0 && dc > 0 && q.rsq > 0.0 && q.rsq < prev_rsq[j]) {
                const double lrate = 0.5 * std::log(q.rsq / prev_rsq[j]) / dc;
                const double lgoal = 0.5 * std::log(c->ctl_host->rtol2 * q.r0sq / q.rsq);
                const int k = (int)std::ceil(lgoal / lrate);
                need = std::max(need, std::min(std::max(k, 1), 8));
            }
            prev_rsq[j] = q.rsq;
            prev_cyc[j] = q.cycles;
        }
        if (all || launched >= max_cycles) break;
        need = std::min(need, max_cycles - launched);
        for (int k = 0; k < need; ++k) HIPCHK(c, hipGraphLaunch(g_next, s));
        launched += need;
    }
    int status = TMG_OK;
    for (int j = 0; j < c->batch; ++j) {
        const InstState &q = c->st_host[j];
        if (q.cycles == 0) {
            // no cycle ran for it (r_0 = 0 or max_cycles = 0): the iterate is u = 0
            HIPCHK(c, hipMemsetAsync(u + c->slab_off_h[0][j] * c->P, 0,
                                     sizeof(double) * c->N[j] * c->P, s));
        }
        if (cycles) cycles[j] = q.cycles;
        if (relres) relres[j] = q.r0sq > 0.0 ? std::sqrt(q.rsq / q.r0sq) : 0.0;
        int sj = TMG_OK;
        if (q.done == 3) sj = TMG_ERR_NONFINITE;
        else if (q.done == 4) sj = TMG_ERR_DIVERGED;
        else if (q.done != 1) sj = TMG_NOT_CONVERGED;
        if (sj < 0) status = std::min(status, sj);
        else if (sj > 0 && status == TMG_OK) status = sj;
    }
    HIPCHK(c, hipStreamSynchronize(s));
    return status;
}

}  // namespace

extern "C" {

void tmg_default_options(tmg_options *o)
{
    if (!o) return;
    o->p = 1;
    o->nu1 = 2;
    o->nu2 = 2;
    o->gamma = 1;
    o->n_coarse = 2;
    o->omega_mode = 0;
    o->omega = 0.5;
    o->precision = 0;
    o->schedule = -1;
}

const char *tmg_error_string(int code)
{
    switch (code) {
    case TMG_OK: return "ok";
    case TMG_NOT_CONVERGED: return "max_cycles reached before the residual tolerance";
    case TMG_ERR_INVALID: return "invalid argument";
    case TMG_ERR_SIZE: return "slab count is not n_coarse * 2^k";
    case TMG_ERR_OMEGA: return "damping parameter outside (0, 1]";
    case TMG_ERR_PARAM: return "lambda and T must be finite and positive";
    case TMG_ERR_OOM: return "device memory allocation failed";
    case TMG_ERR_HIP: return "HIP runtime error";
    case TMG_ERR_NONFINITE: return "non-finite value in the data or the residual";
    case TMG_ERR_DIVERGED: return "residual grew beyond 1e3 times the initial residual";
    case TMG_ERR_UNSUPPORTED: return "option combination not supported";
    default: return "unknown status";
    }
}

int tmg_last_hip_error(tmg_handle h) { return h ? h->last_hip : 0; }

int tmg_setup(tmg_handle *hp, int batch, const int64_t *n_slabs, const double *T,
              const double *lambda, const tmg_options *opt, tmg_stream stream)
{
    if (!hp || !n_slabs || !T || !lambda || !opt || batch < 1) return TMG_ERR_INVALID;
    *hp = nullptr;
    const tmg_options &o = *opt;
    if (o.p < 0 || o.p > TMG_MAX_DEGREE || o.nu1 < 0 || o.nu1 > kMaxSweeps || o.nu2 < 0 ||
        o.nu2 > kMaxSweeps || (o.gamma != 1 && o.gamma != 2) || o.n_coarse < 1 ||
        o.n_coarse > kMaxCoarse || (o.omega_mode != 0 && o.omega_mode != 1))
        return TMG_ERR_INVALID;
    if (o.omega_mode == 1 && !(o.omega > 0.0 && o.omega <= 1.0)) return TMG_ERR_OMEGA;
    if (o.precision != 0) return TMG_ERR_UNSUPPORTED;
    std::vector<int> L(batch);
    for (int j = 0; j < batch; ++j) {
        if (!(std::isfinite(T[j]) && T[j] > 0.0 && std::isfinite(lambda[j]) && lambda[j] > 0.0))
            return TMG_ERR_PARAM;
        int64_t n = n_slabs[j];
        if (n < o.n_coarse || n > (int64_t(1) << 40)) return TMG_ERR_SIZE;
        int lev = 1;
        while (n > o.n_coarse) {
            if (n & 1) return TMG_ERR_SIZE;
            n >>= 1;
            ++lev;
        }
        if (n != o.n_coarse) return TMG_ERR_SIZE;
        L[j] = lev;
    }
    tmg_ctx *c = new (std::nothrow) tmg_ctx;
    if (!c) return TMG_ERR_OOM;
    hipStream_t s = (hipStream_t)stream;
    c->batch = batch;
    c->P = o.p + 1;
    c->opt = o;
    c->N.assign(n_slabs, n_slabs + batch);
    c->T.assign(T, T + batch);
    c->lam.assign(lambda, lambda + batch);
    c->L = L;
    c->Lmax = *std::max_element(L.begin(), L.end());
    const int P = c->P, Lm = c->Lmax;
    const TabLayout TL(P);
    c->tab_stride = TL.stride();

    int rc = TMG_OK;
    auto fail = [&](int code) {
        free_all(c);
        delete c;
        return code;
    };
    if (hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess)
        return fail(TMG_ERR_HIP);

    // level layouts
    c->slab_off_h.assign(Lm, std::vector<int64_t>(batch + 1, 0));
    c->slab_off_d.assign(Lm, nullptr);
    c->level_size.assign(Lm, 0);
    c->fl.assign(Lm, nullptr);
    c->ua.assign(Lm, nullptr);
    c->ub.assign(Lm, nullptr);
    // levels of at most bottom_max slabs run inside the single-work-group
    // bottom kernel (schedule >= 0: bottom_max = 2^schedule, capped)
    const int64_t cap_bottom = (int64_t)kBottomThreads * slabs_per_thread(P);
    c->bottom_max = o.schedule < 0 ? cap_bottom
                                   : std::min<int64_t>(cap_bottom, int64_t(1) << std::min(o.schedule, 40));
    c->lb.assign(batch, 0);
    for (int j = 0; j < batch; ++j) {
        int l = 0;
        while (l < L[j] - 1 && (c->N[j] >> l) > c->bottom_max) ++l;
        c->lb[j] = l;
    }
    c->deep_n.assign(Lm, 0);
    c->bot_visit_n.assign(Lm, 0);
    c->bot_coarse_n.assign(Lm, 0);
    c->bot_visit_d.assign(Lm, nullptr);
    c->bot_coarse_d.assign(Lm, nullptr);
    auto upload_list = [&](const std::vector<int> &v, int **d) -> int {
        if (v.empty()) return TMG_OK;
        int r = dalloc(c, d, v.size());
        if (r) return r;
        if (hipMemcpyAsync(*d, v.data(), sizeof(int) * v.size(), hipMemcpyHostToDevice, s) !=
            hipSuccess)
            return TMG_ERR_HIP;
        return TMG_OK;
    };
    for (int l = 0; l < Lm; ++l) {
        auto &off = c->slab_off_h[l];
        std::vector<int> bv, bc;
        for (int j = 0; j < batch; ++j) {
            off[j + 1] = off[j] + (l < L[j] ? (c->N[j] >> l) : 0);
            if (c->lb[j] == l) (c->lb[j] == L[j] - 1 ? bc : bv).push_back(j);
            if (l < c->lb[j]) c->deep_n[l]++;
        }
        c->level_size[l] = off[batch] * P;
        c->bot_visit_n[l] = (int)bv.size();
        c->bot_coarse_n[l] = (int)bc.size();
        if ((rc = dalloc(c, &c->slab_off_d[l], batch + 1))) return fail(rc);
        if (hipMemcpyAsync(c->slab_off_d[l], off.data(), sizeof(int64_t) * (batch + 1),
                           hipMemcpyHostToDevice, s) != hipSuccess)
            return fail(TMG_ERR_HIP);
        if ((rc = upload_list(bv, &c->bot_visit_d[l]))) return fail(rc);
        if ((rc = upload_list(bc, &c->bot_coarse_d[l]))) return fail(rc);
        if (hipStreamSynchronize(s) != hipSuccess) return fail(TMG_ERR_HIP);
        // buffers: level 0 needs only the ping-pong partner of the user's u
        if (l > 0) {
            if ((rc = dalloc(c, &c->fl[l], c->level_size[l]))) return fail(rc);
            if ((rc = dalloc(c, &c->ua[l], c->level_size[l]))) return fail(rc);
        }
        if (l + 1 < Lm) {
            if ((rc = dalloc(c, &c->ub[l], c->level_size[l]))) return fail(rc);
        }
    }
    // per-level pointer arrays and per-instance level data for the bottom kernel
    {
        std::vector<int> nlev(L.begin(), L.end());
        if ((rc = dalloc(c, &c->lb_d, batch)) || (rc = dalloc(c, &c->nlev_d, batch)) ||
            (rc = dalloc(c, &c->fl_d, Lm)) || (rc = dalloc(c, &c->ua_d, Lm)) ||
            (rc = dalloc(c, &c->ub_d, Lm)) || (rc = dalloc(c, &c->slab_off_dd, Lm)))
            return fail(rc);
        if (hipMemcpyAsync(c->lb_d, c->lb.data(), sizeof(int) * batch, hipMemcpyHostToDevice, s) ||
            hipMemcpyAsync(c->nlev_d, nlev.data(), sizeof(int) * batch, hipMemcpyHostToDevice, s) ||
            hipMemcpyAsync(c->fl_d, c->fl.data(), sizeof(double *) * Lm, hipMemcpyHostToDevice, s) ||
            hipMemcpyAsync(c->ua_d, c->ua.data(), sizeof(double *) * Lm, hipMemcpyHostToDevice, s) ||
            hipMemcpyAsync(c->ub_d, c->ub.data(), sizeof(double *) * Lm, hipMemcpyHostToDevice, s) ||
            hipMemcpyAsync(c->slab_off_dd, c->slab_off_d.data(), sizeof(int64_t *) * Lm,
                           hipMemcpyHostToDevice, s) ||
            hipStreamSynchronize(s))
            return fail(TMG_ERR_HIP);
    }
    // tables, level-major: block (l, j) at (l * batch + j) * stride
    std::vector<double> tf((size_t)Lm * batch * c->tab_stride, 0.0),
        ta((size_t)Lm * batch * c->tab_stride, 0.0);
    for (int l = 0; l < Lm; ++l)
        for (int j = 0; j < batch; ++j) {
            if (l >= L[j]) continue;
            double z = lambda[j] * T[j] / (double)(c->N[j] >> l);
            size_t at = ((size_t)l * batch + j) * c->tab_stride;
            build_level_table(P, z, o.omega_mode, o.omega, false, &tf[at]);
            build_level_table(P, z, o.omega_mode, o.omega, true, &ta[at]);
        }
    std::vector<double> R1T(P * P), R2T(P * P), Rf(2 * P * P), Ra(2 * P * P);
    build_transfer(P, R1T.data(), R2T.data());
    for (int i = 0; i < P * P; ++i) {
        Rf[i] = R1T[i];
        Rf[P * P + i] = R2T[i];
        Ra[i] = R2T[i];
        Ra[P * P + i] = R1T[i];
    }
    std::vector<double> tau(batch);
    for (int j = 0; j < batch; ++j) tau[j] = T[j] / (double)c->N[j];
    if ((rc = dalloc(c, &c->tab_fwd, tf.size())) || (rc = dalloc(c, &c->tab_adj, ta.size())) ||
        (rc = dalloc(c, &c->R_fwd, Rf.size())) || (rc = dalloc(c, &c->R_adj, Ra.size())) ||
        (rc = dalloc(c, &c->st, batch)) || (rc = dalloc(c, &c->st_ops, batch)) ||
        (rc = dalloc(c, &c->ctl, 1)) || (rc = dalloc(c, &c->tau_d, batch)) ||
        (rc = dalloc(c, &c->grad_d, 2 * batch)))
        return fail(rc);
    // partial sums: one slot per level-0 tile at the smallest tile size in use
    int64_t maxtiles = 0;
    for (int j = 0; j < batch; ++j) {
        int tmin = tile_slabs(P) - even_up(kMaxSweeps + 1);
        maxtiles += (c->N[j] + tmin - 1) / tmin;
    }
    c->partial_cap = maxtiles;
    if ((rc = dalloc(c, &c->partial, maxtiles))) return fail(rc);
    if (hipHostMalloc((void **)&c->st_host, sizeof(InstState) * batch) != hipSuccess ||
        hipHostMalloc((void **)&c->ctl_host, sizeof(Control)) != hipSuccess ||
        hipHostMalloc((void **)&c->grad_host, sizeof(double) * 2 * batch) != hipSuccess)
        return fail(TMG_ERR_OOM);
    if (hipMemcpyAsync(c->tab_fwd, tf.data(), tf.size() * 8, hipMemcpyHostToDevice, s) ||
        hipMemcpyAsync(c->tab_adj, ta.data(), ta.size() * 8, hipMemcpyHostToDevice, s) ||
        hipMemcpyAsync(c->R_fwd, Rf.data(), Rf.size() * 8, hipMemcpyHostToDevice, s) ||
        hipMemcpyAsync(c->R_adj, Ra.data(), Ra.size() * 8, hipMemcpyHostToDevice, s) ||
        hipMemcpyAsync(c->tau_d, tau.data(), tau.size() * 8, hipMemcpyHostToDevice, s) ||
        hipMemsetAsync(c->st, 0, sizeof(InstState) * batch, s) ||
        hipStreamSynchronize(s))
        return fail(TMG_ERR_HIP);
    *hp = c;
    return TMG_OK;
}

int tmg_destroy(tmg_handle h)
{
    if (!h) return TMG_ERR_INVALID;
    (void)hipDeviceSynchronize();
    free_all(h);
    delete h;
    return TMG_OK;
}

int tmg_vcycle(tmg_handle c, const double *f, const double *u0, double *u, tmg_stream stream)
{
    if (!c || !f || !u0 || !u) return TMG_ERR_INVALID;
    CycleIO io{f, u0, u, false, false, false};
    return enqueue_cycle(c, io, (hipStream_t)stream);
}

int tmg_solve(tmg_handle c, const double *f, const double *u0, double *u, double rtol,
              int max_cycles, int *cycles, double *relres, tmg_stream stream)
{
    if (!c || !f || !u0 || !u || !(rtol >= 0.0) || max_cycles < 0) return TMG_ERR_INVALID;
    return run_solve(c, f, u0, u, false, rtol, max_cycles, cycles, relres, (hipStream_t)stream);
}

int tmg_adjoint_solve(tmg_handle c, const double *g, const double *u, double *z, double rtol,
                      int max_cycles, double *dlambda, double *du0, int *cycles,
                      double *relres, tmg_stream stream)
{
    if (!c || !g || !z || !(rtol >= 0.0) || max_cycles < 0) return TMG_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    int st = run_solve(c, g, nullptr, z, true, rtol, max_cycles, cycles, relres, s);
    if (st < 0) return st;
    if (u && (dlambda || du0)) {
        HIPCHK(c, launch_grad(c->P, u, z, c->tau_d, c->slab_off_d[0], c->batch, c->grad_d, s));
        HIPCHK(c, hipMemcpyAsync(c->grad_host, c->grad_d, sizeof(double) * 2 * c->batch,
                                 hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        for (int j = 0; j < c->batch; ++j) {
            if (dlambda) dlambda[j] = c->grad_host[2 * j];
            if (du0) du0[j] = c->grad_host[2 * j + 1];
        }
    }
    return st;
}

int tmg_level_info(tmg_handle c, int j, int level, int64_t *n, double *alpha, double *omega)
{
    if (!c || j < 0 || j >= c->batch) return TMG_ERR_INVALID;
    if (level < 0 || level >= c->L[j]) return TMG_ERR_INVALID;
    double z = c->lam[j] * c->T[j] / (double)(c->N[j] >> level);
    std::vector<double> t(c->tab_stride);
    double a = build_level_table(c->P, z, c->opt.omega_mode, c->opt.omega, false, t.data());
    const TabLayout TL(c->P);
    if (n) *n = c->N[j] >> level;
    if (alpha) *alpha = a;
    if (omega) *omega = 1.0 - t[TL.OMC()];
    return c->L[j];
}

int64_t tmg_level_size(tmg_handle c, int level)
{
    if (!c || level < 0 || level >= c->Lmax) return -1;
    return c->level_size[level];
}

int tmg_op_down(tmg_handle c, int level, int trans, int nsweep, const double *f,
                const double *fold_u0, const double *u_in, double *u_out, double *rcout,
                tmg_stream stream)
{
    int rc = check_level_args(c, level);
    if (rc) return rc;
    if (!f || nsweep < 0 || nsweep > kMaxSweeps || (rcout && level + 1 >= c->Lmax) ||
        (fold_u0 && (level != 0 || trans)))
        return TMG_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    const int H = even_up(nsweep + 1), TO = tile_slabs(c->P) - H;
    TileList *tl;
    if ((rc = get_tiles(c, level, rcout ? kHasNext : kAll, TO, s, &tl))) return rc;
    LevelArgs a = base_args(c, level, trans != 0);
    a.f = f;
    a.u0 = fold_u0;
    a.u_in = u_in;
    a.u_out = u_out;
    a.rc = rcout;
    a.tile_off = tl->d_off;
    a.nsweep = nsweep;
    a.halo = H;
    a.tile_out = TO;
    HIPCHK(c, launch_down(c->P, trans != 0, a, tl->ntiles, s));
    return TMG_OK;
}

int tmg_op_up(tmg_handle c, int level, int trans, int nsweep, const double *f,
              const double *fold_u0, const double *u_in, const double *e, double *u_out,
              tmg_stream stream)
{
    int rc = check_level_args(c, level);
    if (rc) return rc;
    if (!f || !u_in || nsweep < 0 || nsweep > kMaxSweeps || (e && level + 1 >= c->Lmax) ||
        (fold_u0 && (level != 0 || trans)))
        return TMG_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    const int H = even_up(nsweep + 1), TO = tile_slabs(c->P) - H;
    TileList *tl;
    if ((rc = get_tiles(c, level, e ? kHasNext : kAll, TO, s, &tl))) return rc;
    LevelArgs a = base_args(c, level, trans != 0);
    a.f = f;
    a.u0 = fold_u0;
    a.u_in = u_in;
    a.e = e;
    a.u_out = u_out;
    a.tile_off = tl->d_off;
    a.nsweep = nsweep;
    a.halo = H;
    a.tile_out = TO;
    HIPCHK(c, launch_up(c->P, trans != 0, a, tl->ntiles, s));
    return TMG_OK;
}

int tmg_op_coarse_solve(tmg_handle c, int level, int trans, const double *r, double *e,
                        tmg_stream stream)
{
    int rc = check_level_args(c, level);
    if (rc) return rc;
    if (!r || !e) return TMG_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    auto key = std::make_tuple(level, 0);
    auto it = c->op_coarse.find(key);
    if (it == c->op_coarse.end()) {
        std::vector<int> list;
        for (int j = 0; j < c->batch; ++j)
            if (level < c->L[j]) {
                if ((c->N[j] >> level) > kMaxCoarse) return TMG_ERR_SIZE;
                list.push_back(j);
            }
        int *d = nullptr;
        if ((rc = dalloc(c, &d, list.size()))) return rc;
        HIPCHK(c, hipMemcpyAsync(d, list.data(), sizeof(int) * list.size(),
                                 hipMemcpyHostToDevice, s));
        HIPCHK(c, hipStreamSynchronize(s));
        it = c->op_coarse.emplace(key, std::make_pair(d, (int)list.size())).first;
    }
    CoarseArgs a{};
    a.r = r;
    a.e = e;
    a.tab = tab_of(c, level, trans != 0);
    a.slab_off = c->slab_off_d[level];
    a.inst = it->second.first;
    a.tab_stride = c->tab_stride;
    HIPCHK(c, launch_coarse(c->P, trans != 0, a, it->second.second, s));
    return TMG_OK;
}

int tmg_op_residual_norm(tmg_handle c, int trans, const double *f, const double *fold_u0,
                         const double *u, double *norms, tmg_stream stream)
{
    if (!c || !f || !u || !norms || (fold_u0 && trans)) return TMG_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    const int H = 2, TO = tile_slabs(c->P) - H;
    TileList *tl;
    int rc = get_tiles(c, 0, kAll, TO, s, &tl);
    if (rc) return rc;
    if (tl->ntiles > c->partial_cap) return TMG_ERR_INVALID;
    LevelArgs a = base_args(c, 0, trans != 0);
    a.f = f;
    a.u0 = fold_u0;
    a.u_in = u;
    a.tile_off = tl->d_off;
    a.norm_off = tl->d_off;
    a.partial = c->partial;
    a.nsweep = 0;
    a.halo = H;
    a.tile_out = TO;
    HIPCHK(c, launch_up(c->P, trans != 0, a, tl->ntiles, s));
    HIPCHK(c, launch_finalize(c->partial, tl->d_off, c->batch, c->st_ops, c->ctl, 1, s));
    HIPCHK(c, hipMemcpyAsync(c->st_host, c->st_ops, sizeof(InstState) * c->batch,
                             hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    for (int j = 0; j < c->batch; ++j) norms[j] = std::sqrt(c->st_host[j].r0sq);
    return TMG_OK;
}

}  // extern "C"
