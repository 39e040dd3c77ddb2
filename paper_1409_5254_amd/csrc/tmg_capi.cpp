// C ABI and host driver of the time-multigrid library (see include/tmg.h).
//
// The driver owns the level hierarchy of every instance, the per-level
// tables, the tile schedules and the captured cycle graphs.
//
// One cycle, for an instance whose levels 0 .. lb-1 run on the streaming
// kernel and lb .. L-1 inside the single-work-group bottom kernel:
//   level 0   : the down leg of this cycle was already done by the previous
//               cycle's fused level-0 pass (or by a separate down leg in the
//               first cycle);
//   1 .. lb-1 : down legs (pre-smoothing + residual + restriction; nothing
//               but the restricted residual is stored);
//   lb        : bottom kernel (gamma visits for a W-cycle);
//   .. 1      : up legs, which recompute the pre-smoothing from the level's
//               right-hand side instead of reading a stored iterate;
//   level 0   : one fused pass: recomputed pre-smoothing, correction,
//               post-smoothing, the residual norm, and the next cycle's
//               pre-smoothing, residual and restriction.
// The level-0 iterate is updated in place; each tile takes its left halo
// from a small per-tile buffer written by the previous pass, so no tile ever
// reads slabs another tile of the same pass writes.  Three graphs (first,
// odd, even: the halo buffers alternate) are captured once per
// (direction, user pointers) and replayed; kernels read the per-instance
// convergence state and return at once for finished instances, so the host
// only synchronises every few cycles.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <thread>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <set>
#include <new>
#include <tuple>
#include <type_traits>
#include <vector>

#include "../../include/tmg.h"
#include "tmg_internal.h"
#include "tmg_tables.h"

using namespace tmg;

static_assert(TMG_NOALLOC_SCRATCH_BYTES == kNoAllocScratchBytes, "scratch size");
static_assert(TMG_NOALLOC_MAX_UNKNOWNS == kNoAllocMaxUnknowns, "no-alloc problem limit");
static_assert(TMG_MAX_DEGREE + 1 == kMaxP, "largest degree");
static_assert(TMG_MAX_TUNED_DEGREE + 1 == kMaxTunedP, "largest degree of the tuned kernels");

namespace {

// kDeep: streaming levels (level < lb_j); kDeepNext: the next level streams
// too (level + 1 < lb_j); kDeepLast: the next level is in the bottom kernel.
// kHasNext2: instances with two more levels (level-wise two-level pass).
// V-cycles group an instance's streaming levels g, g+1, ... (g = 1 or 2)
// into pairs run by two-level launches: kPair<g> marks the first level of a
// pair, kSingle<g> a last level left without a partner.
enum TileKind {
    kDeep = 0, kAll = 1, kHasNext = 2, kDeepNext = 3, kDeepLast = 4, kHasNext2 = 5,
    kPair1 = 6, kSingle1 = 7, kPair2 = 8, kSingle2 = 9,
    kWhole = 10   // level 0 of the instances the bottom kernel holds whole
};

struct TileList {
    int64_t ntiles = 0;
    int64_t *d_off = nullptr;  // [batch+1]
    int *d_inst = nullptr;     // [ntiles] instance of each tile (batch > 1): one load in
                               // place of a binary search over d_off per work-group
    std::vector<int64_t> h_off;       // full lists: d_off on the host
};

// Once most of a batch has finished, the work-groups of its finished
// instances (which leave at once, but still cost a launch slot and a few
// dependent loads each) dominate a cycle.  The later cycles of a solve then
// run on lists of the running instances' tiles only, built on the host from
// the run bits each cycle's summary carries, whenever the running share of
// level-0 tiles has dropped to kActiveShare of the lists in use.  A level-0
// pass reads the left halo of each tile from the slot the pass before
// stored under the tile's number in its list; the first cycle on a new
// generation re-fills those slots from the iterate under the new numbers
// (the values are the iterate's there, so the results do not change).
// The lists of one generation live in a device arena, sent there in one
// copy in stream order from a pinned staging buffer (two, used in turn by
// generations, so that the host never writes one a queued copy still
// reads).  They cover the tile lists the cycles after the first use
// (recorded as they are asked for) and the bottom kernel's instance lists;
// any other list is used in full.
constexpr double kActiveShare = 0.75;
constexpr int kActiveAhead = 2;   // cycles queued past the last summary
struct ActiveSet {
    bool enabled = true;
    bool on = false;                   // the cycles being queued use `lists`
    bool seed = false;                 // the next cycle re-fills the halo slots first
    std::vector<unsigned> run;         // run bits the lists are built for
    int64_t tiles = 0;                 // level-0 tiles of the lists in use
    std::map<std::tuple<int, int, int>, TileList> lists;
    std::vector<int *> bot;            // per level: running instances with lb == level
    std::vector<int> bot_n;
    int *bot_all = nullptr;            // running instances with lb >= 1
    int bot_all_n = 0;
    char *arena = nullptr;             // device
    char *stage[2] = {nullptr, nullptr};   // pinned host
    size_t cap = 0;
    int which = 0;
    hipEvent_t ev[2] = {nullptr, nullptr}; // after the last copy out of stage[k]
    bool is_run(int j) const { return (run[j >> 5] >> (j & 31)) & 1u; }
};

struct GraphKey {
    int kind, trans;
    const void *f, *u0, *u;
    bool operator<(const GraphKey &o) const
    {
        return std::tie(kind, trans, f, u0, u) < std::tie(o.kind, o.trans, o.f, o.u0, o.u);
    }
};

// graph kinds: the first cycle of a solve, and later cycles by halo parity
// kEvenOdd / kEvenOdd2: one / two pairs of an even and an odd cycle in one
// graph (each graph launch costs the GPU ~8 us between cycles)
enum { kFirst = 0, kEven = 1, kOdd = 2, kEvenOdd = 3, kEvenOdd2 = 4 };

// Level buffers of one precision: right-hand side and two iterates per level.
template <typename T>
struct LevelStore {
    std::vector<T *> f, xa, xb;
    T *x(int l, int which) const { return which ? xb[l] : xa[l]; }
};

}  // namespace

struct tmg_ctx {
    int batch = 0, P = 0, S = 0, Lmax = 0;
    // the generic kernels (one slab per thread, tables in LDS): P above the
    // tuned kernels' limit, or the periodic problem; level 0 then runs as a
    // down leg into x0 and an up leg from it, out of place
    bool generic = false;
    double *x0 = nullptr;
    tmg_options opt{};
    std::vector<int64_t> N;
    std::vector<double> T, lam;
    std::vector<int> L;                           // levels of each instance
    std::vector<int> lb;                          // first level of the bottom kernel
    std::vector<std::vector<int64_t>> slab_off_h; // [Lmax][batch+1]
    std::vector<int64_t *> slab_off_d;
    LevelStore<double> d;                         // FP64 hierarchy (plain method)
    LevelStore<float> s;                          // FP32 hierarchy (mixed precision)
    std::vector<int64_t> level_size;              // coefficients per level
    double *hb[2] = {nullptr, nullptr};           // level-0 halo buffers
    int64_t hb_last_off = 0;                      // slots of the one-level pass next to a two-level one
    double *f1b = nullptr;                        // second level-1 right-hand side (two-level passes)
    float *f1b32 = nullptr;                       // the same for the FP32-inner cycle
    int64_t hb_cap = 0;                           // doubles allocated per halo buffer
    bool pairs = true;                            // two-level launches in V-cycles (schedule)
    bool direct = false;                          // cycles after the first launched kernel by kernel
    int span = 0;                                 // >= 3: levels after the first pairs in spans of it
    int span_after = 2;                           // streaming levels before the spans
    int *lb_d = nullptr;                          // [batch] lb on the device (spans)
    double *tab_fwd = nullptr, *tab_adj = nullptr;
    double *R_fwd = nullptr, *R_adj = nullptr;
    float *tab32_fwd = nullptr, *tab32_adj = nullptr;  // the same tables rounded to FP32
    float *R32_fwd = nullptr, *R32_adj = nullptr;
    bool mixed = false;
    int tab_stride = 0;
    int *nlev_d = nullptr;
    std::vector<int *> bot_d;                     // per level: instances with lb == level
    std::vector<int> bot_n;
    int *bot_all_d = nullptr;                     // instances with lb >= 1 (one launch for all)
    int bot_all_n = 0;
    int bot_levels = 0;                           // levels >= 1 with bottom-kernel instances
    void **lvptr_d = nullptr;                     // per level: f, x (first buffer), slab offsets
    std::vector<int> deep_n;                      // per level: instances with level < lb
    int64_t bottom_cap = 0;
    ActiveSet act;
    std::set<std::tuple<int, int, int>> cycle_keys;   // tile lists of cycles after the first
    bool in_cycle = false;                            // enqueue_cycle of such a cycle
    InstState *st = nullptr, *st_ops = nullptr;
    InstState *st_host = nullptr;                 // pinned, batch states (results, op calls)
    Control *ctl = nullptr, *ctl_host = nullptr;  // device / pinned
    HostHead *mirror = nullptr, *mirror_d = nullptr;   // coherent pinned; host / device address
    unsigned *pubn_d = nullptr;                   // copies of a batch's states made (k_publish)
    // the kernels that finish a cycle write the host copy themselves for a
    // single instance; a batch is copied by k_publish after the cycle
    HostHead *mirror1() const { return batch == 1 ? mirror_d : nullptr; }
    int epoch = 0;                                // solves started
    hipEvent_t drain_ev = nullptr;                // recorded after the last launch of a solve
    bool drain_pending = false;
    double *partial = nullptr;
    int64_t partial_cap = 0;
    double *tau_d = nullptr, *grad_d = nullptr, *grad_host = nullptr;
    double *T_d = nullptr;                        // [batch] T_j and N_j: tables built on the
    int64_t *N_d = nullptr;                       // device (tmg_set_lambda)
    bool lam_device = false;                      // lambda last set from a device array
    // The bottom level's visits as one dense operator (one FP64 instance;
    // the gamma visits of a cycle's recursion): D of the bottom level
    // (dense_n unknowns) and its rows' windows, [0] forward and [1] the
    // transposed system's, each valid for the current schedule and tables
    // while dense_ok[.].
    bool dense_on = true;
    bool dense_ok[2] = {false, false};
    int dense_level = -1;
    int64_t dense_n = 0, dense_cap[2] = {0, 0};
    double *dense[2] = {nullptr, nullptr};
    int *dense_win[2] = {nullptr, nullptr};
    bool dense_nomem = false;   // an operator's allocation failed (until the next plan)
    int64_t dense_w[2] = {0, 0};   // the widest span a product's work-group loads
    int *dense_wd = nullptr;       // device copy of the last one measured
    void dense_stale() { dense_ok[0] = dense_ok[1] = false; }
    std::map<std::tuple<int, int, int>, TileList> tiles;
    std::map<int, std::pair<int *, int>> op_coarse;
    std::map<GraphKey, hipGraphExec_t> graphs;
    std::vector<int> cur;                         // capture-time: which iterate buffer is current
    hipStream_t cap = nullptr;
    int last_hip = 0;
    std::vector<void *> allocs;
    // The entry point that allocates nothing (arena != null): every device
    // buffer is carved out of the library's static scratch array; no pinned
    // host memory, streams, events or graphs; the host follows the solve by
    // plain copies of the state into fx_st.
    char *arena = nullptr;
    size_t arena_cap = 0, arena_used = 0;
    InstState fx_st{};
    Control fx_ctl{};
    double fx_grad[2] = {0.0, 0.0};
    bool fixed() const { return arena != nullptr; }

    // halo (even and a multiple of S) and output slabs per tile of each pass
    int rs(int x) const
    {
        const int q = S < 2 ? 2 : S;
        return ((x + q - 1) / q) * q;
    }
    int H_down() const { return rs(opt.nu1 + 1); }
    int H_up() const { return rs(opt.nu1 + opt.nu2); }
    int H_fused() const { return rs(2 * opt.nu1 + opt.nu2 + 1); }
    // two-level launches of V-cycle first visits (levels l, l+1): the down
    // pair loses nu1 slabs at l and nu1 + 1 coarse ones at l+1 and restricts
    // level-(l+1) pairs (a multiple of 4); the up pair loses nu1 + nu2 - 1
    // coarse slabs at l+1, then nu2 at l
    int H_dpair() const
    {
        const int q = S < 4 ? 4 : S;
        return ((3 * opt.nu1 + 2 + q - 1) / q) * q;
    }
    int H_upair() const { return rs(2 * (opt.nu1 + opt.nu2) + opt.nu2); }
    // fused pass that also runs level 1's up leg and level 1's next down
    // leg: level 1's first nu1 + nu2 coarse slabs are wrong, 2 (nu1 + nu2)
    // fine slabs, then nu2 + nu1 + 1 at level 0 and 2 nu1 for level 1's
    // down leg; a multiple of 4 so that level-2 pairs stay inside a tile
    int H_fused2() const
    {
        const int q = S < 4 ? 4 : S;
        return ((3 * (opt.nu1 + opt.nu2) + 1 + 2 * opt.nu1 + q - 1) / q) * q;
    }
    // The W-cycle's fused launch at a level l >= 1: the up leg of a first
    // visit (nu1 + nu2 sweeps), the down leg of the next visit (nu1 sweeps,
    // the residual) and, with next2, level l+1's first down leg from zero
    // on the restricted residual (nu1 sweeps, the residual, restricted once
    // more).  Wrong slabs counted without the saving of a zero start; with
    // next2 in fine slabs, a multiple of 4 so that level-(l+2) pairs stay
    // inside a tile.
    int H_wfused(bool next2) const
    {
        const int w = 2 * opt.nu1 + opt.nu2 + 1;
        return next2 ? r4(2 * ((w + 1) / 2 + opt.nu1 + 1)) : rs(w);
    }
    // V-cycle solves in FP64 fuse level 1's legs into the level-0 pass
    bool fuse_up1() const { return opt.gamma == 1 && !mixed && pairs; }
    // the same for the FP32-inner defect correction
    bool fuse_mix() const { return opt.gamma == 1 && mixed && pairs; }
    // mixed precision, level 0: first down pass, fused pass, single cycle
    int H_mixd() const { return rs(opt.nu1 + 2); }
    int H_mix() const { return rs(2 * opt.nu1 + opt.nu2 + 3); }
    int H_mixv() const { return rs(opt.nu1 + opt.nu2 + 1); }
    // their two-level forms (level 1's inner legs in the tiles; multiples of 4)
    int r4(int x) const
    {
        const int q = S < 4 ? 4 : S;
        return ((x + q - 1) / q) * q;
    }
    int H_mixd2() const { return r4(opt.nu1 + 2 + 2 * opt.nu1); }
    int H_mix2() const { return r4(2 * opt.nu1 + opt.nu2 + 3 + 2 * (opt.nu1 + opt.nu2) + 2 * opt.nu1); }
    // slabs per tile of the streaming launches, and output slabs per tile
    int ts() const { return generic ? kGenThreads : tile_slabs(P); }
    int TO(int H) const { return ts() - H; }
    // generic level-0 up leg with the residual norm: one more slab of halo
    int H_gup0() const { return rs(opt.nu1 + opt.nu2 + 1); }
    // every bottom-kernel level fits one wavefront (one-wavefront work-groups)
    bool small_bottom() const { return bottom_cap <= 64 * bottom_slabs(P); }
    // largest bottom cap: the bottom kernel's level, or the generic kernels'
    // bottom visit
    int64_t max_cap() const
    {
        if (!generic) return bottom_max(P);
        return std::max<int64_t>(opt.n_coarse, gbottom_max(P));
    }
    // generic: the bottom spans several levels (k_gvisit)
    bool gvisit() const { return generic && bottom_cap > opt.n_coarse; }
    // the dense bottom operator applies: one instance in FP64 whose bottom
    // level lies strictly between level 0 and the coarsest (V or W; the
    // generic kernels' bottom visit too, the periodic problem's included)
    bool want_dense() const
    {
        if (!dense_on || batch != 1 || mixed || fixed() || lb.empty()) return false;
        const int l = lb[0];
        return l >= 1 && l < L[0] - 1 && (N[0] >> l) * P <= kDenseMaxN;
    }
    // spans of K levels (k_span, one top-level slab per thread): the down
    // legs lose nu1 + 1 slabs at the top level and, at each level below,
    // half the wrong slabs restricted from above plus nu1 + 1 (the last
    // restriction halves them once more); the up legs lose nu1 + nu2 at the
    // deepest level and twice the wrong slabs prolonged from below plus
    // nu1 + nu2 at each level above.  In top-level slabs, rounded up to a
    // multiple of 2^K so that no coarse slab straddles two tiles.
    int H_sdown(int K) const
    {
        int w = opt.nu1 + 1, h = w;
        for (int k = 1; k < K; ++k) {
            w = (w + 1) / 2 + opt.nu1 + 1;
            h = std::max(h, w << k);
        }
        h = std::max(h, ((w + 1) / 2) << K);
        return ((h + (1 << K) - 1) >> K) << K;
    }
    int H_sup(int K) const
    {
        int w = opt.nu1 + opt.nu2, h = w << (K - 1);
        for (int k = K - 2; k >= 0; --k) {
            w = 2 * w + opt.nu1 + opt.nu2;
            h = std::max(h, w << k);
        }
        return ((h + (1 << K) - 1) >> K) << K;
    }
    // spans of depth K fit a tile with room for output
    bool span_fits(int K) const
    {
        return K >= 3 && K <= kMaxSpan && H_sup(K) <= kSpanThreads - (1 << K) &&
               H_sdown(K) <= kSpanThreads - (1 << K);
    }
};

namespace {

#define HIPCHK(ctx, expr)                                                  \
    do {                                                                   \
        hipError_t e_ = (expr);                                            \
        if (e_ != hipSuccess) {                                            \
            (ctx)->last_hip = (int)e_;                                     \
            return e_ == hipErrorOutOfMemory ? TMG_ERR_OOM : TMG_ERR_HIP;  \
        }                                                                  \
    } while (0)

template <typename T>
int dalloc(tmg_ctx *c, T **p, size_t n)
{
    *p = nullptr;
    if (n == 0) n = 1;
    if (c->arena) {
        // bump allocation in the static scratch, 256-byte aligned
        const size_t bytes = (n * sizeof(T) + 255) & ~size_t(255);
        if (bytes > c->arena_cap - c->arena_used) return TMG_ERR_SIZE;
        *p = reinterpret_cast<T *>(c->arena + c->arena_used);
        c->arena_used += bytes;
        return TMG_OK;
    }
    hipError_t e = hipMalloc((void **)p, n * sizeof(T));
    if (e != hipSuccess) {
        c->last_hip = (int)e;
        return TMG_ERR_OOM;
    }
    c->allocs.push_back(*p);
    return TMG_OK;
}

// Free one allocation made by dalloc (null: nothing).
void dfree(tmg_ctx *c, void *p)
{
    if (!p || c->arena) return;   // the scratch is reclaimed as a whole after the call
    for (size_t i = 0; i < c->allocs.size(); ++i)
        if (c->allocs[i] == p) {
            c->allocs[i] = c->allocs.back();
            c->allocs.pop_back();
            break;
        }
    (void)hipFree(p);
}

bool participates(const tmg_ctx *c, int j, int level, int kind)
{
    if (level >= c->L[j]) return false;
    if (kind == kWhole) return level == 0 && c->lb[j] == 0;
    if (kind == kDeep) return level < c->lb[j];       // streaming kernels in the cycle
    if (kind == kHasNext) return level + 1 < c->L[j]; // level-wise entry points
    if (kind == kHasNext2) return level + 2 < c->L[j];
    if (kind >= kPair1) {
        const int g = kind <= kSingle1 ? 1 : 2;
        if (level < g || ((level - g) & 1)) return false;
        return (kind == kPair1 || kind == kPair2) ? level + 1 < c->lb[j] : level + 1 == c->lb[j];
    }
    if (kind == kDeepNext) return level + 1 < c->lb[j];
    if (kind == kDeepLast) return level < c->lb[j] && level + 1 >= c->lb[j];
    return true;
}

// Tile offsets (prefix sums of ceil(N_jl / tile_out) over participating
// instances) for one (level, kind, tile_out), cached on the device.
TileList *active_tiles(tmg_ctx *c, TileList &full, const std::tuple<int, int, int> &key);

int get_tiles(tmg_ctx *c, int level, int kind, int tile_out, hipStream_t s, TileList **out)
{
    auto key = std::make_tuple(level, kind, tile_out);
    if (c->in_cycle) c->cycle_keys.insert(key);
    auto it = c->tiles.find(key);
    if (it != c->tiles.end()) {
        *out = c->act.on ? active_tiles(c, it->second, key) : &it->second;
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
    std::vector<int> inst;
    if (c->batch > 1 && tl.ntiles > 0) {
        inst.resize(tl.ntiles);
        for (int j = 0; j < c->batch; ++j)
            for (int64_t t = off[j]; t < off[j + 1]; ++t) inst[t] = j;
        if ((rc = dalloc(c, &tl.d_inst, inst.size()))) return rc;
        HIPCHK(c, hipMemcpyAsync(tl.d_inst, inst.data(), inst.size() * sizeof(int),
                                 hipMemcpyHostToDevice, s));
    }
    HIPCHK(c, hipStreamSynchronize(s));
    tl.h_off = std::move(off);
    auto res = c->tiles.emplace(key, std::move(tl));
    *out = c->act.on ? active_tiles(c, res.first->second, key) : &res.first->second;
    return TMG_OK;
}

size_t a256(size_t n) { return (n + 255) & ~size_t(255); }

// The active-set form of a full tile list (the full list itself if the
// generation has none for it: its finished instances leave at once).
TileList *active_tiles(tmg_ctx *c, TileList &full, const std::tuple<int, int, int> &key)
{
    auto it = c->act.lists.find(key);
    return it != c->act.lists.end() ? &it->second : &full;
}

// The bottom kernel's instance list of a level (active-set form while one
// is in use).
void bottom_list(const tmg_ctx *c, int level, const int **inst, int *n)
{
    const ActiveSet &A = c->act;
    const bool act = A.on && level < (int)A.bot_n.size();
    *inst = act ? A.bot[level] : c->bot_d[level];
    *n = act ? A.bot_n[level] : c->bot_n[level];
}

// Starts a generation of active-set lists for the run bits `run` (level-0
// tiles `tiles`): every tile list the cycles of a solve use and the bottom
// kernel's lists, built on the host and sent to the device in one copy
// (each copy costs the stream a switch between engines).
int act_begin(tmg_ctx *c, std::vector<unsigned> &run, int64_t tiles, hipStream_t s)
{
    ActiveSet &A = c->act;
    const int B = c->batch;
    A.run.swap(run);
    std::vector<int> bl;
    std::vector<int> bcount(c->Lmax, 0);
    for (int j = 0; j < B; ++j)
        if (A.is_run(j) && c->lb[j] < c->Lmax) bcount[c->lb[j]]++;
    size_t need = 0;
    for (int l = 0; l < c->Lmax; ++l) need += a256(sizeof(int) * bcount[l]);
    int nall = 0;
    for (int l = 1; l < c->Lmax; ++l) nall += bcount[l];
    need += a256(sizeof(int) * nall);
    std::vector<std::pair<const std::tuple<int, int, int> *, const TileList *>> keys;
    std::vector<int64_t> nrun;
    for (const auto &k : c->cycle_keys) {
        auto it = c->tiles.find(k);
        if (it == c->tiles.end()) continue;
        const std::vector<int64_t> &fo = it->second.h_off;
        int64_t n = 0;
        for (int j = 0; j < B; ++j)
            if (A.is_run(j)) n += fo[j + 1] - fo[j];
        keys.emplace_back(&k, &it->second);
        nrun.push_back(n);
        need += a256(sizeof(int64_t) * (B + 1)) + a256(sizeof(int) * n);
    }
    if (need > A.cap) {
        // nothing queued may still read the arena or a staging buffer
        HIPCHK(c, hipStreamSynchronize(s));
        dfree(c, A.arena);
        A.arena = nullptr;
        for (int k = 0; k < 2; ++k) {
            if (A.stage[k]) (void)hipHostFree(A.stage[k]);
            A.stage[k] = nullptr;
        }
        A.cap = 0;
        const size_t cap = need + need / 2;
        int rc = dalloc(c, &A.arena, cap);
        if (rc) return rc;
        for (int k = 0; k < 2; ++k)
            HIPCHK(c, hipHostMalloc((void **)&A.stage[k], cap, hipHostMallocDefault));
        A.cap = cap;
    }
    for (int k = 0; k < 2; ++k)
        if (!A.ev[k]) HIPCHK(c, hipEventCreateWithFlags(&A.ev[k], hipEventDisableTiming));
    A.which ^= 1;
    // the copy of the generation before last read this staging buffer
    HIPCHK(c, hipEventSynchronize(A.ev[A.which]));
    char *const h = A.stage[A.which];
    size_t used = 0;
    A.lists.clear();
    for (size_t q = 0; q < keys.size(); ++q) {
        const std::vector<int64_t> &fo = keys[q].second->h_off;
        int64_t *off = reinterpret_cast<int64_t *>(h + used);
        const size_t bo = a256(sizeof(int64_t) * (B + 1));
        int *inst = reinterpret_cast<int *>(h + used + bo);
        off[0] = 0;
        for (int j = 0; j < B; ++j) {
            const int64_t m = A.is_run(j) ? fo[j + 1] - fo[j] : 0;
            std::fill(inst + off[j], inst + off[j] + m, j);
            off[j + 1] = off[j] + m;
        }
        TileList tl;
        tl.ntiles = nrun[q];
        tl.d_off = reinterpret_cast<int64_t *>(A.arena + used);
        tl.d_inst = reinterpret_cast<int *>(A.arena + used + bo);
        A.lists.emplace(*keys[q].first, std::move(tl));
        used += bo + a256(sizeof(int) * nrun[q]);
    }
    A.bot.assign(c->Lmax, nullptr);
    A.bot_n.assign(c->Lmax, 0);
    for (int l = 0; l < c->Lmax; ++l) {
        if (bcount[l] == 0) continue;
        int *b = reinterpret_cast<int *>(h + used);
        int n = 0;
        for (int j = 0; j < B; ++j)
            if (c->lb[j] == l && A.is_run(j)) b[n++] = j;
        A.bot[l] = reinterpret_cast<int *>(A.arena + used);
        A.bot_n[l] = n;
        used += a256(sizeof(int) * n);
    }
    {
        int *b = reinterpret_cast<int *>(h + used);
        int n = 0;
        for (int j = 0; j < B; ++j)
            if (c->lb[j] >= 1 && A.is_run(j)) b[n++] = j;
        A.bot_all = reinterpret_cast<int *>(A.arena + used);
        A.bot_all_n = n;
        used += a256(sizeof(int) * n);
    }
    if (used > 0) {
        HIPCHK(c, hipMemcpyAsync(A.arena, h, used, hipMemcpyHostToDevice, s));
        HIPCHK(c, hipEventRecord(A.ev[A.which], s));
    }
    A.tiles = tiles;
    A.on = true;
    A.seed = true;
    return TMG_OK;
}

int64_t tiles_of(const tmg_ctx *c, int level, int kind, int tile_out)
{
    int64_t n = 0;
    for (int j = 0; j < c->batch; ++j)
        if (participates(c, j, level, kind)) n += ((c->N[j] >> level) + tile_out - 1) / tile_out;
    return n;
}

const double *tab_of(const tmg_ctx *c, int level, bool trans)
{
    return (trans ? c->tab_adj : c->tab_fwd) + (int64_t)level * c->batch * c->tab_stride;
}

template <typename T> LevelStore<T> &store(tmg_ctx *c);
template <> LevelStore<double> &store<double>(tmg_ctx *c) { return c->d; }
template <> LevelStore<float> &store<float>(tmg_ctx *c) { return c->s; }

template <typename T> const T *tabT_of(const tmg_ctx *c, int level, bool trans);
template <> const double *tabT_of<double>(const tmg_ctx *c, int level, bool trans)
{
    return tab_of(c, level, trans);
}
template <> const float *tabT_of<float>(const tmg_ctx *c, int level, bool trans)
{
    return (trans ? c->tab32_adj : c->tab32_fwd) + (int64_t)level * c->batch * c->tab_stride;
}
template <typename T> const T *R_of(const tmg_ctx *c, bool trans);
template <> const double *R_of<double>(const tmg_ctx *c, bool trans) { return trans ? c->R_adj : c->R_fwd; }
template <> const float *R_of<float>(const tmg_ctx *c, bool trans) { return trans ? c->R32_adj : c->R32_fwd; }

template <typename T = double>
LegArgsT<T> leg_args(const tmg_ctx *c, int level, bool trans, const TileList *tl, int H)
{
    LegArgsT<T> a{};
    a.tab = tab_of(c, level, trans);
    a.tabT = tabT_of<T>(c, level, trans);
    a.R = R_of<T>(c, trans);
    a.slab_off = c->slab_off_d[level];
    a.cslab_off = level + 1 < c->Lmax ? c->slab_off_d[level + 1] : nullptr;
    a.tile_off = tl->d_off;
    a.tile_inst = tl->d_inst;
    a.n0 = c->N[0] >> level;
    a.batch = c->batch;
    a.generic = c->generic;
    a.periodic = c->opt.periodic;
    a.tab_stride = c->tab_stride;
    a.halo = H;
    a.tile_out = c->TO(H);
    a.touch = level > 0;
    return a;
}

// ---- one cycle ----------------------------------------------------------

struct CycleIO {
    const double *f, *u0;
    double *u;
    bool trans, use_state;
    int kind;      // kFirst / kEven / kOdd (solve); -1: a single warm-started cycle
};

// The initial value enters slab 0 of the forward initial-value problem only
// (the drivers hand periodic problems no u0).
const double *fold_of(const CycleIO &io) { return io.trans ? nullptr : io.u0; }

// A solve's first level-0 down pass also yields the initial residual's norm
// (r_0 = f with u0 folded, u = 0): each launch leaves its tiles' partials,
// and a finalize launch right after it sets its instances' initial state.
// The first finalize of a solve also installs the solve's control block.
struct R0 {
    bool ctl_pending = true;
};

int finalize_r0(tmg_ctx *c, R0 *r0, const TileList *tl, hipStream_t s)
{
    HIPCHK(c, launch_finalize(c->partial, tl->d_off, c->batch, c->st, c->ctl, c->mirror1(), 1, s,
                              r0->ctl_pending ? c->ctl : nullptr,
                              r0->ctl_pending ? c->ctl_host : nullptr));
    r0->ctl_pending = false;
    return TMG_OK;
}

// Bottom kernel for the instances whose bottom part starts at `level`
// (level 0: the caller's FP64 arrays; otherwise the level buffers of T).
template <typename T>
int enqueue_bottom(tmg_ctx *c, const CycleIO &io, int level, const T *x_in, T *x_out,
                   hipStream_t s)
{
    const int *inst;
    int ninst;
    bottom_list(c, level, &inst, &ninst);
    if (ninst == 0) return TMG_OK;
    if constexpr (std::is_same<T, double>::value) {
        // a V-cycle's visit from zero: one product with the dense operator
        const int d = io.trans ? 1 : 0;
        if (c->dense_ok[d] && c->opt.gamma == 1 && !x_in && level == c->dense_level) {
            HIPCHK(c, launch_dense_apply(c->dense[d], c->dense_win[d], store<T>(c).f[level], x_out,
                                         c->dense_n, io.use_state ? c->st : nullptr, s,
                                         c->dense_w[d]));
            return TMG_OK;
        }
    }
    BottomArgsT<T> a{};
    a.f = level == 0 ? reinterpret_cast<const T *>(io.f) : store<T>(c).f[level];
    a.u0 = level == 0 ? fold_of(io) : nullptr;
    a.x_in = x_in;
    a.x_out = x_out;
    a.slab_off = c->slab_off_d[level];
    a.tab = io.trans ? c->tab_adj : c->tab_fwd;
    a.R = io.trans ? c->R_adj : c->R_fwd;
    a.inst = inst;
    a.nlev = c->nlev_d;
    a.st = io.use_state ? c->st : nullptr;
    a.ctl = c->ctl;
    a.mirror = io.use_state ? c->mirror1() : nullptr;
    a.level = level;
    a.batch = c->batch;
    a.tab_stride = c->tab_stride;
    a.nu1 = c->opt.nu1;
    a.nu2 = c->opt.nu2;
    a.gamma = c->opt.gamma;
    a.small = c->small_bottom();
    a.generic = c->generic;
    a.periodic = c->opt.periodic;
    a.visit = c->gvisit();
    HIPCHK(c, launch_bottom<T>(c->P, io.trans, a, ninst, s));
    return TMG_OK;
}

// The bottom kernel for every instance with lb >= 1 in one launch, each at
// its own first bottom level (a V-cycle's first visits, after all down legs
// and before all up legs): the same work as one launch per level.
template <typename T>
int enqueue_bottom_all(tmg_ctx *c, const CycleIO &io, hipStream_t s)
{
    const ActiveSet &A = c->act;
    const int *inst = A.on ? A.bot_all : c->bot_all_d;
    const int n = A.on ? A.bot_all_n : c->bot_all_n;
    if (n == 0) return TMG_OK;
    const int Lm = c->Lmax;
    BottomArgsT<T> a{};
    a.tab = io.trans ? c->tab_adj : c->tab_fwd;
    a.R = io.trans ? c->R_adj : c->R_fwd;
    a.inst = inst;
    a.nlev = c->nlev_d;
    a.st = io.use_state ? c->st : nullptr;
    a.ctl = c->ctl;
    a.mirror = io.use_state ? c->mirror1() : nullptr;
    a.batch = c->batch;
    a.tab_stride = c->tab_stride;
    a.nu1 = c->opt.nu1;
    a.nu2 = c->opt.nu2;
    a.gamma = c->opt.gamma;
    a.lbs = c->lb_d;
    a.f_lv = reinterpret_cast<const T *const *>(c->lvptr_d);
    a.x_lv = reinterpret_cast<T *const *>(c->lvptr_d + Lm);
    a.soff_lv = reinterpret_cast<const int64_t *const *>(c->lvptr_d + 2 * Lm);
    a.small = c->small_bottom();
    a.generic = c->generic;
    a.periodic = c->opt.periodic;
    a.visit = c->gvisit();
    HIPCHK(c, launch_bottom<T>(c->P, io.trans, a, n, s));
    return TMG_OK;
}

// Down leg (streaming instances): nu1 sweeps from the current iterate (zero
// on a first visit), residual, restriction into the next level.
template <typename T>
int enqueue_down(tmg_ctx *c, const CycleIO &io, int level, bool zero, hipStream_t s,
                 int kind = kDeep, R0 *r0 = nullptr)
{
    TileList *tl;
    const int H = c->H_down();
    int rc = get_tiles(c, level, kind, c->TO(H), s, &tl);
    if (rc) return rc;
    if (tl->ntiles == 0) return TMG_OK;
    LevelStore<T> &L = store<T>(c);
    LegArgsT<T> a = leg_args<T>(c, level, io.trans, tl, H);
    a.f = level == 0 ? reinterpret_cast<const T *>(io.f) : L.f[level];
    a.u0 = level == 0 ? fold_of(io) : nullptr;
    a.u_in = zero ? nullptr : (level == 0 ? reinterpret_cast<const T *>(io.u) : L.x(level, c->cur[level]));
    a.rc = L.f[level + 1];
    a.st = io.use_state ? c->st : nullptr;
    a.pre = c->opt.nu1;
    if (r0) {
        a.st = nullptr;   // the state is set after this launch
        a.norm_f = 1;
        a.partial = c->partial;
        a.norm_off = tl->d_off;
    }
    HIPCHK(c, launch_leg<T>(c->P, io.trans, a, tl->ntiles, s));
    return r0 ? finalize_r0(c, r0, tl, s) : TMG_OK;
}

// Up leg at `level` >= 1: the pre-smoothing recomputed from the visit's
// initial iterate, correction with the next level's result, nu2 sweeps.
// A first visit writes the current buffer (nothing is read from it); a
// repeated visit (W-cycle) writes the other one and makes it current.
template <typename T>
int enqueue_up(tmg_ctx *c, const CycleIO &io, int level, bool zero, hipStream_t s,
               int kind = kDeep)
{
    TileList *tl;
    const int H = c->H_up();
    int rc = get_tiles(c, level, kind, c->TO(H), s, &tl);
    if (rc) return rc;
    if (tl->ntiles == 0) return TMG_OK;
    LevelStore<T> &L = store<T>(c);
    LegArgsT<T> a = leg_args<T>(c, level, io.trans, tl, H);
    const int cur = c->cur[level];
    a.f = L.f[level];
    a.u_in = zero ? nullptr : L.x(level, cur);
    a.e = L.x(level + 1, c->cur[level + 1]);
    a.u_out = zero ? L.x(level, cur) : L.x(level, cur ^ 1);
    a.st = io.use_state ? c->st : nullptr;
    a.pre = c->opt.nu1;
    a.post = c->opt.nu2;
    HIPCHK(c, launch_leg<T>(c->P, io.trans, a, tl->ntiles, s));
    if (!zero) c->cur[level] ^= 1;
    return TMG_OK;
}

template <typename T>
int enqueue_coarse_visits(tmg_ctx *c, const CycleIO &io, int l, hipStream_t s, bool skip_up = false);

// A W-cycle's two visits of a level that one instance streams (below).
template <typename T>
int enqueue_w_visits(tmg_ctx *c, const CycleIO &io, int l, bool ready, hipStream_t s);

// skip_up: the up leg of this level runs inside the level-0 pass instead
template <typename T>
int enqueue_visit(tmg_ctx *c, const CycleIO &io, int level, bool zero, hipStream_t s,
                  bool skip_up = false)
{
    int rc = enqueue_down<T>(c, io, level, zero, s);
    if (rc) return rc;
    if ((rc = enqueue_coarse_visits<T>(c, io, level + 1, s))) return rc;
    return skip_up ? TMG_OK : enqueue_up<T>(c, io, level, zero, s);
}

// gamma visits of level l >= 1 from zero: bottom-kernel instances and,
// recursively, the streaming ones.  (When l is an instance's coarsest
// level its visit is the exact solve; repeating it changes nothing.)
template <typename T>
int enqueue_coarse_visits(tmg_ctx *c, const CycleIO &io, int l, hipStream_t s, bool skip_up)
{
    int rc;
    LevelStore<T> &L = store<T>(c);
    c->cur[l] = 0;
    if constexpr (std::is_same<T, double>::value) {
        // the instance's gamma bottom visits from zero in one product
        const int d = io.trans ? 1 : 0;
        if (c->dense_ok[d] && l == c->dense_level) {
            HIPCHK(c, launch_dense_apply(c->dense[d], c->dense_win[d], L.f[l], L.x(l, 0), c->dense_n,
                                         io.use_state ? c->st : nullptr, s, c->dense_w[d]));
            return TMG_OK;
        }
        // one instance's streaming levels of a W-cycle in fused launches
        if (c->opt.gamma == 2 && c->batch == 1 && c->pairs && !c->generic && !skip_up &&
            l < c->lb[0])
            return enqueue_w_visits<T>(c, io, l, false, s);
    }
    for (int g = 0; g < c->opt.gamma; ++g) {
        const int cur = c->cur[l];
        // bottom instances: a first visit starts from zero in place, a repeated
        // one reads the current buffer and writes the other (like enqueue_up)
        if ((rc = enqueue_bottom<T>(c, io, l, g == 0 ? nullptr : L.x(l, cur),
                                    g == 0 ? L.x(l, cur) : L.x(l, cur ^ 1), s)))
            return rc;
        if (c->deep_n[l] > 0) {
            if ((rc = enqueue_visit<T>(c, io, l, g == 0, s, skip_up))) return rc;
        } else if (g > 0) {
            c->cur[l] ^= 1;
        }
    }
    return TMG_OK;
}

// Two-level launches of a V-cycle (first visits from zero) at levels l, l+1.
// The down or up legs of levels level .. level+K-1 in one launch (k_span),
// for every instance that streams `level` (each stops at its bottom level).
template <typename T>
int enqueue_span(tmg_ctx *c, const CycleIO &io, int level, int K, bool down, hipStream_t s)
{
    TileList *tl;
    const int H = down ? c->H_sdown(K) : c->H_sup(K);
    int rc = get_tiles(c, level, kDeep, kSpanThreads - H, s, &tl);
    if (rc) return rc;
    if (tl->ntiles == 0) return TMG_OK;
    LevelStore<T> &L = store<T>(c);
    SpanArgsT<T> a{};
    for (int k = 0; k <= K && level + k < c->Lmax; ++k) {
        a.f[k] = L.f[level + k];
        a.x[k] = L.x(level + k, 0);
        a.slab_off[k] = c->slab_off_d[level + k];
    }
    a.tab = tab_of(c, level, io.trans);
    a.tabT = tabT_of<T>(c, level, io.trans);
    a.tab_level = (int64_t)c->batch * c->tab_stride;
    a.R = R_of<T>(c, io.trans);
    a.tile_off = tl->d_off;
    a.tile_inst = tl->d_inst;
    a.st = io.use_state ? c->st : nullptr;
    a.lb = c->lb_d;
    a.n0 = c->N[0] >> level;
    a.batch = c->batch;
    a.tab_stride = c->tab_stride;
    a.level = level;
    a.K = K;
    a.halo = H;
    a.tile_out = kSpanThreads - H;
    a.nu1 = c->opt.nu1;
    a.nu2 = c->opt.nu2;
    a.up = down ? 0 : 1;
    HIPCHK(c, launch_span<T>(c->P, io.trans, a, tl->ntiles, s));
    return TMG_OK;
}

template <typename T>
int enqueue_pair(tmg_ctx *c, const CycleIO &io, int level, bool down, int kind, hipStream_t s,
                 R0 *r0 = nullptr)
{
    TileList *tl;
    const int H = down ? c->H_dpair() : c->H_upair();
    int rc = get_tiles(c, level, kind, c->TO(H), s, &tl);
    if (rc) return rc;
    if (tl->ntiles == 0) return TMG_OK;
    LevelStore<T> &L = store<T>(c);
    LegArgsT<T> a = leg_args<T>(c, level, io.trans, tl, H);
    a.f = level == 0 ? reinterpret_cast<const T *>(io.f) : L.f[level];
    a.u0 = level == 0 ? fold_of(io) : nullptr;
    a.tab1 = tab_of(c, level + 1, io.trans);
    a.tab1T = tabT_of<T>(c, level + 1, io.trans);
    a.c2slab_off = c->slab_off_d[level + 2];
    a.st = io.use_state ? c->st : nullptr;
    a.pre = c->opt.nu1;
    if (down) {
        a.rc = L.f[level + 1];
        a.f2 = L.f[level + 2];
    } else {
        a.f1 = L.f[level + 1];
        a.e2 = L.x(level + 2, 0);
        a.u_out = L.x(level, 0);
        a.post = c->opt.nu2;
    }
    if (r0) {
        a.st = nullptr;   // the state is set after this launch
        a.norm_f = 1;
        a.partial = c->partial;
        a.norm_off = tl->d_off;
    }
    HIPCHK(c, launch_leg<T>(c->P, io.trans, a, tl->ntiles, s));
    return r0 ? finalize_r0(c, r0, tl, s) : TMG_OK;
}

// The W-cycle's launch between a level's two visits (one instance, l >= 1):
// the up leg of the first visit (from zero) and the down leg of the second
// from its result, restricted into level l+1, and with next2 level l+1's
// first down leg from zero on it, restricted into level l+2.
template <typename T>
int enqueue_w_fused(tmg_ctx *c, const CycleIO &io, int l, bool next2, hipStream_t s)
{
    TileList *tl;
    const int H = c->H_wfused(next2);
    int rc = get_tiles(c, l, next2 ? kDeepNext : kDeep, c->TO(H), s, &tl);
    if (rc) return rc;
    if (tl->ntiles == 0) return TMG_OK;
    LevelStore<T> &L = store<T>(c);
    LegArgsT<T> a = leg_args<T>(c, l, io.trans, tl, H);
    a.f = L.f[l];
    a.e = L.x(l + 1, c->cur[l + 1]);
    a.u_out = L.x(l, c->cur[l]);
    a.rc = L.f[l + 1];
    a.st = io.use_state ? c->st : nullptr;
    a.pre = c->opt.nu1;
    a.post = c->opt.nu2;
    a.next = c->opt.nu1;
    if (next2) {
        a.tab1 = tab_of(c, l + 1, io.trans);
        a.tab1T = tabT_of<T>(c, l + 1, io.trans);
        a.c2slab_off = c->slab_off_d[l + 2];
        a.f2 = L.f[l + 2];
    }
    HIPCHK(c, launch_leg<T>(c->P, io.trans, a, tl->ntiles, s));
    return TMG_OK;
}

// A W-cycle's two visits of a level l >= 1 that one instance streams: each
// visit is down(l), the visits of l+1, up(l), launched as
//   [down(l) + first down(l+1)] ... [up(l) + down(l) + first down(l+1)] ... [up(l)]
// where the first down leg of l+1 (from zero) joins the launch before it
// when l+1 streams too.  `ready`: this level's first down leg ran in the
// caller's launch (which then did not run level l+1's, so the first visit
// of l+1 starts with its own launch).  Every kernel computes what the
// one-level legs compute, in the same order, so the iterates are the same
// to the last bit.
template <typename T>
int enqueue_w_visits(tmg_ctx *c, const CycleIO &io, int l, bool ready, hipStream_t s)
{
    const bool next2 = l + 1 < c->lb[0];
    int rc;
    c->cur[l] = 0;
    if (!ready && (rc = next2 ? enqueue_pair<T>(c, io, l, true, kDeepNext, s)
                              : enqueue_down<T>(c, io, l, true, s)))
        return rc;
    for (int g = 0; g < 2; ++g) {
        // level l+1's first down leg ran in this call's last launch unless
        // that launch was the caller's
        const bool next_ready = g == 1 || !ready;
        if ((rc = next2 ? enqueue_w_visits<T>(c, io, l + 1, next_ready, s)
                        : enqueue_coarse_visits<T>(c, io, l + 1, s, false)))
            return rc;
        if (g == 0 && (rc = enqueue_w_fused<T>(c, io, l, next2, s))) return rc;
    }
    return enqueue_up<T>(c, io, l, false, s);
}


// First level run in spans: after the first span_after streaming levels
// (spans pay only where a launch is latency-bound; the larger levels stay
// in two-level launches, an odd one out in a one-level launch), or none
// (Lmax).
int span_start(const tmg_ctx *c, int first)
{
    return c->pairs && c->span_fits(c->span) ? first + c->span_after : c->Lmax;
}

// Levels >= 1 of a V-cycle (every visit a first visit from zero): all down
// legs from the top, the bottom kernels, all up legs from the bottom, with
// consecutive streaming levels paired into two-level launches (or, with a
// span schedule, the levels after the first pair in spans).  Down and up
// legs start at level down_first / up_first (2 when level 1's legs run
// inside the level-0 pass).
template <typename T>
int enqueue_vcycle_levels(tmg_ctx *c, const CycleIO &io, int down_first, int up_first,
                          hipStream_t s)
{
    int rc;
    LevelStore<T> &L = store<T>(c);
    c->cur.assign(c->Lmax + 1, 0);
    const int dp = down_first == 1 ? kPair1 : kPair2, ds = down_first == 1 ? kSingle1 : kSingle2;
    const int sd = std::min(span_start(c, down_first), c->Lmax);
    if (!c->pairs) {
        for (int l = down_first; l < sd; ++l)
            if ((rc = enqueue_down<T>(c, io, l, true, s))) return rc;
    } else {
        for (int l = down_first; l < sd; l += 2) {
            if (l + 1 == sd) {
                // a lone level before the spans: one leg for every instance
                if ((rc = enqueue_down<T>(c, io, l, true, s))) return rc;
                break;
            }
            if ((rc = enqueue_pair<T>(c, io, l, true, dp, s)) ||
                (rc = enqueue_down<T>(c, io, l, true, s, ds)))
                return rc;
        }
    }
    for (int l = sd; l < c->Lmax; l += c->span)
        if ((rc = enqueue_span<T>(c, io, l, c->span, true, s))) return rc;
    if (c->bot_levels >= 2) {
        if ((rc = enqueue_bottom_all<T>(c, io, s))) return rc;
    } else {
        for (int l = 1; l < c->Lmax; ++l)
            if ((rc = enqueue_bottom<T>(c, io, l, nullptr, L.x(l, 0), s))) return rc;
    }
    if (sd < c->Lmax)
        for (int l = sd + (c->Lmax - 1 - sd) / c->span * c->span; l >= sd; l -= c->span)
            if ((rc = enqueue_span<T>(c, io, l, c->span, false, s))) return rc;
    const int su = std::min(span_start(c, up_first), c->Lmax);
    const int kp = up_first == 1 ? kPair1 : kPair2, ks = up_first == 1 ? kSingle1 : kSingle2;
    if (!c->pairs) {
        for (int l = su - 1; l >= up_first; --l)
            if ((rc = enqueue_up<T>(c, io, l, true, s))) return rc;
        return TMG_OK;
    }
    int top = su - 1;   // the highest level below the spans
    if (su < c->Lmax && ((su - up_first) & 1)) {
        if ((rc = enqueue_up<T>(c, io, top, true, s))) return rc;
        --top;
    }
    for (int l = top; l >= up_first; --l) {
        if ((rc = enqueue_pair<T>(c, io, l, false, kp, s)) ||
            (rc = enqueue_up<T>(c, io, l, true, s, ks)))
            return rc;
    }
    return TMG_OK;
}

// The level-0 halo slots the passes of this cycle read, re-filled from the
// iterate for the tile lists in use (first cycle on an active-set
// generation).
int seed_halos(tmg_ctx *c, const CycleIO &io, hipStream_t s)
{
    const bool fuse = c->mixed ? c->fuse_mix() && c->deep_n[1] > 0
                               : c->fuse_up1() && c->deep_n[1] > 0;
    for (int pass = fuse ? 0 : 1; pass < 2; ++pass) {
        const bool two = pass == 0;
        const int H = c->mixed ? (two ? c->H_mix2() : c->H_mix())
                               : (two ? c->H_fused2() : c->H_fused());
        TileList *tl;
        int rc = get_tiles(c, 0, fuse ? (two ? kDeepNext : kDeepLast) : kDeep, c->TO(H), s, &tl);
        if (rc) return rc;
        const int64_t hoff = fuse && !two ? c->hb_last_off : 0;
        double *hb = (io.kind == kOdd ? c->hb[1] : c->hb[0]) + hoff;
        HIPCHK(c, launch_seed(c->P, io.trans, io.u, hb, tl->d_off, tl->d_inst, c->slab_off_d[0],
                              c->batch, c->N[0], c->TO(H), H, tl->ntiles, s));
    }
    return TMG_OK;
}

// Level-0 part of a cycle of the FP32-inner defect correction (streaming
// instances): see k_mix.  With r0: only the solve's first level-0 down pass
// (with the initial residual's norm); a solve's first cycle leaves that
// pass out.
int enqueue_mixed_level0(tmg_ctx *c, const CycleIO &io, hipStream_t s, R0 *r0 = nullptr)
{
    int rc;
    TileList *tl;
    const bool solve = io.kind >= 0, first = io.kind == kFirst;
    auto margs = [&](int H, TileList *t) {
        MixArgs a{};
        a.f = io.f;
        a.u0 = fold_of(io);
        a.tab = tab_of(c, 0, io.trans);
        a.tab32 = tabT_of<float>(c, 0, io.trans);
        a.R32 = R_of<float>(c, io.trans);
        a.slab_off = c->slab_off_d[0];
        a.cslab_off = c->slab_off_d[1];
        a.tile_off = t->d_off;
        a.tile_inst = t->d_inst;
        a.st = io.use_state ? c->st : nullptr;
        a.n0 = c->N[0];
        a.batch = c->batch;
        a.tab_stride = c->tab_stride;
        a.halo = H;
        a.tile_out = c->TO(H);
        a.pre = c->opt.nu1;
        a.post = c->opt.nu2;
        a.next = c->opt.nu1;
        return a;
    };
    if (!solve) {
        // warm start: seed the halo buffer from the caller's iterate
        const int H = c->H_mixv();
        if ((rc = get_tiles(c, 0, kDeep, c->TO(H), s, &tl))) return rc;
        LegArgs a = leg_args(c, 0, io.trans, tl, H);
        a.f = io.f;
        a.u_in = io.u;
        a.halo_out = c->hb[0];
        HIPCHK(c, launch_leg<double>(c->P, io.trans, a, tl->ntiles, s));
    }
    // two-level passes (as in the FP64 cycle): instances whose level 1
    // streams run level 1's inner legs inside their level-0 passes, with
    // level 1's right-hand side alternating between two buffers
    const bool fuse = solve && c->fuse_mix() && c->deep_n[1] > 0;
    float *f1_in = io.kind == kEven ? c->f1b32 : c->s.f[1];
    float *f1_out = io.kind == kEven ? c->s.f[1] : c->f1b32;
    auto two_level = [&](MixArgs &a) {
        a.tab1 = tab_of(c, 1, io.trans);
        a.tab1_32 = tabT_of<float>(c, 1, io.trans);
        a.c2slab_off = c->slab_off_d[2];
    };
    if (r0 || !solve) {
        // first inner down leg: residual of the iterate, FP32 sweeps, restriction
        for (int pass = fuse ? 0 : 1; pass < 2; ++pass) {
            const bool two = pass == 0;
            const int H = two ? c->H_mixd2() : c->H_mixd();
            if ((rc = get_tiles(c, 0, fuse ? (two ? kDeepNext : kDeepLast) : kDeep, c->TO(H), s,
                                &tl)))
                return rc;
            if (tl->ntiles == 0) continue;
            MixArgs a = margs(H, tl);
            a.u_in = first ? nullptr : io.u;
            a.rc = c->s.f[1];
            if (two) {
                two_level(a);
                a.f2 = c->s.f[2];
            }
            if (r0) {
                // from u = 0 the pass's residual is f itself (u0 folded)
                a.st = nullptr;   // the state is set after this launch
                a.partial = c->partial;
                a.norm_off = tl->d_off;
            }
            HIPCHK(c, launch_mix(c->P, io.trans, a, tl->ntiles, s));
            if (r0 && (rc = finalize_r0(c, r0, tl, s))) return rc;
        }
    }
    if (r0) return TMG_OK;
    if ((rc = c->opt.gamma == 1
                  ? enqueue_vcycle_levels<float>(c, io, fuse ? 2 : 1, fuse ? 2 : 1, s)
                  : enqueue_coarse_visits<float>(c, io, 1, s)))
        return rc;
    for (int pass = fuse ? 0 : 1; pass < 2; ++pass) {
        const bool two = pass == 0;
        const int H = two ? c->H_mix2() : (solve ? c->H_mix() : c->H_mixv());
        if ((rc = get_tiles(c, 0, fuse ? (two ? kDeepNext : kDeepLast) : kDeep, c->TO(H), s, &tl)))
            return rc;
        if (tl->ntiles == 0) continue;
        const int64_t hoff = fuse && !two ? c->hb_last_off : 0;
        MixArgs a = margs(H, tl);
        a.up = 1;
        a.u_in = first ? nullptr : io.u;
        a.halo_in = first ? nullptr : (io.kind == kOdd ? c->hb[1] : c->hb[0]) + hoff;
        if (two) {
            two_level(a);
            a.f1 = f1_in;
            a.e2 = c->s.x(2, c->cur[2]);
        } else {
            a.e = c->s.x(1, c->cur[1]);
        }
        a.u_out = io.u;
        if (solve) {
            a.halo_out = (io.kind == kEven ? c->hb[1] : c->hb[0]) + hoff;
            a.rc = two ? f1_out : c->s.f[1];
            a.f2 = two ? c->s.f[2] : nullptr;
            a.partial = c->partial;
            a.norm_off = tl->d_off;
        }
        HIPCHK(c, launch_mix(c->P, io.trans, a, tl->ntiles, s));
        if (solve && io.use_state)
            HIPCHK(c, launch_finalize(c->partial, tl->d_off, c->batch, c->st, c->ctl, c->mirror1(), 0, s));
    }
    return TMG_OK;
}

// A solve's first level-0 down pass in FP64, with the initial residual's
// norm: with two-level passes, levels 0 and 1 down in one launch for the
// instances whose level 1 streams (the others one level).
int enqueue_first_down(tmg_ctx *c, const CycleIO &io, hipStream_t s, R0 *r0)
{
    int rc;
    if (c->fuse_up1() && c->deep_n[1] > 0) {
        if ((rc = enqueue_pair<double>(c, io, 0, true, kDeepNext, s, r0)) ||
            (rc = enqueue_down<double>(c, io, 0, true, s, kDeepLast, r0)))
            return rc;
        return TMG_OK;
    }
    return enqueue_down<double>(c, io, 0, true, s, kDeep, r0);
}

// Level 0 of a cycle on the generic kernels: a down leg from u (pre sweeps
// stored in x0, residual restricted into level 1's right-hand side), the
// coarse levels, and an up leg from x0 (correction, post sweeps) into u with
// the residual norm of the result.  A solve's first cycle takes its down leg
// from the solve's first level-0 down pass and recomputes the pre sweeps
// from zero in the up leg instead of reading x0.
int enqueue_generic_level0(tmg_ctx *c, const CycleIO &io, hipStream_t s)
{
    int rc;
    TileList *tl;
    const bool first = io.kind == kFirst, solve = io.kind >= 0;
    if (!first) {
        const int H = c->H_down();
        if ((rc = get_tiles(c, 0, kDeep, c->TO(H), s, &tl))) return rc;
        LegArgs a = leg_args(c, 0, io.trans, tl, H);
        a.f = io.f;
        a.u0 = fold_of(io);
        a.u_in = io.u;
        a.u_out = c->x0;
        a.rc = c->d.f[1];
        a.st = io.use_state ? c->st : nullptr;
        a.pre = c->opt.nu1;
        HIPCHK(c, launch_leg<double>(c->P, io.trans, a, tl->ntiles, s));
    }
    if ((rc = c->opt.gamma == 1 ? enqueue_vcycle_levels<double>(c, io, 1, 1, s)
                                : enqueue_coarse_visits<double>(c, io, 1, s)))
        return rc;
    const int H = solve ? c->H_gup0() : c->H_up();
    if ((rc = get_tiles(c, 0, kDeep, c->TO(H), s, &tl))) return rc;
    LegArgs a = leg_args(c, 0, io.trans, tl, H);
    a.f = io.f;
    a.u0 = fold_of(io);
    a.u_in = first ? nullptr : c->x0;
    a.pre = first ? c->opt.nu1 : 0;
    a.e = c->d.x(1, c->cur[1]);
    a.post = c->opt.nu2;
    a.u_out = io.u;
    a.st = io.use_state ? c->st : nullptr;
    if (solve) {
        a.partial = c->partial;
        a.norm_off = tl->d_off;
    }
    HIPCHK(c, launch_leg<double>(c->P, io.trans, a, tl->ntiles, s));
    if (solve && io.use_state)
        HIPCHK(c, launch_finalize(c->partial, tl->d_off, c->batch, c->st, c->ctl, c->mirror1(), 0, s));
    return TMG_OK;
}

int enqueue_cycle(tmg_ctx *c, const CycleIO &io, hipStream_t s)
{
    int rc;
    const bool first = io.kind == kFirst;
    struct InCycle {
        bool &f;
        ~InCycle() { f = false; }
    } in_cycle{c->in_cycle};
    c->in_cycle = io.kind > kFirst;
    if (c->act.on && c->act.seed && io.kind > kFirst && c->deep_n[0] > 0) {
        c->act.seed = false;
        if ((rc = seed_halos(c, io, s))) return rc;
    }
    c->cur.assign(c->Lmax + 1, 0);
    // instances that fit the bottom kernel entirely: the cycle is one launch
    // (FP64 in both precision modes)
    if ((rc = enqueue_bottom<double>(c, io, 0, first ? nullptr : io.u, io.u, s))) return rc;
    if (c->deep_n[0] > 0 && c->generic) {
        if ((rc = enqueue_generic_level0(c, io, s))) return rc;
    } else if (c->deep_n[0] > 0 && c->mixed) {
        if ((rc = enqueue_mixed_level0(c, io, s))) return rc;
    } else if (c->deep_n[0] > 0) {
        TileList *tl;
        const bool solve = io.kind >= 0;
        if (!solve) {
            // warm start: seed the halo buffer from the caller's iterate
            const int H = c->H_up();
            if ((rc = get_tiles(c, 0, kDeep, c->TO(H), s, &tl))) return rc;
            LegArgs a = leg_args(c, 0, io.trans, tl, H);
            a.f = io.f;
            a.u_in = io.u;
            a.halo_out = c->hb[0];
            HIPCHK(c, launch_leg<double>(c->P, io.trans, a, tl->ntiles, s));
        }
        // With fuse2 the instances whose level 1 streams (kDeepNext) run
        // level 1's up leg and next down leg inside their level-0 pass (and
        // the first cycle runs levels 0 and 1 down in one launch); the others
        // (kDeepLast) take level 1's correction from the bottom kernel.
        // Level 1's right-hand side then alternates between two buffers:
        // the pass reads it for this cycle's up leg and writes the next one.
        const bool fuse2 = solve && c->fuse_up1() && c->deep_n[1] > 0;
        double *f1_in = io.kind == kEven ? c->f1b : c->d.f[1];
        double *f1_out = io.kind == kEven ? c->d.f[1] : c->f1b;
        // a solve's first level-0 down pass ran before its first cycle
        // (enqueue_first_down); a warm-started cycle starts from u
        if (!solve && (rc = enqueue_down<double>(c, io, 0, false, s))) return rc;
        if ((rc = c->opt.gamma == 1
                      ? enqueue_vcycle_levels<double>(c, io, fuse2 ? 2 : 1, fuse2 ? 2 : 1, s)
                      : enqueue_coarse_visits<double>(c, io, 1, s)))
            return rc;
        // fused level-0 pass(es)
        for (int pass = fuse2 ? 0 : 1; pass < 2; ++pass) {
            const bool two = pass == 0;
            const int H = two ? c->H_fused2() : (solve ? c->H_fused() : c->H_up());
            const int kind = fuse2 ? (two ? kDeepNext : kDeepLast) : kDeep;
            if ((rc = get_tiles(c, 0, kind, c->TO(H), s, &tl))) return rc;
            if (tl->ntiles == 0) continue;
            const int64_t hoff = fuse2 && !two ? c->hb_last_off : 0;
            LegArgs a = leg_args(c, 0, io.trans, tl, H);
            a.f = io.f;
            a.u0 = fold_of(io);
            a.u_in = first ? nullptr : io.u;
            a.halo_in = first ? nullptr : (io.kind == kOdd ? c->hb[1] : c->hb[0]) + hoff;
            if (two) {
                a.f1 = f1_in;
                a.e2 = c->d.x(2, c->cur[2]);
                a.tab1 = tab_of(c, 1, io.trans);
                a.tab1T = a.tab1;
                a.c2slab_off = c->slab_off_d[2];
            } else {
                a.e = c->d.x(1, c->cur[1]);
            }
            a.u_out = io.u;
            a.st = io.use_state ? c->st : nullptr;
            a.pre = c->opt.nu1;
            a.post = c->opt.nu2;
            if (solve) {
                a.halo_out = (io.kind == kEven ? c->hb[1] : c->hb[0]) + hoff;
                a.rc = two ? f1_out : c->d.f[1];
                a.f2 = two && c->opt.gamma == 1 ? c->d.f[2] : nullptr;
                a.next = c->opt.nu1;
                a.partial = c->partial;
                a.norm_off = tl->d_off;
            }
            HIPCHK(c, launch_leg<double>(c->P, io.trans, a, tl->ntiles, s));
            if (solve && io.use_state)
                HIPCHK(c, launch_finalize(c->partial, tl->d_off, c->batch, c->st, c->ctl, c->mirror1(), 0, s));
        }
    }
    if (io.kind >= 0 && io.use_state && c->batch > 1)
        HIPCHK(c, launch_publish(c->st, c->batch, c->ctl, c->mirror_d, c->pubn_d, s));
    return TMG_OK;
}

// Every tile list a cycle uses, created outside graph capture.
int make_tiles(tmg_ctx *c, hipStream_t s)
{
    TileList *tl;
    int rc;
    for (int l = 0; l < c->Lmax; ++l) {
        if ((rc = get_tiles(c, l, kDeep, c->TO(c->H_down()), s, &tl))) return rc;
        if ((rc = get_tiles(c, l, kDeep, c->TO(c->H_up()), s, &tl))) return rc;
    }
    const int H0[6] = {c->H_fused(), c->H_mixd(), c->H_mix(), c->H_mixv(), c->H_up(),
                       c->H_gup0()};
    for (int H : H0)
        if ((rc = get_tiles(c, 0, kDeep, c->TO(H), s, &tl))) return rc;
    if ((rc = get_tiles(c, 0, kDeepNext, c->TO(c->H_fused2()), s, &tl)) ||
        (rc = get_tiles(c, 0, kDeepLast, c->TO(c->H_fused()), s, &tl)))
        return rc;
    if ((rc = get_tiles(c, 0, kDeepNext, c->TO(c->H_dpair()), s, &tl)) ||
        (rc = get_tiles(c, 0, kDeepLast, c->TO(c->H_down()), s, &tl)) ||
        (rc = get_tiles(c, 0, kDeepNext, c->TO(c->H_mixd2()), s, &tl)) ||
        (rc = get_tiles(c, 0, kDeepLast, c->TO(c->H_mixd()), s, &tl)) ||
        (rc = get_tiles(c, 0, kDeepNext, c->TO(c->H_mix2()), s, &tl)) ||
        (rc = get_tiles(c, 0, kDeepLast, c->TO(c->H_mix()), s, &tl)))
        return rc;
    for (int l = 1; l < c->Lmax; ++l)
        if ((rc = get_tiles(c, l, kPair1, c->TO(c->H_dpair()), s, &tl)) ||
            (rc = get_tiles(c, l, kPair2, c->TO(c->H_dpair()), s, &tl)) ||
            (rc = get_tiles(c, l, kSingle2, c->TO(c->H_down()), s, &tl)) ||
            (rc = get_tiles(c, l, kSingle1, c->TO(c->H_down()), s, &tl)) ||
            (rc = get_tiles(c, l, kPair1, c->TO(c->H_upair()), s, &tl)) ||
            (rc = get_tiles(c, l, kSingle1, c->TO(c->H_up()), s, &tl)) ||
            (rc = get_tiles(c, l, kPair2, c->TO(c->H_upair()), s, &tl)) ||
            (rc = get_tiles(c, l, kSingle2, c->TO(c->H_up()), s, &tl)))
            return rc;
    // one instance's W-cycle: first-visit down pairs and fused launches
    if (c->opt.gamma == 2 && c->batch == 1 && !c->generic)
        for (int l = 1; l < c->Lmax; ++l)
            if ((rc = get_tiles(c, l, kDeepNext, c->TO(c->H_dpair()), s, &tl)) ||
                (rc = get_tiles(c, l, kDeepNext, c->TO(c->H_wfused(true)), s, &tl)) ||
                (rc = get_tiles(c, l, kDeep, c->TO(c->H_wfused(false)), s, &tl)))
                return rc;
    if (c->span_fits(c->span))
        for (int l = 1; l < c->Lmax; ++l)
            if ((rc = get_tiles(c, l, kDeep, kSpanThreads - c->H_sdown(c->span), s, &tl)) ||
                (rc = get_tiles(c, l, kDeep, kSpanThreads - c->H_sup(c->span), s, &tl)))
                return rc;
    return TMG_OK;
}

int get_graph(tmg_ctx *c, const CycleIO &io, hipGraphExec_t *out)
{
    GraphKey key{io.kind, io.trans, io.f, io.u0, io.u};
    auto it = c->graphs.find(key);
    if (it != c->graphs.end()) {
        *out = it->second;
        return TMG_OK;
    }
    int rc = make_tiles(c, c->cap);
    if (rc) return rc;
    hipGraph_t g;
    HIPCHK(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    if (io.kind == kEvenOdd || io.kind == kEvenOdd2) {
        CycleIO e = io, o = io;
        e.kind = kEven;
        o.kind = kOdd;
        for (int r = 0; r < (io.kind == kEvenOdd2 ? 2 : 1) && !rc; ++r) {
            rc = enqueue_cycle(c, e, c->cap);
            if (!rc) rc = enqueue_cycle(c, o, c->cap);
        }
    } else {
        rc = enqueue_cycle(c, io, c->cap);
    }
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

// Waits for the cycles a solve left queued (launched past convergence; they
// do nothing but read the state) before graphs or buffers they name go away.
int drain(tmg_ctx *c)
{
    if (!c->drain_pending) return TMG_OK;
    c->drain_pending = false;
    HIPCHK(c, hipEventSynchronize(c->drain_ev));
    return TMG_OK;
}

// Builds the dense bottom operator where it applies and is not current:
// one work-group per unit load runs the bottom visits (columns of D), then
// the rows' windows.  Launched on s before any cycle that applies it; the
// buffers grow only after a schedule change, which drops every graph.
int ensure_dense(tmg_ctx *c, hipStream_t s, bool trans)
{
    const int d = trans ? 1 : 0;
    if (c->dense_ok[d] || c->dense_nomem || !c->want_dense()) return TMG_OK;
    const int l = c->lb[0];
    const int64_t N = c->N[0] >> l, n = N * c->P;
    int rc;
    if (n * n > c->dense_cap[d]) {
        if ((rc = drain(c))) return rc;
        HIPCHK(c, hipStreamSynchronize(s));
        dfree(c, c->dense[d]);
        dfree(c, c->dense_win[d]);
        c->dense[d] = nullptr;
        c->dense_win[d] = nullptr;
        c->dense_cap[d] = 0;
        if (dalloc(c, &c->dense[d], (size_t)(n * n)) ||
            dalloc(c, &c->dense_win[d], (size_t)(2 * kDenseMaxN))) {
            // no room for the operator: the cycles run the recursion
            dfree(c, c->dense[d]);
            dfree(c, c->dense_win[d]);
            c->dense[d] = nullptr;
            c->dense_win[d] = nullptr;
            c->dense_nomem = true;
            c->last_hip = 0;
            (void)hipGetLastError();   // the failed allocation is no error of this call
            return TMG_OK;
        }
        c->dense_cap[d] = n * n;
    }
    // cycles a solve left queued past convergence may still read D
    if (c->drain_pending) HIPCHK(c, hipStreamWaitEvent(s, c->drain_ev, 0));
    DenseColArgs a{};
    a.tab = trans ? c->tab_adj : c->tab_fwd;   // instance 0
    a.tab_level = (int64_t)c->batch * c->tab_stride;
    a.R = trans ? c->R_adj : c->R_fwd;
    a.D = c->dense[d];
    a.backward = trans ? 1 : 0;
    a.periodic = c->opt.periodic;
    a.N = N;
    a.level = l;
    a.Lc = c->L[0] - 1;
    a.nu1 = c->opt.nu1;
    a.nu2 = c->opt.nu2;
    a.gamma = c->opt.gamma;
    HIPCHK(c, c->generic ? launch_gdense_cols(c->P, a, s) : launch_dense_cols(c->P, a, s));
    HIPCHK(c, launch_dense_window(c->dense[d], n, c->dense_win[d], s));
    // the widest span a product's work-group loads (sets its passes)
    c->dense_w[d] = n;
    if (c->dense_wd || dalloc(c, &c->dense_wd, 1) == TMG_OK) {
        int w = (int)n;
        HIPCHK(c, launch_dense_window_max(c->dense_win[d], n, 1, c->dense_wd, s));
        HIPCHK(c, hipMemcpyAsync(&w, c->dense_wd, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        c->dense_w[d] = w;
    } else {
        c->last_hip = 0;
        (void)hipGetLastError();
    }
    if (c->dense_level != l || c->dense_n != n) c->dense_ok[1 - d] = false;
    c->dense_level = l;
    c->dense_n = n;
    c->dense_ok[d] = true;
    return TMG_OK;
}

void free_all(tmg_ctx *c)
{
    (void)drain(c);
    for (auto &kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
    for (void *p : c->allocs) (void)hipFree(p);
    c->allocs.clear();
    if (c->fixed()) return;   // nothing of its own was allocated
    if (c->st_host) (void)hipHostFree(c->st_host);
    if (c->ctl_host) (void)hipHostFree(c->ctl_host);
    if (c->grad_host) (void)hipHostFree(c->grad_host);
    if (c->mirror) (void)hipHostFree(c->mirror);
    if (c->drain_ev) (void)hipEventDestroy(c->drain_ev);
    for (int k = 0; k < 2; ++k) {
        if (c->act.stage[k]) (void)hipHostFree(c->act.stage[k]);
        if (c->act.ev[k]) (void)hipEventDestroy(c->act.ev[k]);
    }
    if (c->cap) (void)hipStreamDestroy(c->cap);
}

// Solve loop shared by tmg_solve and tmg_adjoint_solve.
// A consistent copy of the host-side summary (see HostHead) and its
// version, or false while the device is writing it.
bool read_summary(const HostHead *h, HostSum *out, long long *ver)
{
    const long long e = __atomic_load_n(&h->end, __ATOMIC_ACQUIRE);
    const HostSum *m = reinterpret_cast<const HostSum *>(h + 1);
    out->running = __atomic_load_n(&m->running, __ATOMIC_RELAXED);
    out->want = __atomic_load_n(&m->want, __ATOMIC_RELAXED);
    out->cycles = __atomic_load_n(&m->cycles, __ATOMIC_RELAXED);
    out->done = __atomic_load_n(&m->done, __ATOMIC_RELAXED);
    __atomic_load(&m->r0sq, &out->r0sq, __ATOMIC_RELAXED);
    __atomic_load(&m->rsq, &out->rsq, __ATOMIC_RELAXED);
    __atomic_load(&m->prev_rsq, &out->prev_rsq, __ATOMIC_RELAXED);
    __atomic_thread_fence(__ATOMIC_ACQUIRE);
    const long long b = __atomic_load_n(&h->begin, __ATOMIC_RELAXED);
    *ver = e;
    return b == e;
}

// The run bits of the summary with version ver (false: the device has
// written a newer one meanwhile).
bool read_run_bits(const HostHead *h, int words, long long ver, std::vector<unsigned> *out)
{
    const long long e = __atomic_load_n(&h->end, __ATOMIC_ACQUIRE);
    const unsigned *b = reinterpret_cast<const unsigned *>(reinterpret_cast<const HostSum *>(h + 1) + 1);
    out->resize(words);
    for (int w = 0; w < words; ++w) (*out)[w] = __atomic_load_n(&b[w], __ATOMIC_RELAXED);
    __atomic_thread_fence(__ATOMIC_ACQUIRE);
    const long long bg = __atomic_load_n(&h->begin, __ATOMIC_RELAXED);
    return e == ver && bg == ver;
}

int run_solve(tmg_ctx *c, const double *f, const double *u0, double *u, bool trans, double rtol,
              int max_cycles, int *cycles, double *relres, hipStream_t s)
{
    // a periodic problem has no initial value
    if (c->opt.periodic) u0 = nullptr;
    // active-set lists last for the cycles of this solve only
    struct ActiveOff {
        ActiveSet &A;
        ~ActiveOff() { A.on = false; }
    } act_off{c->act};
    c->act.on = false;
    TileList *tl;
    int rc = get_tiles(c, 0, kAll, tile_slabs(c->P), s, &tl);
    if (rc) return rc;
    const int words = c->act.enabled && c->batch > 1 ? run_words(c->batch) : 0;
    c->act.tiles = tl->ntiles;
    std::vector<unsigned> bits;
    // cycles the previous solve left queued (on its stream) stay no-ops only
    // while the state they read says finished: this solve resets that state,
    // so its stream waits for them first (nothing to wait for on one stream)
    if (c->drain_pending) HIPCHK(c, hipStreamWaitEvent(s, c->drain_ev, 0));
    if ((rc = ensure_dense(c, s, trans))) return rc;
    c->epoch = c->epoch % (1 << 20) + 1;
    const long long epoch = c->epoch;
    c->ctl_host->rtol2 = rtol * rtol;
    c->ctl_host->max_cycles = max_cycles;
    c->ctl_host->epoch = c->epoch;
    // initial residual r_0 = f (u0 folded), u = 0: its norm comes with the
    // first level-0 down pass of the instances that stream level 0 (that
    // pass is then left out of the first cycle), and from k_norm_f for the
    // instances the bottom kernel holds whole.  The first launch that
    // finishes a norm also installs this solve's control block.
    {
        const CycleIO io0{f, u0, u, trans, true, kFirst};
        R0 r0;
        if (c->bot_n[0] > 0) {
            TileList *tw;
            if ((rc = get_tiles(c, 0, kWhole, tile_slabs(c->P), s, &tw))) return rc;
            HIPCHK(c, launch_norm_f(c->P, f, trans ? nullptr : u0, tab_of(c, 0, trans),
                                    c->tab_stride, c->slab_off_d[0], tw->d_off, tw->d_inst,
                                    c->batch, c->partial, tw->ntiles, s));
            if ((rc = finalize_r0(c, &r0, tw, s))) return rc;
        }
        if (c->deep_n[0] > 0) {
            c->cur.assign(c->Lmax + 1, 0);
            if ((rc = c->mixed ? enqueue_mixed_level0(c, io0, s, &r0)
                               : enqueue_first_down(c, io0, s, &r0)))
                return rc;
        }
    }
    if (c->batch > 1)
        HIPCHK(c, launch_publish(c->st, c->batch, c->ctl, c->mirror_d, c->pubn_d, s));

    // graphs are kept per set of arrays; a full cache is emptied before the
    // five graphs of this solve are fetched, never between them
    hipGraphExec_t g[5];
    if (!c->fixed() && c->graphs.size() + 5 > 30) {
        bool have = true;
        for (int k = 0; k < 5; ++k)
            have = have && c->graphs.count(GraphKey{k, trans, f, u0, u}) > 0;
        if (!have) {
            if ((rc = drain(c))) return rc;
            for (auto &kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
            c->graphs.clear();
        }
    }
    for (int k = 0; k < (c->fixed() ? 0 : c->direct ? 1 : 5); ++k) {
        CycleIO io{f, u0, u, trans, true, k};
        if ((rc = get_graph(c, io, &g[k]))) return rc;
    }
    int launched = 0;
    // cycle 1 has its own graph; cycle n >= 2 reads the halo buffer cycle n-1
    // wrote, and an even cycle with the following odd one (or two such
    // pairs) share one graph launch.  A graph launch leaves the GPU idle for
    // several microseconds at its start; with `direct` the cycles after the
    // first are launched kernel by kernel instead, which pays when the host
    // enqueues a cycle faster than the GPU runs it.
    auto launch = [&](int n) -> int {
        while (n > 0) {
            if (c->fixed() || ((c->direct || c->act.on) && launched > 0)) {
                CycleIO io{f, u0, u, trans, true,
                           launched == 0 ? kFirst : (launched % 2 == 1) ? kEven : kOdd};
                if ((rc = enqueue_cycle(c, io, s))) return rc;
                launched += 1;
                n -= 1;
            } else if (launched == 0) {
                HIPCHK(c, hipGraphLaunch(g[kFirst], s));
                launched = 1;
                n -= 1;
            } else if (launched % 2 == 1 && n >= 4) {
                HIPCHK(c, hipGraphLaunch(g[kEvenOdd2], s));
                launched += 4;
                n -= 4;
            } else if (launched % 2 == 1 && n >= 2) {
                HIPCHK(c, hipGraphLaunch(g[kEvenOdd], s));
                launched += 2;
                n -= 2;
            } else {
                HIPCHK(c, hipGraphLaunch(g[(launched % 2 == 1) ? kEven : kOdd], s));
                launched += 1;
                n -= 1;
            }
        }
        return TMG_OK;
    };

    // After each cycle the device writes a summary into pinned host memory
    // (instances still running, cycles to have queued; see HostHead).  The
    // host follows it there while the stream runs and tops up the queue, so
    // no look at the state stops the GPU.  Cycles queued after an instance
    // converged do nothing for it.
    const int head = std::min(max_cycles, 3);
    if ((rc = launch(head))) return rc;
    HostSum sum{};
    // one instance with nothing of its own allocated: the host reads the
    // state after the queued cycles (a plain copy and a wait), queues up to
    // the count the state predicts, and repeats
    while (c->fixed()) {
        HIPCHK(c, hipMemcpyAsync(&c->fx_st, c->st, sizeof(InstState), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        const InstState q = c->fx_st;
        sum.cycles = q.cycles;
        sum.done = q.done;
        sum.r0sq = q.r0sq;
        sum.rsq = q.rsq;
        if (q.done || q.cycles >= max_cycles) break;
        int want = q.cycles + 2;
        if (q.prev_rsq > 0.0 && q.rsq > 0.0 && q.rsq < q.prev_rsq) {
            const double k =
                std::log(c->ctl_host->rtol2 * q.r0sq / q.rsq) / std::log(q.rsq / q.prev_rsq);
            want = q.cycles + (int)std::fmin(std::fmax(std::ceil(k), 1.0), 64.0);
        }
        want = std::min(std::max(want, launched + 1), max_cycles);
        // every queued cycle has run, so a running instance has cycles == launched
        if (want <= launched) return TMG_ERR_INTERNAL;
        if ((rc = launch(want - launched))) return rc;
    }
    long long last_ver = -1;
    constexpr std::chrono::microseconds kQuiet(2000);
    // Between summaries the host spins for a short while, then yields its
    // core, then sleeps in short steps: the device runs cycles already
    // queued meanwhile, so the host need not answer within microseconds.
    constexpr std::chrono::microseconds kSpin(50), kYield(1000), kNap(20);
    auto since = std::chrono::steady_clock::now(), queried = since;
    while (!c->fixed()) {
        long long ver = 0;
        HostSum q;
        if (__atomic_load_n(&c->mirror->end, __ATOMIC_ACQUIRE) != last_ver &&
            read_summary(c->mirror, &q, &ver) && (ver >> 32) == epoch && ver != last_ver) {
            last_ver = ver;
            sum = q;
            if (c->batch == 1) {
                // the device's running / want_cycles rule for one instance
                sum.running = !q.done && q.cycles < max_cycles;
                sum.want = q.cycles + 2;
                if (q.prev_rsq > 0.0 && q.rsq > 0.0 && q.rsq < q.prev_rsq) {
                    const double k = std::log(c->ctl_host->rtol2 * q.r0sq / q.rsq) /
                                     std::log(q.rsq / q.prev_rsq);
                    const int n = (int)std::fmin(std::fmax(std::ceil(k), 1.0), 64.0);
                    sum.want = q.cycles + (n > 3 ? n - 1 : n);
                }
            }
            if (sum.running == 0) break;
            int want = std::min(std::max(sum.want, 1), max_cycles);
            if (words > 0) {
                // few cycles ahead, so that active-set lists apply soon; a
                // new generation once the running share of level-0 tiles
                // dropped far enough
                want = std::min(want, std::max(sum.cycles + kActiveAhead, 1));
                if (read_run_bits(c->mirror, words, ver, &bits)) {
                    const std::vector<int64_t> &fo = tl->h_off;
                    int64_t r = 0;
                    for (int j = 0; j < c->batch; ++j)
                        if ((bits[j >> 5] >> (j & 31)) & 1u) r += fo[j + 1] - fo[j];
                    if (r > 0 && (double)r <= kActiveShare * (double)c->act.tiles &&
                        (rc = act_begin(c, bits, r, s)))
                        return rc;
                }
            }
            if (want > launched && (rc = launch(want - launched))) return rc;
            since = std::chrono::steady_clock::now();
            continue;
        }
        const auto now = std::chrono::steady_clock::now();
        if (now - since > kYield) std::this_thread::sleep_for(kNap);
        else if (now - since > kSpin) std::this_thread::yield();
        // nothing new for a while: if the stream has drained, every summary
        // it will write is there, so one more read decides (queried rarely:
        // a query is not free for the stream)
        if (now - since > kQuiet && now - queried > kQuiet) {
            queried = now;
            const hipError_t qs = hipStreamQuery(s);
            if (qs == hipSuccess) {
                long long v = 0;
                HostSum r;
                const bool again =
                    !read_summary(c->mirror, &r, &v) || (v >> 32) != epoch || v != last_ver;
                if (!again) {
                    // a drained stream with a running instance: queue one
                    // more cycle, or give up when none is left
                    if (launched >= max_cycles) return TMG_ERR_INTERNAL;
                    if ((rc = launch(1))) return rc;
                }
            } else if (qs != hipErrorNotReady) {
                c->last_hip = (int)qs;
                return TMG_ERR_HIP;
            }
        }
    }
    if (!c->fixed()) {
        HIPCHK(c, hipEventRecord(c->drain_ev, s));
        c->drain_pending = true;
    }
    // per-instance results: the summary holds a single instance's; a batch
    // reads its states once (after the cycles still queued)
    if (c->batch > 1) {
        HIPCHK(c, hipMemcpyAsync(c->st_host, c->st, sizeof(InstState) * c->batch,
                                 hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
    } else {
        c->st_host[0].cycles = sum.cycles;
        c->st_host[0].done = sum.done;
        c->st_host[0].r0sq = sum.r0sq;
        c->st_host[0].rsq = sum.rsq;
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
    return status;
}

// The bottom cap of a schedule id (-1: the largest the bottom kernel holds).
int64_t schedule_cap(int P, int schedule)
{
    return schedule < 0 ? (int64_t)bottom_max(P)
                        : std::min<int64_t>(bottom_max(P), int64_t(1) << std::min(schedule, 40));
}

// First bottom-kernel level of every instance for a bottom cap: the first
// level of at most `cap` slabs (the coarsest level at the latest).
int plan_levels(const std::vector<int> &L, const int64_t *n_slabs, int64_t cap,
                std::vector<int> *lb)
{
    lb->assign(L.size(), 0);
    for (size_t j = 0; j < L.size(); ++j) {
        int l = 0;
        while (l < L[j] - 1 && (n_slabs[j] >> l) > cap) ++l;
        if (L[j] - l > kBottomMaxLevels) return TMG_ERR_SIZE;
        (*lb)[j] = l;
    }
    return TMG_OK;
}

// Install a schedule: the split of every hierarchy between the streaming
// kernels and the bottom kernel (bottom cap) and whether V-cycles use
// two-level launches.  Drops the captured graphs and tile lists of the old
// schedule and sizes the buffers that depend on it.
int apply_plan(tmg_ctx *c, int64_t cap, bool pairs, int span, int span_after, hipStream_t s)
{
    if (c->generic) {
        // the bottom work-group solves the coarsest level, or visits the
        // levels up to gbottom_max(P) slabs (k_gvisit); every level above
        // streams in one-level legs
        cap = std::max<int64_t>(c->opt.n_coarse, std::min(cap, c->max_cap()));
        pairs = false;
        span = 0;
    }
    std::vector<int> lbv;
    int rc = plan_levels(c->L, c->N.data(), cap, &lbv);
    if (rc) return rc;
    if ((rc = drain(c))) return rc;
    HIPCHK(c, hipStreamSynchronize(s));
    for (auto &kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
    for (auto &kv : c->tiles) {
        dfree(c, kv.second.d_off);
        dfree(c, kv.second.d_inst);
    }
    c->tiles.clear();
    c->cycle_keys.clear();
    for (int *p : c->bot_d) dfree(c, p);
    dfree(c, c->bot_all_d);
    c->bot_all_d = nullptr;
    const int Lm = c->Lmax, batch = c->batch, P = c->P;
    c->lb = lbv;
    c->dense_stale();
    c->dense_nomem = false;
    c->bottom_cap = cap;
    c->pairs = pairs;
    c->span = c->span_fits(span) ? span : 0;
    c->span_after = std::max(span_after, 1);   // levels
    if (!c->lb_d && (rc = dalloc(c, &c->lb_d, batch))) return rc;
    HIPCHK(c, hipMemcpyAsync(c->lb_d, c->lb.data(), sizeof(int) * batch, hipMemcpyHostToDevice, s));
    c->deep_n.assign(Lm + 1, 0);
    c->bot_n.assign(Lm + 1, 0);
    c->bot_d.assign(Lm + 1, nullptr);
    for (int l = 0; l < Lm; ++l) {
        std::vector<int> bl;
        for (int j = 0; j < batch; ++j) {
            if (c->lb[j] == l) bl.push_back(j);
            if (l < c->lb[j]) c->deep_n[l]++;
        }
        c->bot_n[l] = (int)bl.size();
        if (!bl.empty()) {
            if ((rc = dalloc(c, &c->bot_d[l], bl.size()))) return rc;
            HIPCHK(c, hipMemcpyAsync(c->bot_d[l], bl.data(), sizeof(int) * bl.size(),
                                     hipMemcpyHostToDevice, s));
        }
    }
    std::vector<int> ball;
    c->bot_levels = 0;
    for (int l = 1; l < Lm; ++l) c->bot_levels += c->bot_n[l] > 0;
    for (int j = 0; j < batch; ++j)
        if (c->lb[j] >= 1) ball.push_back(j);
    c->bot_all_n = (int)ball.size();
    if (!ball.empty()) {
        if ((rc = dalloc(c, &c->bot_all_d, ball.size()))) return rc;
        HIPCHK(c, hipMemcpyAsync(c->bot_all_d, ball.data(), sizeof(int) * ball.size(),
                                 hipMemcpyHostToDevice, s));
    }
    HIPCHK(c, hipStreamSynchronize(s));
    // level-0 halo buffers: one slot of H x P doubles per tile
    const int Hs[5] = {c->H_fused(), c->H_up(), c->H_mix(), c->H_mixv(), c->H_mixd()};
    int64_t hsize = 0;
    for (int H : Hs) hsize = std::max(hsize, tiles_of(c, 0, kDeep, c->TO(H)) * H * P);
    // two-level passes (kDeepNext) and one-level passes (kDeepLast) of one
    // cycle use disjoint slots
    const int Hn = c->mixed ? c->H_mix2() : c->H_fused2(), Hl = c->mixed ? c->H_mix() : c->H_fused();
    c->hb_last_off = tiles_of(c, 0, kDeepNext, c->TO(Hn)) * Hn * P;
    hsize = std::max(hsize, c->hb_last_off + tiles_of(c, 0, kDeepLast, c->TO(Hl)) * Hl * P);
    if (hsize > c->hb_cap) {
        dfree(c, c->hb[0]);
        dfree(c, c->hb[1]);
        c->hb[0] = c->hb[1] = nullptr;
        if ((rc = dalloc(c, &c->hb[0], hsize)) || (rc = dalloc(c, &c->hb[1], hsize))) return rc;
        c->hb_cap = hsize;
    }
    if (c->fuse_up1() && c->deep_n[1] > 0 && !c->f1b &&
        (rc = dalloc(c, &c->f1b, c->level_size[1])))
        return rc;
    if (c->fuse_mix() && c->deep_n[1] > 0 && !c->f1b32 &&
        (rc = dalloc(c, &c->f1b32, c->level_size[1])))
        return rc;
    return TMG_OK;
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
    o->periodic = 0;
}

const char *tmg_error_string(int code)
{
    switch (code) {
    case TMG_OK: return "ok";
    case TMG_NOT_CONVERGED: return "max_cycles reached before the residual tolerance";
    case TMG_ERR_INVALID: return "invalid argument";
    case TMG_ERR_SIZE: return "slab count is not n_coarse * 2^k, or larger than the call takes";
    case TMG_ERR_OMEGA: return "damping parameter outside (0, 1]";
    case TMG_ERR_PARAM: return "lambda and T must be finite and positive";
    case TMG_ERR_OOM: return "device memory allocation failed";
    case TMG_ERR_HIP: return "HIP runtime error";
    case TMG_ERR_NONFINITE: return "non-finite value in the data or the residual";
    case TMG_ERR_DIVERGED: return "residual grew beyond 1e3 times the initial residual";
    case TMG_ERR_UNSUPPORTED: return "option combination not supported";
    case TMG_ERR_INTERNAL: return "internal error: the solve's own state is inconsistent";
    default: return "unknown status";
    }
}

int tmg_last_hip_error(tmg_handle h) { return h ? h->last_hip : 0; }

}  // extern "C"

namespace {

// The generic kernels serve degrees above the tuned kernels' and the
// periodic problem; there every level above the bottom streams in one-level
// legs, and the bottom work-group visits the levels up to gbottom_max(P)
// slabs.
bool uses_generic(const tmg_options &o) { return o.p + 1 > kMaxTunedP || o.periodic != 0; }
int64_t first_cap(const tmg_options &o)
{
    if (!uses_generic(o)) return schedule_cap(o.p + 1, o.schedule);
    // the generic bottom visit up to gbottom_max(P) slabs
    const int64_t gmax = gbottom_max(o.p + 1);
    const int64_t cap = o.schedule < 0 ? gmax
                                       : std::min<int64_t>(gmax, int64_t(1) << std::min(o.schedule, 40));
    return std::max<int64_t>(o.n_coarse, cap);
}

// Argument checks of a set-up (host only): options, lambda, T, and every
// n_slabs[j] = n_coarse * 2^k; L[j] receives the level counts.
int check_problem(int batch, const int64_t *n_slabs, const double *T, const double *lambda,
                  const tmg_options &o, std::vector<int> *Lout)
{
    if (o.p < 0 || o.p > TMG_MAX_DEGREE || o.nu1 < 0 || o.nu1 > kMaxSweeps || o.nu2 < 0 ||
        o.nu2 > kMaxSweeps || (o.gamma != 1 && o.gamma != 2) || o.n_coarse < 1 ||
        o.n_coarse > kMaxCoarse || (o.omega_mode != 0 && o.omega_mode != 1))
        return TMG_ERR_INVALID;
    if (o.omega_mode == 1 && !(o.omega > 0.0 && o.omega <= 1.0)) return TMG_ERR_OMEGA;
    if (o.precision != 0 && o.precision != 1) return TMG_ERR_UNSUPPORTED;
    if (o.periodic != 0 && o.periodic != 1) return TMG_ERR_INVALID;
    // the FP32-inner cycle runs on the tuned kernels only
    if (o.precision == 1 && uses_generic(o)) return TMG_ERR_UNSUPPORTED;
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
    // levels of at most bottom_cap slabs run inside the single-work-group
    // bottom kernel (schedule >= 0: bottom_cap = 2^schedule, capped); an
    // instance's coarsest level always does
    std::vector<int> lbv;
    if (plan_levels(L, n_slabs, first_cap(o), &lbv)) return TMG_ERR_SIZE;
    Lout->swap(L);
    return TMG_OK;
}

// Everything a handle holds for the checked problem: level hierarchy,
// tables, schedule, state, host copies.  On failure the caller releases
// what was made (free_all).
int build_ctx(tmg_ctx *c, int batch, const int64_t *n_slabs, const double *T,
              const double *lambda, const tmg_options &o, const std::vector<int> &L,
              hipStream_t s)
{
    const int P = o.p + 1;
    const int64_t bottom_cap = first_cap(o);
    c->generic = uses_generic(o);
    c->batch = batch;
    c->P = P;
    c->S = c->generic ? 1 : slabs_per_thread(P);
    c->act.enabled = !c->generic;
    c->opt = o;
    c->N.assign(n_slabs, n_slabs + batch);
    c->T.assign(T, T + batch);
    c->lam.assign(lambda, lambda + batch);
    c->L = L;
    c->Lmax = *std::max_element(L.begin(), L.end());
    const int Lm = c->Lmax;
    const TabLayout TL(P);
    c->tab_stride = TL.stride();

    int rc = TMG_OK;
    // the capture stream of the cycle graphs (none without allocations)
    if (!c->fixed() && hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess)
        return TMG_ERR_HIP;

    c->slab_off_h.assign(Lm, std::vector<int64_t>(batch + 1, 0));
    c->slab_off_d.assign(Lm, nullptr);
    c->level_size.assign(Lm, 0);
    c->mixed = o.precision == 1;
    c->d.f.assign(Lm + 1, nullptr);
    c->d.xa.assign(Lm + 1, nullptr);
    c->d.xb.assign(Lm + 1, nullptr);
    c->s.f.assign(Lm + 1, nullptr);
    c->s.xa.assign(Lm + 1, nullptr);
    c->s.xb.assign(Lm + 1, nullptr);
    for (int l = 0; l < Lm; ++l) {
        auto &off = c->slab_off_h[l];
        for (int j = 0; j < batch; ++j) off[j + 1] = off[j] + (l < L[j] ? (c->N[j] >> l) : 0);
        c->level_size[l] = off[batch] * P;
        if ((rc = dalloc(c, &c->slab_off_d[l], batch + 1))) return rc;
        if (hipMemcpyAsync(c->slab_off_d[l], off.data(), sizeof(int64_t) * (batch + 1),
                           hipMemcpyHostToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return TMG_ERR_HIP;
        // coarse-level buffers in the precision of the cycle below level 0
        if (l > 0 && !c->mixed) {
            if ((rc = dalloc(c, &c->d.f[l], c->level_size[l])) ||
                (rc = dalloc(c, &c->d.xa[l], c->level_size[l])) ||
                (rc = dalloc(c, &c->d.xb[l], c->level_size[l])))
                return rc;
        }
        if (l > 0 && c->mixed) {
            if ((rc = dalloc(c, &c->s.f[l], c->level_size[l])) ||
                (rc = dalloc(c, &c->s.xa[l], c->level_size[l])) ||
                (rc = dalloc(c, &c->s.xb[l], c->level_size[l])))
                return rc;
        }
    }
    {
        // per-level arrays of the coarse hierarchy, for one bottom launch
        // over instances at different levels
        std::vector<void *> t(3 * (size_t)Lm, nullptr);
        for (int l = 0; l < Lm; ++l) {
            t[l] = c->mixed ? (void *)c->s.f[l] : (void *)c->d.f[l];
            t[Lm + l] = c->mixed ? (void *)c->s.xa[l] : (void *)c->d.xa[l];
            t[2 * Lm + l] = c->slab_off_d[l];
        }
        if ((rc = dalloc(c, &c->lvptr_d, t.size()))) return rc;
        if (hipMemcpyAsync(c->lvptr_d, t.data(), sizeof(void *) * t.size(), hipMemcpyHostToDevice,
                           s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return TMG_ERR_HIP;
    }
    if (c->generic && (rc = dalloc(c, &c->x0, c->level_size[0]))) return rc;
    if ((rc = apply_plan(c, bottom_cap, !c->generic, 0, 2, s))) return rc;
    // tables, level-major: block (l, j) at (l * batch + j) * stride
    std::vector<double> tf((size_t)Lm * batch * c->tab_stride, 0.0),
        ta((size_t)Lm * batch * c->tab_stride, 0.0);
    for (int l = 0; l < Lm; ++l)
        for (int j = 0; j < batch; ++j) {
            if (l >= L[j]) continue;
            const double z = level_z(lambda[j], T[j], c->N[j], l);
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
    std::vector<int> nlev(L.begin(), L.end());
    if ((rc = dalloc(c, &c->tab_fwd, tf.size())) || (rc = dalloc(c, &c->tab_adj, ta.size())) ||
        (rc = dalloc(c, &c->R_fwd, Rf.size())) || (rc = dalloc(c, &c->R_adj, Ra.size())) ||
        (rc = dalloc(c, &c->st, batch)) || (rc = dalloc(c, &c->st_ops, batch)) ||
        (rc = dalloc(c, &c->ctl, 1)) || (rc = dalloc(c, &c->tau_d, batch)) ||
        (rc = dalloc(c, &c->grad_d, 2 * batch)) || (rc = dalloc(c, &c->nlev_d, batch)) ||
        (rc = dalloc(c, &c->T_d, batch)) || (rc = dalloc(c, &c->N_d, batch)))
        return rc;
    // partial sums: one slot per level-0 tile at the smallest tile size in use
    c->partial_cap = tiles_of(c, 0, kAll, std::min(c->ts(), tile_slabs(P)) - c->rs(3 * kMaxSweeps + 4));
    if ((rc = dalloc(c, &c->partial, c->partial_cap))) return rc;
    const size_t mirror_bytes =
        sizeof(HostHead) + sizeof(HostSum) + sizeof(unsigned) * run_words(batch);
    if (c->fixed()) {
        // one instance: its state, control block and gradients in the context
        c->st_host = &c->fx_st;
        c->ctl_host = &c->fx_ctl;
        c->grad_host = c->fx_grad;
    } else if (hipHostMalloc((void **)&c->st_host, sizeof(InstState) * batch) != hipSuccess ||
        hipHostMalloc((void **)&c->ctl_host, sizeof(Control)) != hipSuccess ||
        hipHostMalloc((void **)&c->grad_host, sizeof(double) * 2 * batch) != hipSuccess ||
        hipHostMalloc((void **)&c->mirror, mirror_bytes,
                      hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess)
        return TMG_ERR_OOM;
    if (c->mirror) std::memset(c->mirror, 0, mirror_bytes);
    if ((rc = dalloc(c, &c->pubn_d, 1)) ||
        hipMemsetAsync(c->pubn_d, 0, sizeof(unsigned), s) != hipSuccess)
        return rc ? rc : TMG_ERR_HIP;
    if (!c->fixed() &&
        (hipHostGetDevicePointer((void **)&c->mirror_d, c->mirror, 0) != hipSuccess ||
         hipEventCreateWithFlags(&c->drain_ev, hipEventDisableTiming) != hipSuccess))
        return TMG_ERR_HIP;
    if (hipMemcpyAsync(c->tab_fwd, tf.data(), tf.size() * 8, hipMemcpyHostToDevice, s) ||
        hipMemcpyAsync(c->tab_adj, ta.data(), ta.size() * 8, hipMemcpyHostToDevice, s) ||
        hipMemcpyAsync(c->R_fwd, Rf.data(), Rf.size() * 8, hipMemcpyHostToDevice, s) ||
        hipMemcpyAsync(c->R_adj, Ra.data(), Ra.size() * 8, hipMemcpyHostToDevice, s) ||
        hipMemcpyAsync(c->tau_d, tau.data(), tau.size() * 8, hipMemcpyHostToDevice, s) ||
        hipMemcpyAsync(c->T_d, T, sizeof(double) * batch, hipMemcpyHostToDevice, s) ||
        hipMemcpyAsync(c->N_d, n_slabs, sizeof(int64_t) * batch, hipMemcpyHostToDevice, s) ||
        hipMemcpyAsync(c->nlev_d, nlev.data(), nlev.size() * sizeof(int), hipMemcpyHostToDevice,
                       s) ||
        hipMemsetAsync(c->st, 0, sizeof(InstState) * batch, s) || hipStreamSynchronize(s))
        return TMG_ERR_HIP;
    if (c->mixed) {
        // FP32 copies of the tables for the inner cycle
        std::vector<float> tf32(tf.begin(), tf.end()), ta32(ta.begin(), ta.end()),
            Rf32(Rf.begin(), Rf.end()), Ra32(Ra.begin(), Ra.end());
        if ((rc = dalloc(c, &c->tab32_fwd, tf32.size())) ||
            (rc = dalloc(c, &c->tab32_adj, ta32.size())) ||
            (rc = dalloc(c, &c->R32_fwd, Rf32.size())) || (rc = dalloc(c, &c->R32_adj, Ra32.size())))
            return rc;
        if (hipMemcpyAsync(c->tab32_fwd, tf32.data(), tf32.size() * 4, hipMemcpyHostToDevice, s) ||
            hipMemcpyAsync(c->tab32_adj, ta32.data(), ta32.size() * 4, hipMemcpyHostToDevice, s) ||
            hipMemcpyAsync(c->R32_fwd, Rf32.data(), Rf32.size() * 4, hipMemcpyHostToDevice, s) ||
            hipMemcpyAsync(c->R32_adj, Ra32.data(), Ra32.size() * 4, hipMemcpyHostToDevice, s) ||
            hipStreamSynchronize(s))
            return TMG_ERR_HIP;
    }
    return TMG_OK;
}

}  // namespace

extern "C" {

int tmg_setup(tmg_handle *hp, int batch, const int64_t *n_slabs, const double *T,
              const double *lambda, const tmg_options *opt, tmg_stream stream)
{
    if (!hp || !n_slabs || !T || !lambda || !opt || batch < 1) return TMG_ERR_INVALID;
    *hp = nullptr;
    std::vector<int> L;
    int rc = check_problem(batch, n_slabs, T, lambda, *opt, &L);
    if (rc) return rc;
    tmg_ctx *c = new (std::nothrow) tmg_ctx;
    if (!c) return TMG_ERR_OOM;
    if ((rc = build_ctx(c, batch, n_slabs, T, lambda, *opt, L, (hipStream_t)stream))) {
        free_all(c);
        delete c;
        return rc;
    }
    *hp = c;
    return TMG_OK;
}

int tmg_solve_noalloc(int64_t n_slabs, double T, double lambda, const tmg_options *opt,
                      const double *f, const double *u0, double *u, double rtol, int max_cycles,
                      int *cycles, double *relres, tmg_stream stream)
{
    if (!opt || !f || !u0 || !u || !(rtol >= 0.0) || max_cycles < 0) return TMG_ERR_INVALID;
    std::vector<int> L;
    int rc = check_problem(1, &n_slabs, &T, &lambda, *opt, &L);
    if (rc) return rc;
    if (n_slabs * (opt->p + 1) > kNoAllocMaxUnknowns) return TMG_ERR_SIZE;
    void *base = nullptr;
    size_t bytes = 0;
    const hipError_t e = noalloc_scratch(&base, &bytes);
    if (e != hipSuccess) return TMG_ERR_HIP;
    hipStream_t s = (hipStream_t)stream;
    tmg_ctx c;
    c.arena = static_cast<char *>(base);
    c.arena_cap = bytes;
    // the scratch keeps the previous call's contents: the set-up clears the
    // state it reads, and no kernel reads a buffer before a launch of the
    // same solve has written it
    rc = build_ctx(&c, 1, &n_slabs, &T, &lambda, *opt, L, s);
    if (!rc) rc = run_solve(&c, f, u0, u, false, rtol, max_cycles, cycles, relres, s);
    if (rc < 0) (void)hipStreamSynchronize(s);   // nothing queued may outlive the call
    free_all(&c);
    return rc;
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
    hipStream_t s = (hipStream_t)stream;
    int rc = make_tiles(c, s);
    if (rc || (rc = ensure_dense(c, s, false))) return rc;
    CycleIO io{f, c->opt.periodic ? nullptr : u0, u, false, false, -1};
    return enqueue_cycle(c, io, s);
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
        TileList *tl;
        const int rc = get_tiles(c, 0, kAll, tile_slabs(c->P), s, &tl);
        if (rc) return rc;
        HIPCHK(c, launch_grad(c->P, u, z, c->tau_d, c->slab_off_d[0], tl->d_off, tl->d_inst,
                              tl->ntiles, c->batch, c->partial, c->grad_d, s));
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

int tmg_autotune(tmg_handle c, const double *f, const double *u0, double *u, int64_t *cap_out,
                 int *pairs_out, int *span_out, int *span_after_out, int *direct_out,
                 tmg_stream stream)
{
    if (!c || !f || !u0 || !u) return TMG_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    struct Cand {
        int64_t cap;
        bool pairs;
        int span, after;
    };
    // in stages, each from the best of the one before: the bottom cap (with
    // two-level launches), then how the streaming levels are launched at
    // that cap, then the launch mode
    std::vector<Cand> cands;
    for (int k = 0; k <= 5; ++k) {
        const int64_t cap = c->max_cap() >> k;
        if (cap < c->opt.n_coarse) break;
        cands.push_back({cap, !c->generic, 0, 2});
    }
    const Cand old{c->bottom_cap, c->pairs, c->span, c->span_after};
    c->direct = false;
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    int rc = TMG_OK;
    float best = -1.0f;
    Cand pick = old;
    constexpr int kCycles = 4;
    // a run that captures the graphs, then the fastest of three timed ones
    // (rtol 0: every instance runs kCycles cycles); milliseconds, or < 0 on
    // an error
    auto timed = [&]() -> float {
        rc = run_solve(c, f, u0, u, false, 0.0, kCycles, nullptr, nullptr, s);
        if (rc < 0) return -1.0f;
        float best_ms = -1.0f;
        for (int rep = 0; rep < 3; ++rep) {
            if (hipEventRecord(e0, s) != hipSuccess) { rc = TMG_ERR_HIP; return -1.0f; }
            rc = run_solve(c, f, u0, u, false, 0.0, kCycles, nullptr, nullptr, s);
            if (rc < 0) return -1.0f;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                rc = TMG_ERR_HIP;
                return -1.0f;
            }
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (best_ms < 0.0f || ms < best_ms) best_ms = ms;
        }
        return best_ms;
    };
    auto run_stage = [&]() {
        for (const Cand &cd : cands) {
            if (apply_plan(c, cd.cap, cd.pairs, cd.span, cd.after, s) != TMG_OK) continue;
            const float ms = timed();
            if (ms < 0.0f) return;
            if (best < 0.0f || ms < best) {
                best = ms;
                pick = cd;
            }
        }
    };
    run_stage();
    if (rc >= 0 && c->opt.gamma == 1 && !c->generic && best >= 0.0f) {
        cands.clear();
        cands.push_back({pick.cap, false, 0, 2});
        for (int K = 3; K <= kMaxSpan; ++K)
            for (int after = 1; after <= 6; ++after)
                if (c->span_fits(K)) cands.push_back({pick.cap, true, K, after});
        run_stage();
        // the caps next to the first stage's pick, with the launch pattern
        // the second stage chose for it
        cands.clear();
        for (int64_t cap : {pick.cap * 2, pick.cap / 2})
            if (cap >= c->opt.n_coarse && cap <= c->max_cap())
                cands.push_back({cap, pick.pairs, pick.span, pick.after});
        if (rc >= 0) run_stage();
    }
    int rc2 = apply_plan(c, pick.cap, pick.pairs, pick.span, pick.after, s);
    // then the same schedule with the cycles after the first launched kernel
    // by kernel
    bool direct = false;
    if (rc >= 0 && rc2 == TMG_OK && best >= 0.0f) {
        c->direct = true;
        const float ms = timed();
        direct = ms >= 0.0f && ms < best;
        c->direct = direct;
        if (direct) {
            // with direct launches the caps next to the pick once more (a
            // graph boundary no longer weighs on the small levels)
            best = ms;
            const Cand base = pick;
            for (int64_t cap : {base.cap * 2, base.cap / 2}) {
                if (cap < c->opt.n_coarse || cap > c->max_cap()) continue;
                if (apply_plan(c, cap, base.pairs, base.span, base.after, s) != TMG_OK) continue;
                c->direct = true;
                const float m2 = timed();
                if (m2 < 0.0f) break;
                if (m2 < best) {
                    best = m2;
                    pick = {cap, base.pairs, base.span, base.after};
                }
            }
            rc2 = apply_plan(c, pick.cap, pick.pairs, pick.span, pick.after, s);
            c->direct = true;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc < 0) return rc;
    if (rc2 != TMG_OK) return rc2;
    if (cap_out) *cap_out = pick.cap;
    if (pairs_out) *pairs_out = pick.pairs ? 1 : 0;
    if (span_out) *span_out = c->span;
    if (span_after_out) *span_after_out = c->span_after;
    if (direct_out) *direct_out = direct ? 1 : 0;
    return TMG_OK;
}

int tmg_set_schedule(tmg_handle c, int64_t bottom_cap, int pairs, int span, int span_after,
                     int direct, tmg_stream stream)
{
    if (!c || bottom_cap < c->opt.n_coarse || bottom_cap > c->max_cap()) return TMG_ERR_INVALID;
    if (c->generic && (pairs || span))
        return TMG_ERR_UNSUPPORTED;   // the generic kernels stream in one-level legs
    if (span != 0 && (!pairs || c->opt.gamma != 1 || !c->span_fits(span) || span_after < 1))
        return TMG_ERR_INVALID;
    const int rc = apply_plan(c, bottom_cap, pairs != 0, span, span_after, (hipStream_t)stream);
    if (rc) return rc;
    c->direct = direct != 0;
    return TMG_OK;
}

int tmg_set_lambda(tmg_handle c, const double *lambda, tmg_stream stream)
{
    if (!c || !lambda) return TMG_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    // cycles a solve left queued past convergence still read the tables
    if (c->drain_pending) HIPCHK(c, hipStreamWaitEvent(s, c->drain_ev, 0));
    HIPCHK(c, launch_set_tables(c->P, lambda, c->T_d, c->N_d, c->nlev_d, c->batch, c->Lmax,
                                c->opt.omega_mode, c->opt.omega, c->tab_stride, c->tab_fwd,
                                c->tab_adj, c->tab32_fwd, c->tab32_adj, s));
    c->lam_device = true;
    c->dense_stale();   // rebuilt from the new tables before the next cycle
    return TMG_OK;
}

int tmg_set_dense_bottom(tmg_handle c, int on, tmg_stream stream)
{
    if (!c) return TMG_ERR_INVALID;
    // graphs captured with the other form are dropped
    const int rc = drain(c);
    if (rc) return rc;
    HIPCHK(c, hipStreamSynchronize((hipStream_t)stream));
    for (auto &kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
    c->dense_on = on != 0;
    c->dense_stale();
    return TMG_OK;
}

int tmg_set_active_set(tmg_handle c, int on)
{
    if (!c) return TMG_ERR_INVALID;
    c->act.enabled = on != 0;
    return TMG_OK;
}

int tmg_level_info(tmg_handle c, int j, int level, int64_t *n, double *alpha, double *omega)
{
    if (!c || j < 0 || j >= c->batch) return TMG_ERR_INVALID;
    if (level < 0 || level >= c->L[j]) return TMG_ERR_INVALID;
    std::vector<double> t(c->tab_stride);
    double a;
    const TabLayout TL(c->P);
    if (c->lam_device) {
        // lambda came from a device array: read the table the device built
        HIPCHK(c, hipDeviceSynchronize());
        HIPCHK(c, hipMemcpy(t.data(), tab_of(c, level, false) + (int64_t)j * c->tab_stride,
                            sizeof(double) * c->tab_stride, hipMemcpyDeviceToHost));
        a = t[TL.ALPHA()];
    } else {
        const double z = level_z(c->lam[j], c->T[j], c->N[j], level);
        a = build_level_table(c->P, z, c->opt.omega_mode, c->opt.omega, false, t.data());
    }
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
    const int H = c->rs(nsweep + 1);
    TileList *tl;
    if ((rc = get_tiles(c, level, rcout ? kHasNext : kAll, c->TO(H), s, &tl))) return rc;
    LegArgs a = leg_args(c, level, trans != 0, tl, H);
    a.f = f;
    a.u0 = fold_u0;
    a.u_in = u_in;
    a.u_out = u_out;
    a.rc = rcout;
    a.pre = nsweep;
    HIPCHK(c, launch_leg<double>(c->P, trans != 0, a, tl->ntiles, s));
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
    const int H = c->rs(nsweep);
    TileList *tl;
    if ((rc = get_tiles(c, level, e ? kHasNext : kAll, c->TO(H), s, &tl))) return rc;
    LegArgs a = leg_args(c, level, trans != 0, tl, H);
    a.f = f;
    a.u0 = fold_u0;
    a.u_in = u_in;
    a.e = e;
    a.u_out = u_out;
    a.post = nsweep;
    HIPCHK(c, launch_leg<double>(c->P, trans != 0, a, tl->ntiles, s));
    return TMG_OK;
}

int tmg_op_down32(tmg_handle c, int level, int trans, int nsweep, const float *f,
                  const float *u_in, float *u_out, float *rcout, tmg_stream stream)
{
    int rc = check_level_args(c, level);
    if (rc) return rc;
    if (!c->mixed) return TMG_ERR_UNSUPPORTED;
    if (!f || nsweep < 0 || nsweep > kMaxSweeps || (rcout && level + 1 >= c->Lmax))
        return TMG_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    const int H = c->rs(nsweep + 1);
    TileList *tl;
    if ((rc = get_tiles(c, level, rcout ? kHasNext : kAll, c->TO(H), s, &tl))) return rc;
    LegArgsT<float> a = leg_args<float>(c, level, trans != 0, tl, H);
    a.f = f;
    a.u_in = u_in;
    a.u_out = u_out;
    a.rc = rcout;
    a.pre = nsweep;
    HIPCHK(c, launch_leg<float>(c->P, trans != 0, a, tl->ntiles, s));
    return TMG_OK;
}

int tmg_op_up32(tmg_handle c, int level, int trans, int nsweep, const float *f,
                const float *u_in, const float *e, float *u_out, tmg_stream stream)
{
    int rc = check_level_args(c, level);
    if (rc) return rc;
    if (!c->mixed) return TMG_ERR_UNSUPPORTED;
    if (!f || !u_in || nsweep < 0 || nsweep > kMaxSweeps || (e && level + 1 >= c->Lmax))
        return TMG_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    const int H = c->rs(nsweep);
    TileList *tl;
    if ((rc = get_tiles(c, level, e ? kHasNext : kAll, c->TO(H), s, &tl))) return rc;
    LegArgsT<float> a = leg_args<float>(c, level, trans != 0, tl, H);
    a.f = f;
    a.u_in = u_in;
    a.e = e;
    a.u_out = u_out;
    a.post = nsweep;
    HIPCHK(c, launch_leg<float>(c->P, trans != 0, a, tl->ntiles, s));
    return TMG_OK;
}

int tmg_op_mix(tmg_handle c, int trans, const double *f, const double *fold_u0,
               const double *u_in, const float *e, double *u_out, float *rcout,
               tmg_stream stream)
{
    if (!c || !f || !u_in || !e || !u_out || !rcout || c->Lmax < 2 || (fold_u0 && trans))
        return TMG_ERR_INVALID;
    if (!c->mixed) return TMG_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    const int H = c->H_mix();
    TileList *tl;
    int rc = get_tiles(c, 0, kHasNext, c->TO(H), s, &tl);
    if (rc) return rc;
    MixArgs a{};
    a.f = f;
    a.u0 = fold_u0;
    a.u_in = u_in;
    a.e = e;
    a.u_out = u_out;
    a.rc = rcout;
    a.tab = tab_of(c, 0, trans != 0);
    a.tab32 = tabT_of<float>(c, 0, trans != 0);
    a.R32 = R_of<float>(c, trans != 0);
    a.slab_off = c->slab_off_d[0];
    a.cslab_off = c->slab_off_d[1];
    a.tile_off = tl->d_off;
    a.tile_inst = tl->d_inst;
    a.n0 = c->N[0];
    a.batch = c->batch;
    a.tab_stride = c->tab_stride;
    a.halo = H;
    a.tile_out = c->TO(H);
    a.pre = c->opt.nu1;
    a.post = c->opt.nu2;
    a.next = c->opt.nu1;
    a.up = 1;
    HIPCHK(c, launch_mix(c->P, trans != 0, a, tl->ntiles, s));
    return TMG_OK;
}

int tmg_op_fused(tmg_handle c, int trans, const double *f, const double *fold_u0,
                 const double *u_in, const double *e, double *u_out, double *rcout,
                 tmg_stream stream)
{
    if (!c || !f || !u_in || !e || !u_out || !rcout || c->Lmax < 2 || (fold_u0 && trans))
        return TMG_ERR_INVALID;
    if (c->generic) return TMG_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    const int H = c->H_fused();
    TileList *tl;
    int rc = get_tiles(c, 0, kHasNext, c->TO(H), s, &tl);
    if (rc) return rc;
    LegArgs a = leg_args(c, 0, trans != 0, tl, H);
    a.f = f;
    a.u0 = fold_u0;
    a.u_in = u_in;
    a.e = e;
    a.u_out = u_out;
    a.rc = rcout;
    a.pre = c->opt.nu1;
    a.post = c->opt.nu2;
    a.next = c->opt.nu1;
    HIPCHK(c, launch_leg<double>(c->P, trans != 0, a, tl->ntiles, s));
    return TMG_OK;
}

int tmg_op_fused2(tmg_handle c, int trans, const double *f, const double *fold_u0,
                  const double *u_in, const double *f1, const double *e2, double *u_out,
                  double *rcout, double *f2, tmg_stream stream)
{
    if (!c || !f || !u_in || !f1 || !e2 || !u_out || !rcout || c->Lmax < 3 || (fold_u0 && trans))
        return TMG_ERR_INVALID;
    if (c->generic) return TMG_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    const int H = c->H_fused2();
    TileList *tl;
    int rc = get_tiles(c, 0, kHasNext2, c->TO(H), s, &tl);
    if (rc) return rc;
    LegArgs a = leg_args(c, 0, trans != 0, tl, H);
    a.f = f;
    a.u0 = fold_u0;
    a.u_in = u_in;
    a.f1 = f1;
    a.e2 = e2;
    a.tab1 = tab_of(c, 1, trans != 0);
    a.tab1T = a.tab1;
    a.c2slab_off = c->slab_off_d[2];
    a.u_out = u_out;
    a.rc = rcout;
    a.f2 = f2;
    a.pre = c->opt.nu1;
    a.post = c->opt.nu2;
    a.next = c->opt.nu1;
    HIPCHK(c, launch_leg<double>(c->P, trans != 0, a, tl->ntiles, s));
    return TMG_OK;
}

int tmg_op_coarse_solve(tmg_handle c, int level, int trans, const double *r, double *e,
                        tmg_stream stream)
{
    int rc = check_level_args(c, level);
    if (rc) return rc;
    if (!r || !e) return TMG_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    auto it = c->op_coarse.find(level);
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
        it = c->op_coarse.emplace(level, std::make_pair(d, (int)list.size())).first;
    }
    CoarseArgs a{};
    a.r = r;
    a.e = e;
    a.generic = c->generic;
    a.periodic = c->opt.periodic;
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
    const int H = c->rs(1);
    TileList *tl;
    int rc = get_tiles(c, 0, kAll, c->TO(H), s, &tl);
    if (rc) return rc;
    if (tl->ntiles > c->partial_cap) return TMG_ERR_INVALID;
    LegArgs a = leg_args(c, 0, trans != 0, tl, H);
    a.f = f;
    a.u0 = fold_u0;
    a.u_in = u;
    a.norm_off = tl->d_off;
    a.partial = c->partial;
    HIPCHK(c, launch_leg<double>(c->P, trans != 0, a, tl->ntiles, s));
    HIPCHK(c, launch_finalize(c->partial, tl->d_off, c->batch, c->st_ops, c->ctl, nullptr, 1, s));
    HIPCHK(c, hipMemcpyAsync(c->st_host, c->st_ops, sizeof(InstState) * c->batch,
                             hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    for (int j = 0; j < c->batch; ++j) norms[j] = std::sqrt(c->st_host[j].r0sq);
    return TMG_OK;
}

}  // extern "C"
