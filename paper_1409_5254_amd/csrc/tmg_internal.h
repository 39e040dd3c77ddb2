// Internal declarations shared by the host driver (tmg_capi.cpp), the table
// builder (tmg_tables.cpp) and the HIP kernels (tmg_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tmg {

constexpr int kMaxP = 21;       // P = p + 1 coefficients per slab (degrees up to 20)
constexpr int kMaxTunedP = 6;   // the register-resident (tuned) kernels take P <= 6
// Work-group (and tile, one slab per thread) of the generic kernels, which
// take any P <= kMaxP and the time-periodic problem.
constexpr int kGenThreads = 256;
constexpr int kThreads = 256;   // work-group size of the scan and reduction kernels
// Work-group size of the streaming (tile) kernels.  Four wavefronts: one
// wavefront per work-group (barrier-free exchange) measured slower on the
// level-0 pass, whose halo share grows fourfold, and no faster on the small
// levels, whose time is launch and memory latency.
constexpr int kLegThreads = 256;
constexpr int kMaxSweeps = 8;
constexpr int64_t kMaxCoarse = 4096;
constexpr int kBottomThreads = 512;   // work-group of the bottom-of-hierarchy kernel

// Slabs held by one thread of a streaming kernel: 32-48 bytes per array and
// thread keeps the most loads in flight per byte on HBM3E.  With S = 1 the
// two fine slabs of a coarse slab sit in neighbouring lanes; otherwise S is
// even and they sit in the same thread.
constexpr int slabs_per_thread(int P) { return P == 1 ? 4 : 2; }
constexpr int tile_slabs(int P) { return kLegThreads * slabs_per_thread(P); }
// Slabs per thread of the bottom kernel (even), the largest level (slabs) it
// holds, and the most levels it can hold (log2(bottom_max) + 1).
constexpr int bottom_slabs(int P) { return P == 1 ? 8 : (P == 2 ? 4 : 2); }
// work-group of the bottom kernel's full form: half of kBottomThreads for
// P >= 5, whose levels would not fit the LDS otherwise
constexpr int bottom_threads(int P) { return P >= 5 ? kBottomThreads / 2 : kBottomThreads; }
constexpr int bottom_max(int P) { return bottom_threads(P) * bottom_slabs(P); }
// Largest level (slabs) of the generic kernels' bottom visit (k_gvisit):
// one slab per thread of kGenThreads, every level's right-hand side and
// iterate in LDS next to one level's table block and the transfer matrices.
constexpr int gbottom_max(int P) { return P <= 10 ? 256 : 128; }
constexpr int kBottomMaxLevels = 13;

// The entry point that allocates nothing (tmg_solve_noalloc) carves every
// device buffer of its solve out of one static device array of this size,
// and takes single instances of at most kNoAllocMaxUnknowns coefficients
// (about 32 bytes of hierarchy, halo and list memory per coefficient, plus
// tables and tile lists).
constexpr size_t kNoAllocScratchBytes = size_t(96) << 20;
constexpr int64_t kNoAllocMaxUnknowns = int64_t(1) << 21;

// Per-(instance, level) table block, doubles, for P coefficients per slab.
// Aop is the diagonal block of the operator (A = K + lambda M, or A^T for the
// transposed system); c the end-value functional (w = c^T u), v the
// injection vector (r = f + v w_left - Aop u).
struct TabLayout {
    int P;
    __host__ __device__ constexpr TabLayout(int P_) : P(P_) {}
    __host__ __device__ constexpr int A() const { return 0; }             // P*P  Aop
    __host__ __device__ constexpr int G() const { return P * P; }         // P*P  omega Aop^{-1}
    __host__ __device__ constexpr int H() const { return 2 * P * P; }     // P    omega Aop^{-1} v
    __host__ __device__ constexpr int C() const { return 2 * P * P + P; } // P    c
    __host__ __device__ constexpr int V() const { return 2 * P * P + 2 * P; } // P  v
    __host__ __device__ constexpr int Q() const { return 2 * P * P + 3 * P; } // P  Aop^{-1} v
    __host__ __device__ constexpr int AI() const { return 2 * P * P + 4 * P; } // P*P Aop^{-1}
    __host__ __device__ constexpr int OMC() const { return 3 * P * P + 4 * P; } // 1 - omega
    __host__ __device__ constexpr int ALPHA() const { return 3 * P * P + 4 * P + 1; }
    __host__ __device__ constexpr int stride() const { return ((3 * P * P + 4 * P + 2 + 3) / 4) * 4; }
};

// Per-instance solve state, written by the finalize kernels.
struct InstState {
    double r0sq;   // ||r_0||^2
    double rsq;    // ||r_k||^2 of the last completed cycle
    double prev_rsq; // ||r_{k-1}||^2 (k >= 2; else -1)
    int cycles;    // completed cycles
    int done;      // 0 running, 1 converged, 2 max cycles, 3 non-finite, 4 diverged
};

struct Control {
    double rtol2;  // rtol^2
    int max_cycles;
    int epoch;     // solve number (tags the host copies of the state)
};

// What the host needs to follow a solve without stopping the stream, in
// fine-grained pinned host memory (a HostHead, then a HostSum), written
// after each cycle: how many instances still run, and how many cycles to
// have queued (the largest count an instance reaches when it converges at
// the rate of its last two cycles).  For a single instance it holds that
// instance's state instead, from which the host works out the same (off the
// GPU's critical path).  begin and end are a sequence lock: the writer
// stores begin = V, the summary, then end = V, with V = epoch * 2^32 + n
// (n differs for every copy of a solve); a reader that finds
// end == begin == V after reading the summary has a consistent copy.
struct HostHead {
    long long begin;
    long long end;
};
struct HostSum {
    int running;   // batch: instances not finished
    int want;      // batch: cycles to have queued
    int cycles;    // single instance: its state; batch: the most cycles run
    int done;
    double r0sq;
    double rsq;
    double prev_rsq;
};
// Batches of at most kRunBits instances: after the HostSum, one bit per
// instance (bit j % 32 of word j / 32) that is set while it runs.
constexpr int kRunBits = 1 << 16;
__host__ __device__ inline int run_words(int batch) { return batch <= kRunBits ? (batch + 31) / 32 : 0; }

// Arguments of the streaming "leg" kernel (one level, all participating
// instances).  Logical slab m of an instance is physical slab N-1-m for the
// transposed system (backward in time).  In order, a leg:
//   loads f (u0 folded at level 0) and the iterate u_in (zero if null; the
//   left halo of a tile from halo_in if given),
//   runs `pre` sweeps, adds the prolongation of e (if e), runs `post` sweeps,
//   stores the tile's output slabs to u_out (and its last `halo` slabs to
//   halo_out), accumulates the squared residual (partial), and, if rc,
//   runs `next` sweeps and stores the restricted residual.
template <typename T>
struct LegArgsT {
    const T *f;
    const double *u0;        // fold values (level 0, forward) or null
    const T *u_in;           // null: zero initial guess
    const T *halo_in;        // null, or per-tile halo slabs written by the previous pass
    const T *e;              // null: no prolongation
    T *u_out;                // null: no store
    T *halo_out;             // null, or per-tile copy of the last `halo` output slabs
    T *rc;                   // null: no restriction
    double *partial;         // null: no residual norm
    const int64_t *norm_off; // [batch+1] partial-sum slots
    const double *tab;       // FP64 table blocks, instance j at tab + j*tab_stride
    const T *tabT;           // the same tables in T
    const T *R;              // R1T (P*P) then R2T (P*P), swapped for backward, in T
    const int64_t *slab_off; // [batch+1] slab offsets of this level
    const int64_t *cslab_off;// [batch+1] slab offsets of the next level
    const int64_t *tile_off; // [batch+1] tile offsets of this launch
    const int *tile_inst;    // [ntiles] instance of each tile (batch > 1)
    const InstState *st;     // per-instance early exit when st[j].done (may be null)
    // Two-level launches (levels l and l+1 of a V-cycle's first visits).
    // Up: with e2 != null the correction of level l+1 is not read from e but
    // computed in the tile as level l+1's up leg: pre sweeps from zero on
    // f1, prolongation of the level-(l+2) correction e2, post sweeps.
    // Down: with rc and f2 != null, level l+1's down leg (next sweeps from
    // zero on the restricted residual, residual) follows, restricted into f2.
    const T *f1;             // level-(l+1) right-hand side
    const T *e2;             // level-(l+2) correction (null: one-level up leg)
    T *f2;                   // level-(l+2) right-hand side (null: one-level down leg)
    const double *tab1;      // level-(l+1) tables (FP64 and in T)
    const T *tab1T;
    const int64_t *c2slab_off; // [batch+1] slab offsets of level l+2
    int64_t n0;              // slabs of instance 0 at this level (used when batch == 1)
    int batch;
    int generic;             // 1: the generic kernel (P > kMaxTunedP, or periodic)
    int periodic;            // 1: u(0) = u(T), slab -1 is slab N-1 (generic kernel only)
    int touch;               // 1: bring every table into the scalar cache at entry
    int tab_stride;
    int halo;                // left halo slabs per tile (even, a multiple of S)
    int tile_out;            // output slabs per tile
    int pre, post, next;     // sweep counts
    int norm_f;              // FP64 first visit at level 0: partial = |f|^2 per tile
                             // (u0 folded), the initial residual's norm; no early exit
};
using LegArgs = LegArgsT<double>;

// A span: the down legs (or the up legs) of up to kMaxSpan consecutive
// levels l .. l+K-1 of a V-cycle's first visits in one launch (see k_span).
// Instance j runs min(K, lb[j] - l) of them.  Level l+k's arrays and tables:
// f[k], x[k], slab_off[k], tab + k * tab_level.
constexpr int kMaxSpan = 4;
constexpr int kSpanThreads = 256;   // one slab of level l per thread
template <typename T>
struct SpanArgsT {
    T *f[kMaxSpan + 1];      // right-hand sides (down: f[0] read, f[1..K] written; up: read)
    T *x[kMaxSpan + 1];      // up: x[K_j] the correction from below (read), x[0] the result
    const int64_t *slab_off[kMaxSpan + 1];
    const double *tab;       // FP64 tables of level l (level l+k at + k * tab_level)
    const T *tabT;
    int64_t tab_level;
    const T *R;
    const int64_t *tile_off;
    const int *tile_inst;    // as in LegArgsT
    const InstState *st;
    const int *lb;           // [batch] first bottom-kernel level of each instance
    int64_t n0;              // slabs of instance 0 at level l (used when batch == 1)
    int batch, tab_stride, level, K, halo, tile_out, nu1, nu2;
    int up;                  // 0: down legs, 1: up legs
};

// Fused level-0 pass of the FP32-inner defect correction (k_mix).
struct MixArgs {
    const double *f;
    const double *u0;
    const double *u_in;      // FP64 iterate (null: zero)
    const double *halo_in;
    const float *e;          // inner correction of level 1
    double *u_out;
    double *halo_out;
    float *rc;               // inner restricted residual for level 1 (null: none)
    double *partial;
    const int64_t *norm_off;
    const double *tab;
    const float *tab32;
    const float *R32;
    const int64_t *slab_off;
    const int64_t *cslab_off;
    const int64_t *tile_off;
    const int *tile_inst;    // as in LegArgsT
    const InstState *st;
    // two-level pass (as in LegArgsT): level 1's inner up leg computed in the
    // tile from f1 and the level-2 inner correction e2 instead of reading e,
    // and level 1's next inner down leg restricted into f2
    const float *f1;
    const float *e2;
    float *f2;
    const double *tab1;      // level-1 tables, FP64 and FP32
    const float *tab1_32;
    const int64_t *c2slab_off; // [batch+1] slab offsets of level 2
    int64_t n0;
    int batch, tab_stride, halo, tile_out, pre, post, next;
    int up;                  // 1: residual, inner up leg and update before the rest
};

struct CoarseArgs {
    const double *r;
    const double *u0;        // fold values (level 0, forward) or null
    double *e;
    const double *tab;
    const double *R;         // transfer matrices (generic kernel's table staging)
    const int64_t *slab_off;
    const int *inst;         // participating instance ids, one work-group each
    const InstState *st;     // may be null
    int tab_stride;
    int generic, periodic;   // as in LegArgsT
};

// One multigrid visit of the levels `level` .. nlev[j]-1 of instance j per
// work-group (see k_bottom), all levels resident in LDS and computed in
// FP64; TIO is the type of the level's arrays in global memory.
template <typename TIO>
struct BottomArgsT {
    const TIO *f;            // right-hand side of level `level` (caller's f at level 0)
    const double *u0;        // fold values (level 0, forward) or null
    const TIO *x_in;         // initial guess at `level` (null: zero)
    TIO *x_out;              // result at `level` (may equal x_in)
    const int64_t *slab_off; // [batch+1] slab offsets of level `level`
    const double *tab;       // tables, block (l, j) at (l * batch + j) * tab_stride
    const double *R;
    const int *inst;         // instances handled, one work-group each
    const int *nlev;         // [batch] levels of each instance
    InstState *st;           // level 0: the work-group also finishes its instance's cycle
    const Control *ctl;
    HostHead *mirror;        // one instance: its host copy after such a cycle (else null)
    int level, batch, tab_stride, nu1, nu2, gamma;
    // With lbs: every instance at its own first bottom level lbs[j] (>= 1,
    // a V-cycle's first visit: x_in and u0 null), with that level's arrays
    // f_lv[l], x_lv[l] (the result) and slab offsets soff_lv[l]; f, x_out,
    // slab_off and level unused.
    const int *lbs;
    const TIO *const *f_lv;
    TIO *const *x_lv;
    const int64_t *const *soff_lv;
    // 1: every instance's first bottom level has at most 64 * bottom_slabs
    // slabs (one wavefront holds it): one-wavefront work-groups
    int small;
    int generic, periodic;   // as in LegArgsT (the generic kernel solves its level exactly)
    int visit;               // generic: the bottom spans several levels (k_gvisit)
};
using BottomArgs = BottomArgsT<double>;

// Host-side launchers (tmg_kernels.hip).  `backward` selects the transposed
// system's backward-in-time indexing.  Return hipSuccess or the launch error.
template <typename T>
hipError_t launch_leg(int P, bool backward, const LegArgsT<T> &a, int64_t ntiles, hipStream_t s);
hipError_t launch_mix(int P, bool backward, const MixArgs &a, int64_t ntiles, hipStream_t s);
template <typename T>
hipError_t launch_span(int P, bool backward, const SpanArgsT<T> &a, int64_t ntiles, hipStream_t s);
hipError_t launch_coarse(int P, bool backward, const CoarseArgs &a, int ninst, hipStream_t s);
// The generic kernels (tmg_generic.h) for any P <= kMaxP; launch_leg,
// launch_bottom and launch_coarse route to them when the arguments say so.
hipError_t launch_gleg(int P, bool backward, const LegArgsT<double> &a, int64_t ntiles,
                       hipStream_t s);
hipError_t launch_gbottom(int P, bool backward, const BottomArgsT<double> &a, int ninst,
                          hipStream_t s);
template <typename TIO>
hipError_t launch_bottom(int P, bool backward, const BottomArgsT<TIO> &a, int ninst, hipStream_t s);

// The gamma visits of a W-cycle's bottom level (one instance, forward, from
// zero) are one linear map of that level's right-hand side: D, n x n with
// n = N P, row-major over the level's unknowns (slab-major).  Its columns
// are the bottom kernel's visits of the unit loads (tmg_bottom.hip); the
// cycle then applies D instead of repeating the recursion below the level.
constexpr int64_t kDenseMaxN = 4096;   // unknowns of the level (D: 128 MiB)
struct DenseColArgs {
    const double *tab;   // the instance's tables: level l at tab + l * tab_level
    const double *R;     // R_1^T, R_2^T
    double *D;           // [n][n]
    int64_t N;           // slabs of level `level` (at most the bottom kernel's)
    int64_t tab_level;
    int level, Lc, nu1, nu2, gamma;   // Lc: the coarsest level
    int backward;   // the transposed system (backward in time; tables and
                    // transfers of the adjoint), D over physical slab order
    int periodic;   // the time-periodic problem (generic kernels only)
};
template <int PP>
hipError_t launch_dense_cols_p(const DenseColArgs &a, hipStream_t s);
hipError_t launch_dense_cols(int P, const DenseColArgs &a, hipStream_t s);
// the same on the generic kernels (k_gvisit's visits; any P <= kMaxP)
template <int PP>
hipError_t launch_gdense_cols_p(const DenseColArgs &a, hipStream_t s);
hipError_t launch_gdense_cols(int P, const DenseColArgs &a, hipStream_t s);
// Row i's window [win[2i], win[2i+1]): the columns from its first to its
// last entry of magnitude above 2^-64 times the row's largest (the start
// rounded down to even; every column if the row holds a non-finite entry).
// The entries outside sum to at most n 2^-64 max_j |D_ij| ||r||_inf, at most
// two units of FP64 rounding of the row's largest product for n <= 4096,
// so the product leaves them out (the operator decays away from its
// diagonal: slabs many decay lengths apart barely couple).
constexpr int kDenseDropExp = -64;
hipError_t launch_dense_window(const double *D, int64_t n, int *win, hipStream_t s);
// *wmax (device) = the widest span of columns a work-group of the product
// loads, over nop operators of n rows (their windows in win, in turn).
hipError_t launch_dense_window_max(const int *win, int64_t n, int nop, int *wmax, hipStream_t s);
// x = D r over the rows' windows (nothing when *st says finished); width:
// launch_dense_window_max's span (n when unknown), which sets the passes
// and the form (one row per wavefront up to 512 columns).
hipError_t launch_dense_apply(const double *D, const int *win, const double *r, double *x,
                              int64_t n, const InstState *st, hipStream_t s, int64_t width);
// nop such products at once: operator y (D + y n^2, win + 2 y n) on
// r + y n into x + y n.
hipError_t launch_dense_apply_batch(const double *D, const int *win, const double *r, double *x,
                                    int64_t n, int nop, hipStream_t s, int64_t width);
// out = Q in for Q [nx][nx] and in, out [nx][n] (row-major).
hipError_t launch_mode_transform(const double *Q, const double *in, double *out, int nx,
                                 int64_t n, hipStream_t s);

// Level-0 halo slots of a tile list (tile_out output slabs and `halo` halo
// slabs per tile) from the iterate u, as the level-0 pass stores them.
hipError_t launch_seed(int P, bool backward, const double *u, double *hb, const int64_t *tile_off,
                       const int *tile_inst, const int64_t *slab_off, int batch, int64_t n0,
                       int tile_out, int halo, int64_t ntiles, hipStream_t s);
hipError_t launch_norm_f(int P, const double *f, const double *u0, const double *tab,
                         int tab_stride, const int64_t *slab_off, const int64_t *tile_off,
                         const int *tile_inst, int batch, double *partial, int64_t ntiles,
                         hipStream_t s);
// With ctl_set (is_r0 only) the launch also writes *val to ctl_set and uses
// it instead of ctl.
hipError_t launch_finalize(const double *partial, const int64_t *norm_off, int batch,
                           InstState *st, const Control *ctl, HostHead *mirror, int is_r0,
                           hipStream_t s, Control *ctl_set = nullptr,
                           const Control *val = nullptr);
// Writes the summary of st[0 .. batch) into the host copy (count: the copies
// made so far).
hipError_t launch_publish(const InstState *st, int batch, const Control *ctl, HostHead *mirror,
                          unsigned *count, hipStream_t s);
// out[2j] = -sum_n z_n^T M_tau u_n, out[2j+1] = v^T z_1 (tau[j]: fine slab length),
// over a level-0 tile list of kLegThreads * S slabs per tile (partial: one
// slot per tile).
hipError_t launch_grad(int P, const double *u, const double *z, const double *tau,
                       const int64_t *slab_off, const int64_t *tile_off, const int *tile_inst,
                       int64_t ntiles, int batch, double *partial, double *out, hipStream_t s);
// Rebuilds the table blocks of every level and instance from lambda (device).
hipError_t launch_set_tables(int P, const double *lam, const double *T, const int64_t *N,
                             const int *nlev, int batch, int Lmax, int omega_mode, double omega,
                             int stride, double *tab_fwd, double *tab_adj, float *t32f,
                             float *t32a, hipStream_t s);

// Device address of the static scratch array on the current device (looked
// up once per device), and its size in bytes.
hipError_t noalloc_scratch(void **ptr, size_t *bytes);

// Host table builder (tmg_tables.cpp).  Fills one table block for a slab of
// step z = lambda*tau (operator K + z diag(1/(2k+1))), transposed if trans.
// omega_mode 0: optimal damping; 1: omega_fixed.  Returns alpha.
double build_level_table(int P, double z, int omega_mode, double omega_fixed, bool trans,
                         double *out);
// R1T, R2T (P*P each, row-major) of the factor-2 transfer.
void build_transfer(int P, double *R1T, double *R2T);

}  // namespace tmg
