/*
 * tmg.h -- C ABI of the MI355X (gfx950) time-multigrid library for
 * discontinuous-Galerkin-in-time discretisations of
 *
 *     u'(t) + lambda u(t) = f(t),  t in (0, T],   u(0) = u0,   lambda > 0
 *
 * following Gander & Neumueller, "Analysis of a time multigrid algorithm for
 * DG-discretizations in time" (arXiv:1409.5254).  The paper's model problem
 * (section 1, eq. chap4_ordinaryDGL) has lambda = 1; the discrete operator
 * depends on lambda and the slab length tau only through z = lambda*tau, so
 * every statement of the paper carries over with tau -> lambda*tau.
 *
 * Discretisation (section 2): N uniform slabs of length tau = T/N, degree-p
 * polynomials on each slab in the Legendre basis psi_k(t) = P_k(xi),
 * xi = 2(t - t_{n-1})/tau - 1, k = 0..p (P = p+1 coefficients per slab).
 * The block lower-bidiagonal system (eq. chap4_generalLinearSystemODE) is
 *     (K + lambda M) u_n - N u_{n-1} = f_n,   n = 1..N,
 * K[k,l] = 1 - 2[l < k, k+l odd], M = tau diag(1/(2k+1)), N = v 1^T with
 * v[k] = (-1)^k; the initial value enters slab 1 as f_1 += u0 v.
 *
 * Multigrid (section 3): nu1 / nu2 damped block Jacobi sweeps
 * (eq. chap4_ODESmoother) with the per-level optimal damping of Lemma
 * chap4_lemma7, factor-2 restriction / prolongation (eqs.
 * chap4_restrictionTime, chap4_prolongationTime), coarse operators
 * rediscretised at 2 tau, applied recursively as a V (gamma = 1) or W
 * (gamma = 2) cycle down to n_coarse slabs, where the system is solved
 * exactly by a parallel prefix scan over the per-slab affine maps of the end
 * values.  Iteration stops at ||f - L u||_2 <= rtol ||f - L 0||_2 per
 * instance (the residual-reduction criterion of section 4.2).
 *
 * DATA LAYOUT.  Every solution / right-hand-side array is float64, on the
 * device, contiguous, [instance][slab][k]: coefficient k of slab n of
 * instance j at  off_j + n*P + k,  off_j = P * sum_{i<j} N_i  (int64).
 * Load vectors f hold f_n[k] = int f(t) psi_k(t) dt over slab n WITHOUT the
 * initial value (the library folds u0).  u0, lambda, T and per-instance
 * outputs are arrays of length `batch`.
 *
 * OWNERSHIP.  The caller owns every array passed in; the library never frees
 * or retains them beyond the call (graphs captured for a set of pointers are
 * re-captured when the pointers change).  The handle owns its tables,
 * hierarchy buffers, graphs and streams.  Every call is ordered on the given
 * stream (a hipStream_t; NULL = the default stream).  tmg_solve and
 * tmg_adjoint_solve return once every instance's outcome is known: the
 * device copies each instance's state into pinned host memory after every
 * cycle and the host follows it there while the stream runs.  Their result
 * is complete in stream order (work enqueued later on the stream sees it;
 * host reads need a synchronisation of the stream); cycles queued past
 * convergence may still be in the stream and change nothing.
 * tmg_vcycle and the tmg_op_* calls are asynchronous.  A handle must not be
 * used from two host threads at once.
 *
 * ERRORS.  0 = TMG_OK; TMG_NOT_CONVERGED (> 0) when max_cycles was reached
 * (outputs valid, relres reports how far it got); negative codes are errors
 * and leave outputs unspecified.  Argument checks run on the host before any
 * device work.
 */
#ifndef TMG_H
#define TMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tmg_ctx *tmg_handle;
typedef void *tmg_stream; /* hipStream_t */

enum {
    TMG_OK = 0,
    TMG_NOT_CONVERGED = 1,
    TMG_ERR_INVALID = -1,     /* null pointer, batch < 1, bad option value        */
    TMG_ERR_SIZE = -2,        /* N_j not n_coarse * 2^k, or too large              */
    TMG_ERR_OMEGA = -3,       /* fixed omega outside (0, 1]                        */
    TMG_ERR_PARAM = -4,       /* lambda or T not finite and > 0                    */
    TMG_ERR_OOM = -5,         /* device allocation failed                          */
    TMG_ERR_HIP = -6,         /* a HIP call failed (see tmg_last_hip_error)        */
    TMG_ERR_NONFINITE = -7,   /* NaN / Inf in the data or the residual             */
    TMG_ERR_DIVERGED = -8,    /* residual grew beyond 1e3 * initial residual       */
    TMG_ERR_UNSUPPORTED = -9, /* option combination not built into the library    */
    TMG_ERR_INTERNAL = -10    /* the library's own solve state is inconsistent (a bug) */
};

typedef struct {
    int p;            /* DG degree, 0 <= p <= TMG_MAX_DEGREE                        */
    int nu1, nu2;     /* pre / post smoothing sweeps, 0..8 (default 2, 2)           */
    int gamma;        /* 1 = V-cycle, 2 = W-cycle                                   */
    int64_t n_coarse; /* coarsest slab count, 1..4096 (default 2)                   */
    int omega_mode;   /* 0 = optimal per level (Lemma chap4_lemma7), 1 = fixed      */
    double omega;     /* damping when omega_mode == 1, in (0, 1]                    */
    int precision;    /* 0 = FP64; 1 = FP32 smoothing / transfers, FP64 residual,
                         FP64 coarsest scan, FP64 outer defect correction          */
    int schedule;     /* kernel schedule id, -1 = library default                   */
    int periodic;     /* 0 = initial-value problem u(0) = u0; 1 = time-periodic
                         u(0) = u(T) (section 3, eq. chap4_periodicBC: the block
                         system with the circulant coupling of eq.
                         chap4_circulantMatrix; u0 is ignored, the coarsest
                         level is solved by the cyclic affine recurrence)       */
} tmg_options;

/* Degrees 0 .. 5 run on register-resident tuned kernels; degrees 6 .. 20, and
 * every periodic problem, on generic kernels (one slab per thread, operators
 * in LDS, FP64 only; the levels above the bottom stream in one-level legs,
 * and one work-group visits the levels of at most 256 slabs for p <= 9, 128
 * above, as the bottom cap allows). */
#define TMG_MAX_DEGREE 20
#define TMG_MAX_TUNED_DEGREE 5

/* Fill *opt with the defaults: p = 1, nu1 = nu2 = 2, V-cycle, n_coarse = 2,
 * optimal damping, FP64, default schedule, initial-value problem. */
void tmg_default_options(tmg_options *opt);

/*
 * Build a solver for `batch` independent instances; instance j has
 * n_slabs[j] slabs on (0, T[j]] and decay rate lambda[j] (host arrays of
 * length batch).  Every n_slabs[j] must equal opt->n_coarse * 2^k (k >= 0).
 * Computes the per-level tables (section 2.1 matrices, alpha = the nonzero
 * eigenvalue of (K + lambda M)^{-1} N per Lemma chap4_theorem2, damping per
 * Lemma chap4_lemma7, transfer matrices R_i^T = M^{-1} Mt^i of section 4.2),
 * allocates the hierarchy (about 2x the fine-level size per array) and
 * uploads everything on stream s.  On success *h owns all device memory.
 */
int tmg_setup(tmg_handle *h, int batch, const int64_t *n_slabs, const double *T,
              const double *lambda, const tmg_options *opt, tmg_stream s);

/*
 * One multigrid cycle in place: u (device, in/out) is the initial guess and
 * receives the result; f the load vectors, u0 the initial values (device,
 * length batch).  The cycle of eq. chap4_errorTwoGridCycle applied
 * recursively.  Asynchronous on s.
 */
int tmg_vcycle(tmg_handle h, const double *f, const double *u0, double *u, tmg_stream s);

/*
 * Solve L u = f from u = 0 with repeated cycles until every instance reaches
 * ||f - L u||_2 <= rtol ||f||_2 (u0 folded) or max_cycles.  cycles[batch]
 * and relres[batch] (host, may be NULL) receive per-instance counts and
 * final relative residuals.  Returns once every instance has finished (see
 * the stream note above): TMG_OK,
 * TMG_NOT_CONVERGED, TMG_ERR_NONFINITE or TMG_ERR_DIVERGED (the worst
 * instance decides).
 */
int tmg_solve(tmg_handle h, const double *f, const double *u0, double *u, double rtol,
              int max_cycles, int *cycles, double *relres, tmg_stream s);

/*
 * Adjoint solve: L^T z = g (device arrays, same layout) backward in time,
 * (L^T z)_n = A^T z_n - 1 (v^T z_{n+1}), by the same multigrid cycle applied
 * to L^T (transposed block Jacobi, the same R and P, backward scan on the
 * coarsest level), from z = 0 to ||g - L^T z|| <= rtol ||g||.  If u
 * (the forward solution, device) is not NULL, also returns for each instance
 *   dlambda[j] = -sum_n z_n^T M_tau u_n   and   du0[j] = v^T z_1
 * (host arrays, may be NULL): the gradients of a loss J(u) with dJ/du = g
 * with respect to lambda and u0; dJ/df = z itself.  Returns as tmg_solve
 * does; blocks until done when gradients are asked for.
 */
int tmg_adjoint_solve(tmg_handle h, const double *g, const double *u, double *z, double rtol,
                      int max_cycles, double *dlambda, double *du0, int *cycles,
                      double *relres, tmg_stream s);

/*
 * Schedule autotuner.  Installs in h the fastest of a few schedules, timed on
 * this hardware with the caller's data: for each candidate it runs four
 * cycles of the solve of L u = f (u0 folded) and keeps the fastest of
 * three runs timed with HIP events.  A schedule is the size up to which an
 * instance's levels run inside the single-work-group bottom kernel
 * (bottom_cap, the largest the bottom kernel holds divided by 1, 2, ...,
 * 32) and whether consecutive levels share two-level launches (V-cycles;
 * for the W-cycle of one instance in FP64, pairs also fuses each level's
 * up leg between its two visits with the next visit's down leg, and each
 * first visit's down leg with the launch before it: the same iterates to
 * the last bit, half the launches), and whether the levels
 * after the first `span_after` streaming levels below level 1 (in pairs, an
 * odd one out alone) run in spans of `span` levels per launch (3 or 4; 0:
 * no spans; V-cycles only), chosen in that order, then the caps next to
 * the chosen one again with the chosen launch pattern; then, for the
 * fastest of those, whether the cycles after the first of a solve are launched kernel
 * by kernel instead of as captured graphs (a graph launch idles the GPU for
 * several microseconds; direct launches pay when the host enqueues a cycle
 * faster than the GPU runs it), the caps next to the pick timed again in
 * that mode.  The solution is the same under every
 * schedule (up to rounding order); only the kernel split and launch mode
 * change.  u (device, same layout as f) is used as scratch and overwritten.
 * *bottom_cap, *pairs, *span, *span_after and *direct (host, may be NULL)
 * receive the choice.  Blocks until done.
 */
int tmg_autotune(tmg_handle h, const double *f, const double *u0, double *u, int64_t *bottom_cap,
                 int *pairs, int *span, int *span_after, int *direct, tmg_stream s);

/*
 * Install a schedule (as chosen by tmg_autotune, e.g. on another handle of
 * the same shape) without timing anything: bottom_cap in [n_coarse, the
 * largest level the bottom kernel holds], pairs, span, span_after and
 * direct as there.  Returns TMG_ERR_INVALID for a bottom_cap out of that
 * range, or a span other than 0 without pairs, for a W-cycle, too deep for
 * the halo the sweep counts need, or with span_after < 1.  Blocks until
 * done.
 */
int tmg_set_schedule(tmg_handle h, int64_t bottom_cap, int pairs, int span, int span_after,
                     int direct, tmg_stream s);

/*
 * New decay rates for the instances of h: lambda is a DEVICE array of length
 * batch (e.g. a learnable parameter).  The per-level tables (section 2.1
 * matrices with z = lambda tau, alpha and the damping of Lemma
 * chap4_lemma7, as tmg_setup builds them, to the same bits) are rebuilt by a
 * kernel on stream s, so nothing is read back to the host and no buffer,
 * schedule or graph is rebuilt (a W-cycle's dense bottom operator, see
 * tmg_set_dense_bottom, is recomputed from the new tables by kernels before
 * the next cycle, in place).  Later calls on h see the new tables in
 * stream order (work on another stream must be ordered after s by the
 * caller).  A lambda that is not finite and positive leaves non-finite
 * tables: the next solve then returns TMG_ERR_NONFINITE.  Returns
 * TMG_ERR_INVALID for a null handle or array.
 */
int tmg_set_lambda(tmg_handle h, const double *lambda, tmg_stream s);

/*
 * Active sets of a batch (on by default; a single instance has none).  Once
 * the running instances of a batch hold at most three quarters of its
 * level-0 tiles, the later cycles of a solve launch work-groups for their
 * tiles only, and are launched kernel by kernel; the lists are rebuilt each
 * time that share drops by as much again.  Results are bitwise the same
 * with it on or off: an instance's tiles and every reduction over them are
 * the same, and the cycles after an instance finished leave it untouched
 * either way.  With it on, fewer cycles are queued ahead of the last one
 * the host has seen finish.  Batches above 65536 instances never use it.
 * Returns TMG_ERR_INVALID for a null handle.
 */
int tmg_set_active_set(tmg_handle h, int on);

/*
 * The bottom level's visits as one dense operator (on by default).  The
 * gamma visits of a level that the cycle's recursion makes from a zero
 * iterate (the recursion of eq. chap4_errorTwoGridCycle, section 3, applied
 * below that level, with the exact solve on the coarsest; one visit for a
 * V-cycle, two for a W-cycle) form one fixed linear map of that level's
 * right-hand side.  Where it applies (one instance, FP64, solves, adjoint
 * solves (the transposed system's own operator) and cycles, a bottom level
 * strictly between level 0 and the coarsest with
 * at most 4096 unknowns, which every bottom_cap of tmg_set_schedule gives) the
 * library builds the map's matrix once per schedule and set of tables
 * (n x n doubles, n = slabs x (p + 1), at most 128 MiB of device memory;
 * one bottom-kernel visit per unit load, before the first cycle that uses
 * it) and applies it at each visit instead of the recursion.  The map
 * decays away from its diagonal (slabs many decay lengths apart barely
 * couple), so each row's product covers only the columns from its first to
 * its last entry above 2^-64 times the row's largest magnitude: the entries
 * left out contribute at most n 2^-64 max_j |D_ij| max_j |r_j|, two units
 * of FP64 rounding of the row's largest product.  The result is the same
 * cycle up to rounding (the product also sums in another order than the
 * recursion).  on = 0 runs the recursion at every visit.  Drops the graphs
 * captured so far (waits for the handle's queued work and for stream s).
 * Returns TMG_ERR_INVALID for a null handle.
 */
int tmg_set_dense_bottom(tmg_handle h, int on, tmg_stream s);

/*
 * For callers that cannot allocate device memory (code that must not call
 * hipMalloc: tight serving loops, harnesses that forbid allocation): the
 * solve of tmg_solve for ONE instance (n_slabs slabs on (0, T], decay rate
 * lambda, options *opt) without a handle.  Every buffer the solve's kernels
 * need beyond f, u0 and u (level hierarchy, tables, tile lists, halo slots,
 * norm partials, state) is carved out of a static device array of the
 * library (TMG_NOALLOC_SCRATCH_BYTES per device, held from the library's
 * load to the end of the process).  The call allocates no device or pinned
 * host memory and creates no streams, events or graphs; it rebuilds the
 * tables and schedule (default schedule, cycles launched kernel by kernel;
 * a W-cycle's bottom visits run the recursion, without the dense operator
 * of tmg_set_dense_bottom) on every call, and it blocks until the solve is
 * done.
 * f, u0 (length 1) and u are device arrays as for tmg_solve; cycles and
 * relres (host, may be NULL) receive one value each.  Returns as tmg_solve,
 * or TMG_ERR_SIZE when n_slabs * (p + 1) exceeds TMG_NOALLOC_MAX_UNKNOWNS.
 * Every call on one device shares that device's array and keeps the last
 * call's contents there: calls that overlap on one device (other host
 * threads, or work queued on several streams at once) race and must be
 * serialised by the caller.
 */
#define TMG_NOALLOC_SCRATCH_BYTES (96u << 20)
#define TMG_NOALLOC_MAX_UNKNOWNS (1 << 21)
int tmg_solve_noalloc(int64_t n_slabs, double T, double lambda, const tmg_options *opt,
                      const double *f, const double *u0, double *u, double rtol, int max_cycles,
                      int *cycles, double *relres, tmg_stream s);

/* Release every resource of h (synchronises its streams first). */
int tmg_destroy(tmg_handle h);

/* Static, NUL-terminated description of a status code. */
const char *tmg_error_string(int code);

/* The last hipError_t seen by h (0 if none). */
int tmg_last_hip_error(tmg_handle h);

/* ------------------------------------------------------------------------
 * Level-wise entry points: the individual kernels of one cycle, on all
 * instances of h at hierarchy level `level` (0 = finest).  Arrays are device
 * arrays laid out like the level: [instance][slab][k] with instance j holding
 * n_slabs[j] >> level slabs (instances whose hierarchy is shorter are
 * skipped).  `trans` = 1 selects the transposed (adjoint, backward-in-time)
 * operator.  Used for kernel-by-kernel verification and timing; all are
 * asynchronous on s.
 * --------------------------------------------------------------------- */

/* Number of levels of instance j (level 0 .. n-1), its slab count and
 * the alpha / omega used there; returns the level count or an error. */
int tmg_level_info(tmg_handle h, int j, int level, int64_t *n_slabs, double *alpha,
                   double *omega);

/* Total coefficients (sum over instances of (n_slabs[j] >> level) * P). */
int64_t tmg_level_size(tmg_handle h, int level);

/*
 * Down leg: nsweep damped block Jacobi sweeps u_out = S^nsweep u_in for
 * L_level u = f (u_in == NULL: zero initial guess), then the residual
 * r = f - L u_out and its restriction rc = R r (eq. chap4_restrictionTime)
 * into the next level's layout (rc may be NULL to skip).  If fold_u0 != NULL
 * (level 0 only), the initial values are folded into slab 1 of f on the fly.
 */
int tmg_op_down(tmg_handle h, int level, int trans, int nsweep, const double *f,
                const double *fold_u0, const double *u_in, double *u_out, double *rc,
                tmg_stream s);

/*
 * Up leg: u_out = S^nsweep (u_in + P e) (eq. chap4_prolongationTime) with e
 * in the next level's layout; fold_u0 as for tmg_op_down.
 */
int tmg_op_up(tmg_handle h, int level, int trans, int nsweep, const double *f,
              const double *fold_u0, const double *u_in, const double *e, double *u_out,
              tmg_stream s);

/*
 * The fused level-0 pass of a cycle (forward or transposed): starting from
 * u_in, nu1 damped block Jacobi sweeps (recomputing the pre-smoothing), the
 * correction u += P e with e in level 1's layout, nu2 sweeps -> u_out; then,
 * continuing from u_out, nu1 sweeps of the next cycle, the residual and its
 * restriction -> rc (level 1's layout).  This is the pass every cycle after
 * the first runs at level 0 (there with u updated in place).  u_in and u_out
 * must not overlap.  fold_u0 as for tmg_op_down.
 */
int tmg_op_fused(tmg_handle h, int trans, const double *f, const double *fold_u0,
                 const double *u_in, const double *e, double *u_out, double *rc, tmg_stream s);

/*
 * The two-level form of the fused level-0 pass that V-cycle solves in FP64
 * run for instances whose level 1 is a streaming level: level 1's correction
 * is not read but computed tile by tile as level 1's up leg of a first visit
 * (nu1 sweeps from zero on f1, the correction u1 += P e2 with e2 in level
 * 2's layout, nu2 sweeps; eqs. chap4_ODESmoother, chap4_prolongationTime),
 * then the level-0 work of tmg_op_fused, which writes level 1's next
 * right-hand side rc.  If f2 != NULL, level 1's next down leg follows in the
 * same tiles (nu1 sweeps from zero on rc, residual, restriction; eq.
 * chap4_restrictionTime) into f2 (level 2's layout).  f1 is level 1's
 * right-hand side, e2 level 2's correction; instances with fewer than three
 * levels are skipped.  u_in and u_out must not overlap, nor f1 and rc;
 * fold_u0 as for tmg_op_down.
 */
int tmg_op_fused2(tmg_handle h, int trans, const double *f, const double *fold_u0,
                  const double *u_in, const double *f1, const double *e2, double *u_out,
                  double *rc, double *f2, tmg_stream s);

/*
 * The reduced-precision kernels of the FP32-inner defect correction
 * (precision = 1 handles only; TMG_ERR_UNSUPPORTED otherwise), for
 * verification against FP64: the down and up legs of tmg_op_down /
 * tmg_op_up with float arrays (FP32 storage and sweeps, the residual in
 * FP64 arithmetic from the FP32 operands, FP32 transfers), and the level-0
 * pass of an outer iteration (k_mix): r = f - L u_in in FP64, rounded to
 * FP32; the inner up leg on L e = r (nu1 sweeps from zero, the correction
 * P e with e in level 1's layout, nu2 sweeps, FP32); u_out = u_in + e_inner
 * in FP64; then the next inner down leg from u_out (r' = f - L u_out in FP64
 * rounded to FP32, nu1 FP32 sweeps from zero, inner residual in FP64
 * arithmetic, FP32 restriction) into rc (level 1's layout).  u_in and u_out
 * must not overlap.  fold_u0 as for tmg_op_down (level 0, forward).
 */
int tmg_op_down32(tmg_handle h, int level, int trans, int nsweep, const float *f,
                  const float *u_in, float *u_out, float *rc, tmg_stream s);
int tmg_op_up32(tmg_handle h, int level, int trans, int nsweep, const float *f,
                const float *u_in, const float *e, float *u_out, tmg_stream s);
int tmg_op_mix(tmg_handle h, int trans, const double *f, const double *fold_u0,
               const double *u_in, const float *e, double *u_out, float *rc, tmg_stream s);

/* Exact solve L_level e = r on every instance by the parallel affine prefix
 * scan (forward in time; backward for trans = 1).  Requires
 * n_slabs[j] >> level <= 4096. */
int tmg_op_coarse_solve(tmg_handle h, int level, int trans, const double *r, double *e,
                        tmg_stream s);

/* Per-instance residual norms ||f - L u||_2 at level 0 (host output array of
 * length batch; blocks).  fold_u0 as above. */
int tmg_op_residual_norm(tmg_handle h, int trans, const double *f, const double *fold_u0,
                         const double *u, double *norms, tmg_stream s);

/* ------------------------------------------------------------------------
 * Space-time heat equation (the paper's closing section: the time multigrid
 * applied to u_t = u_xx + f, with the spatial problem solved inside every
 * block Jacobi step).
 *
 *     u_t - u_xx = f  on (0,1) x (0,T],   u(0,t) = u(1,t) = 0,   u(x,0) = u0(x),
 *
 * second-order finite differences on nx interior points x_i = i h,
 * h = 1/(nx+1), and at every point the DG-in-time discretisation of the
 * header's first part (N slabs of degree p).  The slab block couples the
 * points of a slab, I (x) K + L_h (x) M with L_h = tridiag(-1, 2, -1)/h^2;
 * the cycle is that of section 3 (block Jacobi over whole slabs, each block
 * solved exactly by block elimination over the points; factor-2 transfers
 * in time at every point; the coarse operator rediscretised at 2 tau on the
 * same spatial grid; forward substitution on the coarsest level).  Damping:
 * omega_mode 0 takes Lemma chap4_lemma7's value at the smallest eigenvalue
 * of L_h (the slowest spatial mode) per level, 1 the fixed opt->omega.
 *
 * LAYOUT.  f and u are device arrays [point][slab][k]: coefficient k of
 * slab n at point i at (i*N + n)*P + k; f holds the load vectors at every
 * point without the initial value; u0 is a device array of nx values.
 * Options used: p (0 .. TMG_MAX_TUNED_DEGREE), nu1, nu2, gamma, n_coarse,
 * omega_mode, omega; precision and periodic must be 0.  N must be
 * n_coarse * 2^k with k >= 1.  Errors as above; calls are ordered on s and
 * tmg_heat_solve blocks (it reads the residual norm after every cycle).
 * --------------------------------------------------------------------- */
typedef struct tmg_heat_ctx *tmg_heat_handle;
#define TMG_HEAT_MAX_POINTS 4096

int tmg_heat_setup(tmg_heat_handle *h, int64_t n_slabs, int nx, double T,
                   const tmg_options *opt, tmg_stream s);
/* One cycle in place on u (the initial guess). */
int tmg_heat_vcycle(tmg_heat_handle h, const double *f, const double *u0, double *u,
                    tmg_stream s);
/* Solve from u = 0 to ||f - L u||_2 <= rtol ||f||_2 (u0 folded) or max_cycles. */
int tmg_heat_solve(tmg_heat_handle h, const double *f, const double *u0, double *u, double rtol,
                   int max_cycles, int *cycles, double *relres, tmg_stream s);
int tmg_heat_destroy(tmg_heat_handle h);
int tmg_heat_last_hip_error(tmg_heat_handle h);
/*
 * The coarse levels by sine modes (on by default).  The cycle acts on each
 * eigenvector of L_h separately: the slab block I (x) K + L_h (x) M, the
 * residual and the transfers in time are all diagonal in them.  Mode k
 * (eigenvalue 4 sin^2(pi k h/2)/h^2) follows the scalar problem of the
 * header's first part with that lambda and this cycle's damping.  So the
 * visits of the first level of at most 256 slabs above the coarsest (the
 * per-mode operators within 1 GiB of device memory) are: the orthonormal
 * sine transform over the points, for each mode the scalar problem's
 * visit operator (tabulated at setup, as by tmg_set_dense_bottom), and the
 * inverse transform.  That is the same cycle up to rounding, and replaces
 * every level below with three launches.  on = 0 runs those levels' legs.
 * Returns TMG_ERR_INVALID for a null handle.
 */
int tmg_heat_set_mode_solve(tmg_heat_handle h, int on);

#ifdef __cplusplus
}
#endif

#endif /* TMG_H */
