/*
 * FP64 CPU oracle for the time-multigrid solve of DG-in-time discretisations
 * of u' + lambda*u = f on (0,T], u(0) = u0 (Gander & Neumueller, "Analysis of
 * a time multigrid algorithm for DG-discretizations in time", SIAM preprint,
 * arXiv:1409.5254).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this file.  It shares no code,
 * header, table or constant with the HIP library, and the HIP library never
 * calls it.
 *
 * Plain and slow on purpose: every slab matrix is built from its integral
 * definition by Gauss-Legendre quadrature, every block solve is a dense
 * Gaussian elimination, and every multigrid step follows the paper's formulas
 * in the paper's order.  Build with -O2 -ffp-contract=off (no fused
 * multiply-add, no fast-math).
 *
 * Notation follows the paper: P = p_t + 1 dofs per slab, K, M, N the slab
 * stiffness(+jump), mass and upwind-coupling matrices, L the block
 * lower-bidiagonal system matrix, D its block diagonal, R/P restriction and
 * prolongation.  The paper fixes lambda = 1; here K + M becomes K + lambda*M.
 * Matrices are row-major, entry [k][l] at k*P + l (k = test index, l = trial
 * index).  Vectors are slab-major, coefficient k of slab n at n*P + k.
 *
 * The multigrid pieces (slab operators, smoother, transfers, two-grid error
 * propagator) are in section 3 of the paper; the discretisation in section 2.
 * Nothing in this file carries a "parity unpinned" caveat: every exported
 * function is pinned by the CPU tests against closed forms printed in the
 * paper, exact identities, dense brute force or the Fourier symbol.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXP 32

/* ---------------------------------------------------------------------- */
/* Legendre polynomials and Gauss-Legendre quadrature                      */
/* ---------------------------------------------------------------------- */

/* P_k(x) by Bonnet's recurrence (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}. */
static double legendre(int k, double x)
{
    double pm = 1.0, pc = x;
    if (k == 0) return 1.0;
    for (int j = 1; j < k; ++j) {
        double pn = ((2.0 * j + 1.0) * x * pc - j * pm) / (j + 1.0);
        pm = pc;
        pc = pn;
    }
    return pc;
}

/* P_k'(x) from P'_{j+1} = P'_{j-1} + (2j+1) P_j. */
static double legendre_d(int k, double x)
{
    if (k == 0) return 0.0;
    double dm = 0.0, dc = 1.0; /* P_0', P_1' */
    for (int j = 1; j < k; ++j) {
        double dn = dm + (2.0 * j + 1.0) * legendre(j, x);
        dm = dc;
        dc = dn;
    }
    return dc;
}

/* q-point Gauss-Legendre rule on [-1,1]: Newton iteration on P_q. */
static void gauss_legendre(int q, double *x, double *w)
{
    for (int i = 0; i < q; ++i) {
        double z = cos(M_PI * (i + 0.75) / (q + 0.5));
        for (int it = 0; it < 100; ++it) {
            double dz = legendre(q, z) / legendre_d(q, z);
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        double d = legendre_d(q, z);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * d * d);
    }
}

/* ---------------------------------------------------------------------- */
/* Dense linear algebra (P x P)                                            */
/* ---------------------------------------------------------------------- */

/* Solve A x = b (trans = 0) or A^T x = b (trans = 1) by Gaussian
 * elimination with partial pivoting.  Returns 0, or -1 if A is singular. */
static int dense_solve(int P, const double *A, int trans, const double *b, double *x)
{
    double a[OR_MAXP * OR_MAXP], y[OR_MAXP];
    for (int i = 0; i < P; ++i) {
        for (int j = 0; j < P; ++j) a[i * P + j] = trans ? A[j * P + i] : A[i * P + j];
        y[i] = b[i];
    }
    for (int c = 0; c < P; ++c) {
        int piv = c;
        for (int i = c + 1; i < P; ++i)
            if (fabs(a[i * P + c]) > fabs(a[piv * P + c])) piv = i;
        if (a[piv * P + c] == 0.0) return -1;
        if (piv != c) {
            for (int j = 0; j < P; ++j) {
                double t = a[c * P + j];
                a[c * P + j] = a[piv * P + j];
                a[piv * P + j] = t;
            }
            double t = y[c];
            y[c] = y[piv];
            y[piv] = t;
        }
        for (int i = c + 1; i < P; ++i) {
            double m = a[i * P + c] / a[c * P + c];
            for (int j = c; j < P; ++j) a[i * P + j] -= m * a[c * P + j];
            y[i] -= m * y[c];
        }
    }
    for (int i = P - 1; i >= 0; --i) {
        double s = y[i];
        for (int j = i + 1; j < P; ++j) s -= a[i * P + j] * x[j];
        x[i] = s / a[i * P + i];
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Slab matrices (section 2.1) and level data                              */
/* ---------------------------------------------------------------------- */

typedef struct {
    int P;
    int64_t N;     /* slabs on this level */
    double tau;    /* slab length */
    double lam;
    double K[OR_MAXP * OR_MAXP], M[OR_MAXP * OR_MAXP], Nm[OR_MAXP * OR_MAXP];
    double A[OR_MAXP * OR_MAXP]; /* K + lambda*M, the diagonal block of L */
    double alpha;                /* nonzero eigenvalue of A^{-1} N */
    double omega;                /* damping used on this level */
    int periodic;                /* u(0) = u(T): slab 0 couples to slab N-1 */
} or_level;

/*
 * Slab matrices of the DG variational form (section 2.1) for the Legendre
 * basis psi_k(t) = P_k(xi), xi = 2(t - t_{n-1})/tau - 1:
 *   K[k,l] = -int psi_l d/dt psi_k dt + psi_l(t_n) psi_k(t_n),
 *   M[k,l] =  int psi_l psi_k dt,
 *   N[k,l] =  psi_l^{n-1}(t_{n-1}) psi_k^n(t_{n-1}).
 * The integrals are evaluated by Gauss-Legendre quadrature (exact here).
 */
static void slab_matrices(int P, double tau, double lam, or_level *lv)
{
    lv->periodic = 0;
    int q = P + 2;
    double x[OR_MAXP + 2], w[OR_MAXP + 2];
    gauss_legendre(q, x, w);
    lv->P = P;
    lv->tau = tau;
    lv->lam = lam;
    for (int k = 0; k < P; ++k)
        for (int l = 0; l < P; ++l) {
            double sk = 0.0, sm = 0.0;
            for (int i = 0; i < q; ++i) {
                /* d/dt psi_k = (2/tau) P_k'(xi), dt = (tau/2) dxi */
                sk += w[i] * legendre(l, x[i]) * legendre_d(k, x[i]);
                sm += w[i] * legendre(l, x[i]) * legendre(k, x[i]);
            }
            lv->K[k * P + l] = -sk + legendre(l, 1.0) * legendre(k, 1.0);
            lv->M[k * P + l] = 0.5 * tau * sm;
            lv->Nm[k * P + l] = legendre(l, 1.0) * legendre(k, -1.0);
            lv->A[k * P + l] = lv->K[k * P + l] + lam * lv->M[k * P + l];
        }
    /* alpha: the only nonzero eigenvalue of the rank-one matrix A^{-1} N
     * (Lemma chap4_theorem2), i.e. its trace. */
    double tr = 0.0;
    for (int l = 0; l < P; ++l) {
        double col[OR_MAXP], y[OR_MAXP];
        for (int k = 0; k < P; ++k) col[k] = lv->Nm[k * P + l];
        dense_solve(P, lv->A, 0, col, y);
        tr += y[l];
    }
    lv->alpha = tr;
}

/* Optimal damping of Lemma chap4_lemma7. */
static double omega_star(double alpha)
{
    return alpha >= 0.0 ? 1.0 / (1.0 + alpha * alpha) : 1.0;
}

/*
 * Local prolongation matrices R_1^T = M^{-1} Mt^1 and R_2^T = M^{-1} Mt^2
 * (eqs. chap4_restrictionTime, chap4_prolongationTime), with
 *   Mt^1[k,l] = int_0^tau      psit_l(t) psi_k(t)       dt,
 *   Mt^2[k,l] = int_tau^{2tau} psit_l(t) psi_k(t - tau) dt,
 * psit the coarse basis on (0, 2tau) and psi the fine basis on (0, tau).
 * (The source prints psi_k(t + tau) in Mt^2; the fine basis function of the
 * second fine slab is psi_k(t - tau), which is the reading taken.)
 */
static void transfer_matrices(int P, double *R1T, double *R2T)
{
    int q = P + 2;
    double x[OR_MAXP + 2], w[OR_MAXP + 2];
    gauss_legendre(q, x, w);
    const double tau = 1.0; /* cancels in M^{-1} Mt */
    double M[OR_MAXP * OR_MAXP], T1[OR_MAXP * OR_MAXP], T2[OR_MAXP * OR_MAXP];
    for (int k = 0; k < P; ++k)
        for (int l = 0; l < P; ++l) {
            double sm = 0.0, s1 = 0.0, s2 = 0.0;
            for (int i = 0; i < q; ++i) {
                /* fine slab t = tau (xi + 1)/2; first half: coarse coordinate
                 * t/tau - 1 = (xi - 1)/2; second half: (xi + 1)/2. */
                sm += w[i] * legendre(l, x[i]) * legendre(k, x[i]);
                s1 += w[i] * legendre(l, 0.5 * (x[i] - 1.0)) * legendre(k, x[i]);
                s2 += w[i] * legendre(l, 0.5 * (x[i] + 1.0)) * legendre(k, x[i]);
            }
            M[k * P + l] = 0.5 * tau * sm;
            T1[k * P + l] = 0.5 * tau * s1;
            T2[k * P + l] = 0.5 * tau * s2;
        }
    for (int l = 0; l < P; ++l) {
        double c1[OR_MAXP], c2[OR_MAXP], y1[OR_MAXP], y2[OR_MAXP];
        for (int k = 0; k < P; ++k) {
            c1[k] = T1[k * P + l];
            c2[k] = T2[k * P + l];
        }
        dense_solve(P, M, 0, c1, y1);
        dense_solve(P, M, 0, c2, y2);
        for (int k = 0; k < P; ++k) {
            R1T[k * P + l] = y1[k];
            R2T[k * P + l] = y2[k];
        }
    }
}

/* ---------------------------------------------------------------------- */
/* Operators on one level                                                  */
/* ---------------------------------------------------------------------- */

/* (L u)_n = A u_n - N u_{n-1}, u_{-1} = 0 (eq. chap4_generalLinearSystemODE;
 * the initial value enters the right-hand side of the first slab).  For the
 * periodic problem u(0) = u(T) (eq. chap4_equationLinearSystemODEPeriodic)
 * the circulant coupling of eq. chap4_circulantMatrix makes u_{-1} = u_{N-1}. */
static void apply_L(const or_level *lv, const double *u, double *out)
{
    int P = lv->P;
    for (int64_t n = 0; n < lv->N; ++n)
        for (int k = 0; k < P; ++k) {
            double s = 0.0;
            for (int l = 0; l < P; ++l) s += lv->A[k * P + l] * u[n * P + l];
            int64_t left = n > 0 ? n - 1 : (lv->periodic ? lv->N - 1 : -1);
            if (left >= 0)
                for (int l = 0; l < P; ++l) s -= lv->Nm[k * P + l] * u[left * P + l];
            out[n * P + k] = s;
        }
}

/* (L^T z)_n = A^T z_n - N^T z_{n+1}, z_N = 0 (periodic: z_N = z_0). */
static void apply_LT(const or_level *lv, const double *z, double *out)
{
    int P = lv->P;
    for (int64_t n = 0; n < lv->N; ++n)
        for (int k = 0; k < P; ++k) {
            double s = 0.0;
            for (int l = 0; l < P; ++l) s += lv->A[l * P + k] * z[n * P + l];
            int64_t right = n + 1 < lv->N ? n + 1 : (lv->periodic ? 0 : -1);
            if (right >= 0)
                for (int l = 0; l < P; ++l) s -= lv->Nm[l * P + k] * z[right * P + l];
            out[n * P + k] = s;
        }
}

/* r = f - L u (trans = 0) or r = g - L^T z (trans = 1). */
static void residual(const or_level *lv, int trans, const double *f, const double *u, double *r)
{
    int64_t n = lv->N * lv->P;
    if (trans) apply_LT(lv, u, r);
    else apply_L(lv, u, r);
    for (int64_t i = 0; i < n; ++i) r[i] = f[i] - r[i];
}

/* Block substitution (trans = 0, forward in time):
 *   A u_n = f_n + N u_{n-1},  with u_{-1} := y for the first slab,
 * or backward substitution for the transposed system (trans = 1):
 *   A^T z_n = g_n + N^T z_{n+1},  with z_N := y for the last slab.
 * f == NULL stands for a zero right-hand side, y == NULL for a zero
 * coupling at the boundary. */
static void substitute(const or_level *lv, int trans, const double *f, const double *y, double *u)
{
    int P = lv->P;
    int64_t N = lv->N;
    double rhs[OR_MAXP];
    if (!trans) {
        for (int64_t n = 0; n < N; ++n) {
            const double *prev = n > 0 ? u + (n - 1) * P : y;
            for (int k = 0; k < P; ++k) {
                double s = f ? f[n * P + k] : 0.0;
                if (prev)
                    for (int l = 0; l < P; ++l) s += lv->Nm[k * P + l] * prev[l];
                rhs[k] = s;
            }
            dense_solve(P, lv->A, 0, rhs, u + n * P);
        }
    } else {
        for (int64_t n = N - 1; n >= 0; --n) {
            const double *next = n + 1 < N ? u + (n + 1) * P : y;
            for (int k = 0; k < P; ++k) {
                double s = f ? f[n * P + k] : 0.0;
                if (next)
                    for (int l = 0; l < P; ++l) s += lv->Nm[l * P + k] * next[l];
                rhs[k] = s;
            }
            dense_solve(P, lv->A, 1, rhs, u + n * P);
        }
    }
}

/* Exact solve.  Initial-value problem: the substitution itself.  Periodic
 * problem (eq. chap4_equationLinearSystemODEPeriodic): the substitution is
 * affine in the coupled boundary slab y (u_{N-1} that slab 0 sees, or z_0
 * that slab N-1 sees for the transposed system): the slab it ends on is
 * Phi y + psi, psi from the substitution with y = 0 and column k of Phi from
 * the substitution of the homogeneous system with y = e_k.  The periodic
 * solution has y = Phi y + psi, so y solves (I - Phi) y = psi, and one more
 * substitution with that y gives it. */
static void direct(const or_level *lv, int trans, const double *f, double *u)
{
    if (!lv->periodic) {
        substitute(lv, trans, f, NULL, u);
        return;
    }
    int P = lv->P;
    int64_t N = lv->N;
    const int64_t end = trans ? 0 : N - 1;   /* the slab the substitution ends on */
    double Phi[OR_MAXP * OR_MAXP], psi[OR_MAXP], e[OR_MAXP], y[OR_MAXP];
    double IminusPhi[OR_MAXP * OR_MAXP];
    substitute(lv, trans, f, NULL, u);
    for (int k = 0; k < P; ++k) psi[k] = u[end * P + k];
    for (int c = 0; c < P; ++c) {
        for (int k = 0; k < P; ++k) e[k] = (k == c) ? 1.0 : 0.0;
        substitute(lv, trans, NULL, e, u);
        for (int k = 0; k < P; ++k) Phi[k * P + c] = u[end * P + k];
    }
    for (int k = 0; k < P; ++k)
        for (int c = 0; c < P; ++c) IminusPhi[k * P + c] = (k == c ? 1.0 : 0.0) - Phi[k * P + c];
    dense_solve(P, IminusPhi, 0, psi, y);
    substitute(lv, trans, f, y, u);
}

/* One damped block Jacobi step (eq. chap4_ODESmoother):
 *   u <- u + omega D^{-1} (f - L u),  D = blockdiag(A);
 * transposed variant: z <- z + omega D^{-T} (g - L^T z). */
static void jacobi(const or_level *lv, int trans, double omega, const double *f, double *u)
{
    int P = lv->P;
    int64_t n = lv->N * P;
    double *r = malloc(sizeof(double) * n);
    residual(lv, trans, f, u, r);
    for (int64_t s = 0; s < lv->N; ++s) {
        double d[OR_MAXP];
        dense_solve(P, lv->A, trans, r + s * P, d);
        for (int k = 0; k < P; ++k) u[s * P + k] += omega * d[k];
    }
    free(r);
}

/* rc = R r: rc_m = R_1 r_{2m} + R_2 r_{2m+1}, R_i = (R_i^T)^T
 * (eq. chap4_restrictionTime, 0-based slab pairs). */
static void restrict_r(int P, const double *R1T, const double *R2T, int64_t Nc, const double *r,
                       double *rc)
{
    for (int64_t m = 0; m < Nc; ++m)
        for (int k = 0; k < P; ++k) {
            double s = 0.0;
            for (int l = 0; l < P; ++l)
                s += R1T[l * P + k] * r[(2 * m) * P + l] + R2T[l * P + k] * r[(2 * m + 1) * P + l];
            rc[m * P + k] = s;
        }
}

/* u += P e: u_{2m} += R_1^T e_m, u_{2m+1} += R_2^T e_m (eq. chap4_prolongationTime). */
static void prolong_add(int P, const double *R1T, const double *R2T, int64_t Nc, const double *e,
                        double *u)
{
    for (int64_t m = 0; m < Nc; ++m)
        for (int k = 0; k < P; ++k) {
            double s1 = 0.0, s2 = 0.0;
            for (int l = 0; l < P; ++l) {
                s1 += R1T[k * P + l] * e[m * P + l];
                s2 += R2T[k * P + l] * e[m * P + l];
            }
            u[(2 * m) * P + k] += s1;
            u[(2 * m + 1) * P + k] += s2;
        }
}

/* ---------------------------------------------------------------------- */
/* Hierarchy and cycle                                                     */
/* ---------------------------------------------------------------------- */

typedef struct {
    int P, nlev;
    int nu1, nu2, gamma;
    int lb64;     /* mixed-precision reference: first level run in FP64 (nlev-1 by default) */
    or_level *lv; /* lv[0] finest (the paper's level L), lv[nlev-1] coarsest */
    double R1T[OR_MAXP * OR_MAXP], R2T[OR_MAXP * OR_MAXP];
} or_hier;

/* Level sizes N, N/2, ..., n_coarse.  Returns -1 unless N = n_coarse * 2^k. */
static int build_hier(or_hier *H, int p, int64_t N, double T, double lam, int nu1, int nu2,
                      int gamma, int64_t n_coarse, int omega_mode, double omega_fixed,
                      int periodic)
{
    if (p < 0 || p + 1 > OR_MAXP || N < 1 || n_coarse < 1 || T <= 0.0) return -1;
    int nlev = 1;
    int64_t m = N;
    while (m > n_coarse) {
        if (m % 2) return -1;
        m /= 2;
        ++nlev;
    }
    if (m != n_coarse) return -1;
    H->P = p + 1;
    H->nlev = nlev;
    H->nu1 = nu1;
    H->nu2 = nu2;
    H->gamma = gamma;
    H->lb64 = nlev - 1;
    H->lv = calloc((size_t)nlev, sizeof(or_level));
    for (int l = 0; l < nlev; ++l) {
        int64_t Nl = N >> l;
        slab_matrices(p + 1, T / (double)Nl, lam, &H->lv[l]);
        H->lv[l].N = Nl;
        H->lv[l].omega = omega_mode == 0 ? omega_star(H->lv[l].alpha) : omega_fixed;
        H->lv[l].periodic = periodic;
    }
    transfer_matrices(p + 1, H->R1T, H->R2T);
    return 0;
}

static void free_hier(or_hier *H) { free(H->lv); }

/*
 * One multigrid cycle on level l for L_l u = f (trans = 1: for L_l^T),
 * in place on u.  Two-grid structure of eq. chap4_errorTwoGridCycle applied
 * recursively: nu1 smoothing steps, residual, restriction, gamma cycles on
 * the coarse error equation from a zero initial guess (an exact solve when
 * the next level is the coarsest), prolongation and correction, nu2
 * smoothing steps.  The coarse operator is the rediscretisation at 2*tau.
 */
static void cycle(const or_hier *H, int l, int trans, const double *f, double *u)
{
    const or_level *lv = &H->lv[l];
    int P = H->P;
    if (l == H->nlev - 1) {
        direct(lv, trans, f, u);
        return;
    }
    for (int s = 0; s < H->nu1; ++s) jacobi(lv, trans, lv->omega, f, u);
    int64_t Nc = lv->N / 2;
    double *r = malloc(sizeof(double) * lv->N * P);
    double *rc = malloc(sizeof(double) * Nc * P);
    double *e = calloc((size_t)(Nc * P), sizeof(double));
    residual(lv, trans, f, u, r);
    restrict_r(P, H->R1T, H->R2T, Nc, r, rc);
    if (l + 1 == H->nlev - 1)
        direct(&H->lv[l + 1], trans, rc, e);
    else
        for (int g = 0; g < H->gamma; ++g) cycle(H, l + 1, trans, rc, e);
    prolong_add(P, H->R1T, H->R2T, Nc, e, u);
    for (int s = 0; s < H->nu2; ++s) jacobi(lv, trans, lv->omega, f, u);
    free(r);
    free(rc);
    free(e);
}

static double norm2(int64_t n, const double *x)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += x[i] * x[i];
    return sqrt(s);
}

/* ---------------------------------------------------------------------- */
/* Exported API (ctypes)                                                   */
/* ---------------------------------------------------------------------- */

int or_max_dofs(void) { return OR_MAXP; }

/* Slab tables for one level: K, M, N, A = K + lambda*M (P*P each), alpha,
 * the optimal omega, and the level-independent R1T, R2T (P*P each). */
int or_tables(int p, double tau, double lam, double *K, double *M, double *Nm, double *A,
              double *alpha, double *omega, double *R1T, double *R2T)
{
    if (p < 0 || p + 1 > OR_MAXP) return -1;
    or_level lv;
    int P = p + 1;
    slab_matrices(P, tau, lam, &lv);
    memcpy(K, lv.K, sizeof(double) * P * P);
    memcpy(M, lv.M, sizeof(double) * P * P);
    memcpy(Nm, lv.Nm, sizeof(double) * P * P);
    memcpy(A, lv.A, sizeof(double) * P * P);
    *alpha = lv.alpha;
    *omega = omega_star(lv.alpha);
    transfer_matrices(P, R1T, R2T);
    return 0;
}

/* Legendre end values used for the initial-value fold: vL[k] = psi_k(t_{n-1}^+). */
static void fold_u0(int P, double u0, double *f)
{
    /* upwind term u_tau^0(t_0) v(t_0) with u_tau^0(t_0) := u0 (eq. chap4_discreteVarFormODE, n = 1) */
    for (int k = 0; k < P; ++k) f[k] += u0 * legendre(k, -1.0);
}

/* f_out = f with the initial value folded into slab 0. */
int or_fold(int p, int64_t N, double u0, const double *f, double *f_out)
{
    memcpy(f_out, f, sizeof(double) * N * (p + 1));
    fold_u0(p + 1, u0, f_out);
    return 0;
}

/* out = L u (trans = 0) or L^T u (trans = 1) on N slabs of length tau;
 * periodic: the circulant system of eq. chap4_equationLinearSystemODEPeriodic. */
int or_apply(int p, int64_t N, double tau, double lam, int trans, const double *u, double *out,
             int periodic)
{
    or_level lv;
    slab_matrices(p + 1, tau, lam, &lv);
    lv.N = N;
    lv.periodic = periodic;
    if (trans) apply_LT(&lv, u, out);
    else apply_L(&lv, u, out);
    return 0;
}

/* r = f - L u (or g - L^T z). */
int or_residual(int p, int64_t N, double tau, double lam, int trans, const double *f,
                const double *u, double *r, int periodic)
{
    or_level lv;
    slab_matrices(p + 1, tau, lam, &lv);
    lv.N = N;
    lv.periodic = periodic;
    residual(&lv, trans, f, u, r);
    return 0;
}

/* nsweep damped block Jacobi steps in place on u (omega <= 0: optimal omega). */
int or_sweeps(int p, int64_t N, double tau, double lam, int trans, double omega, int nsweep,
              const double *f, double *u, int periodic)
{
    or_level lv;
    slab_matrices(p + 1, tau, lam, &lv);
    lv.N = N;
    lv.periodic = periodic;
    if (omega <= 0.0) omega = omega_star(lv.alpha);
    for (int s = 0; s < nsweep; ++s) jacobi(&lv, trans, omega, f, u);
    return 0;
}

int or_restrict(int p, int64_t Nc, const double *r, double *rc)
{
    double R1T[OR_MAXP * OR_MAXP], R2T[OR_MAXP * OR_MAXP];
    transfer_matrices(p + 1, R1T, R2T);
    restrict_r(p + 1, R1T, R2T, Nc, r, rc);
    return 0;
}

int or_prolong_add(int p, int64_t Nc, const double *e, double *u)
{
    double R1T[OR_MAXP * OR_MAXP], R2T[OR_MAXP * OR_MAXP];
    transfer_matrices(p + 1, R1T, R2T);
    prolong_add(p + 1, R1T, R2T, Nc, e, u);
    return 0;
}

/* Exact solve of L u = f (trans = 0, forward) or L^T z = g (trans = 1, backward);
 * periodic: of the circulant system. */
int or_direct(int p, int64_t N, double tau, double lam, int trans, const double *f, double *u,
              int periodic)
{
    or_level lv;
    slab_matrices(p + 1, tau, lam, &lv);
    lv.N = N;
    lv.periodic = periodic;
    direct(&lv, trans, f, u);
    return 0;
}

/* Per-level alpha and omega of the hierarchy (arrays of length nlev). */
int or_levels(int p, int64_t N, double T, double lam, int64_t n_coarse, int omega_mode,
              double omega_fixed, double *alpha, double *omega)
{
    or_hier H;
    if (build_hier(&H, p, N, T, lam, 2, 2, 1, n_coarse, omega_mode, omega_fixed, 0)) return -1;
    for (int l = 0; l < H.nlev; ++l) {
        alpha[l] = H.lv[l].alpha;
        omega[l] = H.lv[l].omega;
    }
    int n = H.nlev;
    free_hier(&H);
    return n;
}

/* ncyc cycles in place on u for L u = f (already folded) or L^T z = g. */
int or_cycles(int p, int64_t N, double T, double lam, int nu1, int nu2, int gamma,
              int64_t n_coarse, int omega_mode, double omega_fixed, int trans, int ncyc,
              const double *f, double *u, int periodic)
{
    or_hier H;
    if (build_hier(&H, p, N, T, lam, nu1, nu2, gamma, n_coarse, omega_mode, omega_fixed,
                   periodic))
        return -1;
    for (int c = 0; c < ncyc; ++c) cycle(&H, 0, trans, f, u);
    free_hier(&H);
    return 0;
}

/*
 * Multigrid solve from u = 0 until ||f - L u||_2 <= rtol ||f||_2 (relative
 * residual reduction, as measured in section 4's experiments), or max_cycles.
 * f is already folded.  hist (optional, length max_cycles + 1) receives the
 * residual norms.  Returns the number of cycles; *relres the final ratio.
 */
int or_solve(int p, int64_t N, double T, double lam, int nu1, int nu2, int gamma,
             int64_t n_coarse, int omega_mode, double omega_fixed, int trans, const double *f,
             double rtol, int max_cycles, double *u, double *relres, double *hist, int periodic)
{
    or_hier H;
    if (build_hier(&H, p, N, T, lam, nu1, nu2, gamma, n_coarse, omega_mode, omega_fixed,
                   periodic))
        return -1;
    int64_t n = N * (p + 1);
    double *r = malloc(sizeof(double) * n);
    memset(u, 0, sizeof(double) * n);
    double r0 = norm2(n, f), rk = r0;
    if (hist) hist[0] = r0;
    int k = 0;
    while (k < max_cycles && rk > rtol * r0) {
        cycle(&H, 0, trans, f, u);
        ++k;
        residual(&H.lv[0], trans, f, u, r);
        rk = norm2(n, r);
        if (hist) hist[k] = rk;
    }
    *relres = r0 > 0.0 ? rk / r0 : 0.0;
    free(r);
    free_hier(&H);
    return k;
}

/* ---------------------------------------------------------------------- */
/* Space-time heat equation (section 6, Conclusions)                        */
/* ---------------------------------------------------------------------- */
/*
 * u_t - u_xx = f on (0,1) x (0,T], u = 0 at x = 0, 1, u(x,0) = u0(x), with
 * second-order finite differences on nx interior points x_i = i h,
 * h = 1/(nx+1), L_h = tridiag(-1, 2, -1) / h^2, and the DG-in-time
 * discretisation of the ODE part on every spatial point.  The slab system
 * couples all points of a slab:
 *     (I (x) K + L_h (x) M) U_n - (I (x) N) U_{n-1} = F_n,
 * U_n ordered [point][k].  Arrays are [point][slab][k]: coefficient k of slab
 * n at point i at (i*N + n)*P + k.  The time multigrid of section 3 applies
 * with block Jacobi over whole slabs (every block solved exactly: the dense
 * slab block is LU-factored once per level), time restriction and
 * prolongation at every point, the coarse operator rediscretised at 2 tau on
 * the same spatial grid, and forward substitution on the coarsest level.
 */
typedef struct {
    int P, nx;
    int64_t N;
    double tau, h;
    or_level t;   /* K, M (tau-scaled), N of the time slab */
    double *LU;   /* (nx P)^2 LU factors of the slab block */
    int *piv;
    double omega;
} or_heat_level;

/* LU factorisation with partial pivoting of a dense n x n matrix (in place). */
static void lu_factor(int n, double *a, int *piv)
{
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int i = c + 1; i < n; ++i)
            if (fabs(a[(int64_t)i * n + c]) > fabs(a[(int64_t)p * n + c])) p = i;
        piv[c] = p;
        if (p != c)
            for (int j = 0; j < n; ++j) {
                double t = a[(int64_t)c * n + j];
                a[(int64_t)c * n + j] = a[(int64_t)p * n + j];
                a[(int64_t)p * n + j] = t;
            }
        for (int i = c + 1; i < n; ++i) {
            double m = a[(int64_t)i * n + c] / a[(int64_t)c * n + c];
            a[(int64_t)i * n + c] = m;
            for (int j = c + 1; j < n; ++j) a[(int64_t)i * n + j] -= m * a[(int64_t)c * n + j];
        }
    }
}

static void lu_solve(int n, const double *a, const int *piv, const double *b, double *x)
{
    for (int i = 0; i < n; ++i) x[i] = b[i];
    for (int c = 0; c < n; ++c) {
        if (piv[c] != c) {
            double t = x[c];
            x[c] = x[piv[c]];
            x[piv[c]] = t;
        }
        for (int i = c + 1; i < n; ++i) x[i] -= a[(int64_t)i * n + c] * x[c];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = x[i];
        for (int j = i + 1; j < n; ++j) s -= a[(int64_t)i * n + j] * x[j];
        x[i] = s / a[(int64_t)i * n + i];
    }
}

/* Smallest eigenvalue of L_h: (4/h^2) sin^2(pi h / 2). */
static double heat_lambda1(int nx)
{
    const double h = 1.0 / (nx + 1), s = sin(M_PI * h / 2.0);
    return 4.0 * s * s / (h * h);
}

/* alpha (the nonzero eigenvalue of A^{-1} N, Lemma chap4_theorem2) of the
 * time slab at the smallest eigenvalue of L_h: the damping of Lemma
 * chap4_lemma7 is taken there, for the slowest spatial mode. */
static double heat_alpha(int P, double tau, int nx)
{
    or_level lv;
    slab_matrices(P, tau, heat_lambda1(nx), &lv);
    return lv.alpha;
}

static void heat_level_init(or_heat_level *hl, int P, int nx, int64_t N, double tau)
{
    hl->P = P;
    hl->nx = nx;
    hl->N = N;
    hl->tau = tau;
    hl->h = 1.0 / (nx + 1);
    slab_matrices(P, tau, 1.0, &hl->t);
    const int n = nx * P;
    hl->LU = calloc((size_t)n * n, sizeof(double));
    hl->piv = calloc((size_t)n, sizeof(int));
    const double ih2 = 1.0 / (hl->h * hl->h);
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < nx; ++j) {
            double L = (i == j) ? 2.0 * ih2 : ((i - j == 1 || j - i == 1) ? -ih2 : 0.0);
            for (int k = 0; k < P; ++k)
                for (int l = 0; l < P; ++l) {
                    double v = L * hl->t.M[k * P + l];
                    if (i == j) v += hl->t.K[k * P + l];
                    hl->LU[(int64_t)(i * P + k) * n + (j * P + l)] = v;
                }
        }
    lu_factor(n, hl->LU, hl->piv);
    hl->omega = omega_star(heat_alpha(P, tau, nx));
}

static void heat_level_free(or_heat_level *hl)
{
    free(hl->LU);
    free(hl->piv);
}

/* (L U) at every point and slab: K u_{i,n} + M (L_h u)_{i,n} - N u_{i,n-1}. */
static void heat_apply(const or_heat_level *hl, const double *u, double *out)
{
    const int P = hl->P, nx = hl->nx;
    const int64_t N = hl->N;
    const double ih2 = 1.0 / (hl->h * hl->h);
    for (int i = 0; i < nx; ++i)
        for (int64_t n = 0; n < N; ++n) {
            const double *ui = u + ((int64_t)i * N + n) * P;
            double lu[OR_MAXP];
            for (int l = 0; l < P; ++l) {
                double s = 2.0 * ui[l];
                if (i > 0) s -= u[((int64_t)(i - 1) * N + n) * P + l];
                if (i + 1 < nx) s -= u[((int64_t)(i + 1) * N + n) * P + l];
                lu[l] = s * ih2;
            }
            for (int k = 0; k < P; ++k) {
                double s = 0.0;
                for (int l = 0; l < P; ++l) s += hl->t.K[k * P + l] * ui[l] + hl->t.M[k * P + l] * lu[l];
                if (n > 0)
                    for (int l = 0; l < P; ++l) s -= hl->t.Nm[k * P + l] * ui[l - P];
                out[((int64_t)i * N + n) * P + k] = s;
            }
        }
}

static void heat_residual(const or_heat_level *hl, const double *f, const double *u, double *r)
{
    const int64_t n = (int64_t)hl->nx * hl->N * hl->P;
    heat_apply(hl, u, r);
    for (int64_t i = 0; i < n; ++i) r[i] = f[i] - r[i];
}

/* Gather slab n of every point into [point][k] (and scatter back). */
static void heat_gather(const or_heat_level *hl, const double *a, int64_t n, double *s)
{
    for (int i = 0; i < hl->nx; ++i)
        for (int k = 0; k < hl->P; ++k) s[i * hl->P + k] = a[((int64_t)i * hl->N + n) * hl->P + k];
}
static void heat_scatter(const or_heat_level *hl, const double *s, int64_t n, double *a)
{
    for (int i = 0; i < hl->nx; ++i)
        for (int k = 0; k < hl->P; ++k) a[((int64_t)i * hl->N + n) * hl->P + k] = s[i * hl->P + k];
}

/* One damped block Jacobi step over whole slabs (eq. chap4_ODESmoother with
 * the space-time slab block as D): u <- u + omega D^{-1} (f - L u). */
static void heat_jacobi(const or_heat_level *hl, double omega, const double *f, double *u)
{
    const int P = hl->P, n = hl->nx * P;
    const int64_t tot = (int64_t)hl->N * n;
    double *r = malloc(sizeof(double) * tot);
    double *rs = malloc(sizeof(double) * n), *d = malloc(sizeof(double) * n);
    heat_residual(hl, f, u, r);
    for (int64_t s = 0; s < hl->N; ++s) {
        heat_gather(hl, r, s, rs);
        lu_solve(n, hl->LU, hl->piv, rs, d);
        for (int i = 0; i < hl->nx; ++i)
            for (int k = 0; k < P; ++k) u[((int64_t)i * hl->N + s) * P + k] += omega * d[i * P + k];
    }
    free(r);
    free(rs);
    free(d);
}

/* Exact solve: forward substitution over the slabs, each slab block solved exactly. */
static void heat_direct(const or_heat_level *hl, const double *f, double *u)
{
    const int P = hl->P, n = hl->nx * P;
    double *rs = malloc(sizeof(double) * n), *d = malloc(sizeof(double) * n);
    for (int64_t s = 0; s < hl->N; ++s) {
        heat_gather(hl, f, s, rs);
        if (s > 0)
            for (int i = 0; i < hl->nx; ++i)
                for (int k = 0; k < P; ++k) {
                    double t = 0.0;
                    for (int l = 0; l < P; ++l)
                        t += hl->t.Nm[k * P + l] * u[((int64_t)i * hl->N + s - 1) * P + l];
                    rs[i * P + k] += t;
                }
        lu_solve(n, hl->LU, hl->piv, rs, d);
        heat_scatter(hl, d, s, u);
    }
    free(rs);
    free(d);
}

typedef struct {
    int P, nx, nlev, nu1, nu2, gamma;
    or_heat_level *lv;
    double R1T[OR_MAXP * OR_MAXP], R2T[OR_MAXP * OR_MAXP];
} or_heat_hier;

static int heat_build(or_heat_hier *H, int p, int nx, int64_t N, double T, int nu1, int nu2,
                      int gamma, int64_t n_coarse, int omega_mode, double omega_fixed)
{
    if (p < 0 || p + 1 > OR_MAXP || nx < 1 || N < 1 || n_coarse < 1 || T <= 0.0) return -1;
    int nlev = 1;
    int64_t m = N;
    while (m > n_coarse) {
        if (m % 2) return -1;
        m /= 2;
        ++nlev;
    }
    if (m != n_coarse) return -1;
    H->P = p + 1;
    H->nx = nx;
    H->nlev = nlev;
    H->nu1 = nu1;
    H->nu2 = nu2;
    H->gamma = gamma;
    H->lv = calloc((size_t)nlev, sizeof(or_heat_level));
    for (int l = 0; l < nlev; ++l) {
        heat_level_init(&H->lv[l], p + 1, nx, N >> l, T / (double)(N >> l));
        if (omega_mode == 1) H->lv[l].omega = omega_fixed;
    }
    transfer_matrices(p + 1, H->R1T, H->R2T);
    return 0;
}

static void heat_free(or_heat_hier *H)
{
    for (int l = 0; l < H->nlev; ++l) heat_level_free(&H->lv[l]);
    free(H->lv);
}

/* One cycle on level l (eq. chap4_errorTwoGridCycle applied recursively, as
 * in `cycle`), the transfers applied at every spatial point. */
static void heat_cycle(const or_heat_hier *H, int l, const double *f, double *u)
{
    const or_heat_level *lv = &H->lv[l];
    const int P = H->P, nx = H->nx;
    if (l == H->nlev - 1) {
        heat_direct(lv, f, u);
        return;
    }
    for (int s = 0; s < H->nu1; ++s) heat_jacobi(lv, lv->omega, f, u);
    const int64_t N = lv->N, Nc = N / 2;
    double *r = malloc(sizeof(double) * nx * N * P);
    double *rc = malloc(sizeof(double) * nx * Nc * P);
    double *e = calloc((size_t)(nx * Nc * P), sizeof(double));
    heat_residual(lv, f, u, r);
    for (int i = 0; i < nx; ++i)
        restrict_r(P, H->R1T, H->R2T, Nc, r + (int64_t)i * N * P, rc + (int64_t)i * Nc * P);
    if (l + 1 == H->nlev - 1)
        heat_direct(&H->lv[l + 1], rc, e);
    else
        for (int g = 0; g < H->gamma; ++g) heat_cycle(H, l + 1, rc, e);
    for (int i = 0; i < nx; ++i)
        prolong_add(P, H->R1T, H->R2T, Nc, e + (int64_t)i * Nc * P, u + (int64_t)i * N * P);
    for (int s = 0; s < H->nu2; ++s) heat_jacobi(lv, lv->omega, f, u);
    free(r);
    free(rc);
    free(e);
}

/* f_out = f with u0_i (-1)^k added to slab 0 of every point i. */
int or_heat_fold(int p, int nx, int64_t N, const double *u0, const double *f, double *f_out)
{
    const int P = p + 1;
    memcpy(f_out, f, sizeof(double) * nx * N * P);
    for (int i = 0; i < nx; ++i) fold_u0(P, u0[i], f_out + (int64_t)i * N * P);
    return 0;
}

int or_heat_apply(int p, int nx, int64_t N, double tau, const double *u, double *out)
{
    or_heat_level hl;
    heat_level_init(&hl, p + 1, nx, N, tau);
    heat_apply(&hl, u, out);
    heat_level_free(&hl);
    return 0;
}

int or_heat_residual(int p, int nx, int64_t N, double tau, const double *f, const double *u,
                     double *r)
{
    or_heat_level hl;
    heat_level_init(&hl, p + 1, nx, N, tau);
    heat_residual(&hl, f, u, r);
    heat_level_free(&hl);
    return 0;
}

/* nsweep block Jacobi steps in place (omega <= 0: the level's damping). */
int or_heat_sweeps(int p, int nx, int64_t N, double tau, double omega, int nsweep,
                   const double *f, double *u)
{
    or_heat_level hl;
    heat_level_init(&hl, p + 1, nx, N, tau);
    if (omega <= 0.0) omega = hl.omega;
    for (int s = 0; s < nsweep; ++s) heat_jacobi(&hl, omega, f, u);
    heat_level_free(&hl);
    return 0;
}

int or_heat_direct(int p, int nx, int64_t N, double tau, const double *f, double *u)
{
    or_heat_level hl;
    heat_level_init(&hl, p + 1, nx, N, tau);
    heat_direct(&hl, f, u);
    heat_level_free(&hl);
    return 0;
}

/* Per-level damping (array of length nlev); returns nlev. */
int or_heat_levels(int p, int nx, int64_t N, double T, int64_t n_coarse, int omega_mode,
                   double omega_fixed, double *omega)
{
    or_heat_hier H;
    if (heat_build(&H, p, nx, N, T, 2, 2, 1, n_coarse, omega_mode, omega_fixed)) return -1;
    for (int l = 0; l < H.nlev; ++l) omega[l] = H.lv[l].omega;
    const int n = H.nlev;
    heat_free(&H);
    return n;
}

int or_heat_cycles(int p, int nx, int64_t N, double T, int nu1, int nu2, int gamma,
                   int64_t n_coarse, int omega_mode, double omega_fixed, int ncyc,
                   const double *f, double *u)
{
    or_heat_hier H;
    if (heat_build(&H, p, nx, N, T, nu1, nu2, gamma, n_coarse, omega_mode, omega_fixed))
        return -1;
    for (int c = 0; c < ncyc; ++c) heat_cycle(&H, 0, f, u);
    heat_free(&H);
    return 0;
}

/* Multigrid solve from u = 0 to ||f - L u||_2 <= rtol ||f||_2 (f folded). */
int or_heat_solve(int p, int nx, int64_t N, double T, int nu1, int nu2, int gamma,
                  int64_t n_coarse, int omega_mode, double omega_fixed, const double *f,
                  double rtol, int max_cycles, double *u, double *relres, double *hist)
{
    or_heat_hier H;
    if (heat_build(&H, p, nx, N, T, nu1, nu2, gamma, n_coarse, omega_mode, omega_fixed))
        return -1;
    const int64_t n = (int64_t)nx * N * (p + 1);
    double *r = malloc(sizeof(double) * n);
    memset(u, 0, sizeof(double) * n);
    double r0 = norm2(n, f), rk = r0;
    if (hist) hist[0] = r0;
    int k = 0;
    while (k < max_cycles && rk > rtol * r0) {
        heat_cycle(&H, 0, f, u);
        ++k;
        heat_residual(&H.lv[0], f, u, r);
        rk = norm2(n, r);
        if (hist) hist[k] = rk;
    }
    *relres = r0 > 0.0 ? rk / r0 : 0.0;
    free(r);
    heat_free(&H);
    return k;
}

/* ---------------------------------------------------------------------- */
/* Mixed precision reference (FP32 inner cycle, FP64 outer correction)    */
/* ---------------------------------------------------------------------- */

/* FP32 copy of a level: the same matrices rounded to float. */
typedef struct {
    int P;
    int64_t N;
    float A[OR_MAXP * OR_MAXP], Nm[OR_MAXP * OR_MAXP];
    float omega;
} or_level32;

static int dense_solve32(int P, const float *A, const float *b, float *x)
{
    float a[OR_MAXP * OR_MAXP], y[OR_MAXP];
    for (int i = 0; i < P; ++i) {
        for (int j = 0; j < P; ++j) a[i * P + j] = A[i * P + j];
        y[i] = b[i];
    }
    for (int c = 0; c < P; ++c) {
        int piv = c;
        for (int i = c + 1; i < P; ++i)
            if (fabsf(a[i * P + c]) > fabsf(a[piv * P + c])) piv = i;
        if (a[piv * P + c] == 0.0f) return -1;
        if (piv != c) {
            for (int j = 0; j < P; ++j) {
                float t = a[c * P + j];
                a[c * P + j] = a[piv * P + j];
                a[piv * P + j] = t;
            }
            float t = y[c];
            y[c] = y[piv];
            y[piv] = t;
        }
        for (int i = c + 1; i < P; ++i) {
            float m = a[i * P + c] / a[c * P + c];
            for (int j = c; j < P; ++j) a[i * P + j] -= m * a[c * P + j];
            y[i] -= m * y[c];
        }
    }
    for (int i = P - 1; i >= 0; --i) {
        float s = y[i];
        for (int j = i + 1; j < P; ++j) s -= a[i * P + j] * x[j];
        x[i] = s / a[i * P + i];
    }
    return 0;
}

/* FP32 damped block Jacobi step: u <- u + omega D^{-1}(f - L u), all float. */
static void jacobi32(const or_level32 *lv, const float *f, float *u)
{
    int P = lv->P;
    int64_t N = lv->N;
    float *r = malloc(sizeof(float) * N * P);
    for (int64_t n = 0; n < N; ++n)
        for (int k = 0; k < P; ++k) {
            float s = 0.0f;
            for (int l = 0; l < P; ++l) s += lv->A[k * P + l] * u[n * P + l];
            if (n > 0)
                for (int l = 0; l < P; ++l) s -= lv->Nm[k * P + l] * u[(n - 1) * P + l];
            r[n * P + k] = f[n * P + k] - s;
        }
    for (int64_t n = 0; n < N; ++n) {
        float d[OR_MAXP];
        dense_solve32(P, lv->A, r + n * P, d);
        for (int k = 0; k < P; ++k) u[n * P + k] += lv->omega * d[k];
    }
    free(r);
}

/*
 * Mixed-precision cycle on level l: smoothing, restriction and prolongation
 * in FP32 (storage and arithmetic); the intra-cycle residual in FP64
 * arithmetic from the FP32 operands, stored as FP32.  A visit of a level
 * l >= H->lb64 runs in FP64 arithmetic from the FP32 right-hand side and
 * iterate and stores its result as FP32: by default (lb64 = the coarsest
 * level) only the coarsest solve; a smaller lb64 also computes the levels
 * above it in FP64, as a solver that keeps its small levels on chip does.
 */
static void cycle32(const or_hier *H, const or_level32 *L32, int l, const float *f, float *u)
{
    const or_level *lv = &H->lv[l];
    int P = H->P;
    int64_t N = lv->N;
    if (l >= H->lb64) {
        double *f64 = malloc(sizeof(double) * N * P), *u64 = malloc(sizeof(double) * N * P);
        for (int64_t i = 0; i < N * P; ++i) {
            f64[i] = (double)f[i];
            u64[i] = (double)u[i];
        }
        cycle(H, l, 0, f64, u64);
        for (int64_t i = 0; i < N * P; ++i) u[i] = (float)u64[i];
        free(f64);
        free(u64);
        return;
    }
    for (int s = 0; s < H->nu1; ++s) jacobi32(&L32[l], f, u);
    int64_t Nc = N / 2;
    double *u64 = malloc(sizeof(double) * N * P), *f64 = malloc(sizeof(double) * N * P);
    double *r64 = malloc(sizeof(double) * N * P);
    for (int64_t i = 0; i < N * P; ++i) {
        u64[i] = (double)u[i];
        f64[i] = (double)f[i];
    }
    residual(lv, 0, f64, u64, r64);
    float *r = malloc(sizeof(float) * N * P), *rc = malloc(sizeof(float) * Nc * P);
    float *e = calloc((size_t)(Nc * P), sizeof(float));
    for (int64_t i = 0; i < N * P; ++i) r[i] = (float)r64[i];
    float R1T[OR_MAXP * OR_MAXP], R2T[OR_MAXP * OR_MAXP];
    for (int i = 0; i < P * P; ++i) {
        R1T[i] = (float)H->R1T[i];
        R2T[i] = (float)H->R2T[i];
    }
    for (int64_t m = 0; m < Nc; ++m)
        for (int k = 0; k < P; ++k) {
            float s = 0.0f;
            for (int j = 0; j < P; ++j)
                s += R1T[j * P + k] * r[(2 * m) * P + j] + R2T[j * P + k] * r[(2 * m + 1) * P + j];
            rc[m * P + k] = s;
        }
    if (l + 1 == H->nlev - 1)
        cycle32(H, L32, l + 1, rc, e);
    else
        for (int g = 0; g < H->gamma; ++g) cycle32(H, L32, l + 1, rc, e);
    for (int64_t m = 0; m < Nc; ++m)
        for (int k = 0; k < P; ++k) {
            float s1 = 0.0f, s2 = 0.0f;
            for (int j = 0; j < P; ++j) {
                s1 += R1T[k * P + j] * e[m * P + j];
                s2 += R2T[k * P + j] * e[m * P + j];
            }
            u[(2 * m) * P + k] += s1;
            u[(2 * m + 1) * P + k] += s2;
        }
    for (int s = 0; s < H->nu2; ++s) jacobi32(&L32[l], f, u);
    free(u64);
    free(f64);
    free(r64);
    free(r);
    free(rc);
    free(e);
}

/*
 * Defect correction: repeat { r = f - L u (FP64); stop if ||r|| <= rtol ||f||;
 * one FP32-inner cycle on L e = r from e = 0; u += e (FP64) }.
 * Returns the number of outer iterations (each is one cycle).
 */
/* FP32 copies of every level of H. */
static or_level32 *levels32(const or_hier *H)
{
    int P = H->P;
    or_level32 *L32 = calloc((size_t)H->nlev, sizeof(or_level32));
    for (int l = 0; l < H->nlev; ++l) {
        L32[l].P = P;
        L32[l].N = H->lv[l].N;
        L32[l].omega = (float)H->lv[l].omega;
        for (int i = 0; i < P * P; ++i) {
            L32[l].A[i] = (float)H->lv[l].A[i];
            L32[l].Nm[i] = (float)H->lv[l].Nm[i];
        }
    }
    return L32;
}

/* lb64 in [0, nlev-1] selects the first level visited in FP64 (see
 * cycle32); any other value keeps the default (the coarsest level). */
static void set_lb64(or_hier *H, int lb64)
{
    if (lb64 >= 0 && lb64 < H->nlev) H->lb64 = lb64;
}

/*
 * One FP32-inner cycle on L e = r from e = 0 (r rounded to FP32 first); the
 * correction e is returned in double.  This is the inner step of the
 * defect correction below.
 */
int or_cycle_mixed(int p, int64_t N, double T, double lam, int nu1, int nu2, int gamma,
                   int64_t n_coarse, int omega_mode, double omega_fixed, int lb64,
                   const double *r, double *e)
{
    or_hier H;
    if (build_hier(&H, p, N, T, lam, nu1, nu2, gamma, n_coarse, omega_mode, omega_fixed, 0))
        return -1;
    set_lb64(&H, lb64);
    or_level32 *L32 = levels32(&H);
    int64_t n = N * H.P;
    float *r32 = malloc(sizeof(float) * n), *e32 = malloc(sizeof(float) * n);
    for (int64_t i = 0; i < n; ++i) {
        r32[i] = (float)r[i];
        e32[i] = 0.0f;
    }
    cycle32(&H, L32, 0, r32, e32);
    for (int64_t i = 0; i < n; ++i) e[i] = (double)e32[i];
    free(r32);
    free(e32);
    free(L32);
    free_hier(&H);
    return 0;
}

int or_solve_mixed(int p, int64_t N, double T, double lam, int nu1, int nu2, int gamma,
                   int64_t n_coarse, int omega_mode, double omega_fixed, int lb64,
                   const double *f, double rtol, int max_cycles, double *u, double *relres,
                   double *hist)
{
    or_hier H;
    if (build_hier(&H, p, N, T, lam, nu1, nu2, gamma, n_coarse, omega_mode, omega_fixed, 0))
        return -1;
    set_lb64(&H, lb64);
    or_level32 *L32 = levels32(&H);
    int64_t n = N * H.P;
    double *r = malloc(sizeof(double) * n);
    float *r32 = malloc(sizeof(float) * n), *e32 = malloc(sizeof(float) * n);
    memset(u, 0, sizeof(double) * n);
    double r0 = norm2(n, f), rk = r0;
    if (hist) hist[0] = r0;
    int k = 0;
    while (k < max_cycles && rk > rtol * r0) {
        residual(&H.lv[0], 0, f, u, r);
        for (int64_t i = 0; i < n; ++i) {
            r32[i] = (float)r[i];
            e32[i] = 0.0f;
        }
        cycle32(&H, L32, 0, r32, e32);
        for (int64_t i = 0; i < n; ++i) u[i] += (double)e32[i];
        ++k;
        residual(&H.lv[0], 0, f, u, r);
        rk = norm2(n, r);
        if (hist) hist[k] = rk;
    }
    *relres = r0 > 0.0 ? rk / r0 : 0.0;
    free(r);
    free(r32);
    free(e32);
    free(L32);
    free_hier(&H);
    return k;
}

/* ---------------------------------------------------------------------- */
/* Gradients of J = 1/2 sum_n (w_n - y_n)^2, w_n = u_n(t_n^-)              */
/* ---------------------------------------------------------------------- */

/*
 * Given the forward solution u of L u = f(u0) and the adjoint solution z of
 * L^T z = g with g_n[k] = (w_n - y_n) psi_k(t_n^-), the gradients are
 *   dJ/df = z,  dJ/du0 = sum_k psi_k(t_0^+) z_0[k],
 *   dJ/dlambda = -sum_n z_n^T M_tau u_n   (dL/dlambda = blockdiag(M_tau)).
 */
int or_adjoint_rhs(int p, int64_t N, const double *u, const double *y, double *g, double *J)
{
    int P = p + 1;
    double s = 0.0;
    for (int64_t n = 0; n < N; ++n) {
        double w = 0.0;
        for (int k = 0; k < P; ++k) w += legendre(k, 1.0) * u[n * P + k];
        double d = w - y[n];
        s += 0.5 * d * d;
        for (int k = 0; k < P; ++k) g[n * P + k] = d * legendre(k, 1.0);
    }
    *J = s;
    return 0;
}

int or_gradients(int p, int64_t N, double tau, double lam, const double *u, const double *z,
                 double *dlam, double *du0)
{
    or_level lv;
    int P = p + 1;
    slab_matrices(P, tau, lam, &lv);
    double s = 0.0;
    for (int64_t n = 0; n < N; ++n)
        for (int k = 0; k < P; ++k)
            for (int l = 0; l < P; ++l) s += z[n * P + k] * lv.M[k * P + l] * u[n * P + l];
    *dlam = -s;
    double d = 0.0;
    for (int k = 0; k < P; ++k) d += legendre(k, -1.0) * z[k];
    *du0 = d;
    return 0;
}
