// Per-level slab tables from closed forms for the unnormalised Legendre
// basis psi_k(t) = P_k(xi), xi = 2(t - t_{n-1})/tau - 1 (section 2.1):
//   K[k,l] = 1 - 2 [l < k and k + l odd]   (from -int psi_l psi_k' + psi_l psi_k at t_n)
//   M      = tau diag(1/(2k+1))
//   N      = v 1^T,  v[k] = P_k(-1) = (-1)^k,  1[k] = P_k(1) = 1
// so that the diagonal block is A = K + z diag(1/(2k+1)) with z = lambda tau.
// One routine for the host (set-up) and the device (tmg_set_lambda), with
// floating-point contraction off so that both produce the same bits.
#pragma once

#include <hip/hip_runtime.h>

#include "tmg_internal.h"

namespace tmg {

// Gauss-Jordan inverse with partial pivoting (P <= kMaxP, well conditioned).
__host__ __device__ inline void table_invert(int P, const double *A, double *Ainv)
{
#pragma clang fp contract(off)
    double a[kMaxP][2 * kMaxP];
    for (int i = 0; i < P; ++i)
        for (int j = 0; j < P; ++j) {
            a[i][j] = A[i * P + j];
            a[i][P + j] = (i == j) ? 1.0 : 0.0;
        }
    for (int c = 0; c < P; ++c) {
        int piv = c;
        for (int i = c + 1; i < P; ++i)
            if (fabs(a[i][c]) > fabs(a[piv][c])) piv = i;
        if (piv != c)
            for (int j = 0; j < 2 * P; ++j) {
                const double t = a[c][j];
                a[c][j] = a[piv][j];
                a[piv][j] = t;
            }
        const double d = a[c][c];
        for (int j = 0; j < 2 * P; ++j) a[c][j] /= d;
        for (int i = 0; i < P; ++i) {
            if (i == c) continue;
            const double m = a[i][c];
            if (m != 0.0)
                for (int j = 0; j < 2 * P; ++j) a[i][j] -= m * a[c][j];
        }
    }
    for (int i = 0; i < P; ++i)
        for (int j = 0; j < P; ++j) Ainv[i * P + j] = a[i][P + j];
}

// One table block (see TabLayout) for a slab of step z = lambda tau,
// transposed if trans; omega_mode 0: the damping of Lemma chap4_lemma7,
// 1: omega_fixed.  Returns alpha, the nonzero eigenvalue of A^{-1} v c^T.
__host__ __device__ inline double level_table(int P, double z, int omega_mode, double omega_fixed,
                                              bool trans, double *out)
{
#pragma clang fp contract(off)
    const TabLayout L(P);
    for (int i = 0; i < L.stride(); ++i) out[i] = 0.0;
    double A[kMaxP * kMaxP], Ai[kMaxP * kMaxP];
    for (int k = 0; k < P; ++k)
        for (int l = 0; l < P; ++l) {
            const double K = (l < k && ((k + l) & 1)) ? -1.0 : 1.0;
            const double M = (k == l) ? z / (2.0 * k + 1.0) : 0.0;
            // transposed system: diagonal block A^T
            if (trans) A[l * P + k] = K + M;
            else A[k * P + l] = K + M;
        }
    table_invert(P, A, Ai);
    double ones[kMaxP], alt[kMaxP];
    for (int k = 0; k < P; ++k) {
        ones[k] = 1.0;
        alt[k] = (k & 1) ? -1.0 : 1.0;
    }
    // forward: w = 1^T u, injection v = (-1)^k; transposed: w = v^T z, injection 1
    const double *c = trans ? alt : ones;
    const double *v = trans ? ones : alt;
    double q[kMaxP];
    for (int k = 0; k < P; ++k) {
        double s = 0.0;
        for (int l = 0; l < P; ++l) s += Ai[k * P + l] * v[l];
        q[k] = s;
    }
    // alpha = c^T A^{-1} v: the nonzero eigenvalue of the rank-one A^{-1} v c^T
    double alpha = 0.0;
    for (int k = 0; k < P; ++k) alpha += c[k] * q[k];
    // damping of Lemma chap4_lemma7
    const double omega = omega_mode == 0 ? (alpha >= 0.0 ? 1.0 / (1.0 + alpha * alpha) : 1.0)
                                         : omega_fixed;
    for (int i = 0; i < P * P; ++i) {
        out[L.A() + i] = A[i];
        out[L.G() + i] = omega * Ai[i];
        out[L.AI() + i] = Ai[i];
    }
    for (int k = 0; k < P; ++k) {
        out[L.H() + k] = omega * q[k];
        out[L.C() + k] = c[k];
        out[L.V() + k] = v[k];
        out[L.Q() + k] = q[k];
    }
    out[L.OMC()] = 1.0 - omega;
    out[L.ALPHA()] = alpha;
    return alpha;
}

// Step z of level l of an instance with n slabs on (0, T] and decay rate
// lambda (the same expression on host and device).
__host__ __device__ inline double level_z(double lambda, double T, int64_t n, int l)
{
#pragma clang fp contract(off)
    return lambda * T / (double)(n >> l);
}

}  // namespace tmg
