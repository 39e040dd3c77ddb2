// Host-side construction of the per-level slab tables and the transfer
// matrices, from closed forms for the unnormalised Legendre basis
// psi_k(t) = P_k(xi), xi = 2(t - t_{n-1})/tau - 1 (section 2.1):
//   K[k,l] = 1 - 2 [l < k and k + l odd]   (from -int psi_l psi_k' + psi_l psi_k at t_n)
//   M      = tau diag(1/(2k+1))
//   N      = v 1^T,  v[k] = P_k(-1) = (-1)^k,  1[k] = P_k(1) = 1
// so that the diagonal block is A = K + z diag(1/(2k+1)) with z = lambda tau.
#include <cmath>
#include <cstring>

#include "tmg_internal.h"

namespace tmg {

namespace {

// Gauss-Jordan inverse with partial pivoting (P <= kMaxP, well conditioned).
void invert(int P, const double *A, double *Ainv)
{
    double a[kMaxP][2 * kMaxP];
    for (int i = 0; i < P; ++i)
        for (int j = 0; j < P; ++j) {
            a[i][j] = A[i * P + j];
            a[i][P + j] = (i == j) ? 1.0 : 0.0;
        }
    for (int c = 0; c < P; ++c) {
        int piv = c;
        for (int i = c + 1; i < P; ++i)
            if (std::fabs(a[i][c]) > std::fabs(a[piv][c])) piv = i;
        if (piv != c)
            for (int j = 0; j < 2 * P; ++j) std::swap(a[c][j], a[piv][j]);
        double d = a[c][c];
        for (int j = 0; j < 2 * P; ++j) a[c][j] /= d;
        for (int i = 0; i < P; ++i) {
            if (i == c) continue;
            double m = a[i][c];
            if (m != 0.0)
                for (int j = 0; j < 2 * P; ++j) a[i][j] -= m * a[c][j];
        }
    }
    for (int i = 0; i < P; ++i)
        for (int j = 0; j < P; ++j) Ainv[i * P + j] = a[i][P + j];
}

}  // namespace

double build_level_table(int P, double z, int omega_mode, double omega_fixed, bool trans,
                         double *out)
{
    const TabLayout L(P);
    std::memset(out, 0, sizeof(double) * L.stride());
    double A[kMaxP * kMaxP], Ai[kMaxP * kMaxP];
    for (int k = 0; k < P; ++k)
        for (int l = 0; l < P; ++l) {
            double K = (l < k && ((k + l) & 1)) ? -1.0 : 1.0;
            double M = (k == l) ? z / (2.0 * k + 1.0) : 0.0;
            // transposed system: diagonal block A^T
            if (trans) A[l * P + k] = K + M;
            else A[k * P + l] = K + M;
        }
    invert(P, A, Ai);
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
    double omega = omega_mode == 0 ? (alpha >= 0.0 ? 1.0 / (1.0 + alpha * alpha) : 1.0)
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

// Column l of R1T (R2T) holds the Legendre coefficients of the coarse basis
// function P_l restricted to the first (second) fine slab, written in the
// fine coordinate xi: P_l((xi - 1)/2) and P_l((xi + 1)/2).  Built with
// Bonnet's recurrence on Legendre coefficient vectors, using
// xi P_k = ((k+1) P_{k+1} + k P_{k-1}) / (2k+1).
void build_transfer(int P, double *R1T, double *R2T)
{
    for (int half = 0; half < 2; ++half) {
        double shift = half == 0 ? -1.0 : 1.0;
        double *R = half == 0 ? R1T : R2T;
        double prev[kMaxP + 1] = {0}, cur[kMaxP + 1] = {0};
        cur[0] = 1.0;  // P_0(y) = 1
        for (int k = 0; k < P; ++k) R[k * P + 0] = cur[k];
        // y = (xi + shift)/2 as an operator on Legendre coefficient vectors
        auto mul_y = [&](const double *in, double *out) {
            double t[kMaxP + 2] = {0};
            for (int k = 0; k <= kMaxP; ++k) {
                if (in[k] == 0.0) continue;
                if (k + 1 <= kMaxP) t[k + 1] += in[k] * (k + 1.0) / (2.0 * k + 1.0);
                if (k >= 1) t[k - 1] += in[k] * k / (2.0 * k + 1.0);
            }
            for (int k = 0; k <= kMaxP; ++k) out[k] = 0.5 * (t[k] + shift * in[k]);
        };
        for (int l = 0; l + 1 < P; ++l) {
            // P_{l+1}(y) = ((2l+1) y P_l(y) - l P_{l-1}(y)) / (l+1)
            double yc[kMaxP + 1], next[kMaxP + 1];
            mul_y(cur, yc);
            for (int k = 0; k <= kMaxP; ++k)
                next[k] = ((2.0 * l + 1.0) * yc[k] - l * prev[k]) / (l + 1.0);
            for (int k = 0; k <= kMaxP; ++k) {
                prev[k] = cur[k];
                cur[k] = next[k];
            }
            for (int k = 0; k < P; ++k) R[k * P + (l + 1)] = cur[k];
        }
    }
}

}  // namespace tmg
