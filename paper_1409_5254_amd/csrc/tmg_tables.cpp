// Host-side construction of the per-level slab tables (the closed forms of
// tmg_tables.h) and the factor-2 transfer matrices.
#include <cmath>

#include "tmg_tables.h"

namespace tmg {

double build_level_table(int P, double z, int omega_mode, double omega_fixed, bool trans,
                         double *out)
{
    return level_table(P, z, omega_mode, omega_fixed, trans, out);
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
