// Shared declarations of the space-time heat equation's kernels
// (tmg_heat.hip) and driver (tmg_heat_capi.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tmg {

constexpr int kHeatThreads = 64;   // one wavefront per tile of as many slabs
constexpr int kHeatMaxChunks = 8;  // wavefronts sharing a tile in a partitioned leg
// LDS of a partitioned leg: the chunk end exchange and the level's four
// per-point tables (read from global memory when they do not fit)
constexpr size_t kHeatPartLdsBytes = 64 * 1024;
inline size_t heat_part_lds_bytes(int P, int nx, int chunks)
{
    return sizeof(double) * ((size_t)2 * chunks * kHeatThreads * P + (size_t)4 * nx * P * P);
}

// One leg of the heat cycle on one level (see k_hleg), or the coarsest
// level's exact solve (k_hcoarse: f, u0, u_out, Cinv, G, Md, ih2, ws, N, nx).
struct HeatArgs {
    const double *f;        // right-hand side of the level, [point][slab][k]
    const double *u0;       // [nx] initial values entering slab 0 (zeros above level 0)
    const double *u_in;     // iterate (null: zero)
    const double *e;        // next level's correction to prolongate (null: none)
    double *u_out;          // result (null: none)
    double *rc;             // restricted residual into the next level (null: none)
    double *partial;        // per-tile squared residual (null: none)
    const double *Cinv;     // [nx][P*P] C_i^{-1} of the block elimination over the points
    const double *G;        // [nx][P*P] C_i^{-1} E
    const double *K;        // [P*P] the slab's K
    const double *Md;       // [P] diagonal of the slab's M (tau / (2k + 1))
    const double *R;        // R_1^T then R_2^T (P*P each)
    double *ws;             // workspace, 2 nx kHeatThreads P doubles per tile
    int64_t N, Nc;          // slabs of this level and of the next
    double ih2;             // 1 / h^2
    double omc, om;         // 1 - omega, omega
    int nx, halo, tile_out, sweeps, norm_f;
    // partitioned legs (k_hlegp): `chunks` chunks of the points, the
    // elimination factors restarted at each chunk's first point, the spikes
    // and the reduced system's inverse ((2 chunks P)^2)
    int chunks;
    const double *Cl, *Gl, *SL, *SR, *Minv;
};

// lean: the variant with fewer registers per wavefront (more resident), for
// launches with more tiles than two wavefronts per SIMD
hipError_t launch_hleg(int P, const HeatArgs &a, int64_t ntiles, bool lean, hipStream_t s);
// a leg whose spatial solves are partitioned over a.chunks wavefronts (sweeps >= 1)
hipError_t launch_hlegp(int P, const HeatArgs &a, int64_t ntiles, hipStream_t s);
hipError_t launch_hcoarse(int P, const HeatArgs &a, hipStream_t s);
hipError_t launch_hsum(const double *partial, int64_t n, double *out, hipStream_t s);

}  // namespace tmg
