// Coarse-level scan, halo seeding, norms, convergence state and host
// summary, adjoint gradients, and the static scratch of the entry point that
// allocates nothing.
#include <hip/hip_runtime.h>

#include <mutex>

#include "tmg_kernels.h"
#include "tmg_tables.h"

namespace tmg {

hipError_t launch_coarse(int P, bool backward, const CoarseArgs &a, int ninst, hipStream_t s)
{
    if (ninst <= 0) return hipSuccess;
    if (a.generic) {
        TMG_DISPATCH_PALL(P, { return launch_gcoarse_p<PP>(backward, a, a.periodic, ninst, s); })
        return hipErrorInvalidValue;
    }
    TMG_DISPATCH_P(P, {
        if (backward) hipLaunchKernelGGL((k_coarse<PP, true>), dim3(ninst), dim3(kThreads), 0, s, a);
        else hipLaunchKernelGGL((k_coarse<PP, false>), dim3(ninst), dim3(kThreads), 0, s, a);
    })
    return hipGetLastError();
}

template <typename TIO>
hipError_t launch_bottom(int P, bool backward, const BottomArgsT<TIO> &a, int ninst, hipStream_t s)
{
    if (ninst <= 0) return hipSuccess;
    if (a.generic) {
        if constexpr (std::is_same<TIO, double>::value) return launch_gbottom(P, backward, a, ninst, s);
        else return hipErrorInvalidValue;
    }
    TMG_DISPATCH_P(P, { return launch_bottom_p<TIO, PP>(backward, a, ninst, s); })
    return hipErrorInvalidValue;
}

hipError_t launch_gleg(int P, bool backward, const LegArgsT<double> &a, int64_t ntiles,
                       hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    TMG_DISPATCH_PALL(P, { return launch_gleg_p<PP>(backward, a, ntiles, s); })
    return hipErrorInvalidValue;
}

hipError_t launch_gbottom(int P, bool backward, const BottomArgsT<double> &a, int ninst,
                          hipStream_t s)
{
    if (ninst <= 0) return hipSuccess;
    TMG_DISPATCH_PALL(P, { return launch_gbottom_p<PP>(backward, a, ninst, s); })
    return hipErrorInvalidValue;
}
template hipError_t launch_bottom<double>(int, bool, const BottomArgsT<double> &, int, hipStream_t);
template hipError_t launch_bottom<float>(int, bool, const BottomArgsT<float> &, int, hipStream_t);

hipError_t launch_seed(int P, bool backward, const double *u, double *hb, const int64_t *tile_off,
                       const int *tile_inst, const int64_t *slab_off, int batch, int64_t n0,
                       int tile_out, int halo, int64_t ntiles, hipStream_t s)
{
    const int64_t n = ntiles * halo;
    if (n <= 0) return hipSuccess;
    const dim3 grid((unsigned)((n + kThreads - 1) / kThreads)), block(kThreads);
    TMG_DISPATCH_P(P, {
        if (backward)
            hipLaunchKernelGGL((k_seed<PP, true>), grid, block, 0, s, u, hb, tile_off, tile_inst,
                               slab_off, batch, n0, tile_out, halo, n);
        else
            hipLaunchKernelGGL((k_seed<PP, false>), grid, block, 0, s, u, hb, tile_off, tile_inst,
                               slab_off, batch, n0, tile_out, halo, n);
    })
    return hipGetLastError();
}

hipError_t launch_norm_f(int P, const double *f, const double *u0, const double *tab,
                         int tab_stride, const int64_t *slab_off, const int64_t *tile_off,
                         const int *tile_inst, int batch, double *partial, int64_t ntiles,
                         hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    TMG_DISPATCH_PALL(P, {
        hipLaunchKernelGGL((k_norm_f<PP>), dim3((unsigned)ntiles), dim3(kLegThreads), 0, s, f, u0, tab,
                           tab_stride, slab_off, tile_off, tile_inst, batch, partial);
    })
    return hipGetLastError();
}

hipError_t launch_finalize(const double *partial, const int64_t *norm_off, int batch,
                           InstState *st, const Control *ctl, HostHead *mirror, int is_r0,
                           hipStream_t s, Control *ctl_set, const Control *val)
{
    Control v{};
    if (val) v = *val;
    hipLaunchKernelGGL(k_finalize, dim3(batch), dim3(kFinThreads), 0, s, partial, norm_off, st, ctl,
                       mirror, is_r0, ctl_set, v);
    return hipGetLastError();
}

hipError_t launch_publish(const InstState *st, int batch, const Control *ctl, HostHead *mirror,
                          unsigned *count, hipStream_t s)
{
    hipLaunchKernelGGL(k_publish, dim3(1), dim3(kFinThreads), 0, s, st, batch, ctl, mirror, count);
    return hipGetLastError();
}

// ---- the static scratch of the entry point that allocates nothing --------
// One array per device, held from the library's load to the end of the
// process.  Host code never names it in a launch or copy: its device
// address, looked up once per device with that device current, is what
// the driver hands out (the name itself is a host-side stand-in).
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

hipError_t noalloc_scratch(void **ptr, size_t *bytes)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    *bytes = kNoAllocScratchBytes;
    return hipSuccess;
}

hipError_t launch_grad(int P, const double *u, const double *z, const double *tau,
                       const int64_t *slab_off, const int64_t *tile_off, const int *tile_inst,
                       int64_t ntiles, int batch, double *partial, double *out, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    TMG_DISPATCH_PALL(P, {
        hipLaunchKernelGGL((k_grad_partial<PP>), dim3((unsigned)ntiles), dim3(kLegThreads), 0, s,
                           u, z, slab_off, tile_off, tile_inst, batch, partial);
        hipLaunchKernelGGL((k_grad_finish<PP>), dim3(batch), dim3(kThreads), 0, s, partial,
                           tile_off, z, tau, slab_off, out);
    })
    return hipGetLastError();
}

// Every (level, instance) table block rebuilt from lambda (device), one
// thread per block: the forward and transposed FP64 tables and, for the
// FP32-inner cycle, their FP32 roundings.  A lambda that is not finite and
// positive leaves NaN tables, so the next solve ends non-finite.
__global__ void k_set_tables(int P, const double *__restrict__ lam, const double *__restrict__ T,
                             const int64_t *__restrict__ N, const int *__restrict__ nlev,
                             int batch, int Lmax, int omega_mode, double omega, int stride,
                             double *__restrict__ tab_fwd, double *__restrict__ tab_adj,
                             float *__restrict__ t32f, float *__restrict__ t32a)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)Lmax * batch) return;
    const int l = (int)(idx / batch), j = (int)(idx - (int64_t)l * batch);
    if (l >= nlev[j]) return;
    const int64_t at = idx * stride;   // block (l, j) at (l * batch + j) * stride
    double *tf = tab_fwd + at, *ta = tab_adj + at;
    const double lj = lam[j];
    if (isfinite(lj) && lj > 0.0) {
        const double z = level_z(lj, T[j], N[j], l);
        level_table(P, z, omega_mode, omega, false, tf);
        level_table(P, z, omega_mode, omega, true, ta);
    } else {
        for (int i = 0; i < stride; ++i) tf[i] = ta[i] = __builtin_nan("");
    }
    if (t32f)
        for (int i = 0; i < stride; ++i) {
            t32f[at + i] = (float)tf[i];
            t32a[at + i] = (float)ta[i];
        }
}

hipError_t launch_set_tables(int P, const double *lam, const double *T, const int64_t *N,
                             const int *nlev, int batch, int Lmax, int omega_mode, double omega,
                             int stride, double *tab_fwd, double *tab_adj, float *t32f,
                             float *t32a, hipStream_t s)
{
    const int64_t n = (int64_t)Lmax * batch;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_set_tables, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, P, lam, T, N,
                       nlev, batch, Lmax, omega_mode, omega, stride, tab_fwd, tab_adj, t32f, t32a);
    return hipGetLastError();
}

}  // namespace tmg
