// Span kernels (k_span): several consecutive small levels per launch.
#include <hip/hip_runtime.h>

#include "tmg_kernels.h"

namespace tmg {

template hipError_t launch_span<double>(int, bool, const SpanArgsT<double> &, int64_t, hipStream_t);
template hipError_t launch_span<float>(int, bool, const SpanArgsT<float> &, int64_t, hipStream_t);

}  // namespace tmg
