// Streaming leg kernels (k_leg), FP64 instantiations.
#include <hip/hip_runtime.h>

#include "tmg_kernels.h"

namespace tmg {

template hipError_t launch_leg<double>(int, bool, const LegArgsT<double> &, int64_t, hipStream_t);

}  // namespace tmg
