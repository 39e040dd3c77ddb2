// Streaming leg kernels (k_leg), FP32 instantiations (the inner cycle of the
// FP32-inner defect correction).
#include <hip/hip_runtime.h>

#include "tmg_kernels.h"

namespace tmg {

template hipError_t launch_leg<float>(int, bool, const LegArgsT<float> &, int64_t, hipStream_t);

}  // namespace tmg
