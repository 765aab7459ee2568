// peak.h -- launcher of the vector FMA rate microbenchmark (peak.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace vc {

// blocks x 256 lanes, eight FMA chains of `steps` each; out holds one value
// per lane (fp64 ? double : float)
hipError_t launch_fma_rate(void *out, int fp64, int blocks, int steps, hipStream_t s);

}  // namespace vc
