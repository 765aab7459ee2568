// peak.hip -- vector FMA rate of the device, the compute roof of the cell
// kernels' roofline (the cell kernels are bound by FP64 vector arithmetic).
//
// Every lane runs eight independent FMA chains, x <- x * a + b, for a given
// number of steps: enough independent work per wave to keep the SIMDs
// issuing every cycle.  a and b are kernel arguments, so the chains cannot
// be folded, and one store per lane keeps them live.  FP32 runs as plain
// v_fma_f32 (the library is built without packed FP32 instructions), so its
// rate is the unpacked one.
#include "peak.h"

namespace vc {

namespace {

template <typename T>
__global__ __launch_bounds__(256) void k_fma_rate(T *out, int steps, T a, T b)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    T x0 = (T)t * (T)1e-9, x1 = x0 + (T)1, x2 = x0 + (T)2, x3 = x0 + (T)3;
    T x4 = x0 + (T)4, x5 = x0 + (T)5, x6 = x0 + (T)6, x7 = x0 + (T)7;
    for (int i = 0; i < steps; i++) {
        x0 = fma(x0, a, b);
        x1 = fma(x1, a, b);
        x2 = fma(x2, a, b);
        x3 = fma(x3, a, b);
        x4 = fma(x4, a, b);
        x5 = fma(x5, a, b);
        x6 = fma(x6, a, b);
        x7 = fma(x7, a, b);
    }
    out[t] = ((x0 + x1) + (x2 + x3)) + ((x4 + x5) + (x6 + x7));
}

}  // namespace

hipError_t launch_fma_rate(void *out, int fp64, int blocks, int steps, hipStream_t s)
{
    if (fp64) k_fma_rate<double><<<blocks, 256, 0, s>>>((double *)out, steps, 0.999999, 1e-7);
    else k_fma_rate<float><<<blocks, 256, 0, s>>>((float *)out, steps, 0.999999f, 1e-7f);
    return hipGetLastError();
}

}  // namespace vc
