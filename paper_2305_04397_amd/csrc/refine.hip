// Device helper of the assignment check after an FP32 solve: the values of
// the re-solved (column, model) pairs at their initial states.
#include "common.h"
#include "kern.h"

namespace morap {
namespace k {

__global__ void gather_values_kernel(int n, const int64_t* __restrict__ idx, const double* __restrict__ x,
                                     double* __restrict__ out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int64_t i = idx[q];
    out[q] = i >= 0 ? x[i] : 0.0;
}

void gather_values(hipStream_t s, int n, const int64_t* idx, const double* x, double* out) {
    if (n <= 0) return;
    hipLaunchKernelGGL(gather_values_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, idx, x, out);
    MORAP_HIP(hipGetLastError());
}

}  // namespace k
}  // namespace morap
