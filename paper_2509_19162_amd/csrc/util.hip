// Small bookkeeping kernels of the layer pipeline.
#include "internal.h"

namespace cg {

namespace {

__global__ void clear_words_kernel(uint32_t *__restrict__ a, uint32_t na,
                                   uint64_t *__restrict__ b, uint32_t nb) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < na) a[i] = 0;
    if (i < nb) b[i] = 0;
}

}  // namespace

void launch_clear(uint32_t *a, uint32_t na, uint64_t *b, uint32_t nb, hipStream_t s) {
    const uint32_t n = na > nb ? na : nb;
    if (!n) return;
    hipLaunchKernelGGL(clear_words_kernel, dim3((n + 255) / 256), dim3(256), 0, s, a, na, b, nb);
    CG_HIP(hipGetLastError());
}

}  // namespace cg
