// Zero-fill of small device buffers by a kernel rather than hipMemsetAsync,
// so that a caller capturing the encoder calls into a HIP graph gets kernel
// nodes only (memset nodes have misbehaved on graph replays).
#include <algorithm>

#include "sc_internal.h"

namespace sc {

__global__ __launch_bounds__(256) void zero_words_kernel(uint32_t *__restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

hipError_t launch_zero_words(void *p, int64_t nwords, hipStream_t st) {
    if (nwords <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((nwords + 255) / 256, 1024);
    hipLaunchKernelGGL(zero_words_kernel, dim3((unsigned)blocks), dim3(256), 0, st, (uint32_t *)p, nwords);
    return hipGetLastError();
}

}  // namespace sc
