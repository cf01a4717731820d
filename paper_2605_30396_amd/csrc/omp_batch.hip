// Batch-OMP over one dictionary: a persistent grid of 4-wave workgroups
// walks the 16-signal tiles (tile body in omp_core.h), then a scan pass
// refits the supports flagged as ill-conditioned in FP64.
//
// alpha0 modes:
//   A0_VALU         FP32 FMAs from the feature-major dictionary
//   A0_MFMA_F32     v_mfma_f32_16x16x4_f32, FP32 operands (same precision)
//   A0_MFMA_BF16X6  v_mfma_f32_16x16x32_bf16 on three-part BF16 splits of D
//                   and x, six products summed in FP32: correlations of FP32
//                   accuracy from BF16 matrix cores (half the matrix-core time
//                   of A0_MFMA_F32).
#include <algorithm>

#include "omp_batch_impl.h"

namespace sc {

__global__ __launch_bounds__(kOmpThreads) void omp_refit_kernel(DictDev dict, OmpParams p) {
    __shared__ RefitScratch ws[kOmpWaves];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const unsigned long long nref = refit_scan(dict, p, (int64_t)blockIdx.x * kOmpWaves + wave,
                                               (int64_t)gridDim.x * kOmpWaves, ws[wave], lane);
    if (p.stats && lane == 0 && nref) atomicAdd(p.stats + 2, nref);
}

hipError_t launch_omp_refit(const DictDev &dict, const OmpParams &p, hipStream_t st) {
    const int64_t nchunks = (p.N + 63) / 64;   // upper bound in list mode
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>((nchunks + kOmpWaves - 1) / kOmpWaves,
                                                                (int64_t)device_cus() * 4));
    hipLaunchKernelGGL(omp_refit_kernel, dim3((unsigned)grid), dim3(kOmpThreads), 0, st, dict, p);
    return hipGetLastError();
}

// (E, KMAX) pairs with a compiled register-resident pursuit, for each alpha0 mode.
hipError_t launch_omp_batch(const DictDev &dict, const OmpParams &p, int kmax, int a0mode, int row_cache,
                            hipStream_t st) {
    switch (a0mode) {
        case A0_VALU: return launch_omp_batch_valu(dict, p, kmax, row_cache, st);
        case A0_MFMA_F32: return launch_omp_batch_mfma(dict, p, kmax, row_cache, st);
        case A0_MFMA_BF16X6: return launch_omp_batch_bf16(dict, p, kmax, row_cache, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace sc
