// Batch-OMP kernels with the A0_MFMA_BF16X6 correlation stage.
#include "omp_batch_impl.h"

namespace sc {

hipError_t launch_omp_batch_bf16(const DictDev &dict, const OmpParams &p, int kmax, int row_cache,
                                 hipStream_t st) {
    return launch_batch_mode<A0_MFMA_BF16X6>(dict, p, kmax, row_cache, st);
}

}  // namespace sc
