// One-pass CSC encoder kernels with the split-BF16 MFMA correlation stage.
#include "omp_csc_impl.h"

namespace sc {

hipError_t launch_omp_csc_bf16(const DictDev &dict, const OmpParams &p, int kmax, int row_cache, int64_t *colptr,
                               int32_t *rows, float *vals, int64_t cap, void *ws, hipStream_t st) {
    return launch_csc_mode<A0_MFMA_BF16X6>(dict, p, kmax, row_cache, colptr, rows, vals, cap, ws, st);
}

}  // namespace sc
