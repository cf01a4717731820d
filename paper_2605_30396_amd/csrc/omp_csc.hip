// The one-pass CSC encoder: column-pointer refit pass, workspace size and the
// dispatch over correlation stages (kernels in omp_csc_impl.h, instantiated
// per stage in omp_csc_{valu,mfma,bf16}.hip).
#include "omp_csc_impl.h"

namespace sc {

hipError_t launch_omp_csc_valu(const DictDev &dict, const OmpParams &p, int kmax, int row_cache, int64_t *colptr,
                               int32_t *rows, float *vals, int64_t cap, void *ws, hipStream_t st);
hipError_t launch_omp_csc_mfma(const DictDev &dict, const OmpParams &p, int kmax, int row_cache, int64_t *colptr,
                               int32_t *rows, float *vals, int64_t cap, void *ws, hipStream_t st);
hipError_t launch_omp_csc_bf16(const DictDev &dict, const OmpParams &p, int kmax, int row_cache, int64_t *colptr,
                               int32_t *rows, float *vals, int64_t cap, void *ws, hipStream_t st);

// Columns flagged with colptr[i] = -(offset + 1): FP64 refit of their
// coefficients in place, then the pointer is restored.
__global__ __launch_bounds__(kOmpThreads) void omp_csc_refit_kernel(DictDev dict, OmpParams p, int64_t *colptr,
                                                                    const int32_t *__restrict__ rows,
                                                                    float *__restrict__ vals, int64_t cap) {
    __shared__ RefitScratch ws[kOmpWaves];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t N = p.N, nchunks = (N + 63) / 64;
    unsigned long long nref = 0;
    for (int64_t c = (int64_t)blockIdx.x * kOmpWaves + wave; c < nchunks; c += (int64_t)gridDim.x * kOmpWaves) {
        const int64_t i = c * 64 + lane;
        const int64_t v = i < N ? colptr[i] : 0;
        uint64_t flagged = ballot(v < 0);
        while (flagged) {
            const int l = __ffsll((unsigned long long)flagged) - 1;
            flagged &= flagged - 1;
            const int64_t sig = c * 64 + l;
            const int64_t off = -__shfl(v, l, 64) - 1;
            const int64_t nxv = colptr[sig + 1];   // may be flagged too (or being restored)
            const int64_t nx = nxv < 0 ? -nxv - 1 : nxv;
            const int n = __builtin_amdgcn_readfirstlane((int)(nx - off));
            if (off + n <= cap) {
                const double r2 = refit_codes(dict, p.X + sig * dict.d, rows + off, vals + off, n, ws[wave], lane);
                if (lane == 0 && p.resid) p.resid[sig] = (float)sqrt(r2);
            }
            if (lane == 0) colptr[sig] = off;
            nref += 1;
        }
    }
    if (p.stats && lane == 0 && nref) atomicAdd(p.stats + 2, nref);
}

size_t csc_encode_workspace_bytes(int64_t N) {
    const int64_t ntiles = (N + kCscTile - 1) / kCscTile;
    return 256 + sizeof(uint64_t) * (size_t)ntiles;
}

hipError_t launch_omp_csc(const DictDev &dict, const OmpParams &p, int kmax, int a0mode, int row_cache,
                          int64_t *colptr, int32_t *rows, float *vals, int64_t cap, void *ws, hipStream_t st) {
    hipError_t e;
    switch (a0mode) {
        case A0_VALU: e = launch_omp_csc_valu(dict, p, kmax, row_cache, colptr, rows, vals, cap, ws, st); break;
        case A0_MFMA_F32: e = launch_omp_csc_mfma(dict, p, kmax, row_cache, colptr, rows, vals, cap, ws, st); break;
        case A0_MFMA_BF16X6: e = launch_omp_csc_bf16(dict, p, kmax, row_cache, colptr, rows, vals, cap, ws, st); break;
        default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess || !p.fp64_refit) return e;
    int dev = 0, ncu = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t nchunks = (p.N + 63) / 64;
    const int64_t rgrid = std::max<int64_t>(1, std::min<int64_t>((nchunks + kOmpWaves - 1) / kOmpWaves, (int64_t)ncu * 4));
    hipLaunchKernelGGL(omp_csc_refit_kernel, dim3((unsigned)rgrid), dim3(kOmpThreads), 0, st, dict, p, colptr, rows,
                       vals, cap);
    return hipGetLastError();
}

}  // namespace sc
