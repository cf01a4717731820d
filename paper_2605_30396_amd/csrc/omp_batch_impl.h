// Single-dictionary Batch-OMP kernel and its launchers, instantiated per
// alpha0 mode in omp_batch_{valu,mfma,bf16}.hip (compiled in parallel).
#pragma once
#include <algorithm>

#include "omp_core.h"

namespace sc {

// Workgroup shape: the matrix-core correlations (FP32 or split BF16) of
// dictionaries of 128..512 atoms run 8 waves on 32-signal tiles, so every
// dictionary read from the cache feeds twice the signals (the correlation
// stage is bound by those reads); the LDS tile (75 KB at K = 512) still lets
// two workgroups share a compute unit.  Every other case runs 4 waves on
// 16-signal tiles.
template <int E, int MODE>
struct BatchShape {
    static constexpr int NW = ((MODE == A0_MFMA_F32 || MODE == A0_MFMA_BF16X6) && E >= 2 && E <= 8) ? 8 : kOmpWaves;
    static constexpr int T = 4 * NW;
};

template <int E, int KMAX, int MODE, int RCQ>
__global__ __launch_bounds__((64 * BatchShape<E, MODE>::NW)) __attribute__((amdgpu_waves_per_eu(4)))
void omp_batch_kernel(DictDev dict, OmpParams p) {
    constexpr int NW = BatchShape<E, MODE>::NW, T = BatchShape<E, MODE>::T;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    OmpTally tally;
    int64_t Nsig = p.N;
    if (p.rows) Nsig = min<int64_t>(Nsig, (int64_t)*p.nrows);
    const int64_t ntiles = (Nsig + T - 1) / T;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t s0 = tile * T;
        const int nt = (int)min<int64_t>(T, Nsig - s0);
        // thread-derived addresses are recomputed per tile rather than held
        // live across the loop
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        omp_tile<E, KMAX, T, MODE == A0_MFMA_BF16X6, RCQ, NW>(dict, p, MODE, s0, nt, smem_raw, tid, tally);
    }
    // counters: one pair of atomics per workgroup (device-wide atomics on one
    // address serialise, and every wave ends at about the same time)
    __shared__ unsigned long long red[NW][2];
    if (p.stats) {
        if ((threadIdx.x & 63) == 0) {
            red[threadIdx.x >> 6][0] = tally.sig;
            red[threadIdx.x >> 6][1] = tally.atoms;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long sg = 0, at = 0;
            for (int w = 0; w < NW; ++w) {
                sg += red[w][0];
                at += red[w][1];
            }
            if (sg) {
                atomicAdd(p.stats + 0, sg);
                atomicAdd(p.stats + 1, at);
            }
        }
    }
}

inline int device_cus() {
    int dev = 0, ncu = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    return ncu;
}

template <int E, int KMAX, int MODE, int RCQ>
static hipError_t launch_batch_t(const DictDev &dict, const OmpParams &p, hipStream_t st) {
    constexpr int Kp = 64 * E, NW = BatchShape<E, MODE>::NW, T = BatchShape<E, MODE>::T;
    const size_t smem = omp_tile_lds(T, Kp, MODE == A0_MFMA_BF16X6);
    auto kern = omp_batch_kernel<E, KMAX, MODE, RCQ>;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const int64_t ntiles = (p.N + T - 1) / T;   // upper bound in list mode
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)kern, 64 * NW, smem) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    const int64_t grid = std::min<int64_t>(ntiles, (int64_t)device_cus() * per_cu);
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(64 * NW), smem, st, dict, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !p.fp64_refit) return e;
    return launch_omp_refit(dict, p, st);
}

// row_cache: 0 or 4 Gram rows kept in registers (4 only for E <= 8)
template <int MODE>
static hipError_t launch_batch_mode(const DictDev &dict, const OmpParams &p, int kmax, int row_cache,
                                    hipStream_t st) {
#define SC_CASE(EE, KK)                                                                  \
    if (dict.E == EE && kmax == KK) {                                                    \
        if constexpr (EE <= 8)                                                           \
            if (row_cache > 0) return launch_batch_t<EE, KK, MODE, 4>(dict, p, st);      \
        return launch_batch_t<EE, KK, MODE, 0>(dict, p, st);                             \
    }
    SC_CASE(1, 4) SC_CASE(1, 8) SC_CASE(1, 12) SC_CASE(1, 16) SC_CASE(1, 24) SC_CASE(1, 32)
    SC_CASE(2, 4) SC_CASE(2, 8) SC_CASE(2, 12) SC_CASE(2, 16) SC_CASE(2, 24) SC_CASE(2, 32)
    SC_CASE(4, 4) SC_CASE(4, 8) SC_CASE(4, 12) SC_CASE(4, 16) SC_CASE(4, 24) SC_CASE(4, 32)
    SC_CASE(8, 4) SC_CASE(8, 8) SC_CASE(8, 12) SC_CASE(8, 16) SC_CASE(8, 24) SC_CASE(8, 32)
    SC_CASE(12, 4) SC_CASE(12, 8) SC_CASE(12, 12) SC_CASE(12, 16)
    SC_CASE(16, 4) SC_CASE(16, 8) SC_CASE(16, 12) SC_CASE(16, 16)
#undef SC_CASE
    return hipErrorInvalidValue;
}

}  // namespace sc
