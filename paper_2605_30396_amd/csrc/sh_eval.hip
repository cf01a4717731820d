// Radiance straight from sparse codes (Sec. 2.2 of the paper).
//
// For a Gaussian with code {(idx_t, coef_t)} and view direction w:
//   rgb_c(w) = sum_t coef_t * sum_{j<nb} D[idx_t][c*nb + j] * Y_j(w)
// The dense SH vector is never formed in memory: each thread reads its
// Gaussian's codes once from HBM, and the shared dictionary is staged in LDS
// (it is read k times per Gaussian, the codes once).  The memory-traffic
// argument is the paper's Eq. (2)-(3): per Gaussian the codes (8k bytes)
// replace the 180 bytes of FP32 rest coefficients.
#include "sc_internal.h"
#include "sh_basis.h"

namespace sc {

constexpr int kShThreads = 1024;
constexpr int kAtomStride = 48;                 // 45 floats padded to a multiple of 4
constexpr int kShLdsAtoms = (128 * 1024) / (kAtomStride * 4);   // atoms staged in LDS

template <int NB, bool LDS>
__global__ __launch_bounds__(kShThreads) void sh_eval_kernel(const float *__restrict__ D, int K,
                                                             const int32_t *__restrict__ idx,
                                                             const float *__restrict__ coef,
                                                             const int32_t *__restrict__ count, int64_t N, int k,
                                                             const float *__restrict__ dirs, int64_t M, int shared,
                                                             float *__restrict__ rgb) {
    constexpr int d = 3 * NB;
    extern __shared__ __align__(16) float sD[];
    if (LDS) {
        for (int q = threadIdx.x; q < K * kAtomStride; q += kShThreads) {
            int j = q / kAtomStride, i = q - j * kAtomStride;
            sD[q] = i < d ? D[(size_t)j * d + i] : 0.f;
        }
        __syncthreads();
    }
    const int64_t items = shared ? N * M : N;
    for (int64_t it = (int64_t)blockIdx.x * kShThreads + threadIdx.x; it < items;
         it += (int64_t)gridDim.x * kShThreads) {
        const int64_t g = shared ? it / M : it;
        const int64_t m = shared ? it - g * M : it;
        const int cnt = count[g];
        float r = 0.f, gr = 0.f, b = 0.f;
        if (cnt < 0) {
            r = gr = b = __builtin_nanf("");
        } else {
            float x = dirs[3 * m], y = dirs[3 * m + 1], z = dirs[3 * m + 2];
            const float inv = rsqrtf(x * x + y * y + z * z);
            x *= inv;
            y *= inv;
            z *= inv;
            float Y[NB];
            sh_basis<NB>(x, y, z, Y);
            const int n = cnt < k ? cnt : k;
            const int32_t *ix = idx + g * k;
            const float *cf = coef + g * k;
            for (int t = 0; t < n; ++t) {
                const int j = ix[t];
                if (j < 0 || j >= K) continue;
                const float c = cf[t];
                const float *a = LDS ? sD + j * kAtomStride : D + (size_t)j * d;
                float s0 = 0.f, s1 = 0.f, s2 = 0.f;
#pragma unroll
                for (int q = 0; q < NB; ++q) {
                    s0 = fmaf(a[q], Y[q], s0);
                    s1 = fmaf(a[NB + q], Y[q], s1);
                    s2 = fmaf(a[2 * NB + q], Y[q], s2);
                }
                r = fmaf(c, s0, r);
                gr = fmaf(c, s1, gr);
                b = fmaf(c, s2, b);
            }
        }
        rgb[3 * it] = r;
        rgb[3 * it + 1] = gr;
        rgb[3 * it + 2] = b;
    }
}

template <int NB>
static hipError_t launch_sh_t(const DictDev &dict, const int32_t *idx, const float *coef, const int32_t *count,
                              int64_t N, int k, const float *dirs, int64_t M, int shared, float *rgb,
                              hipStream_t st) {
    int dev = 0, ncu = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t items = shared ? N * M : N;
    int64_t blocks = std::min<int64_t>((items + kShThreads - 1) / kShThreads, (int64_t)ncu);
    if (blocks < 1) blocks = 1;
    if (dict.K <= kShLdsAtoms) {
        size_t smem = sizeof(float) * (size_t)dict.K * kAtomStride;
        auto kern = sh_eval_kernel<NB, true>;
        static bool attr = false;
        if (!attr) {
            hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               128 * 1024);
            if (e != hipSuccess) return e;
            attr = true;
        }
        hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(kShThreads), smem, st, dict.D, dict.K, idx, coef,
                           count, N, k, dirs, M, shared, rgb);
    } else {
        hipLaunchKernelGGL((sh_eval_kernel<NB, false>), dim3((unsigned)blocks), dim3(kShThreads), 0, st, dict.D,
                           dict.K, idx, coef, count, N, k, dirs, M, shared, rgb);
    }
    return hipGetLastError();
}

hipError_t launch_sh_eval(const DictDev &dict, const int32_t *idx, const float *coef, const int32_t *count,
                          int64_t N, int k, const float *dirs, int64_t M, int shared, float *rgb,
                          hipStream_t st) {
    switch (dict.d) {
        case 9: return launch_sh_t<3>(dict, idx, coef, count, N, k, dirs, M, shared, rgb, st);
        case 24: return launch_sh_t<8>(dict, idx, coef, count, N, k, dirs, M, shared, rgb, st);
        case 45: return launch_sh_t<15>(dict, idx, coef, count, N, k, dirs, M, shared, rgb, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace sc
