// Radiance straight from sparse codes (Sec. 2.2 of the paper).
//
// For a Gaussian with code {(idx_t, coef_t)} and view direction w:
//   rgb_c(w) = sum_t coef_t * sum_{j<nb} D[idx_t][c*nb + j] * Y_j(w)
// The dense SH vector is never formed in memory: each thread reads its
// Gaussian's codes once from HBM, and the shared dictionary is staged in LDS
// (it is read k times per Gaussian, the codes once).  The memory-traffic
// argument is the paper's Eq. (2)-(3): per Gaussian the codes (8k bytes)
// replace the 180 bytes of FP32 rest coefficients.
#include <cstdint>

#include "sc_internal.h"
#include "sh_basis.h"

namespace sc {

constexpr int kShThreads = 1024;
// LDS row of an atom: 45 floats padded to 52, a multiple of 4 (16-byte rows
// for vector reads) whose quotient 13 is odd, so atom rows start on 16
// different 4-bank groups of the 64 banks and the random atoms that the
// lanes of a wave read at once seldom share a bank (a 48-float row has only
// 4 starting groups: one atom in 16 per group, 4-way conflicts).
constexpr int kAtomStride = 52;
constexpr int kShLdsAtoms = (128 * 1024) / (kAtomStride * 4);   // atoms staged in LDS

// KV > 0: code rows of k = 4 KV entries are read as KV 16-byte vectors, and
// the next item's count, direction and codes are requested before the current
// item is evaluated (one HBM round trip in flight per thread); KV = 0 reads
// rows of any width entry by entry.
template <int NB, bool LDS, int KV>
__global__ __launch_bounds__(kShThreads) void sh_eval_kernel(const float *__restrict__ D, int K,
                                                             const int32_t *__restrict__ idx,
                                                             const float *__restrict__ coef,
                                                             const int32_t *__restrict__ count, int64_t N, int k,
                                                             const float *__restrict__ dirs, int64_t M, int shared,
                                                             float *__restrict__ rgb) {
    constexpr int d = 3 * NB;
    constexpr int KR = KV > 0 ? 4 * KV : 1;
    extern __shared__ __align__(16) float sD[];
    if (LDS) {
        for (int q = threadIdx.x; q < K * kAtomStride; q += kShThreads) {
            int j = q / kAtomStride, i = q - j * kAtomStride;
            sD[q] = i < d ? D[(size_t)j * d + i] : 0.f;
        }
        __syncthreads();
    }
    const int64_t items = shared ? N * M : N;
    const int64_t stride = (int64_t)gridDim.x * kShThreads;
    struct Item {
        int cnt;
        float x, y, z;
        int jv[KR];
        float cv[KR];
    };
    auto fetch = [&](int64_t it, Item &q) {
        if (it >= items) return;
        const int64_t g = shared ? it / M : it;
        const int64_t m = shared ? it - g * M : it;
        q.cnt = count[g];
        q.x = dirs[3 * m];
        q.y = dirs[3 * m + 1];
        q.z = dirs[3 * m + 2];
        if constexpr (KV > 0) {
            const int4 *iv = reinterpret_cast<const int4 *>(idx + g * k);
            const float4 *fv = reinterpret_cast<const float4 *>(coef + g * k);
#pragma unroll
            for (int v = 0; v < KV; ++v) {
                const int4 a = iv[v];
                const float4 c = fv[v];
                q.jv[4 * v] = a.x, q.jv[4 * v + 1] = a.y, q.jv[4 * v + 2] = a.z, q.jv[4 * v + 3] = a.w;
                q.cv[4 * v] = c.x, q.cv[4 * v + 1] = c.y, q.cv[4 * v + 2] = c.z, q.cv[4 * v + 3] = c.w;
            }
        }
    };
    int64_t it = (int64_t)blockIdx.x * kShThreads + threadIdx.x;
    Item cur{};
    fetch(it, cur);
    for (; it < items; it += stride) {
        Item nxt{};
        fetch(it + stride, nxt);
        const int64_t g = shared ? it / M : it;
        const int cnt = cur.cnt;
        float r = 0.f, gr = 0.f, b = 0.f;
        if (cnt < 0) {
            r = gr = b = __builtin_nanf("");
        } else {
            float x = cur.x, y = cur.y, z = cur.z;
            const float inv = rsqrtf(x * x + y * y + z * z);
            x *= inv;
            y *= inv;
            z *= inv;
            float Y[NB];
            sh_basis<NB>(x, y, z, Y);
            const int n = cnt < k ? cnt : k;
            auto atom = [&](int j, float c) {
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
            };
            if constexpr (KV > 0) {
#pragma unroll
                for (int t = 0; t < KR; ++t) {
                    const int j = cur.jv[t];
                    if (t < n && j >= 0 && j < K) atom(j, cur.cv[t]);
                }
            } else {
                const int32_t *ix = idx + g * k;
                const float *cf = coef + g * k;
                for (int t = 0; t < n; ++t) {
                    const int j = ix[t];
                    if (j < 0 || j >= K) continue;
                    atom(j, cf[t]);
                }
            }
        }
        rgb[3 * it] = r;
        rgb[3 * it + 1] = gr;
        rgb[3 * it + 2] = b;
        cur = nxt;
    }
}

template <int NB, int KV>
static hipError_t launch_sh_kv(const DictDev &dict, const int32_t *idx, const float *coef, const int32_t *count,
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
        auto kern = sh_eval_kernel<NB, true, KV>;
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
        hipLaunchKernelGGL((sh_eval_kernel<NB, false, KV>), dim3((unsigned)blocks), dim3(kShThreads), 0, st,
                           dict.D, dict.K, idx, coef, count, N, k, dirs, M, shared, rgb);
    }
    return hipGetLastError();
}

// Vector code rows need k = 4, 8 or 12 and 16-byte aligned idx / coef (wider
// rows would not fit the double-buffered registers of a 1024-thread block).
template <int NB>
static hipError_t launch_sh_t(const DictDev &dict, const int32_t *idx, const float *coef, const int32_t *count,
                              int64_t N, int k, const float *dirs, int64_t M, int shared, float *rgb,
                              hipStream_t st) {
    const bool al = ((reinterpret_cast<uintptr_t>(idx) | reinterpret_cast<uintptr_t>(coef)) & 15) == 0;
    const int kv = (al && k % 4 == 0 && k <= 12) ? k / 4 : 0;
    switch (kv) {
        case 1: return launch_sh_kv<NB, 1>(dict, idx, coef, count, N, k, dirs, M, shared, rgb, st);
        case 2: return launch_sh_kv<NB, 2>(dict, idx, coef, count, N, k, dirs, M, shared, rgb, st);
        case 3: return launch_sh_kv<NB, 3>(dict, idx, coef, count, N, k, dirs, M, shared, rgb, st);
        default: return launch_sh_kv<NB, 0>(dict, idx, coef, count, N, k, dirs, M, shared, rgb, st);
    }
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
