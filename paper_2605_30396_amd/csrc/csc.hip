// Compressed-sparse-column storage of the codes and the consumers that read
// it (Sec. 2.2: only the non-zeros of each Gaussian's code and their atom
// indices are stored, column by column, because the codes have different
// lengths).
//
// Packing is two stream-ordered passes over the padded codes:
//   colptr[i] = sum_{g < i} max(count[g], 0)      (exclusive scan, int64)
//   rows[colptr[i] + t] = idx[i][t], vals[...] = coef[i][t]   (t < count[i])
// The scan: per-block sums (4096 signals per block), one workgroup scanning
// the block sums, then each block scans its own signals from its offset.
//
// Consumers: radiance of the view-dependent SH part from CSC columns (the
// same sum as the padded-code kernel), and the full per-Gaussian colour of
// the 3DGS renderer from CSC: view direction from the Gaussian's position
// and the camera centre, degree-0 term C0 * DC, + 0.5, clamped at 0.
#include "sc_internal.h"
#include "sh_basis.h"

namespace sc {

constexpr int kCscThreads = 256;
constexpr int kCscPerThread = 16;                         // consecutive signals per thread
constexpr int kCscBlock = kCscThreads * kCscPerThread;    // 4096 signals per block

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Inclusive scan over the 64 lanes of a wave.
__device__ __forceinline__ int64_t wave_scan_i64(int64_t v, int lane) {
    for (int off = 1; off < 64; off <<= 1) {
        const int64_t u = __shfl_up(v, off, 64);
        if (lane >= off) v += u;
    }
    return v;
}

__device__ __forceinline__ int nz(int c) { return c > 0 ? c : 0; }

__global__ __launch_bounds__(kCscThreads) void csc_block_sums_kernel(const int32_t *__restrict__ count, int64_t N,
                                                                     int64_t *__restrict__ bsum) {
    __shared__ int64_t part[kCscThreads / 64];
    const int64_t i0 = (int64_t)blockIdx.x * kCscBlock + (int64_t)threadIdx.x * kCscPerThread;
    int64_t s = 0;
    for (int q = 0; q < kCscPerThread; ++q)
        if (i0 + q < N) s += nz(count[i0 + q]);
    s = wave_sum_i64(s);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int w = 0; w < kCscThreads / 64; ++w) t += part[w];
        bsum[blockIdx.x] = t;
    }
}

// Exclusive scan of nb block sums in place (one workgroup); the total goes
// to *total.
__global__ __launch_bounds__(1024) void csc_scan_sums_kernel(int64_t *__restrict__ bsum, int64_t nb,
                                                             int64_t *__restrict__ total) {
    __shared__ int64_t wtot[16];
    __shared__ int64_t carry_sh;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) carry_sh = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < nb; c0 += 1024) {
        const int64_t i = c0 + tid;
        const int64_t v = i < nb ? bsum[i] : 0;
        const int64_t inc = wave_scan_i64(v, lane);
        if (lane == 63) wtot[wave] = inc;
        __syncthreads();
        int64_t before = carry_sh;
        for (int w = 0; w < wave; ++w) before += wtot[w];
        if (i < nb) bsum[i] = before + inc - v;
        __syncthreads();
        if (tid == 0) {
            int64_t t = 0;
            for (int w = 0; w < 16; ++w) t += wtot[w];
            carry_sh += t;
        }
        __syncthreads();
    }
    if (tid == 0) *total = carry_sh;
}

__global__ __launch_bounds__(kCscThreads) void csc_colptr_kernel(const int32_t *__restrict__ count, int64_t N,
                                                                 const int64_t *__restrict__ boff,
                                                                 int64_t *__restrict__ colptr) {
    __shared__ int64_t wtot[kCscThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t i0 = (int64_t)blockIdx.x * kCscBlock + (int64_t)tid * kCscPerThread;
    int c[kCscPerThread];
    int64_t s = 0;
#pragma unroll
    for (int q = 0; q < kCscPerThread; ++q) {
        c[q] = i0 + q < N ? nz(count[i0 + q]) : 0;
        s += c[q];
    }
    const int64_t inc = wave_scan_i64(s, lane);
    if (lane == 63) wtot[wave] = inc;
    __syncthreads();
    int64_t off = boff[blockIdx.x] + inc - s;
    for (int w = 0; w < wave; ++w) off += wtot[w];
#pragma unroll
    for (int q = 0; q < kCscPerThread; ++q) {
        if (i0 + q < N) colptr[i0 + q] = off;
        off += c[q];
    }
}

// One thread per (signal, slot).
__global__ void csc_fill_kernel(const int32_t *__restrict__ idx, const float *__restrict__ coef,
                                const int32_t *__restrict__ count, int64_t N, int k,
                                const int64_t *__restrict__ colptr, int32_t *__restrict__ rows,
                                float *__restrict__ vals) {
    const int64_t total = N * k;
    for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < total;
         it += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = it / k;
        const int t = (int)(it - i * k);
        if (t < nz(count[i])) {
            const int64_t o = colptr[i] + t;
            rows[o] = idx[it];
            vals[o] = coef[it];
        }
    }
}

// LDS row of an atom: 45 floats padded to 52 (16-byte rows; the odd quotient
// 13 spreads the rows of random atoms over 16 starting bank groups, where a
// 48-float row would give 4 and 4-way bank conflicts).
constexpr int kStride = 52;

// The view-dependent radiance of one CSC column at unit direction (x, y, z).
template <int NB, bool LDS>
__device__ __forceinline__ void csc_column_rgb(const float *__restrict__ D, const float *__restrict__ sD, int K,
                                               const int32_t *__restrict__ rows, const float *__restrict__ vals,
                                               int64_t c0, int64_t c1, float x, float y, float z, float &r,
                                               float &gr, float &b) {
    constexpr int d = 3 * NB;
    float Y[NB];
    sh_basis<NB>(x, y, z, Y);
    r = gr = b = 0.f;
    for (int64_t e = c0; e < c1; ++e) {
        const int j = rows[e];
        if (j < 0 || j >= K) continue;
        const float c = vals[e];
        const float *a = LDS ? sD + j * kStride : D + (size_t)j * d;
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

// mode 0: per-Gaussian or shared directions (like sh_eval_sparse);
// mode 1: the 3DGS colour from positions, DC terms and a camera centre.
template <int NB, bool LDS, int MODE>
__global__ __launch_bounds__(1024) void csc_eval_kernel(const float *__restrict__ D, int K,
                                                        const int64_t *__restrict__ colptr,
                                                        const int32_t *__restrict__ rows,
                                                        const float *__restrict__ vals, int64_t N,
                                                        const float *__restrict__ dirs, int64_t M, int shared,
                                                        const float *__restrict__ pos, const float *__restrict__ dc,
                                                        float cx, float cy, float cz, float *__restrict__ rgb) {
    constexpr int d = 3 * NB;
    extern __shared__ __align__(16) float sD[];
    if (LDS) {
        for (int q = threadIdx.x; q < K * kStride; q += blockDim.x) {
            const int j = q / kStride, i = q - j * kStride;
            sD[q] = i < d ? D[(size_t)j * d + i] : 0.f;
        }
        __syncthreads();
    }
    const int64_t items = (MODE == 0 && shared) ? N * M : N;
    for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < items;
         it += (int64_t)gridDim.x * blockDim.x) {
        const int64_t g = (MODE == 0 && shared) ? it / M : it;
        float x, y, z;
        if (MODE == 0) {
            const int64_t m = shared ? it - g * M : it;
            x = dirs[3 * m];
            y = dirs[3 * m + 1];
            z = dirs[3 * m + 2];
        } else {
            x = pos[3 * g] - cx;
            y = pos[3 * g + 1] - cy;
            z = pos[3 * g + 2] - cz;
        }
        const float n2 = x * x + y * y + z * z;
        const float inv = n2 > 0.f ? rsqrtf(n2) : 0.f;
        float r, gr, b;
        csc_column_rgb<NB, LDS>(D, sD, K, rows, vals, colptr[g], colptr[g + 1], x * inv, y * inv, z * inv, r, gr, b);
        if (MODE == 1) {
            r = fmaxf(fmaf(kShC0, dc[3 * g], r) + 0.5f, 0.f);
            gr = fmaxf(fmaf(kShC0, dc[3 * g + 1], gr) + 0.5f, 0.f);
            b = fmaxf(fmaf(kShC0, dc[3 * g + 2], b) + 0.5f, 0.f);
        }
        rgb[3 * it] = r;
        rgb[3 * it + 1] = gr;
        rgb[3 * it + 2] = b;
    }
}

static int csc_cus() {
    int dev = 0, ncu = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    return ncu;
}

int64_t csc_workspace_blocks(int64_t N) { return (N + kCscBlock - 1) / kCscBlock; }

hipError_t launch_csc_colptr(const int32_t *count, int64_t N, int64_t *colptr, int64_t *bsum, hipStream_t st) {
    const int64_t nb = csc_workspace_blocks(N);
    if (nb > 0) {
        hipLaunchKernelGGL(csc_block_sums_kernel, dim3((unsigned)nb), dim3(kCscThreads), 0, st, count, N, bsum);
    }
    hipLaunchKernelGGL(csc_scan_sums_kernel, dim3(1), dim3(1024), 0, st, bsum, nb, colptr + N);
    if (nb > 0) {
        hipLaunchKernelGGL(csc_colptr_kernel, dim3((unsigned)nb), dim3(kCscThreads), 0, st, count, N, bsum, colptr);
    }
    return hipGetLastError();
}

hipError_t launch_csc_fill(const int32_t *idx, const float *coef, const int32_t *count, int64_t N, int k,
                           const int64_t *colptr, int32_t *rows, float *vals, hipStream_t st) {
    const int64_t total = N * k;
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, (int64_t)csc_cus() * 16));
    hipLaunchKernelGGL(csc_fill_kernel, dim3((unsigned)blocks), dim3(256), 0, st, idx, coef, count, N, k, colptr,
                       rows, vals);
    return hipGetLastError();
}

template <int NB, int MODE>
static hipError_t launch_csc_eval_t(const DictDev &dict, const int64_t *colptr, const int32_t *rows,
                                    const float *vals, int64_t N, const float *dirs, int64_t M, int shared,
                                    const float *pos, const float *dc, const float *cam, float *rgb,
                                    hipStream_t st) {
    const int64_t items = (MODE == 0 && shared) ? N * M : N;
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((items + 1023) / 1024, (int64_t)csc_cus()));
    const float cx = cam ? cam[0] : 0.f, cy = cam ? cam[1] : 0.f, cz = cam ? cam[2] : 0.f;
    constexpr int kLdsAtoms = (128 * 1024) / (kStride * 4);
    if (dict.K <= kLdsAtoms) {
        const size_t smem = sizeof(float) * (size_t)dict.K * kStride;
        auto kern = csc_eval_kernel<NB, true, MODE>;
        static bool attr = false;
        if (!attr) {
            hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               128 * 1024);
            if (e != hipSuccess) return e;
            attr = true;
        }
        hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(1024), smem, st, dict.D, dict.K, colptr, rows, vals, N,
                           dirs, M, shared, pos, dc, cx, cy, cz, rgb);
    } else {
        hipLaunchKernelGGL((csc_eval_kernel<NB, false, MODE>), dim3((unsigned)blocks), dim3(1024), 0, st, dict.D,
                           dict.K, colptr, rows, vals, N, dirs, M, shared, pos, dc, cx, cy, cz, rgb);
    }
    return hipGetLastError();
}

hipError_t launch_csc_eval(const DictDev &dict, const int64_t *colptr, const int32_t *rows, const float *vals,
                           int64_t N, const float *dirs, int64_t M, int shared, const float *pos, const float *dc,
                           const float *cam, float *rgb, hipStream_t st) {
    const bool colour = pos != nullptr;
#define SC_CSC(NB)                                                                                      \
    return colour ? launch_csc_eval_t<NB, 1>(dict, colptr, rows, vals, N, dirs, M, shared, pos, dc, cam, rgb, st) \
                  : launch_csc_eval_t<NB, 0>(dict, colptr, rows, vals, N, dirs, M, shared, pos, dc, cam, rgb, st);
    switch (dict.d) {
        case 9: SC_CSC(3)
        case 24: SC_CSC(8)
        case 45: SC_CSC(15)
        default: return hipErrorInvalidValue;
    }
#undef SC_CSC
}

}  // namespace sc
