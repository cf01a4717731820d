// Training of the support proposer on the GPU: forward with saved
// activations, binary cross-entropy on logits against the multi-hot OMP
// support, backpropagation through the three layers, and Adam.
//
// All matrix products go through one MFMA GEMM kernel (one wave per 32 x 32
// output tile) with fused epilogues:
//   STORE  C = acc (+ bias)
//   GELU   a = acc + bias is saved, h = GELU(a) is the next layer's input
//   DGELU  C = acc * GELU'(a_saved)          (backprop through the activation)
// Products with few output tiles and a long reduction (the weight gradients,
// reduced over the batch) are split along K: each slice writes its partial
// tile to a workspace and a second kernel adds the slices in a fixed order
// and applies the epilogue, so the result stays deterministic.
// Two precisions: BF16 operands on v_mfma_f32_32x32x16_bf16 (production: the
// same rounding points as the inference kernel), or FP32 operands on
// v_mfma_f32_32x32x2_f32 (used to check the gradients against the FP64
// oracle).  Operands are addressed with arbitrary element strides so the
// transposed products of the backward pass need no copies.
#include <algorithm>

#include "mfma.h"
#include "sc_internal.h"
#include "wave.h"

namespace sc {

typedef float floatx1 __attribute__((ext_vector_type(1)));

template <bool F32>
__global__ __launch_bounds__(64) void gemm_kernel(GemmArgs g) {
    const int lane = threadIdx.x;
    const int n0 = blockIdx.x * 32, m0 = blockIdx.y * 32;
    const int lr = lane & 31, lh = lane >> 5;
    const int kspan = g.K / (int)gridDim.z, kbeg = blockIdx.z * kspan, kend = kbeg + kspan;
    floatx16 acc = floatx16{};
    if (F32) {
        const float *A = (const float *)g.A;
        const float *B = (const float *)g.B;
        for (int k0 = kbeg; k0 < kend; k0 += 2) {
            const float a = A[(int64_t)(m0 + lr) * g.sam + (int64_t)(k0 + lh) * g.sak];
            const float b = B[(int64_t)(k0 + lh) * g.sbk + (int64_t)(n0 + lr) * g.sbn];
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
        }
    } else {
        const uint16_t *A = (const uint16_t *)g.A;
        const uint16_t *B = (const uint16_t *)g.B;
        for (int k0 = kbeg; k0 < kend; k0 += 16) {
            bf16x8 a, b;
            if (g.sak == 1) {
                a = ld_bf16x8(A + (int64_t)(m0 + lr) * g.sam + k0 + 8 * lh);
            } else {
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    a[q] = __builtin_bit_cast(__bf16, A[(int64_t)(m0 + lr) * g.sam + (int64_t)(k0 + 8 * lh + q) * g.sak]);
            }
            if (g.sbk == 1) {
                b = ld_bf16x8(B + (int64_t)(n0 + lr) * g.sbn + k0 + 8 * lh);
            } else {
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    b[q] = __builtin_bit_cast(__bf16, B[(int64_t)(k0 + 8 * lh + q) * g.sbk + (int64_t)(n0 + lr) * g.sbn]);
            }
            acc = mfma32(a, b, acc);
        }
    }
    const int j = n0 + lr;
    if (gridDim.z > 1) {   // split-K slice: raw partial tile, epilogue after the reduction
        float *P = g.part + (size_t)blockIdx.z * g.M * g.N;
#pragma unroll
        for (int r = 0; r < 16; ++r) P[(size_t)(m0 + 8 * (r >> 2) + 4 * lh + (r & 3)) * g.N + j] = acc[r];
        return;
    }
    if (j >= g.Nvalid) return;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = m0 + 8 * (r >> 2) + 4 * lh + (r & 3);
        float v = acc[r];
        if (g.epi == EPI_STORE) {
            if (g.bias) v += g.bias[j];
        } else if (g.epi == EPI_GELU) {
            v += g.bias[j];
            g.Cpre[(int64_t)i * g.ldc + j] = v;
            v = gelu_f(v);
        } else {
            v *= gelu_grad_f(g.aux[(int64_t)i * g.ldc + j]);
        }
        if (g.Cf) g.Cf[(int64_t)i * g.ldc + j] = v;
        if (g.Ch) {
            if (F32)
                ((float *)g.Ch)[(int64_t)i * g.ldh + j] = v;
            else
                ((uint16_t *)g.Ch)[(int64_t)i * g.ldh + j] = bf16_bits(v);
        }
    }
}

// C = sum over slices of the partial tiles (+ bias), STORE epilogue.
__global__ __launch_bounds__(256) void splitk_reduce_kernel(GemmArgs g, int S) {
    const int64_t mn = (int64_t)g.M * g.N;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < mn; t += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(t / g.N), j = (int)(t - (int64_t)i * g.N);
        if (j >= g.Nvalid) continue;
        float v = 0.f;
        for (int s = 0; s < S; ++s) v += g.part[(size_t)s * mn + t];
        if (g.bias) v += g.bias[j];
        g.Cf[(int64_t)i * g.ldc + j] = v;
    }
}

int gemm_splits(int M, int N, int K) {
    const int tiles = (M / 32) * (N / 32);
    int s = 1;
    while (tiles * s < 512 && K % (32 * s) == 0 && K / (2 * s) >= 64) s *= 2;
    return s;
}

hipError_t launch_gemm(const GemmArgs &g, bool f32, hipStream_t st) {
    if (g.M % 32 || g.N % 32 || g.K % 16) return hipErrorInvalidValue;
    int S = 1;
    if (g.part && g.epi == EPI_STORE && g.Cf && !g.Ch) S = gemm_splits(g.M, g.N, g.K);
    dim3 grid(g.N / 32, g.M / 32, S);
    if (f32)
        hipLaunchKernelGGL(gemm_kernel<true>, grid, dim3(64), 0, st, g);
    else
        hipLaunchKernelGGL(gemm_kernel<false>, grid, dim3(64), 0, st, g);
    if (S > 1) {
        const int64_t mn = (int64_t)g.M * g.N;
        hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)std::min<int64_t>((mn + 255) / 256, 1024)), dim3(256),
                           0, st, g, S);
    }
    return hipGetLastError();
}

// Batch rows -> x / ||x|| (zero padded to 64 features), BF16 or FP32.
template <bool F32>
__global__ void train_prep_kernel(const float *__restrict__ X, const int32_t *__restrict__ rows, int64_t B, int d,
                                  void *__restrict__ xh) {
    const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int f = threadIdx.x & 63;
    if (b >= B) return;
    const int64_t r = rows ? (int64_t)rows[b] : b;
    const float v = f < d ? X[r * d + f] : 0.f;
    const float ss = wave_sum(v * v);
    const float nrm = sqrtf(ss);
    const float o = (nrm > 0.f && isfinite(nrm)) ? v / nrm : 0.f;
    if (F32)
        ((float *)xh)[b * 64 + f] = o;
    else
        ((uint16_t *)xh)[b * 64 + f] = bf16_bits(o);
}

// dz = (w y (sigma(z) - 1) + (1 - y) sigma(z)) / (B K), y = multi-hot OMP support;
// loss accumulated into *loss (mean over the B K entries).  A wave takes 64
// consecutive logits of one row (K is a multiple of 64): lane q < count holds
// the row's q-th support atom and the membership test reads it by lane index.
// Waves stride over the B K / 64 chunks with a bounded grid, so the loss takes
// one atomic per block.
constexpr int kBceBlocks = 128;   // few blocks: one loss atomic each on a single address
template <bool F32>
__global__ __launch_bounds__(256) void bce_grad_kernel(const float *__restrict__ Z, int64_t B, int K,
                                                       const int32_t *__restrict__ rows,
                                                       const int32_t *__restrict__ sup,
                                                       const int32_t *__restrict__ cnt, int kcap, float pos_weight,
                                                       void *__restrict__ dz, float *__restrict__ loss) {
    __shared__ float part[4];
    const int lane = threadIdx.x & 63;
    const int64_t nchunk = B * K / 64;
    const float inv = 1.f / ((float)B * (float)K);
    float l = 0.f;
    for (int64_t ch = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); ch < nchunk; ch += (int64_t)gridDim.x * 4) {
        const int64_t t = ch * 64 + lane;
        const int64_t b = (ch * 64) / K;
        const int j = (int)(t - b * K);
        const int64_t r = rows ? (int64_t)rows[b] : b;
        const int c = min(max(cnt[r], 0), kcap);
        const int myatom = lane < c ? sup[r * kcap + lane] : -1;
        bool y = false;
        for (int q = 0; q < c; ++q) y |= __shfl(myatom, q, 64) == j;
        const float z = Z[t];
        const float sp = fmaxf(z, 0.f) + log1pf(__expf(-fabsf(z)));   // softplus(z)
        const float sig = 1.f / (1.f + __expf(-z));
        float g;
        if (y) {
            l += pos_weight * (sp - z);
            g = pos_weight * (sig - 1.f) * inv;
        } else {
            l += sp;
            g = sig * inv;
        }
        if (F32)
            ((float *)dz)[t] = g;
        else
            ((uint16_t *)dz)[t] = bf16_bits(g);
    }
    if (loss) {
        l = wave_sum(l);
        if (lane == 0) part[threadIdx.x >> 6] = l;
        __syncthreads();
        if (threadIdx.x == 0) {
            const float s = (part[0] + part[1]) + (part[2] + part[3]);
            if (s != 0.f) atomicAdd(loss, s * inv);
        }
    }
}

// out[j] = sum_i A[i * ld + j] over M rows (bias gradients).  One block per
// 64 columns; its 16 waves take every 16th row, so 16 row streams are in
// flight per column group, and the 16 partial sums are added in a fixed order
// (deterministic result).
template <bool F32>
__global__ __launch_bounds__(1024) void colsum_kernel(const void *__restrict__ A, int64_t M, int N, int64_t ld,
                                                      float *__restrict__ out) {
    __shared__ float part[16][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + lane;
    float s = 0.f;
    if (j < N) {
#pragma unroll 8
        for (int64_t i = w; i < M; i += 16)
            s += F32 ? ((const float *)A)[i * ld + j] : bf16_to_f32(((const uint16_t *)A)[i * ld + j]);
    }
    part[w][lane] = s;
    __syncthreads();
    if (w == 0 && j < N) {
        float t = 0.f;
#pragma unroll
        for (int q = 0; q < 16; ++q) t += part[q][lane];
        out[j] = t;
    }
}

// Adam, in place on the FP32 master parameters (bias-corrected step sizes
// passed from the host).
__global__ void adam_kernel(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                            const float *__restrict__ g, int64_t n, float lr_t, float beta1, float beta2,
                            float eps_hat) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = beta1 * m[i] + (1.f - beta1) * gi;
        const float vi = beta2 * v[i] + (1.f - beta2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr_t * mi / (sqrtf(vi) + eps_hat);
    }
}

hipError_t launch_train_prep(const float *X, const int32_t *rows, int64_t B, int d, void *xh, bool f32,
                             hipStream_t st) {
    dim3 grid((unsigned)((B + 3) / 4));
    if (f32)
        hipLaunchKernelGGL(train_prep_kernel<true>, grid, dim3(256), 0, st, X, rows, B, d, xh);
    else
        hipLaunchKernelGGL(train_prep_kernel<false>, grid, dim3(256), 0, st, X, rows, B, d, xh);
    return hipGetLastError();
}

hipError_t launch_bce_grad(const float *Z, int64_t B, int K, const int32_t *rows, const int32_t *sup,
                           const int32_t *cnt, int kcap, float pos_weight, void *dz, float *loss, bool f32,
                           hipStream_t st) {
    if (K % 64) return hipErrorInvalidValue;
    const int64_t n = B * K;
    dim3 grid((unsigned)std::min<int64_t>((n + 255) / 256, kBceBlocks));
    if (f32)
        hipLaunchKernelGGL(bce_grad_kernel<true>, grid, dim3(256), 0, st, Z, B, K, rows, sup, cnt, kcap, pos_weight, dz,
                           loss);
    else
        hipLaunchKernelGGL(bce_grad_kernel<false>, grid, dim3(256), 0, st, Z, B, K, rows, sup, cnt, kcap, pos_weight,
                           dz, loss);
    return hipGetLastError();
}

hipError_t launch_colsum(const void *A, int64_t M, int N, int64_t ld, float *out, bool f32, hipStream_t st) {
    dim3 grid((N + 63) / 64);
    if (f32)
        hipLaunchKernelGGL(colsum_kernel<true>, grid, dim3(1024), 0, st, A, M, N, ld, out);
    else
        hipLaunchKernelGGL(colsum_kernel<false>, grid, dim3(1024), 0, st, A, M, N, ld, out);
    return hipGetLastError();
}

hipError_t launch_adam(float *p, float *m, float *v, const float *g, int64_t n, float lr_t, float beta1, float beta2,
                       float eps_hat, hipStream_t st) {
    hipLaunchKernelGGL(adam_kernel, dim3(1024), dim3(256), 0, st, p, m, v, g, n, lr_t, beta1, beta2, eps_hat);
    return hipGetLastError();
}

}  // namespace sc
