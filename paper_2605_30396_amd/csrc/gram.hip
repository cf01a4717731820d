// Dictionary set-up kernels: atom checks, device layouts and the Gram matrix
// G = D^T D that Batch-OMP reads one row per selected atom.
#include "sc_internal.h"

namespace sc {

// Round-to-nearest-even FP32 -> BF16 (inputs are finite: the atoms are checked).
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// One thread per atom: finiteness, unit norm (Eq. (1)), optional rescaling.
// status bit 0: non-finite entry, bit 1: norm off by more than 1e-4 (or zero
// norm when normalising).
__global__ void dict_check_kernel(const float *__restrict__ D, int d, int K, int normalize,
                                  float *__restrict__ Dc, int *__restrict__ status) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= K) return;
    const float *a = D + (size_t)j * d;
    double s = 0.0;
    bool finite = true;
    for (int i = 0; i < d; ++i) {
        float v = a[i];
        finite &= isfinite(v);
        s += (double)v * v;
    }
    if (!finite) {
        atomicOr(status, 1);
        return;
    }
    double nrm = sqrt(s);
    if (normalize) {
        if (nrm == 0.0) {
            atomicOr(status, 2);
            return;
        }
        for (int i = 0; i < d; ++i) Dc[(size_t)j * d + i] = (float)((double)a[i] / nrm);
    } else {
        if (fabs(nrm - 1.0) > 1e-4) atomicOr(status, 2);
        for (int i = 0; i < d; ++i) Dc[(size_t)j * d + i] = a[i];
    }
}

// DT: d x Kp feature-major; Dbf: Kp x 64 BF16, Dlo and Dl2 the BF16
// roundings of what the previous parts leave (D = Dbf + Dlo + Dl2 to ~2^-27
// relative), all three in the operand order of the split-BF16 correlation; D48: K x 48 FP32 atom-major; Dr: Kp x dpad FP32 in
// FP32 MFMA operand order; Dbfo: Dbf in BF16 MFMA operand order; all zero
// padded.
__global__ void dict_layout_kernel(const float *__restrict__ Dc, int d, int K, int Kp, float *__restrict__ DT,
                                   uint16_t *__restrict__ Dbf, uint16_t *__restrict__ Dlo, uint16_t *__restrict__ Dl2,
                                   float *__restrict__ D48, float *__restrict__ Dr, int dpad,
                                   uint16_t *__restrict__ Dbfo) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= Kp * 64) return;
    int j = t / 64, i = t % 64;   // atom, feature
    float v = (j < K && i < d) ? Dc[(size_t)j * d + i] : 0.f;
    const uint16_t hi = f32_to_bf16(v);
    const float r1 = v - __uint_as_float((uint32_t)hi << 16);
    const uint16_t mid = f32_to_bf16(r1);
    const size_t o = op_order_bf16x32(j, i);
    Dbf[o] = hi;
    Dbfo[op_order_index(j, i, 64)] = hi;
    Dlo[o] = mid;
    Dl2[o] = f32_to_bf16(r1 - __uint_as_float((uint32_t)mid << 16));
    if (i < d) DT[(size_t)i * Kp + j] = v;
    if (j < K && i < 48) D48[(size_t)j * 48 + i] = v;
    if (i < dpad) Dr[op_order_f32(j, i, dpad)] = v;
}

// G[j][l] = <a_j, a_l>, summed in FP64 and rounded once; columns l >= K are 0.
// G64 keeps the FP64 sums (the products of FP32 entries are exact in FP64).
__global__ void gram_kernel(const float *__restrict__ Dc, int d, int K, int Kp, float *__restrict__ G,
                            double *__restrict__ G64) {
    int l = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y;
    if (l >= Kp) return;
    float g = 0.f;
    if (l < K) {
        const float *a = Dc + (size_t)j * d;
        const float *b = Dc + (size_t)l * d;
        double s = 0.0;
        for (int i = 0; i < d; ++i) s += (double)a[i] * (double)b[i];
        g = (float)s;
        G64[(size_t)j * K + l] = s;
    }
    G[(size_t)j * Kp + l] = g;
}

hipError_t launch_dict_check(const float *D, int d, int K, int normalize, float *Dcopy, int *status,
                             hipStream_t st) {
    dict_check_kernel<<<(K + 255) / 256, 256, 0, st>>>(D, d, K, normalize, Dcopy, status);
    return hipGetLastError();
}

hipError_t launch_dict_layouts(const float *Dcopy, int d, int K, int Kp, float *DT, uint16_t *Dbf, uint16_t *Dlo,
                               uint16_t *Dl2, float *D48, float *Dr, int dpad, uint16_t *Dbfo, hipStream_t st) {
    int n = Kp * 64;
    dict_layout_kernel<<<(n + 255) / 256, 256, 0, st>>>(Dcopy, d, K, Kp, DT, Dbf, Dlo, Dl2, D48, Dr, dpad, Dbfo);
    return hipGetLastError();
}

hipError_t launch_gram(const float *Dcopy, int d, int K, int Kp, float *G, double *G64, hipStream_t st) {
    dim3 grid((Kp + 255) / 256, K);
    gram_kernel<<<grid, 256, 0, st>>>(Dcopy, d, K, Kp, G, G64);
    return hipGetLastError();
}

}  // namespace sc
