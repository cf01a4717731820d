// BF16 MFMA helpers for gfx950 (64-lane waves).
//
// v_mfma_f32_32x32x16_bf16, lane l (checked on hardware):
//   A (32 x 16): row l % 32, k = 8 (l / 32) + q, q = 0..7
//   B (16 x 32): col l % 32, k = 8 (l / 32) + q
//   C (32 x 32): value r (0..15) is row 8 (r / 4) + 4 (l / 32) + r % 4, col l % 32
// v_mfma_f32_16x16x32_bf16, lane l:
//   A (16 x 32): row l % 16, k = 8 (l / 16) + q
//   B (32 x 16): col l % 16, k = 8 (l / 16) + q
//   C (16 x 16): value r (0..3) is row 4 (l / 16) + r, col l % 16
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sc {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16x8 ld_bf16x8(const uint16_t *p) {
    uint4 v = *reinterpret_cast<const uint4 *>(p);
    return __builtin_bit_cast(bf16x8, v);
}

__device__ __forceinline__ floatx16 mfma32(bf16x8 a, bf16x8 b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ floatx4 mfma16(bf16x8 a, bf16x8 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Round-to-nearest-even FP32 -> BF16 bits (the hardware conversion).
__device__ __forceinline__ uint16_t bf16_bits(float f) {
    return __builtin_bit_cast(uint16_t, (__bf16)f);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Two FP32 values rounded to BF16 (round to nearest even) in one packed
// conversion: a in the low half, b in the high half.
typedef float floatx2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t bf16_pack2(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((floatx2){a, b}, bf16x2));
}

// Phi(t), the standard normal CDF, and exp(-t^2/2), via a rational fit of
// erfc of the form of Abramowitz & Stegun 7.1.26 with coefficients fitted for
// this library (max |error| of erf ~1.2e-8 before FP32 rounding):
//   erfc(u) = tt P(tt) exp(-u^2),  tt = 1 / (1 + p u),  u = |t| / sqrt 2 >= 0.
// For t < 0, Phi(t) = erfc(u)/2 is formed without cancellation.
// h = erfc(u) / 2 = Phi(-|t|) and g = exp(-t^2 / 2).  1 / sqrt 2 is folded
// into p (tt = 1 / (1 + (p / sqrt 2) |t|)) and the polynomial's coefficients
// are halved (an exact scaling, so tt * P * g is erfc(u) / 2 directly).
__device__ __forceinline__ void erfc_half_and_gauss(float t, float &h, float &g) {
    const float tt = __builtin_amdgcn_rcpf(fmaf(0.2053894377894869f, fabsf(t), 1.f));
    float P = 0.6933924019619302f;
    P = fmaf(P, tt, -1.428651480896066f);
    P = fmaf(P, tt, 1.679207553849397f);
    P = fmaf(P, tt, -0.8579665555316653f);
    P = fmaf(P, tt, 0.36832632086264155f);
    P = fmaf(P, tt, 0.0456917654774965f);
    g = __builtin_amdgcn_exp2f(t * t * -0.7213475204444817f);   // 2^(-t^2 log2(e) / 2)
    h = tt * P * g;
}

__device__ __forceinline__ void phi_and_gauss(float t, float &Phi, float &g) {
    float h;
    erfc_half_and_gauss(t, h, g);
    Phi = t >= 0.f ? 1.f - h : h;
}

// GELU(t) = t Phi(t) (the exact, erf form) = max(t, 0) - |t| h for either
// sign of t, with h = Phi(-|t|).
__device__ __forceinline__ float gelu_f(float t) {
    float h, g;
    erfc_half_and_gauss(t, h, g);
    return fmaf(-fabsf(t), h, fmaxf(t, 0.f));
}

// d/dt GELU = Phi(t) + t phi(t),  phi(t) = exp(-t^2/2) / sqrt(2 pi).
__device__ __forceinline__ float gelu_grad_f(float t) {
    float Phi, g;
    phi_and_gauss(t, Phi, g);
    return Phi + t * 0.39894228040143268f * g;
}

// Order-preserving map of a float to uint32 (larger float -> larger key).
__device__ __forceinline__ uint32_t order_key(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

}  // namespace sc
