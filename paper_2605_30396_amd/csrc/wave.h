// Wavefront-level primitives for gfx950 (64-lane waves).
//
// Reductions use DPP row operations inside each 16-lane row and read the four
// row results with v_readlane, so the result is wave-uniform.  Every caller
// must run them with all 64 lanes active.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sc {

constexpr int kWave = 64;

template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ float readlane_f(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

__device__ __forceinline__ int readlane_i(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }

// v with lane `lane` replaced by the wave-uniform x (v_writelane_b32: no exec
// mask or lane compare needed).  x and lane must be wave-uniform: x is passed
// in a scalar register and the lane in M0 (an instruction may read only one
// SGPR besides M0).  The compiler has no builtin for this instruction, hence
// the asm; it reads and writes registers only.
__device__ __forceinline__ int writelane_i(int x, int lane, int v) {
    x = __builtin_amdgcn_readfirstlane(x);   // free when x is already scalar
    asm("v_writelane_b32 %0, %1, m0" : "+v"(v) : "s"(x), "{m0}"(lane));
    return v;
}
__device__ __forceinline__ float writelane_f(float x, int lane, float v) {
    return __int_as_float(writelane_i(__float_as_int(x), lane, __float_as_int(v)));
}

// Lane 0's value, known to the compiler as wave-uniform (callers pass values
// that are equal on every lane, so branches on them need no exec masking).
__device__ __forceinline__ float readfirstlane_f(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// DPP controls: quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror, row_mirror
#define SC_DPP_QP1032 0xB1
#define SC_DPP_QP2301 0x4E
#define SC_DPP_HMIRROR 0x141
#define SC_DPP_MIRROR 0x140

// Max over the wave of non-NaN inputs (callers pass finite values).
__device__ __forceinline__ float wave_max(float v) {
    v = fmaxf(v, dpp_f<SC_DPP_QP1032>(v));
    v = fmaxf(v, dpp_f<SC_DPP_QP2301>(v));
    v = fmaxf(v, dpp_f<SC_DPP_HMIRROR>(v));
    v = fmaxf(v, dpp_f<SC_DPP_MIRROR>(v));
    return fmaxf(fmaxf(readlane_f(v, 0), readlane_f(v, 16)), fmaxf(readlane_f(v, 32), readlane_f(v, 48)));
}

__device__ __forceinline__ float wave_sum(float v) {
    v += dpp_f<SC_DPP_QP1032>(v);
    v += dpp_f<SC_DPP_QP2301>(v);
    v += dpp_f<SC_DPP_HMIRROR>(v);
    v += dpp_f<SC_DPP_MIRROR>(v);
    return (readlane_f(v, 0) + readlane_f(v, 16)) + (readlane_f(v, 32) + readlane_f(v, 48));
}

// Sum over lanes [0, NL) (NL a multiple of 16; the other rows are not read).
template <int NL>
__device__ __forceinline__ float lanes_sum(float v) {
    static_assert(NL % 16 == 0 && NL >= 16 && NL <= 64, "whole 16-lane rows");
    v += dpp_f<SC_DPP_QP1032>(v);
    v += dpp_f<SC_DPP_QP2301>(v);
    v += dpp_f<SC_DPP_HMIRROR>(v);
    v += dpp_f<SC_DPP_MIRROR>(v);
    float r = readlane_f(v, 0);
    if constexpr (NL > 16) r += readlane_f(v, 16);
    if constexpr (NL > 32) r += readlane_f(v, 32);
    if constexpr (NL > 48) r += readlane_f(v, 48);
    return r;
}

__device__ __forceinline__ double wave_sum_d(double v) {
    // FP64 reduction through 32-bit halves (DPP moves 32 bits)
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}

// Unsigned maximum over the wave (wave-uniform result).
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
    v = max(v, dpp_u<SC_DPP_QP1032>(v));
    v = max(v, dpp_u<SC_DPP_QP2301>(v));
    v = max(v, dpp_u<SC_DPP_HMIRROR>(v));
    v = max(v, dpp_u<SC_DPP_MIRROR>(v));
    const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)v, 0), b = (uint32_t)__builtin_amdgcn_readlane((int)v, 16);
    const uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)v, 32), e = (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
    return max(max(a, b), max(c, e));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int lane_id() { return __lane_id(); }

}  // namespace sc
