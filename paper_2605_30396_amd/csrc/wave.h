// Wavefront-level primitives for gfx950 (64-lane waves).
//
// Reductions use DPP row operations inside each 16-lane row, then the two
// row broadcasts (lane 15 of each row into the next, lane 31 into rows 2
// and 3) so that lane 63 holds the wave's result, read with one v_readlane:
// the result is wave-uniform and stays in a scalar register.  Every caller
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

// DPP controls: quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror, row_mirror,
// row_bcast:15, row_bcast:31
#define SC_DPP_QP1032 0xB1
#define SC_DPP_QP2301 0x4E
#define SC_DPP_HMIRROR 0x141
#define SC_DPP_MIRROR 0x140
#define SC_DPP_BCAST15 0x142
#define SC_DPP_BCAST31 0x143

// The row broadcasts: rows not in the row mask receive `idle` (the identity
// of the reduction).
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_bcast_f(float v, float idle) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(idle), __float_as_int(v), CTRL, ROWS, 0xF, false));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_bcast_u(uint32_t v, uint32_t idle) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)idle, (int)v, CTRL, ROWS, 0xF, false);
}

// Max over the wave of non-NaN inputs (callers pass finite values).
__device__ __forceinline__ float wave_max(float v) {
    v = fmaxf(v, dpp_f<SC_DPP_QP1032>(v));
    v = fmaxf(v, dpp_f<SC_DPP_QP2301>(v));
    v = fmaxf(v, dpp_f<SC_DPP_HMIRROR>(v));
    v = fmaxf(v, dpp_f<SC_DPP_MIRROR>(v));
    v = fmaxf(v, dpp_bcast_f<SC_DPP_BCAST15, 0xA>(v, v));
    v = fmaxf(v, dpp_bcast_f<SC_DPP_BCAST31, 0xC>(v, v));
    return readlane_f(v, 63);
}

__device__ __forceinline__ float wave_sum(float v) {
    v += dpp_f<SC_DPP_QP1032>(v);
    v += dpp_f<SC_DPP_QP2301>(v);
    v += dpp_f<SC_DPP_HMIRROR>(v);
    v += dpp_f<SC_DPP_MIRROR>(v);
    v += dpp_bcast_f<SC_DPP_BCAST15, 0xA>(v, -0.f);
    v += dpp_bcast_f<SC_DPP_BCAST31, 0xC>(v, -0.f);
    return readlane_f(v, 63);
}

// Sum over lanes [0, NL) for NL = 16, 32 or 64 (the other rows are not read).
template <int NL>
__device__ __forceinline__ float lanes_sum(float v) {
    static_assert(NL == 16 || NL == 32 || NL == 64, "one, two or four 16-lane rows");
    v += dpp_f<SC_DPP_QP1032>(v);
    v += dpp_f<SC_DPP_QP2301>(v);
    v += dpp_f<SC_DPP_HMIRROR>(v);
    v += dpp_f<SC_DPP_MIRROR>(v);
    if constexpr (NL == 16) {
        return readlane_f(v, 0);
    } else if constexpr (NL == 32) {
        v += dpp_bcast_f<SC_DPP_BCAST15, 0xA>(v, -0.f);
        return readlane_f(v, 31);
    } else {
        v += dpp_bcast_f<SC_DPP_BCAST15, 0xA>(v, -0.f);
        v += dpp_bcast_f<SC_DPP_BCAST31, 0xC>(v, -0.f);
        return readlane_f(v, 63);
    }
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
    v = max(v, dpp_bcast_u<SC_DPP_BCAST15, 0xA>(v, 0u));
    v = max(v, dpp_bcast_u<SC_DPP_BCAST31, 0xC>(v, 0u));
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int lane_id() { return __lane_id(); }

}  // namespace sc
