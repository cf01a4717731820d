// The tolerance-controlled encoder writing CSC directly (Sec. 2.2 stores the
// variable-length codes column by column; Sec. 3.2 varies their length by the
// tolerance): one pass over the signals, no padded N x k codes in memory.
//
// Workgroups take 16- or 32-signal tiles in increasing order from a ticket
// counter, so every tile below the one a workgroup holds has been taken by a
// running workgroup.  A tile's codes are encoded into an LDS stage (the same
// tile body as the padded encoder) and its number of non-zeros is published
// in a per-tile descriptor; its column offset is found by looking back over
// the descriptors of the tiles before it (decoupled look-back: a descriptor
// holds either the tile's own count, or the inclusive count of every tile up
// to it).  The columns are then written at their offsets, in signal order.
// Only the descriptors (8 bytes per tile) live in the workspace.
//
// A code whose support is ill-conditioned is written with its FP32
// coefficients and its column pointer stored as -(offset + 1); the refit pass
// solves those columns again in FP64 and restores the pointer.
#pragma once
#include <algorithm>

#include "omp_core.h"

namespace sc {

constexpr int kCscTile = 16;
constexpr uint64_t kDescAgg = 1ull << 62;     // descriptor holds the tile's own count
constexpr uint64_t kDescIncl = 2ull << 62;    // descriptor holds the inclusive count
constexpr uint64_t kDescVal = (1ull << 62) - 1;
constexpr long kLookBackSpins = 1l << 24;     // bound on the wait for one predecessor

// Workspace header; the descriptors follow at byte 256.
struct CscHeader {
    int ticket;
    int error;   // set when a look-back wait exceeded its bound
};

__device__ __forceinline__ int code_nnz(int c) { return c >= 0 ? c : (c < -1 ? -c - 2 : 0); }

__device__ __forceinline__ uint64_t desc_load(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void desc_store(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Tile t publishes its own count agg as soon as its codes are staged (tile 0
// publishes its inclusive count at once).
__device__ __forceinline__ void publish_count(uint64_t *desc, int64_t t, int64_t agg) {
    desc_store(desc + t, (t == 0 ? kDescIncl : kDescAgg) | (uint64_t)agg);
}

// Exclusive offset of tile t (own count agg), from the descriptors of the
// tiles before it; publishes t's inclusive count.  Called by one lane.
__device__ __forceinline__ int64_t look_back(uint64_t *desc, int64_t t, int64_t agg, int *error) {
    if (t == 0) return 0;
    int64_t excl = 0, j = t - 1;
    long spins = 0;
    for (;;) {
        const uint64_t v = desc_load(desc + j);
        if (v & kDescIncl) {
            excl += (int64_t)(v & kDescVal);
            break;
        }
        if (v & kDescAgg) {
            excl += (int64_t)(v & kDescVal);
            --j;   // tile 0 always publishes an inclusive count, so j stays >= 0
            continue;
        }
        if (++spins > kLookBackSpins) {   // never expected: the predecessor's workgroup is running
            atomicOr(error, 1);
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    desc_store(desc + t, kDescIncl | (uint64_t)(excl + agg));
    return excl;
}

// Tile shape: with a matrix-core correlation stage and 128..512 atoms, 8
// waves on 32-signal tiles (as the padded encoder) when the tile and its two
// code stages still let two workgroups share a compute unit, and then held to
// 128 VGPRs so that both fit; otherwise 4 waves on 16-signal tiles.
template <int E, int KMAX, int MODE>
struct CscShape {
    static constexpr bool wide =
        (MODE == A0_MFMA_F32 || MODE == A0_MFMA_BF16X6) && E >= 2 && E <= 8 &&
        omp_tile_lds(32, 64 * E, MODE == A0_MFMA_BF16X6) + 2 * sizeof(int32_t) * (2 * 32 * KMAX + 32) <= 80 * 1024;
    static constexpr int NW = wide ? 8 : kOmpWaves;
    static constexpr int T = wide ? 32 : kCscTile;
};

// Per workgroup a two-deep pipeline: tile i is encoded into one LDS stage
// and its count published; then tile i-1 (in the other stage) gets its
// offset and is written out.  By then the tiles before i-1 have had a whole
// tile's time to publish their counts, so the look-back seldom waits, and a
// slow tile does not stall the workgroups behind it.
template <int E, int KMAX, int MODE, int RCQ>
__global__ __launch_bounds__((64 * CscShape<E, KMAX, MODE>::NW))
__attribute__((amdgpu_waves_per_eu(CscShape<E, KMAX, MODE>::wide ? 4 : 1))) void omp_csc_kernel(
    DictDev dict, OmpParams p, int64_t *__restrict__ colptr, int32_t *__restrict__ rows, float *__restrict__ vals,
    int64_t cap, CscHeader *hdr, uint64_t *desc) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int Kp = 64 * E;
    constexpr int T = CscShape<E, KMAX, MODE>::T, NW = CscShape<E, KMAX, MODE>::NW;
    constexpr int kStageWords = 2 * T * KMAX + T;   // idx, coef, count of one stage
    const size_t tile_lds = omp_tile_lds(T, Kp, MODE == A0_MFMA_BF16X6);
    int32_t *stage_base = reinterpret_cast<int32_t *>(smem_raw + tile_lds);
    __shared__ int64_t col_off[T];
    __shared__ int64_t tile_sh;
    OmpTally tally;
    const int64_t N = p.N, ntiles = (N + T - 1) / T;
    const int k = p.k;
    int64_t prev = -1;   // the staged tile waiting for its offset (wave-uniform)
    int buf = 0;
    for (;;) {
        __syncthreads();   // the previous tile's stage and offsets are consumed
        if (threadIdx.x == 0) tile_sh = atomicAdd(&hdr->ticket, 1);
        __syncthreads();
        const int64_t t = tile_sh;
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        const int lane = tid & 63, wave = tid >> 6;
        if (t < ntiles) {   // encode tile t into stage `buf`, publish its count
            int32_t *sb = stage_base + buf * kStageWords;
            const CodeStage stage{sb, reinterpret_cast<float *>(sb + T * KMAX), sb + 2 * T * KMAX};
            const int64_t s0 = t * T;
            const int nt = (int)min<int64_t>(T, N - s0);
            omp_tile<E, KMAX, T, MODE == A0_MFMA_BF16X6, RCQ, NW>(dict, p, MODE, s0, nt, smem_raw, tid, tally, &stage);
            __syncthreads();
            if (wave == 0) {
                int64_t c = lane < nt ? code_nnz(stage.cnt[lane]) : 0;
#pragma unroll
                for (int off = 1; off < T; off <<= 1) c += __shfl_xor(c, off, 64);
                if (lane == 0) publish_count(desc, t, c);
            }
        }
        if (prev >= 0) {   // offset of tile prev, then its columns
            const int32_t *sb = stage_base + (buf ^ 1) * kStageWords;
            const int32_t *st_idx = sb;
            const float *st_coef = reinterpret_cast<const float *>(sb + T * KMAX);
            const int32_t *st_cnt = sb + 2 * T * KMAX;
            const int64_t s0 = prev * T;
            const int nt = (int)min<int64_t>(T, N - s0);
            if (wave == 0) {
                const int64_t c = lane < nt ? code_nnz(st_cnt[lane]) : 0;
                int64_t incl = c;
#pragma unroll
                for (int off = 1; off < T; off <<= 1) {
                    const int64_t u = __shfl_up(incl, off, 64);
                    if (lane >= off) incl += u;
                }
                const int64_t agg = __shfl(incl, T - 1, 64);
                int64_t excl = 0;
                if (lane == 0) excl = look_back(desc, prev, agg, &hdr->error);
                excl = __shfl(excl, 0, 64);
                if (lane < T) col_off[lane] = excl + incl - c;
                if (lane == 0 && prev == ntiles - 1) colptr[N] = excl + agg;
            }
            __syncthreads();
            for (int s = wave; s < nt; s += NW) {
                const int cnt = st_cnt[s];
                const int n = code_nnz(cnt);
                const int64_t o = col_off[s];
                if (lane < n && o + lane < cap) {
                    rows[o + lane] = st_idx[s * k + lane];
                    vals[o + lane] = st_coef[s * k + lane];
                }
                if (lane == 0) colptr[s0 + s] = cnt < -1 ? -(o + 1) : o;   // flagged for the FP64 refit
            }
        }
        if (t >= ntiles) break;
        prev = t;
        buf ^= 1;
    }
    if (p.stats) {   // one pair of atomics per workgroup
        __shared__ unsigned long long red[NW][2];
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

template <int E, int KMAX, int MODE, int RCQ>
static hipError_t launch_csc_t(const DictDev &dict, const OmpParams &p, int64_t *colptr, int32_t *rows, float *vals,
                               int64_t cap, void *ws, hipStream_t st) {
    constexpr int Kp = 64 * E;
    constexpr int T = CscShape<E, KMAX, MODE>::T, NW = CscShape<E, KMAX, MODE>::NW;
    const size_t smem = omp_tile_lds(T, Kp, MODE == A0_MFMA_BF16X6) +
                        2 * sizeof(int32_t) * (2 * T * KMAX + T);   // two code stages
    auto kern = omp_csc_kernel<E, KMAX, MODE, RCQ>;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)kern, 64 * NW, smem) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    int dev = 0, ncu = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t ntiles = (p.N + T - 1) / T;
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(ntiles, (int64_t)ncu * per_cu));
    CscHeader *hdr = reinterpret_cast<CscHeader *>(ws);
    uint64_t *desc = reinterpret_cast<uint64_t *>(reinterpret_cast<unsigned char *>(ws) + 256);
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(64 * NW), smem, st, dict, p, colptr, rows, vals, cap, hdr,
                       desc);
    return hipGetLastError();
}

template <int MODE>
static hipError_t launch_csc_mode(const DictDev &dict, const OmpParams &p, int kmax, int row_cache, int64_t *colptr,
                                  int32_t *rows, float *vals, int64_t cap, void *ws, hipStream_t st) {
#define SC_CASE(EE, KK)                                                                                   \
    if (dict.E == EE && kmax == KK) {                                                                     \
        if constexpr (EE <= 8)                                                                            \
            if (row_cache > 0) return launch_csc_t<EE, KK, MODE, 4>(dict, p, colptr, rows, vals, cap, ws, st); \
        return launch_csc_t<EE, KK, MODE, 0>(dict, p, colptr, rows, vals, cap, ws, st);                  \
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
