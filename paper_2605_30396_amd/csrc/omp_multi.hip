// Batch-OMP over many scenes in one persistent launch.
//
// Every scene has its own dictionary (K <= 512), sparsity cap (k <= 16),
// tolerance and outputs.  The scenes' 16- or 32-signal tiles are numbered
// scene after scene (the host orders the scenes, by default with the most
// expensive tiles first) and a grid of workgroups sized to fill the device
// takes them one at a time from an atomic counter, so uneven scenes balance
// without a launch per scene.  A tile runs the same body as the
// single-dictionary encoder (omp_core.h), picked by the scene's class
// (E = Kp / 64 in {1, 2, 4, 8}, KMAX in {4, 8, 12, 16}); the correlation
// stage (VALU or FP32 MFMA) is chosen per launch.
// The scene descriptors travel as kernel arguments; the dictionary layout is
// read from its device copy in the handle.
#include <string.h>

#include <algorithm>

#include "omp_core.h"

namespace sc {

constexpr int kMaxScenes = SC_MAX_SCENES;

struct SceneDesc {
    const DictDev *dict;
    const float *X;
    int32_t *idx;
    float *coef;
    int32_t *count;
    float *resid;
    unsigned long long *stats;
    int64_t N;
    int64_t tile_begin;   // first tile of the scene in the launch's numbering
    int k;
    float eps;
    int flags;            // bit 0: eps relative to ||x||, bit 1: FP64 refit, bits 8..15: d
    int cls;              // 4 * log2(E) + KMAX / 4 - 1
};

struct MultiArgs {
    SceneDesc sc[kMaxScenes];
    int n;
    int pad;
    int64_t total_tiles;
    int *counter;         // zeroed before the launch
};
static_assert(sizeof(MultiArgs) <= 3072, "kernel arguments must stay well inside 4 KiB");

__device__ __forceinline__ OmpParams scene_params(const SceneDesc &s) {
    OmpParams p;
    p.X = s.X;
    p.N = s.N;
    p.rows = nullptr;
    p.nrows = nullptr;
    p.k = s.k;
    p.eps = s.eps;
    p.relative = s.flags & 1;
    p.fp64_refit = (s.flags >> 1) & 1;
    p.kappa_max = 1e3f;
    p.idx = s.idx;
    p.coef = s.coef;
    p.count = s.count;
    p.resid = s.resid;
    p.stats = s.stats;
    return p;
}

// 32-signal tiles run on 8 waves (the wider tile halves the dictionary reads
// per signal of the correlation stage), and so do 16-signal tiles with the
// matrix-core correlation stage (its accumulators then take half the
// registers per wave); 16-signal tiles with the VALU stage run on 4.
template <int T, int MODE>
constexpr int multi_waves() { return (T == 32 || MODE == A0_MFMA_F32) ? 8 : kOmpWaves; }

// Gram rows a class body keeps in registers when the launch asks for the row
// cache.  The merged kernel holds a few more live values across its tile
// loop than the single-dictionary kernel, and the largest bodies are at the
// 128-register limit there already: the 512-atom bodies keep two rows up to
// a cap of 12 (four spill) and none at 16.
template <int E, int KMAX, int RCQ>
constexpr int multi_rows() { return RCQ == 0 ? 0 : E <= 4 ? RCQ : KMAX <= 12 ? 2 : 0; }

template <int T, int RCQ, int MODE>
__global__ __launch_bounds__((64 * multi_waves<T, MODE>())) __attribute__((amdgpu_waves_per_eu(4)))
void omp_multi_kernel(MultiArgs a) {
    constexpr int NW = multi_waves<T, MODE>();
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int64_t tile_sh;
    OmpTally tally;
    int cur = -1;
    const int tid = threadIdx.x;
    auto flush = [&]() {
        if (cur >= 0 && (tid & 63) == 0 && tally.sig && a.sc[cur].stats) {
            atomicAdd(a.sc[cur].stats + 0, tally.sig);
            atomicAdd(a.sc[cur].stats + 1, tally.atoms);
        }
        tally = OmpTally{};
    };
    if (tid == 0) tile_sh = (int64_t)atomicAdd(a.counter, 1);
    __syncthreads();
    int64_t tile = tile_sh;
    while (tile < a.total_tiles) {
        // the next tile's number is fetched while this tile is encoded; it
        // reaches tile_sh after the tile body, whose first barrier every
        // thread passes only after reading the current number
        int nxt = 0;
        if (tid == 0) nxt = atomicAdd(a.counter, 1);
        int si = 0;
        for (int q = 1; q < a.n; ++q) si += a.sc[q].tile_begin <= tile ? 1 : 0;
        if (si != cur) {
            flush();
            cur = si;
        }
        const SceneDesc &sd = a.sc[si];
        DictDev dict = *sd.dict;
        dict.d = sd.flags >> 8;   // from the kernel arguments: the tile loads need not wait for *sd.dict
        int tidv = tid;   // recomputed per tile rather than held live
        asm volatile("" : "+v"(tidv));
        const OmpParams p = scene_params(sd);
        const int64_t s0 = (tile - sd.tile_begin) * T;
        const int nt = (int)min<int64_t>(T, sd.N - s0);
#define SC_BODY(EI, EE, KK)                                                                            \
    case 4 * EI + KK / 4 - 1:                                                                          \
        omp_tile<EE, KK, T, false, multi_rows<EE, KK, RCQ>(), NW>(dict, p, MODE, s0, nt, smem_raw, tidv, tally); \
        break;
        switch (sd.cls) {
            SC_BODY(0, 1, 4) SC_BODY(0, 1, 8) SC_BODY(0, 1, 12) SC_BODY(0, 1, 16)
            SC_BODY(1, 2, 4) SC_BODY(1, 2, 8) SC_BODY(1, 2, 12) SC_BODY(1, 2, 16)
            SC_BODY(2, 4, 4) SC_BODY(2, 4, 8) SC_BODY(2, 4, 12) SC_BODY(2, 4, 16)
            SC_BODY(3, 8, 4) SC_BODY(3, 8, 8) SC_BODY(3, 8, 12) SC_BODY(3, 8, 16)
            default: __syncthreads(); break;   // (classes are checked on the host) the body's barrier
        }
#undef SC_BODY
        if (tid == 0) tile_sh = (int64_t)nxt;
        __syncthreads();
        tile = tile_sh;
    }
    flush();
}

// FP64 refit of the flagged supports of every scene that asked for it.
__global__ __launch_bounds__(kOmpThreads) void omp_multi_refit_kernel(MultiArgs a) {
    __shared__ RefitScratch ws[kOmpWaves];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t gw = (int64_t)blockIdx.x * kOmpWaves + wave, nw = (int64_t)gridDim.x * kOmpWaves;
    for (int q = 0; q < a.n; ++q) {
        const SceneDesc &sd = a.sc[q];
        if (!((sd.flags >> 1) & 1)) continue;
        const DictDev dict = *sd.dict;
        const unsigned long long nref = refit_scan(dict, scene_params(sd), gw, nw, ws[wave], lane);
        if (sd.stats && lane == 0 && nref) atomicAdd(sd.stats + 2, nref);
    }
}

__global__ void zero_counter_kernel(int *c) {
    if (threadIdx.x == 0) c[0] = 0;
}

static int multi_cus() {
    int dev = 0, ncu = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    return ncu;
}

template <int T, int RCQ, int MODE>
static hipError_t launch_multi_t(const MultiArgs &a, int max_kp, int wg_per_cu, hipStream_t st) {
    const size_t smem = omp_tile_lds(T, max_kp, false);
    auto kern = omp_multi_kernel<T, RCQ, MODE>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    int per_cu = 0;
    constexpr int nthreads = 64 * multi_waves<T, MODE>();
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)kern, nthreads, smem) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    if (wg_per_cu > 0) per_cu = std::min(per_cu, wg_per_cu);
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(a.total_tiles, (int64_t)multi_cus() * per_cu));
    hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(64), 0, st, a.counter);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(nthreads), smem, st, a);
    return hipGetLastError();
}

// Host side: descriptors from the validated scenes, in the order given by
// `order` (indices into `scenes`).
hipError_t launch_omp_multi(const sc_scene *scenes, const int *order, int n, int a0mode, int tile, int row_cache,
                            int wg_per_cu, int *counter, hipStream_t st) {
    MultiArgs a;
    memset(&a, 0, sizeof(a));
    a.n = n;
    a.counter = counter;
    int64_t t0 = 0;
    int max_kp = 64;
    bool any_refit = false;
    for (int q = 0; q < n; ++q) {
        const sc_scene &s = scenes[order[q]];
        const sc_dict h = s.dict;
        SceneDesc &d = a.sc[q];
        d.dict = h->ddev;
        d.X = s.X;
        d.idx = s.idx;
        d.coef = s.coef;
        d.count = s.count;
        d.resid = s.resid;
        d.stats = h->stats;
        d.N = s.N;
        d.tile_begin = t0;
        d.k = s.k;
        d.eps = s.eps;
        d.flags = ((s.flags & SC_EPS_RELATIVE) ? 1 : 0) | ((s.flags & SC_NO_FP64_REFIT) ? 0 : 2) | (h->dev.d << 8);
        const int E = h->dev.E;
        const int ei = E == 1 ? 0 : E == 2 ? 1 : E == 4 ? 2 : 3;
        d.cls = 4 * ei + pick_kmax(s.k) / 4 - 1;
        t0 += (s.N + tile - 1) / tile;
        max_kp = std::max(max_kp, h->dev.Kp);
        any_refit |= (d.flags & 2) != 0;
    }
    a.total_tiles = t0;
    if (t0 == 0) return hipSuccess;
    hipError_t e;
    const bool mf = a0mode == A0_MFMA_F32;
    if (tile == 32) {
        if (row_cache)
            e = mf ? launch_multi_t<32, 4, A0_MFMA_F32>(a, max_kp, wg_per_cu, st)
                   : launch_multi_t<32, 4, A0_VALU>(a, max_kp, wg_per_cu, st);
        else
            e = mf ? launch_multi_t<32, 0, A0_MFMA_F32>(a, max_kp, wg_per_cu, st)
                   : launch_multi_t<32, 0, A0_VALU>(a, max_kp, wg_per_cu, st);
    } else {
        if (row_cache)
            e = mf ? launch_multi_t<16, 4, A0_MFMA_F32>(a, max_kp, wg_per_cu, st)
                   : launch_multi_t<16, 4, A0_VALU>(a, max_kp, wg_per_cu, st);
        else
            e = mf ? launch_multi_t<16, 0, A0_MFMA_F32>(a, max_kp, wg_per_cu, st)
                   : launch_multi_t<16, 0, A0_VALU>(a, max_kp, wg_per_cu, st);
    }
    if (e != hipSuccess || !any_refit) return e;
    int64_t nchunks = 0;
    for (int q = 0; q < n; ++q) nchunks = std::max<int64_t>(nchunks, (a.sc[q].N + 63) / 64);
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>((nchunks + kOmpWaves - 1) / kOmpWaves,
                                                                (int64_t)multi_cus() * 4));
    hipLaunchKernelGGL(omp_multi_refit_kernel, dim3((unsigned)grid), dim3(kOmpThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace sc
