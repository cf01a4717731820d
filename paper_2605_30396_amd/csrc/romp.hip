// Restricted Batch-OMP over per-signal candidate atoms (the proposer's list),
// with the explicit-residual acceptance test that routes misses to the full
// encoder.
//
// Eight lanes serve one signal (8 signals per wave); lane g of a group owns
// candidates 4g .. 4g+3 of the signal's list, which is sorted by atom index,
// so the lowest (lane, entry) with the largest |alpha| is the lowest atom
// index.  Group reductions use DPP inside each 8-lane half-row; values of the
// winning lane are fetched with ds_bpermute.  The pursuit is the same
// Batch-OMP as the full encoder (alpha0 = D_C^T x, Gram-row update of the
// orthonormalised correlations, incremental Cholesky), restricted to C.
//
// After the pursuit the coefficients are solved, the residual ||x - D_I g|| is
// computed explicitly in FP32, and the code is accepted if it is <= eps (or
// eps ||x||); otherwise the signal index is appended to the fallback list.
#include "sc_internal.h"
#include "wave.h"

namespace sc {

constexpr int kRCpl = 4;           // candidates per lane (n_cand <= 32)
constexpr int kRThreads = 256;
constexpr int kMissQ = 256;        // fallback rows queued per wave before one atomic reserves their slots
// Dictionary staged in LDS (LDSD): one 16-wave workgroup per compute unit
// reads the candidate rows from its own copy of D48 (K x 48 FP32, 96 KB at
// K = 512) instead of gathering them from L2, which bounded the correlation
// stage; the miss queues are shorter to make room.
constexpr int kRWavesL = 16;
constexpr int kMissQL = 64;

template <int KMAX>
struct GroupScratch {
    float L[KMAX * KMAX];
    float c[KMAX];
    float gam[KMAX];
    int sel[KMAX];
    float x[48];
    int cand[8 * kRCpl];
};

template <int KMAX>
struct RompWaveScratch {
    GroupScratch<KMAX> g[8];
    double Gd[KMAX * KMAX];
    double zd[KMAX];
};

__device__ __forceinline__ float grp_max(float v) {
    v = fmaxf(v, dpp_f<SC_DPP_QP1032>(v));
    v = fmaxf(v, dpp_f<SC_DPP_QP2301>(v));
    v = fmaxf(v, dpp_f<SC_DPP_HMIRROR>(v));
    return v;
}

__device__ __forceinline__ float grp_sum(float v) {
    v += dpp_f<SC_DPP_QP1032>(v);
    v += dpp_f<SC_DPP_QP2301>(v);
    v += dpp_f<SC_DPP_HMIRROR>(v);
    return v;
}

__device__ __forceinline__ float shfl_f(float v, int src) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}
__device__ __forceinline__ int shfl_i(int v, int src) { return __builtin_amdgcn_ds_bpermute(src << 2, v); }

template <int N>
using vecr = float __attribute__((ext_vector_type(N)));

// gamma = L^-T c (group lane 0).
template <int KMAX>
__device__ __forceinline__ void grp_back_substitute(GroupScratch<KMAX> &gs, int n, int g) {
    __builtin_amdgcn_wave_barrier();
    if (g == 0) {
        for (int t = n - 1; t >= 0; --t) {
            float s = gs.c[t];
            for (int u = t + 1; u < n; ++u) s -= gs.L[u * KMAX + t] * gs.gam[u];
            gs.gam[t] = s / gs.L[t * KMAX + t];
        }
    }
    __builtin_amdgcn_wave_barrier();
}

// ||x - D_I gamma||^2 over the group (lane g holds features g, g+8, ...).
// The atom rows are read in batches of BT steps with every load of a batch in
// flight at once (steps past n read atom 0 with a zero weight).
template <int KMAX, int BT>
__device__ __forceinline__ float grp_resid2(const GroupScratch<KMAX> &gs, int n, const float *__restrict__ D48, int d,
                                            int g) {
    float r[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) r[q] = gs.x[g + 8 * q];   // zero beyond d
#pragma unroll
    for (int t0 = 0; t0 < KMAX; t0 += BT) {
        if (__ballot(t0 < n) != 0) {   // some active group still has steps here
            float a[BT][6], gt[BT];
#pragma unroll
            for (int u = 0; u < BT; ++u) {
                const int t = t0 + u;
                const bool on = t < n;
                const int j = on ? gs.sel[t < KMAX ? t : 0] : 0;
                gt[u] = on ? gs.gam[t < KMAX ? t : 0] : 0.f;
#pragma unroll
                for (int q = 0; q < 6; ++q) a[u][q] = D48[(size_t)j * 48 + g + 8 * q];
            }
#pragma unroll
            for (int u = 0; u < BT; ++u)
#pragma unroll
                for (int q = 0; q < 6; ++q) r[q] = fmaf(-a[u][q], gt[u], r[q]);
        }
    }
    float acc = 0.f;
#pragma unroll
    for (int q = 0; q < 6; ++q) acc = fmaf(r[q], r[q], acc);
    (void)d;
    return grp_sum(acc);
}

template <int KMAX, bool LDSD>
__global__ __launch_bounds__(LDSD ? 64 * kRWavesL : kRThreads) void omp_restricted_kernel(
    DictDev dict, const float *__restrict__ D48g, RompParams p) {
    constexpr int NWV = LDSD ? kRWavesL : kRThreads / 64;   // waves per workgroup
    constexpr int MQ = LDSD ? kMissQL : kMissQ;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    RompWaveScratch<KMAX> *wsAll = reinterpret_cast<RompWaveScratch<KMAX> *>(smem_raw);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const float *__restrict__ D48 = D48g;
    if constexpr (LDSD) {   // the workgroup's copy of the dictionary rows, after the wave scratch
        static_assert(sizeof(RompWaveScratch<KMAX>) % 16 == 0, "16-byte aligned dictionary copy");
        float *Ds = reinterpret_cast<float *>(smem_raw + sizeof(RompWaveScratch<KMAX>) * NWV);
        for (int q = tid; q < dict.K * 12; q += 64 * NWV)
            reinterpret_cast<float4 *>(Ds)[q] = reinterpret_cast<const float4 *>(D48g)[q];
        __syncthreads();
        D48 = Ds;
    }
    const int g = lane & 7, grp = lane >> 3;
    RompWaveScratch<KMAX> &ws = wsAll[wave];
    GroupScratch<KMAX> &gs = ws.g[grp];
    const int d = dict.d, Kp = dict.Kp, k = p.k, nc = p.n_cand;
    const float *__restrict__ G = dict.G;
    const float nanv = __builtin_nanf("");
    unsigned long long n_sig = 0, n_atoms = 0, n_miss = 0, n_refit = 0;
    // per-wave queue of fallback rows (wave-uniform fill level nq)
    __shared__ int32_t miss_queue[NWV][MQ];
    int32_t *mq = miss_queue[wave];
    int nq = 0;
    auto flush_misses = [&]() {
        if (nq == 0) return;
        __builtin_amdgcn_wave_barrier();
        int base = 0;
        if (lane == 0) base = atomicAdd(p.miss_count, nq);
        base = __builtin_amdgcn_readfirstlane(base);
        for (int q = lane; q < nq; q += 64) p.miss_rows[base + q] = mq[q];
        __builtin_amdgcn_wave_barrier();
        nq = 0;
    };
    using vR = vecr<kRCpl>;

    const int64_t ngroups = (p.N + 7) / 8;
    const int64_t gwave = (int64_t)blockIdx.x * NWV + wave;
    const int64_t wstride = (int64_t)gridDim.x * NWV;
    for (int64_t wg = gwave; wg < ngroups; wg += wstride) {
        const int64_t sig = wg * 8 + grp;
        const bool valid = sig < p.N;
        // ---- signal and candidates: every load issued before the first use ----
        float xr[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const int f = g + 8 * q;
            xr[q] = (valid && f < d) ? p.X[sig * d + f] : 0.f;
        }
        // a candidate outside [0, K) reads as -1 (no candidate)
        int cid[kRCpl];
#pragma unroll
        for (int e = 0; e < kRCpl; ++e) {
            const int q = g * kRCpl + e;
            const int c = (valid && q < nc) ? p.cand[sig * nc + q] : -1;
            cid[e] = (unsigned)c < (unsigned)dict.K ? c : -1;
        }
        int first = valid ? p.cand[sig * nc] : 0;
        first = (unsigned)first < (unsigned)dict.K ? first : -1;
        float xx_part = 0.f;
        bool fin = true;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            fin &= isfinite(xr[q]);
            gs.x[g + 8 * q] = xr[q];
            xx_part = fmaf(xr[q], xr[q], xx_part);
        }
        int nf = fin ? 0 : 1;
        nf |= __builtin_amdgcn_update_dpp(0, nf, SC_DPP_QP1032, 0xF, 0xF, false);
        nf |= __builtin_amdgcn_update_dpp(0, nf, SC_DPP_QP2301, 0xF, 0xF, false);
        nf |= __builtin_amdgcn_update_dpp(0, nf, SC_DPP_HMIRROR, 0xF, 0xF, false);
        const float xx = grp_sum(xx_part);
        const bool cand_ok = first >= 0;
        __builtin_amdgcn_wave_barrier();
        // ---- alpha0 over the candidates ----
        // Lane g takes features 4g .. 4g+3 and 32+2g, 33+2g of every candidate
        // (one 16-byte and one 8-byte load), so the group's eight lanes read
        // one contiguous 192-byte dictionary row together (scattered per-lane
        // rows cost one cache-line access per lane); the partial dots are
        // summed over the group and each candidate's sum is kept by the lane
        // that owns it in the pursuit.
#pragma unroll
        for (int e = 0; e < kRCpl; ++e) gs.cand[g * kRCpl + e] = cid[e];
        __builtin_amdgcn_wave_barrier();
        const float4 xa = *reinterpret_cast<const float4 *>(gs.x + 4 * g);
        const float2 xb = *reinterpret_cast<const float2 *>(gs.x + 32 + 2 * g);
        vR al;
#pragma unroll
        for (int e = 0; e < kRCpl; ++e) al[e] = 0.f;
        constexpr int kCB = 2;   // candidates per batch of loads (4 would cost a wave per SIMD at k = 8)
        static_assert((8 * kRCpl) % kCB == 0, "candidate batches");
#pragma unroll
        for (int b = 0; b < 8 * kRCpl / kCB; ++b) {
            if (kCB * b >= nc) break;   // uniform: slots past the list are -1 (NaN below)
            float4 da[kCB];
            float2 db[kCB];
#pragma unroll
            for (int u = 0; u < kCB; ++u) {
                const int c = gs.cand[kCB * b + u];
                const float *row = D48 + (size_t)(c < 0 ? 0 : c) * 48;
                da[u] = *reinterpret_cast<const float4 *>(row + 4 * g);
                db[u] = *reinterpret_cast<const float2 *>(row + 32 + 2 * g);
            }
#pragma unroll
            for (int u = 0; u < kCB; ++u) {
                float part = fmaf(da[u].x, xa.x, fmaf(da[u].y, xa.y, fmaf(da[u].z, xa.z, da[u].w * xa.w)));
                part = fmaf(db[u].x, xb.x, fmaf(db[u].y, xb.y, part));
                part = grp_sum(part);
                const int cq = kCB * b + u;   // owned by lane cq / kRCpl, entry cq % kRCpl
                if (g == cq / kRCpl) al[cq % kRCpl] = part;
            }
        }
#pragma unroll
        for (int e = 0; e < kRCpl; ++e)
            if (cid[e] < 0) al[e] = nanv;

        const float xnorm = sqrtf(xx);
        const float eps_abs = p.relative ? p.eps * xnorm : p.eps;
        const float eps2 = eps_abs * eps_abs;
        const float band = 1e-5f * xx;
        const float brk = 1e-6f * xnorm;
        bool active = valid && !nf && cand_ok && xx > 0.f;
        bool explicit_done = false;
        float rr_expl = 0.f;
        float rr = xx;
        float lmax = 0.f, lmin = 3.4e38f;
        int n = 0;
        vR B[KMAX];

#pragma unroll
        for (int it = 0; it < KMAX; ++it) {
            if (active) {
                bool go = it < p.kcap;
                if (go && eps2 > 0.f) {
                    if (rr <= eps2 - band) {
                        go = false;
                    } else if (rr <= eps2 + band) {
                        grp_back_substitute<KMAX>(gs, it, g);
                        float re = grp_resid2<KMAX, 2>(gs, it, D48, d, g);
                        if (re <= eps2) {
                            explicit_done = true;
                            rr_expl = re;
                            go = false;
                        }
                    }
                }
                float m = -1.f;
                int ei = 0;
#pragma unroll
                for (int e = 0; e < kRCpl; ++e) {
                    float v = fabsf(al[e]);
                    if (v > m) {
                        m = v;
                        ei = e;
                    }
                }
                const float mx = grp_max(m);
                if (go && !(mx > brk)) go = false;
                const uint64_t bal = __ballot(go && m == mx);
                const int gbits = (int)((bal >> (grp * 8)) & 0xFFull);
                const int owner = grp * 8 + (__ffs(gbits) - 1);
                float myal = al[0];
                int myc = cid[0];
#pragma unroll
                for (int e = 1; e < kRCpl; ++e)
                    if (ei == e) {
                        myal = al[e];
                        myc = cid[e];
                    }
                const int es = shfl_i(ei, go ? owner : lane);
                const int j = shfl_i(myc, go ? owner : lane);
                // the Gram gathers of the step read row jl (j itself whenever
                // the step is taken); up to a cap of 4 they are issued here,
                // before the shuffles below, from an in-range row (at caps
                // 5..8 the registers they hold early would cost a wave per SIMD)
                constexpr bool kEarly = KMAX <= 4;
                float gjj = 0.f;
                vR gjc;
                if constexpr (kEarly) {
                    const int jl = (unsigned)j < (unsigned)dict.K ? j : 0;
                    const float *__restrict__ Gj = G + (size_t)jl * Kp;
                    gjj = Gj[jl];
#pragma unroll
                    for (int e = 0; e < kRCpl; ++e) gjc[e] = Gj[cid[e] >= 0 ? cid[e] : 0];
                }
                const float aj = shfl_f(myal, go ? owner : lane);
                float wsq = 0.f;
                float w[KMAX];
#pragma unroll
                for (int t = 0; t < it; ++t) {
                    float bv = B[t][0];
#pragma unroll
                    for (int e = 1; e < kRCpl; ++e)
                        if (es == e) bv = B[t][e];
                    w[t] = shfl_f(bv, go ? owner : lane);
                    wsq = fmaf(w[t], w[t], wsq);
                }
                if (go) {
                    if constexpr (!kEarly) gjj = G[(size_t)j * Kp + j];
                    const float l2 = gjj - wsq;
                    if (!(l2 > 1e-9f * gjj)) {
                        go = false;
                    } else {
                        const float ell = sqrtf(l2);
                        const float inv = 1.f / ell;
                        const float cn = aj * inv;
                        rr = fmaf(-cn, cn, rr);
                        lmax = fmaxf(lmax, ell);
                        lmin = fminf(lmin, ell);
                        vR bn;
#pragma unroll
                        for (int e = 0; e < kRCpl; ++e) {
                            if constexpr (kEarly)
                                bn[e] = cid[e] >= 0 ? gjc[e] : 0.f;
                            else
                                bn[e] = cid[e] >= 0 ? G[(size_t)j * Kp + cid[e]] : 0.f;
                        }
#pragma unroll
                        for (int t = 0; t < it; ++t) bn -= w[t] * B[t];
                        bn *= inv;
                        B[it] = bn;
                        al -= cn * bn;
                        if (lane == owner) {
#pragma unroll
                            for (int e = 0; e < kRCpl; ++e)
                                if (es == e) al[e] = nanv;
                        }
                        if (g == 0) {
                            for (int t = 0; t < it; ++t) gs.L[it * KMAX + t] = w[t];
                            gs.L[it * KMAX + it] = ell;
                            gs.c[it] = cn;
                            gs.sel[it] = j;
                        }
                        n = it + 1;
                    }
                }
                active = go;
            }
        }
        __builtin_amdgcn_wave_barrier();

        // ---- finalise ----
        // A code whose tracked ||r||^2 is clearly above eps^2 (beyond the FP32
        // band) is a miss: no coefficients or explicit residual are needed.
        const bool ok_sig = valid && !nf && cand_ok;
        const bool need = ok_sig && (explicit_done || xx == 0.f || rr <= eps2 + band);
        if (__ballot(need) != 0) grp_back_substitute<KMAX>(gs, n, g);
        bool want_refit = need && n > 0 && p.fp64_refit && (lmax / lmin) * (lmax / lmin) > p.kappa_max;
        // FP64 refits, one group at a time (rare)
        uint64_t rb = __ballot(want_refit && g == 0);
        while (rb) {
            const int gl = __ffsll((unsigned long long)rb) - 1;
            rb &= rb - 1;
            GroupScratch<KMAX> &gq = ws.g[gl >> 3];
            const int nq = shfl_i(n, gl);
            for (int q = lane; q < nq * nq; q += 64) {
                int t = q / nq, u = q % nq;
                double s = 0.0;
                for (int i = 0; i < d; ++i)
                    s += (double)D48[(size_t)gq.sel[t] * 48 + i] * (double)D48[(size_t)gq.sel[u] * 48 + i];
                ws.Gd[t * KMAX + u] = s;
            }
            if (lane < nq) {
                double s = 0.0;
                for (int i = 0; i < d; ++i) s += (double)D48[(size_t)gq.sel[lane] * 48 + i] * (double)gq.x[i];
                ws.zd[lane] = s;
            }
            __builtin_amdgcn_wave_barrier();
            if (lane == 0) {
                double *Gd = ws.Gd, *z = ws.zd;
                for (int t = 0; t < nq; ++t)
                    for (int u = 0; u <= t; ++u) {
                        double s = Gd[t * KMAX + u];
                        for (int v = 0; v < u; ++v) s -= Gd[t * KMAX + v] * Gd[u * KMAX + v];
                        Gd[t * KMAX + u] = (u == t) ? sqrt(fmax(s, 1e-300)) : s / Gd[u * KMAX + u];
                    }
                for (int t = 0; t < nq; ++t) {
                    double s = z[t];
                    for (int u = 0; u < t; ++u) s -= Gd[t * KMAX + u] * z[u];
                    z[t] = s / Gd[t * KMAX + t];
                }
                for (int t = nq - 1; t >= 0; --t) {
                    double s = z[t];
                    for (int u = t + 1; u < nq; ++u) s -= Gd[u * KMAX + t] * z[u];
                    z[t] = s / Gd[t * KMAX + t];
                }
                for (int t = 0; t < nq; ++t) gq.gam[t] = (float)z[t];
            }
            __builtin_amdgcn_wave_barrier();
        }
        if (want_refit) {
            explicit_done = false;
            if (g == 0) n_refit += 1;
        }
        float re = 3.4e38f;
        if (__ballot(need && !explicit_done) != 0) re = grp_resid2<KMAX, 4>(gs, need ? n : 0, D48, d, g);
        if (explicit_done) re = rr_expl;
        if (!need) re = 3.4e38f;
        const bool accept = valid && !nf && cand_ok && (re <= eps2 || xx == 0.f);
        const bool miss = valid && !nf && !accept;
        if (valid) {
            int32_t *oidx = p.idx + sig * k;
            float *ocoef = p.coef + sig * k;
            if (nf) {
                for (int t = g; t < k; t += 8) {
                    oidx[t] = -1;
                    ocoef[t] = 0.f;
                }
                if (g == 0) {
                    p.count[sig] = -1;
                    if (p.resid) p.resid[sig] = nanv;
                }
            } else if (accept) {
                for (int t = g; t < k; t += 8) {
                    oidx[t] = t < n ? gs.sel[t] : -1;
                    ocoef[t] = t < n ? gs.gam[t] : 0.f;
                }
                if (g == 0) {
                    p.count[sig] = n;
                    if (p.resid) p.resid[sig] = sqrtf(re);
                    n_sig += 1;
                    n_atoms += n;
                }
            }
        }
        // misses of the wave's 8 signals are queued in LDS; the queue is
        // flushed to the fallback list with one atomic per kMissQ entries
        const uint64_t mb = __ballot(miss && g == 0);
        if (mb) {
            const int cm = __popcll(mb);
            if (nq + cm > MQ) flush_misses();
            if (miss && g == 0) {
                mq[nq + __popcll(mb & ((1ull << lane) - 1ull))] = (int32_t)sig;
                n_miss += 1;
            }
            nq += cm;
        }
        __builtin_amdgcn_wave_barrier();
    }
    flush_misses();
    if (p.stats) {   // one atomic per counter and workgroup
        __shared__ unsigned int red[NWV][4];
        const unsigned long long v[4] = {n_sig, n_atoms, n_refit, n_miss};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            unsigned int t = (unsigned int)v[c];
            t += __shfl_xor(t, 8);
            t += __shfl_xor(t, 16);
            t += __shfl_xor(t, 32);
            if (lane == 0) red[wave][c] = t;
        }
        __syncthreads();
        if (tid < 4) {
            unsigned long long t = 0;
            for (int w = 0; w < NWV; ++w) t += red[w][tid];
            if (t) atomicAdd(p.stats + tid, t);
        }
    }
}

template <int KMAX, bool LDSD>
static hipError_t launch_romp_t(const DictDev &dict, const float *D48, const RompParams &p, size_t smem, int ncu,
                                hipStream_t st) {
    constexpr int NWV = LDSD ? kRWavesL : kRThreads / 64;
    auto kern = omp_restricted_kernel<KMAX, LDSD>;
    static size_t attr = 0;   // largest dynamic LDS size set so far
    if (smem > attr) {
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e != hipSuccess) return e;
        attr = smem;
    }
    const int64_t nw = (p.N + 7) / 8;
    const int64_t grid = LDSD ? std::max<int64_t>(1, std::min<int64_t>((nw + NWV - 1) / NWV, (int64_t)ncu))
                              : std::max<int64_t>(1, std::min<int64_t>((nw + 3) / 4, (int64_t)ncu * 8));
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(64 * NWV), smem, st, dict, D48, p);
    return hipGetLastError();
}

template <int KMAX>
static hipError_t launch_romp_k(const DictDev &dict, const float *D48, const RompParams &p, hipStream_t st) {
    int dev = 0, ncu = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    constexpr size_t lds_max = 160 * 1024;   // LDS of a gfx950 workgroup
    // static LDS of the staged form: miss queues and the counter reduction
    constexpr size_t kStaticL = sizeof(int32_t) * kRWavesL * kMissQL + sizeof(unsigned int) * kRWavesL * 4;
    const size_t smemL = sizeof(RompWaveScratch<KMAX>) * kRWavesL + sizeof(float) * 48 * (size_t)dict.K;
    if constexpr (KMAX <= 4) {
        if (smemL + kStaticL <= lds_max)
            return launch_romp_t<KMAX, true>(dict, D48, p, smemL, ncu, st);
    }
    return launch_romp_t<KMAX, false>(dict, D48, p, sizeof(RompWaveScratch<KMAX>) * (kRThreads / 64), ncu, st);
}

hipError_t launch_omp_restricted(const DictDev &dict, const float *D48, const RompParams &p, int kmax, hipStream_t st) {
    if (p.n_cand > 8 * kRCpl) return hipErrorInvalidValue;
    switch (kmax) {
        case 4: return launch_romp_k<4>(dict, D48, p, st);
        case 8: return launch_romp_k<8>(dict, D48, p, st);
        case 12: return launch_romp_k<12>(dict, D48, p, st);
        case 16: return launch_romp_k<16>(dict, D48, p, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace sc
