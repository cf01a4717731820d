// FP32 Batch-OMP on gfx950: one 64-lane wave per signal, correlations in
// registers.
//
// OMP (Sec. 2.1 of the paper) selects, step by step, the atom most correlated
// with the residual and refits x on the selected atoms by least squares.
// Batch-OMP reaches the same result from the Gram matrix G = D^T D without
// ever forming the residual:
//
//   alpha0 = D^T x                       (once per signal)
//   step n: j = argmax_{j not selected} |alpha_j|
//           w = first n-1 entries of the new Cholesky row of G_II
//           l = sqrt(G_jj - |w|^2)                      (new diagonal entry)
//           c_n = alpha_j / l                           (forward substitution)
//           B_n = (G[j,:] - sum_t w_t B_t) / l          (Gram-row update)
//           alpha -= c_n B_n
//           ||r||^2 -= c_n^2
//   gamma = L^-T c                                       (back substitution)
//
// B_t = D^T q_t are the correlations of the orthonormalised atoms q_t, so
// w_t = B_t[j] is read straight from the registers of the lane owning atom j,
// and alpha = alpha0 - G_I gamma is maintained incrementally: one Gram row is
// read per step.
//
// Work layout: a workgroup of 4 waves takes tiles of 16 signals.  The tile's
// alpha0 = D^T X_tile (Kp x 16) is computed by all 256 threads from the
// feature-major dictionary (L2-resident) and the tile held in LDS, then each
// wave encodes 4 signals.  Lane l owns atoms l*E .. l*E+E-1 (Kp = 64 E), so
// ties in the argmax resolve to the lowest atom index by taking the lowest
// lane, then the lowest entry.  Selected atoms are poisoned with NaN, which no
// '>' comparison ever picks.
#include "sc_internal.h"
#include "wave.h"

namespace sc {

constexpr int kTileS = 16;   // signals per workgroup tile
constexpr int kOmpWaves = 4;
constexpr int kOmpThreads = 64 * kOmpWaves;

template <int N>
using vecf = float __attribute__((ext_vector_type(N)));

// Per-wave LDS scratch of the pursuit (KMAX x KMAX Cholesky factor etc.).
template <int KMAX>
struct WaveScratch {
    float L[KMAX * KMAX];  // row n: w_0..w_{n-1}, l_n
    float c[KMAX];         // forward-substituted right-hand side
    float gam[KMAX];       // coefficients
    int sel[KMAX];         // selected atoms, in order
    double Gd[KMAX * KMAX];  // FP64 refit workspace
    double zd[KMAX];
};

// gamma = L^-T c for the first n rows, computed by lane 0 into LDS.
template <int KMAX>
__device__ __forceinline__ void back_substitute(WaveScratch<KMAX> &ws, int n) {
    __builtin_amdgcn_wave_barrier();
    if (lane_id() == 0) {
        for (int t = n - 1; t >= 0; --t) {
            float s = ws.c[t];
            for (int u = t + 1; u < n; ++u) s -= ws.L[u * KMAX + t] * ws.gam[u];
            ws.gam[t] = s / ws.L[t * KMAX + t];
        }
    }
    __builtin_amdgcn_wave_barrier();
}

// ||x - D_I gamma||^2 with lane i < d holding x_i.
template <int KMAX>
__device__ __forceinline__ float explicit_resid2(const WaveScratch<KMAX> &ws, int n, const float *__restrict__ D,
                                                 int d, float xv, int lane) {
    float r = 0.f;
    if (lane < d) {
        r = xv;
        for (int t = 0; t < n; ++t) r -= D[(size_t)ws.sel[t] * d + lane] * ws.gam[t];
    }
    return wave_sum(r * r);
}

// FP64 refit of gamma on the selected atoms: G_II gamma = D_I^T x, with G_II
// and D_I^T x summed in FP64 and solved by Cholesky (lane 0, into LDS).
template <int KMAX>
__device__ void refit_fp64(WaveScratch<KMAX> &ws, int n, const float *__restrict__ D, int d,
                           const float *__restrict__ xs /* LDS, stride kTileS */, int lane) {
    __builtin_amdgcn_wave_barrier();
    for (int q = lane; q < n * n; q += 64) {
        int t = q / n, u = q % n;
        const float *a = D + (size_t)ws.sel[t] * d;
        const float *b = D + (size_t)ws.sel[u] * d;
        double s = 0.0;
        for (int i = 0; i < d; ++i) s += (double)a[i] * (double)b[i];
        ws.Gd[t * KMAX + u] = s;
    }
    if (lane < n) {
        const float *a = D + (size_t)ws.sel[lane] * d;
        double s = 0.0;
        for (int i = 0; i < d; ++i) s += (double)a[i] * (double)xs[i * kTileS];
        ws.zd[lane] = s;
    }
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) {
        double *Gd = ws.Gd, *z = ws.zd;
        for (int t = 0; t < n; ++t) {          // G = R R^T, R lower, in place
            for (int u = 0; u <= t; ++u) {
                double s = Gd[t * KMAX + u];
                for (int v = 0; v < u; ++v) s -= Gd[t * KMAX + v] * Gd[u * KMAX + v];
                Gd[t * KMAX + u] = (u == t) ? sqrt(fmax(s, 1e-300)) : s / Gd[u * KMAX + u];
            }
        }
        for (int t = 0; t < n; ++t) {          // R y = z
            double s = z[t];
            for (int u = 0; u < t; ++u) s -= Gd[t * KMAX + u] * z[u];
            z[t] = s / Gd[t * KMAX + t];
        }
        for (int t = n - 1; t >= 0; --t) {     // R^T g = y
            double s = z[t];
            for (int u = t + 1; u < n; ++u) s -= Gd[u * KMAX + t] * z[u];
            z[t] = s / Gd[t * KMAX + t];
        }
        for (int t = 0; t < n; ++t) ws.gam[t] = (float)z[t];
    }
    __builtin_amdgcn_wave_barrier();
}

// alpha0 tile: A0[s][j] = sum_i DT[i][j] * Xt[i][s] for the 16 tile signals.
template <int E>
__device__ __forceinline__ void alpha0_tile(const float *__restrict__ DT, int d, const float *__restrict__ Xt,
                                            float *__restrict__ A0, int tid) {
    constexpr int Kp = 64 * E;
    constexpr int KpP = Kp < 256 ? Kp : 256;   // atoms covered by one pass of 256 threads
    constexpr int SG = 256 / KpP;              // signal groups
    constexpr int JS = Kp / KpP;               // atom slots per thread
    constexpr int SQ = kTileS / SG;            // signals per thread
    const int j0 = tid % KpP, sg = tid / KpP;
    float acc[JS][SQ];
#pragma unroll
    for (int r = 0; r < JS; ++r)
#pragma unroll
        for (int q = 0; q < SQ; ++q) acc[r][q] = 0.f;
    for (int i = 0; i < d; ++i) {
        float dv[JS];
#pragma unroll
        for (int r = 0; r < JS; ++r) dv[r] = DT[(size_t)i * Kp + j0 + r * KpP];
#pragma unroll
        for (int q = 0; q < SQ; ++q) {
            float xv = Xt[i * kTileS + sg + q * SG];
#pragma unroll
            for (int r = 0; r < JS; ++r) acc[r][q] = fmaf(dv[r], xv, acc[r][q]);
        }
    }
#pragma unroll
    for (int r = 0; r < JS; ++r)
#pragma unroll
        for (int q = 0; q < SQ; ++q) A0[(sg + q * SG) * Kp + j0 + r * KpP] = acc[r][q];
}

template <int E, int KMAX>
__global__ __launch_bounds__(kOmpThreads) void omp_fp32_kernel(DictDev dict, OmpParams p) {
    constexpr int Kp = 64 * E;
    using vE = vecf<E>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float *A0 = reinterpret_cast<float *>(smem_raw);                   // [16][Kp]
    float *Xt = A0 + kTileS * Kp;                                      // [64][16]
    WaveScratch<KMAX> *wsAll = reinterpret_cast<WaveScratch<KMAX> *>(Xt + 64 * kTileS);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    WaveScratch<KMAX> &ws = wsAll[wave];
    const int d = dict.d, K = dict.K, k = p.k;
    const float *__restrict__ G = dict.G;
    const float *__restrict__ Dg = dict.D;
    const float nanv = __builtin_nanf("");
    unsigned long long n_sig = 0, n_atoms = 0, n_refit = 0;

    const int64_t ntiles = (p.N + kTileS - 1) / kTileS;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t s0 = tile * kTileS;
        const int nt = (int)min<int64_t>(kTileS, p.N - s0);
        __syncthreads();
        // coalesced read of the tile's nt*d contiguous floats, stored transposed
        const float *__restrict__ Xtile = p.X + s0 * d;
        for (int f = tid; f < nt * d; f += kOmpThreads) {
            int s = f / d, i = f - s * d;
            Xt[i * kTileS + s] = Xtile[f];
        }
        __syncthreads();
        alpha0_tile<E>(dict.DT, d, Xt, A0, tid);
        __syncthreads();

        for (int s = wave; s < nt; s += kOmpWaves) {
            const int64_t sig = s0 + s;
            const float xv = lane < d ? Xt[lane * kTileS + s] : 0.f;
            const bool bad = lane < d && !isfinite(xv);
            int32_t *oidx = p.idx + sig * k;
            float *ocoef = p.coef + sig * k;
            if (ballot(bad) != 0) {
                for (int t = lane; t < k; t += 64) {
                    oidx[t] = -1;
                    ocoef[t] = 0.f;
                }
                if (lane == 0) {
                    p.count[sig] = -1;
                    if (p.resid) p.resid[sig] = nanv;
                }
                continue;
            }
            const float xx = wave_sum(xv * xv);
            const float xnorm = sqrtf(xx);
            const float eps_abs = p.relative ? p.eps * xnorm : p.eps;
            const float eps2 = eps_abs * eps_abs;
            const float band = 1e-5f * xx;
            const float brk = 1e-6f * xnorm;

            vE al;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int j = lane * E + e;
                al[e] = j < K ? A0[s * Kp + j] : nanv;
            }
            vE B[KMAX];
            float rr = xx;
            float lmax = 0.f, lmin = 3.4e38f;
            int n = 0;
            bool explicit_done = false;
            float rr_expl = 0.f;
            bool active = xx > 0.f;

            // Fully unrolled over the sparsity cap (so B[] stays in registers);
            // `active` turns the remaining steps into skipped uniform branches.
#pragma unroll
            for (int it = 0; it < KMAX; ++it) {
                if (!active) continue;
                if (it >= k) {
                    active = false;
                    continue;
                }
                // ---- stop test (before the selection) ----
                if (eps2 > 0.f) {
                    if (rr <= eps2 - band) {
                        active = false;
                        continue;
                    }
                    if (rr <= eps2 + band) {
                        back_substitute<KMAX>(ws, it);
                        float re = explicit_resid2<KMAX>(ws, it, Dg, d, xv, lane);
                        if (re <= eps2) {
                            explicit_done = true;
                            rr_expl = re;
                            active = false;
                            continue;
                        }
                    }
                }
                // ---- selection: argmax |alpha| over unselected atoms ----
                float m = -1.f;
                int ei = 0;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    float v = fabsf(al[e]);
                    if (v > m) {
                        m = v;
                        ei = e;
                    }
                }
                const float mx = wave_max(m);
                if (!(mx > brk)) {
                    active = false;
                    continue;
                }
                const uint64_t bal = ballot(m == mx);
                const int wl = __ffsll((unsigned long long)bal) - 1;
                const int es = readlane_i(ei, wl);
                const int j = wl * E + es;
                const float aj = readlane_f(al[es], wl);
                float w[KMAX];
                float wsq = 0.f;
#pragma unroll
                for (int t = 0; t < it; ++t) {
                    w[t] = readlane_f(B[t][es], wl);
                    wsq = fmaf(w[t], w[t], wsq);
                }
                const float gjj = G[(size_t)j * Kp + j];
                const float l2 = gjj - wsq;
                if (!(l2 > 1e-9f * gjj)) {   // numerically dependent atom
                    active = false;
                    continue;
                }
                const float ell = sqrtf(l2);
                const float inv = 1.f / ell;
                const float cn = aj * inv;
                rr = fmaf(-cn, cn, rr);
                lmax = fmaxf(lmax, ell);
                lmin = fminf(lmin, ell);
                // ---- Gram-row update of the correlations ----
                vE bn;
#pragma unroll
                for (int e = 0; e < E; ++e) bn[e] = G[(size_t)j * Kp + lane * E + e];
#pragma unroll
                for (int t = 0; t < it; ++t) bn -= w[t] * B[t];
                bn *= inv;
                B[it] = bn;
                al -= cn * bn;
                if (lane == wl) al[es] = nanv;
                // ---- record the Cholesky row, c_n and the atom ----
                __builtin_amdgcn_wave_barrier();
                if (lane < it) {
                    float wv = 0.f;
#pragma unroll
                    for (int t = 0; t < it; ++t)
                        if (lane == t) wv = w[t];
                    ws.L[it * KMAX + lane] = wv;
                }
                if (lane == 0) {
                    ws.L[it * KMAX + it] = ell;
                    ws.c[it] = cn;
                    ws.sel[it] = j;
                }
                __builtin_amdgcn_wave_barrier();
                n = it + 1;
            }

            // ---- finalise: coefficients, optional FP64 refit, residual ----
            back_substitute<KMAX>(ws, n);
            if (n > 0 && p.fp64_refit) {
                float kap = (lmax / lmin) * (lmax / lmin);
                if (kap > p.kappa_max) {
                    refit_fp64<KMAX>(ws, n, Dg, d, Xt + s, lane);
                    n_refit += 1;
                    explicit_done = false;
                }
            }
            float re = explicit_done ? rr_expl : explicit_resid2<KMAX>(ws, n, Dg, d, xv, lane);
            for (int t = lane; t < k; t += 64) {
                oidx[t] = t < n ? ws.sel[t] : -1;
                ocoef[t] = t < n ? ws.gam[t] : 0.f;
            }
            if (lane == 0) {
                p.count[sig] = n;
                if (p.resid) p.resid[sig] = sqrtf(re);
            }
            n_sig += 1;
            n_atoms += n;
            __builtin_amdgcn_wave_barrier();
        }
    }
    if (p.stats && lane == 0 && n_sig) {
        atomicAdd(p.stats + 0, n_sig);
        atomicAdd(p.stats + 1, n_atoms);
        if (n_refit) atomicAdd(p.stats + 2, n_refit);
    }
}

template <int E, int KMAX>
static hipError_t launch_fp32_t(const DictDev &dict, const OmpParams &p, hipStream_t st) {
    constexpr int Kp = 64 * E;
    size_t smem = sizeof(float) * (kTileS * Kp + 64 * kTileS) + sizeof(WaveScratch<KMAX>) * kOmpWaves;
    auto kern = omp_fp32_kernel<E, KMAX>;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    int64_t ntiles = (p.N + kTileS - 1) / kTileS;
    int dev = 0, ncu = 256;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    int64_t grid = std::min<int64_t>(ntiles, (int64_t)ncu * 16);
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(kOmpThreads), smem, st, dict, p);
    return hipGetLastError();
}

// (E, KMAX) pairs with a compiled register-resident pursuit.
hipError_t launch_omp_fp32(const DictDev &dict, const OmpParams &p, int kmax, hipStream_t st) {
#define SC_CASE(EE, KK) \
    if (dict.E == EE && kmax == KK) return launch_fp32_t<EE, KK>(dict, p, st);
    SC_CASE(1, 4) SC_CASE(1, 8) SC_CASE(1, 12) SC_CASE(1, 16) SC_CASE(1, 24) SC_CASE(1, 32)
    SC_CASE(2, 4) SC_CASE(2, 8) SC_CASE(2, 12) SC_CASE(2, 16) SC_CASE(2, 24) SC_CASE(2, 32)
    SC_CASE(4, 4) SC_CASE(4, 8) SC_CASE(4, 12) SC_CASE(4, 16) SC_CASE(4, 24) SC_CASE(4, 32)
    SC_CASE(8, 4) SC_CASE(8, 8) SC_CASE(8, 12) SC_CASE(8, 16)
    SC_CASE(12, 4) SC_CASE(12, 8) SC_CASE(12, 12)
    SC_CASE(16, 4) SC_CASE(16, 8)
#undef SC_CASE
    return hipErrorInvalidValue;
}

}  // namespace sc
