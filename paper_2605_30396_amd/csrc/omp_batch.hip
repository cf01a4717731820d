// Batch-OMP on gfx950: one 64-lane wave per signal, correlations and the
// Cholesky factor in registers.
//
// OMP (Sec. 2.1 of the paper) selects, step by step, the atom most correlated
// with the residual and refits x on the selected atoms by least squares.
// Batch-OMP reaches the same result from the Gram matrix G = D^T D without
// forming the residual:
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
// Register layout of one wave: lane l owns atoms l*E .. l*E+E-1 (Kp = 64 E)
// of alpha and of every B_t, so ties in the argmax resolve to the lowest atom
// index by taking the lowest lane, then the lowest entry; selected atoms are
// poisoned with NaN, which no '>' comparison picks.  Lane t also keeps step
// t's scalars (c_t, l_tt, the atom) and column t of L (L[u][t], u > t), so
// the triangular solves and the explicit residual run lane-parallel.
//
// Work layout: a workgroup of 4 waves takes tiles of 16 signals.  The tile's
// alpha0 = D^T X_tile (Kp x 16) is computed by the whole workgroup into LDS,
// then each wave encodes 4 signals.  alpha0 modes:
//   A0_VALU         FP32 FMAs from the feature-major dictionary
//   A0_MFMA_F32     v_mfma_f32_16x16x4_f32, FP32 operands (same precision)
//   A0_MFMA_BF16X3  v_mfma_f32_16x16x32_bf16 on the split D = Dh + Dl,
//                   x = xh + xl: Dh xh + Dl xh + Dh xl, relative error ~2^-16.
//                   The pursuit then runs on these correlations, and the
//                   coefficients are refit from D_I^T x computed in FP32, so
//                   the BF16 error affects only near-tie selections; the stop
//                   test near eps is taken on the explicit FP32 residual.
#include "mfma.h"
#include "sc_internal.h"
#include "wave.h"

namespace sc {

constexpr int kTileS = 16;   // signals per workgroup tile
constexpr int kXhs = 72;     // LDS row stride (BF16) of the split signal tile
constexpr int kOmpWaves = 4;
constexpr int kOmpThreads = 64 * kOmpWaves;

template <int N>
using vecf = float __attribute__((ext_vector_type(N)));

// Per-wave LDS scratch of the (rare) FP64 refit.
template <int KMAX>
struct WaveScratch {
    int sel[KMAX];
    float gam[KMAX];
    double Gd[KMAX * KMAX];
    double zd[KMAX];
};

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

// alpha0 tile on FP32 MFMA: wave w computes the 16-atom blocks w, w+4, ...
// with independent accumulators interleaved over the k-steps.  The A operand
// (16 atoms x 4 features) is read from the feature-major dictionary, so each
// load covers 4 runs of 16 consecutive atoms.
template <int E>
__device__ __forceinline__ void alpha0_mfma_f32(const float *__restrict__ DT, int d, const float *__restrict__ Xt,
                                                float *__restrict__ A0, int wave, int lane) {
    constexpr int Kp = 64 * E, MT = Kp / 16, NB = MT / kOmpWaves;   // blocks per wave
    const int lr = lane & 15, kq = lane >> 4;
    floatx4 acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = floatx4{0.f, 0.f, 0.f, 0.f};
    const int dk = (d + 3) & ~3;
#pragma unroll 2
    for (int k0 = 0; k0 < dk; k0 += 4) {
        const int f = k0 + kq;
        const float bx = Xt[f * kTileS + lr];
        const float *row = DT + (size_t)(f < d ? f : 0) * Kp + lr;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const float a = f < d ? row[(wave + kOmpWaves * b) * 16] : 0.f;
            acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bx, acc[b], 0, 0, 0);
        }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b)
        *reinterpret_cast<floatx4 *>(A0 + lr * Kp + (wave + kOmpWaves * b) * 16 + 4 * kq) = acc[b];
}

// alpha0 tile as the split BF16 product Dh xh + Dl xh + Dh xl (features padded to 64).
template <int E>
__device__ __forceinline__ void alpha0_mfma_bf16x3(const uint16_t *__restrict__ Dh, const uint16_t *__restrict__ Dl,
                                                   const uint16_t *__restrict__ Xh, const uint16_t *__restrict__ Xl,
                                                   float *__restrict__ A0, int wave, int lane) {
    constexpr int Kp = 64 * E, MT = Kp / 16, NB = MT / kOmpWaves;
    const int lr = lane & 15, kq = lane >> 4;
    floatx4 acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k0 = 0; k0 < 64; k0 += 32) {
        const bf16x8 bh = ld_bf16x8(Xh + lr * kXhs + k0 + 8 * kq);
        const bf16x8 bl = ld_bf16x8(Xl + lr * kXhs + k0 + 8 * kq);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int atom = (wave + kOmpWaves * b) * 16 + lr;
            const bf16x8 ah = ld_bf16x8(Dh + (size_t)atom * 64 + k0 + 8 * kq);
            const bf16x8 al = ld_bf16x8(Dl + (size_t)atom * 64 + k0 + 8 * kq);
            acc[b] = mfma16(al, bh, acc[b]);
            acc[b] = mfma16(ah, bl, acc[b]);
            acc[b] = mfma16(ah, bh, acc[b]);
        }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b)
        *reinterpret_cast<floatx4 *>(A0 + lr * Kp + (wave + kOmpWaves * b) * 16 + 4 * kq) = acc[b];
}

template <int E, int KMAX, int MODE>
__global__ __launch_bounds__(kOmpThreads) void omp_batch_kernel(DictDev dict, OmpParams p) {
    constexpr int Kp = 64 * E;
    constexpr bool kRefit = MODE == A0_MFMA_BF16X3;
    using vE = vecf<E>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float *A0 = reinterpret_cast<float *>(smem_raw);                   // [16][Kp]
    float *Xt = A0 + kTileS * Kp;                                      // [64][16]
    uint16_t *Xh = reinterpret_cast<uint16_t *>(Xt + 64 * kTileS);     // [16][72] BF16 high part
    uint16_t *Xl = Xh + kTileS * kXhs;                                 // [16][72] BF16 low part
    WaveScratch<KMAX> *wsAll = reinterpret_cast<WaveScratch<KMAX> *>(Xl + kTileS * kXhs);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    WaveScratch<KMAX> &ws = wsAll[wave];
    const int d = dict.d, K = dict.K, k = p.k;
    const float *__restrict__ G = dict.G;
    const float *__restrict__ Dg = dict.D;
    const float nanv = __builtin_nanf("");
    unsigned long long n_sig = 0, n_atoms = 0, n_refit = 0;

    // feature rows >= d of the tile stay zero (the MFMA products read 48 or 64)
    for (int q = tid; q < 64 * kTileS; q += kOmpThreads) Xt[q] = 0.f;

    const int64_t Nsig = p.rows ? (int64_t)(*p.nrows) : p.N;
    const int64_t ntiles = (Nsig + kTileS - 1) / kTileS;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t s0 = tile * kTileS;
        const int nt = (int)min<int64_t>(kTileS, Nsig - s0);
        __syncthreads();
        // coalesced read of the tile's nt*d floats (rows gathered through the
        // list in fallback mode), stored transposed
        if (p.rows) {
            for (int f = tid; f < nt * d; f += kOmpThreads) {
                int s = f / d, i = f - s * d;
                Xt[i * kTileS + s] = p.X[(int64_t)p.rows[s0 + s] * d + i];
            }
        } else {
            const float *__restrict__ Xtile = p.X + s0 * d;
            for (int f = tid; f < nt * d; f += kOmpThreads) {
                int s = f / d, i = f - s * d;
                Xt[i * kTileS + s] = Xtile[f];
            }
        }
        __syncthreads();
        if (MODE == A0_VALU) {
            alpha0_tile<E>(dict.DT, d, Xt, A0, tid);
        } else if (MODE == A0_MFMA_F32) {
            alpha0_mfma_f32<E>(dict.DT, d, Xt, A0, wave, lane);
        } else {
            for (int q = tid; q < kTileS * 64; q += kOmpThreads) {
                const int s = q >> 6, f = q & 63;
                const float v = Xt[f * kTileS + s];
                const uint16_t hi = bf16_bits(v);
                Xh[s * kXhs + f] = hi;
                Xl[s * kXhs + f] = bf16_bits(v - bf16_to_f32(hi));
            }
            __syncthreads();
            alpha0_mfma_bf16x3<E>(dict.Dbf, dict.Dlo, Xh, Xl, A0, wave, lane);
        }
        __syncthreads();

        for (int s = wave; s < nt; s += kOmpWaves) {
            const int64_t sig = p.rows ? (int64_t)p.rows[s0 + s] : s0 + s;
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
            // tracked-residual uncertainty: FP32 rounding, or the ~2^-16
            // error of the split-BF16 correlations
            const float band = (kRefit ? 1e-4f : 1e-5f) * xx;
            const float brk = 1e-6f * xnorm;

            vE al;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int j = lane * E + e;
                al[e] = j < K ? A0[s * Kp + j] : nanv;
            }
            vE B[KMAX];
            // lane t: step t's scalars, column t (and row t) of L
            float Lcol[KMAX], Lrow[KMAX];
#pragma unroll
            for (int u = 0; u < KMAX; ++u) {
                Lcol[u] = 0.f;
                Lrow[u] = 0.f;
            }
            float cval = 0.f, lval = 1.f, linv = 1.f, gam_l = 0.f;
            int selv = -1;
            float rr = xx;
            float lmax = 0.f, lmin = 3.4e38f;
            int n = 0;
            bool explicit_done = false;
            float rr_expl = 0.f;
            bool active = xx > 0.f;

            // c_t = L^-1 (D_I^T x): z recomputed in FP32 from the signal (BF16 refit)
            auto refit_c = [&](int nn) {
                float z = 0.f;
                if (lane < nn) {
                    const float *a = dict.D48 + (size_t)selv * 48;
                    for (int i = 0; i < d; ++i) z = fmaf(a[i], Xt[i * kTileS + s], z);
                }
                float acc = 0.f;
#pragma unroll
                for (int t = 0; t < KMAX; ++t) {
                    if (t < nn) {
                        const float yt = readlane_f((z - acc) * linv, t);
                        if (lane == t) cval = yt;
                        acc = fmaf(Lrow[t], yt, acc);
                    }
                }
            };
            // gamma = L^-T c, lane t receives gamma_t
            auto back_substitute = [&](int nn) {
                float acc = 0.f;
#pragma unroll
                for (int t = KMAX - 1; t >= 0; --t) {
                    if (t < nn) {
                        const float gt = readlane_f((cval - acc) * linv, t);
                        if (lane == t) gam_l = gt;
                        acc = fmaf(Lcol[t], gt, acc);
                    }
                }
            };
            // ||x - D_I gamma||^2 (lane i < d holds x_i)
            auto explicit_resid2 = [&](int nn) {
                float r = xv;
#pragma unroll
                for (int t = 0; t < KMAX; ++t) {
                    if (t < nn) {
                        const int st = readlane_i(selv, t);
                        const float gt = readlane_f(gam_l, t);
                        if (lane < d) r = fmaf(-Dg[(size_t)st * d + lane], gt, r);
                    }
                }
                return wave_sum(lane < d ? r * r : 0.f);
            };

            // Fully unrolled over the sparsity cap (so the per-step arrays stay
            // in registers); `active` skips the remaining steps uniformly.
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
                        if (kRefit) refit_c(it);
                        back_substitute(it);
                        const float re = explicit_resid2(it);
                        if (re <= eps2) {
                            explicit_done = true;
                            rr_expl = re;
                            active = false;
                            continue;
                        }
                    }
                }
                // ---- selection: argmax |alpha| over unselected atoms ----
                // lane maximum (NaN-poisoned entries are ignored by fmax),
                // wave maximum, lowest lane holding it, lowest entry in it
                float m = fabsf(al[0]);
#pragma unroll
                for (int e = 1; e < E; ++e) m = fmaxf(m, fabsf(al[e]));
                if (!(m >= 0.f)) m = -1.f;   // all entries poisoned
                const float mx = wave_max(m);
                if (!(mx > brk)) {
                    active = false;
                    continue;
                }
                int ei = E - 1;
                float sv = al[E - 1];
#pragma unroll
                for (int e = E - 2; e >= 0; --e) {
                    const bool hit = fabsf(al[e]) == m;
                    ei = hit ? e : ei;
                    sv = hit ? al[e] : sv;
                }
                const uint64_t bal = ballot(m == mx);
                const int wl = __ffsll((unsigned long long)bal) - 1;
                const int es = readlane_i(ei, wl);
                const int j = wl * E + es;
                const float aj = readlane_f(sv, wl);
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
                const float inv = __builtin_amdgcn_rcpf(ell);
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
                // ---- keep L row `it` distributed: lane t < it gets w_t ----
                float wmine = 0.f;
#pragma unroll
                for (int t = 0; t < it; ++t) wmine = lane == t ? w[t] : wmine;
                Lcol[it] = wmine;
                if (kRefit) {
#pragma unroll
                    for (int t = 0; t < it; ++t) Lrow[t] = lane == it ? w[t] : Lrow[t];
                }
                if (lane == it) {
                    cval = cn;
                    lval = ell;
                    linv = inv;
                    selv = j;
                }
                n = it + 1;
            }

            // ---- finalise: coefficients, optional FP64 refit, residual ----
            if (kRefit) refit_c(n);
            back_substitute(n);
            if (n > 0 && p.fp64_refit) {
                const float kap = (lmax / lmin) * (lmax / lmin);
                if (kap > p.kappa_max) {
                    if (lane < n) ws.sel[lane] = selv;
                    refit_fp64<KMAX>(ws, n, Dg, d, Xt + s, lane);
                    if (lane < n) gam_l = ws.gam[lane];
                    n_refit += 1;
                    explicit_done = false;
                }
            }
            const float re = explicit_done ? rr_expl : explicit_resid2(n);
            if (lane < k) {
                oidx[lane] = lane < n ? selv : -1;
                ocoef[lane] = lane < n ? gam_l : 0.f;
            }
            if (lane == 0) {
                p.count[sig] = n;
                if (p.resid) p.resid[sig] = sqrtf(re);
            }
            n_sig += 1;
            n_atoms += n;
        }
    }
    if (p.stats && lane == 0 && n_sig) {
        atomicAdd(p.stats + 0, n_sig);
        atomicAdd(p.stats + 1, n_atoms);
        if (n_refit) atomicAdd(p.stats + 2, n_refit);
    }
}

template <int E, int KMAX, int MODE>
static hipError_t launch_batch_t(const DictDev &dict, const OmpParams &p, hipStream_t st) {
    constexpr int Kp = 64 * E;
    size_t smem = sizeof(float) * (kTileS * Kp + 64 * kTileS) + sizeof(uint16_t) * 2 * kTileS * kXhs +
                  sizeof(WaveScratch<KMAX>) * kOmpWaves;
    auto kern = omp_batch_kernel<E, KMAX, MODE>;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    int64_t ntiles = (p.N + kTileS - 1) / kTileS;   // upper bound in fallback mode
    int dev = 0, ncu = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    int64_t grid = std::min<int64_t>(ntiles, (int64_t)ncu * 16);
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(kOmpThreads), smem, st, dict, p);
    return hipGetLastError();
}

template <int MODE>
static hipError_t launch_batch_mode(const DictDev &dict, const OmpParams &p, int kmax, hipStream_t st) {
#define SC_CASE(EE, KK) \
    if (dict.E == EE && kmax == KK) return launch_batch_t<EE, KK, MODE>(dict, p, st);
    SC_CASE(1, 4) SC_CASE(1, 8) SC_CASE(1, 12) SC_CASE(1, 16) SC_CASE(1, 24) SC_CASE(1, 32)
    SC_CASE(2, 4) SC_CASE(2, 8) SC_CASE(2, 12) SC_CASE(2, 16) SC_CASE(2, 24) SC_CASE(2, 32)
    SC_CASE(4, 4) SC_CASE(4, 8) SC_CASE(4, 12) SC_CASE(4, 16) SC_CASE(4, 24) SC_CASE(4, 32)
    SC_CASE(8, 4) SC_CASE(8, 8) SC_CASE(8, 12) SC_CASE(8, 16)
    SC_CASE(12, 4) SC_CASE(12, 8) SC_CASE(12, 12)
    SC_CASE(16, 4) SC_CASE(16, 8)
#undef SC_CASE
    return hipErrorInvalidValue;
}

// (E, KMAX) pairs with a compiled register-resident pursuit, for each alpha0 mode.
hipError_t launch_omp_batch(const DictDev &dict, const OmpParams &p, int kmax, int a0mode, hipStream_t st) {
    if (a0mode == A0_MFMA_BF16X3 && dict.d > 48) a0mode = A0_MFMA_F32;   // the FP32 refit reads 48-wide rows
    switch (a0mode) {
        case A0_VALU: return launch_batch_mode<A0_VALU>(dict, p, kmax, st);
        case A0_MFMA_F32: return launch_batch_mode<A0_MFMA_F32>(dict, p, kmax, st);
        case A0_MFMA_BF16X3: return launch_batch_mode<A0_MFMA_BF16X3>(dict, p, kmax, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace sc
