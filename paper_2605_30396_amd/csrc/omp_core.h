// Batch-OMP tile encoder on gfx950, shared by the single-dictionary kernel
// and the multi-scene persistent kernel.
//
// OMP (Sec. 2.1, Eq. (1)) picks, step by step, the atom most correlated with
// the residual and refits x on the picked atoms by least squares.  Batch-OMP
// reaches the same codes from alpha0 = D^T x and the Gram matrix G = D^T D
// without forming the residual:
//
//   alpha = alpha0 - G_I gamma                 (correlations of the residual)
//   j     = argmax_{j not in I} |alpha_j|
//   w     = Li G[I, j],  l = sqrt(G_jj - |w|^2)       (Li = L^-1, G_II = L L^T)
//   c_j   = alpha_j / l
//   new row of Li = (-(w^T Li), 1) / l
//   gamma += c_j (new row of Li),   ||r||^2 -= c_j^2   (gamma = Li^T c)
//
// One 64-lane wave encodes one signal.  Lane l owns atoms l*E .. l*E+E-1
// (Kp = 64 E) of alpha0; the Gram rows of the selected atoms are re-read
// (from L2) whenever alpha is formed, so the per-wave register state is
// O(E + k) and several waves fit on a SIMD.  Lane t keeps step t's atom,
// gamma_t, and row t and column t of Li, so each step costs every lane O(1)
// per selected atom, with no serial substitution.
//
// Selection key: the bits of |alpha_j| with the low 10 mantissa bits replaced
// by (1023 - j) and bit 31 set while the atom is selectable, so one unsigned
// wave maximum gives the atom, and entries whose magnitudes agree to 2^-13
// relative resolve to the lowest index.  Padding atoms have bit 31 clear;
// selected atoms keep it (their correlation is zero up to rounding) and are
// masked only when one of them wins.
//
// A support whose Cholesky condition estimate (max L_ii / min L_ii)^2 exceeds
// kappa_max leaves count = -(2 + n) and the FP32 coefficients; a separate
// pass (refit_scan) solves it again in FP64 and writes the final count.
#pragma once
#include "mfma.h"
#include "sc_internal.h"
#include "wave.h"

namespace sc {

constexpr int kOmpWaves = 4;
constexpr int kOmpThreads = 64 * kOmpWaves;
constexpr int kXhs = 72;                              // LDS row stride (BF16) of the split signal tile
constexpr uint32_t kKeyIdx = 1023u;                   // atom index bits of a selection key
constexpr uint32_t kKeyMag = 0x7FFFFFFFu & ~kKeyIdx;  // magnitude bits of a selection key
constexpr uint32_t kKeyLive = 0x80000000u;            // set while the atom may still be selected

// Row stride (floats) of the alpha0 tile in LDS: 4 floats past Kp, so the
// 16 rows an MFMA result writes at once start 16 bytes apart and spread over
// the banks instead of hitting the same ones.
__host__ __device__ constexpr int a0_stride(int Kp) { return Kp + 4; }

// Row stride (floats) of the feature-major signal tile Xt[64][T]: 4 past T,
// so a column read (lane = feature) or the tile store spreads over 16 bank
// groups instead of the 4 that a stride of T = 16 maps to, and rows stay 16
// bytes aligned for the vector reads of the VALU correlation.
__host__ __device__ constexpr int xt_stride(int T) { return T + 4; }

// The three BF16 signal parts [T][kXhs] of the split-BF16 correlations live
// inside the alpha0 tile when it is large enough: they are read only before
// the tile is written.
__host__ __device__ constexpr bool split_in_a0(int T, int Kp) {
    return 3 * T * kXhs * (int)sizeof(uint16_t) <= T * a0_stride(Kp) * (int)sizeof(float);
}

// LDS bytes of one workgroup: alpha0 tile [T][a0_stride(Kp)], signal tile
// [64][xt_stride(T)], and for the split-BF16 correlations the three BF16
// signal parts when they do not fit inside the alpha0 tile.
__host__ __device__ constexpr size_t omp_tile_lds(int T, int Kp, bool split) {
    return sizeof(float) * ((size_t)T * a0_stride(Kp) + 64 * (size_t)xt_stride(T)) +
           (split && !split_in_a0(T, Kp) ? sizeof(uint16_t) * 3 * T * kXhs : 0);
}

struct OmpTally {
    unsigned long long sig = 0, atoms = 0;
};

// Signals s0 .. s0+nt-1 of the call (through `rows` when given), stored
// feature-major Xt[i][s]; features >= d and columns >= nt are zero.  A thread
// holds at most NE = T * 64 / NT elements of the tile (d <= 64); all of its
// loads (the listed row numbers first, then the signal entries) are issued
// from clamped addresses before any is used, so the tile costs one or two
// memory round trips instead of one or two per element.
template <int T, int NW = kOmpWaves>
__device__ __forceinline__ void load_tile(const OmpParams &p, int d, int64_t s0, int nt, float *Xt, int tid) {
    constexpr int NT = 64 * NW;
    constexpr int NE = (T * 64 + NT - 1) / NT;
    // element f = s d + i of the tile; (s, i) stepped along with f (one
    // division per thread, not one per element)
    const int dq = NT / d, dr = NT - dq * d;
    int s = tid / d, i = tid - (tid / d) * d;
    int se[NE], ie[NE];
    bool ok[NE];
#pragma unroll
    for (int e = 0; e < NE; ++e) {
        ok[e] = tid + e * NT < nt * d;
        se[e] = ok[e] ? s : 0;
        ie[e] = ok[e] ? i : 0;
        s += dq;
        i += dr;
        if (i >= d) {
            i -= d;
            ++s;
        }
    }
    float v[NE];
    if (p.rows) {   // a listed row outside [0, N) reads as zeros (and is not encoded)
        int64_t r[NE];
#pragma unroll
        for (int e = 0; e < NE; ++e) r[e] = p.rows[s0 + se[e]];
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            const bool in = ok[e] && (uint64_t)r[e] < (uint64_t)p.N;
            v[e] = p.X[(in ? r[e] : 0) * d + ie[e]];
            v[e] = in ? v[e] : 0.f;
        }
    } else {
        const float *__restrict__ Xtile = p.X + s0 * d;
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            v[e] = Xtile[ok[e] ? tid + e * NT : 0];
            v[e] = ok[e] ? v[e] : 0.f;
        }
    }
#pragma unroll
    for (int e = 0; e < NE; ++e)
        if (ok[e]) Xt[ie[e] * xt_stride(T) + se[e]] = v[e];
    for (int q = tid; q < 64 * T; q += NT) {
        const int i = q / T, s = q - i * T;
        if (i >= d || s >= nt) Xt[i * xt_stride(T) + s] = 0.f;
    }
}

// alpha0 tile on VALU: A0[s][j] = sum_i DT[i][j] Xt[i][s].  The dictionary
// rows are read from L2 four features ahead of their use (a ring of four row
// slices in registers), so the L2 latency overlaps the FMAs of the features
// in between instead of stalling every feature.
template <int E, int T, int NW = kOmpWaves>
__device__ __forceinline__ void alpha0_valu(const float *__restrict__ DT, int d, const float *__restrict__ Xt,
                                            float *__restrict__ A0, int tid) {
    constexpr int Kp = 64 * E, NT = 64 * NW;
    constexpr int KpP = Kp < NT ? Kp : NT;   // atoms covered by one pass of the workgroup
    constexpr int SG = NT / KpP;             // signal groups
    constexpr int JS = Kp / KpP;                               // atom slots per thread
    constexpr int SQ = T / SG;                                 // signals per thread
    constexpr int PF = 4;                                      // prefetch distance (features)
    static_assert(Kp % KpP == 0 && T % SG == 0, "tile shape");
    const int j0 = tid % KpP, sg = tid / KpP;
    const float *__restrict__ dp = DT + j0;
    float acc[JS][SQ];
#pragma unroll
    for (int r = 0; r < JS; ++r)
#pragma unroll
        for (int q = 0; q < SQ; ++q) acc[r][q] = 0.f;
    float ring[PF][JS];
#pragma unroll
    for (int u = 0; u < PF; ++u) {
        const int i = u < d ? u : d - 1;
#pragma unroll
        for (int r = 0; r < JS; ++r) ring[u][r] = dp[(size_t)i * Kp + r * KpP];
    }
    for (int i0 = 0; i0 < d; i0 += PF) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int i = i0 + u;
            if (i < d) {
                float xv[SQ];
                if constexpr (SG == 1 && SQ % 4 == 0) {
#pragma unroll
                    for (int q4 = 0; q4 < SQ / 4; ++q4) {
                        const float4 v = *reinterpret_cast<const float4 *>(Xt + i * xt_stride(T) + 4 * q4);
                        xv[4 * q4] = v.x;
                        xv[4 * q4 + 1] = v.y;
                        xv[4 * q4 + 2] = v.z;
                        xv[4 * q4 + 3] = v.w;
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < SQ; ++q) xv[q] = Xt[i * xt_stride(T) + sg + q * SG];
                }
#pragma unroll
                for (int q = 0; q < SQ; ++q)
#pragma unroll
                    for (int r = 0; r < JS; ++r) acc[r][q] = fmaf(ring[u][r], xv[q], acc[r][q]);
                const int inext = i + PF < d ? i + PF : d - 1;
#pragma unroll
                for (int r = 0; r < JS; ++r) ring[u][r] = dp[(size_t)inext * Kp + r * KpP];
            }
        }
    }
#pragma unroll
    for (int r = 0; r < JS; ++r)
#pragma unroll
        for (int q = 0; q < SQ; ++q) A0[(sg + q * SG) * a0_stride(Kp) + j0 + r * KpP] = acc[r][q];
}

// alpha0 tile on FP32 MFMA (v_mfma_f32_16x16x4_f32): wave w computes the
// 16-atom blocks w, w+NW, ... for every 16-signal column block; when there
// are fewer atom blocks than waves, NW / MT waves share an atom block and
// split the column blocks between them, waves past the last column block
// staying idle (each output element takes the same MFMA sequence either way,
// so the values do not depend on the wave count).
// The contraction runs over 16-feature chunks whose four k-steps take features
// 4 kq + s (s = 0..3) in lane group kq, so the A operands of a whole chunk are
// one 16-byte read per lane.  Dr holds the dictionary in that operand order
// (op_order_f32: per 16-atom block and chunk, 64 lanes x 4 floats, 1 KB
// contiguous), so a wave's read is eight whole cache lines; the next chunk is
// read while the current one is multiplied.  B operands come from the
// feature-major signal tile in LDS.
template <int E, int T, int NW>
struct MfmaF32Split {
    static constexpr int MT = 16 * E / 4, CB = T / 16;
    static constexpr int WPB = MT >= NW ? 1 : NW / MT;          // waves per atom block
    static constexpr int NB = MT >= NW ? MT / NW : 1;
    static constexpr int CBW = CB >= WPB ? CB / WPB : 1;        // column blocks per wave
    static constexpr bool ok = T % 16 == 0 && (MT >= NW ? MT % NW == 0
                                                        : NW % MT == 0 && (CB % WPB == 0 || WPB % CB == 0));
};

template <int E, int T, int NW = kOmpWaves>
__device__ __forceinline__ void alpha0_mfma_f32(const float *__restrict__ Dr, int dpad, const float *__restrict__ Xt,
                                                float *__restrict__ A0, int wave, int lane) {
    using S = MfmaF32Split<E, T, NW>;
    constexpr int Kp = 64 * E, MT = S::MT, NB = S::NB, CB = S::CBW;
    static_assert(S::ok, "MFMA tile shape");
    const int lr = lane & 15, kq = lane >> 4;
    const int ab0 = MT >= NW ? wave : wave % MT;            // first atom block of this wave
    const int cb0 = MT >= NW ? 0 : (wave / MT) * CB;        // first column block of this wave
    if (cb0 >= S::CB) return;   // more waves than (atom block, column block) pairs: this one is idle
    floatx4 acc[NB][CB];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int c = 0; c < CB; ++c) acc[b][c] = floatx4{0.f, 0.f, 0.f, 0.f};
    const float *rowp[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) rowp[b] = Dr + ((size_t)(ab0 + NW * b) * (dpad / 16) * 64 + lane) * 4;
    floatx4 an[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) an[b] = *reinterpret_cast<const floatx4 *>(rowp[b]);
    for (int f0 = 0; f0 < dpad; f0 += 16) {
        floatx4 a[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) a[b] = an[b];
        if (f0 + 16 < dpad) {
#pragma unroll
            for (int b = 0; b < NB; ++b) an[b] = *reinterpret_cast<const floatx4 *>(rowp[b] + 16 * (f0 + 16));
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int f = f0 + 4 * kq + q;
            float bx[CB];
#pragma unroll
            for (int c = 0; c < CB; ++c) bx[c] = Xt[f * xt_stride(T) + (cb0 + c) * 16 + lr];
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int c = 0; c < CB; ++c)
                    acc[b][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[b][q], bx[c], acc[b][c], 0, 0, 0);
        }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int c = 0; c < CB; ++c)
            *reinterpret_cast<floatx4 *>(A0 + ((cb0 + c) * 16 + lr) * a0_stride(Kp) + (ab0 + NW * b) * 16 + 4 * kq) =
                acc[b][c];
}

// alpha0 tile from BF16 matrix cores at FP32 accuracy: D and x are each
// split into three BF16 parts (v = vh + vm + vl, every part the rounding of
// what the previous ones leave), and the six products whose scale is at least
// 2^-16 are summed in FP32, smallest first:
//   Dm xm + Dl xh + Dh xl + Dm xh + Dh xm + Dh xh.
// The products left out (Dm xl, Dl xm, Dl xl) and the parts' own rounding
// are each <= 2^-27 |a_i x_i|, so they add <= 4 2^-27 ||x|| for a unit atom;
// the FP32 accumulation error is that of an FP32 dot product.  Features are
// padded to 64 (two k-steps of v_mfma_f32_16x16x32_bf16).  The waves split
// the 16-atom blocks and 16-signal column blocks as the FP32 stage does
// (MfmaF32Split); the dictionary parts are stored in the operand order of
// this MFMA (op_order_bf16x32: per 16-atom block and 32-feature k-step, 64
// lanes x 8 values, 1 KB contiguous), and the signal parts [3][T][kXhs] come
// from LDS.
template <int E, int T, int NW = kOmpWaves>
__device__ __forceinline__ void alpha0_mfma_bf16x6(const uint16_t *__restrict__ Dh, const uint16_t *__restrict__ Dm,
                                                   const uint16_t *__restrict__ Dl, const uint16_t *__restrict__ Xh,
                                                   float *__restrict__ A0, int wave, int lane) {
    using S = MfmaF32Split<E, T, NW>;
    constexpr int Kp = 64 * E, MT = S::MT, NB = S::NB, CB = S::CBW;
    static_assert(S::ok, "MFMA tile shape");
    const uint16_t *Xm = Xh + T * kXhs, *Xl = Xm + T * kXhs;
    const int lr = lane & 15, kq = lane >> 4;
    const int ab0 = MT >= NW ? wave : wave % MT;            // first atom block of this wave
    const int cb0 = MT >= NW ? 0 : (wave / MT) * CB;        // first column block of this wave
    const bool busy = cb0 < S::CB;   // waves past the last column block stay idle
    floatx4 acc[NB][CB];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int c = 0; c < CB; ++c) acc[b][c] = floatx4{0.f, 0.f, 0.f, 0.f};
    if (busy) {
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            bf16x8 bh[CB], bm[CB], bl[CB];
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                const int row = ((cb0 + c) * 16 + lr) * kXhs + 32 * ks + 8 * kq;
                bh[c] = ld_bf16x8(Xh + row);
                bm[c] = ld_bf16x8(Xm + row);
                bl[c] = ld_bf16x8(Xl + row);
            }
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const size_t off = (((size_t)(ab0 + NW * b) * 2 + ks) * 64 + lane) * 8;
                const bf16x8 ah = ld_bf16x8(Dh + off);
                const bf16x8 am = ld_bf16x8(Dm + off);
                const bf16x8 al = ld_bf16x8(Dl + off);
#pragma unroll
                for (int c = 0; c < CB; ++c) {
                    acc[b][c] = mfma16(am, bm[c], acc[b][c]);
                    acc[b][c] = mfma16(al, bh[c], acc[b][c]);
                    acc[b][c] = mfma16(ah, bl[c], acc[b][c]);
                    acc[b][c] = mfma16(am, bh[c], acc[b][c]);
                    acc[b][c] = mfma16(ah, bm[c], acc[b][c]);
                    acc[b][c] = mfma16(ah, bh[c], acc[b][c]);
                }
            }
        }
    }
    __syncthreads();   // every wave has read the signal parts, which may share the alpha0 tile
    if (busy) {
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int c = 0; c < CB; ++c)
                *reinterpret_cast<floatx4 *>(A0 + ((cb0 + c) * 16 + lr) * a0_stride(Kp) + (ab0 + NW * b) * 16 +
                                             4 * kq) = acc[b][c];
    }
}

// The E Gram-row entries of this lane (16-byte aligned for E % 4 == 0).
template <int E>
__device__ __forceinline__ void load_row(const float *__restrict__ p, float (&v)[E]) {
    if constexpr (E % 4 == 0) {
#pragma unroll
        for (int q = 0; q < E / 4; ++q) {
            const float4 f = reinterpret_cast<const float4 *>(p)[q];
            v[4 * q] = f.x;
            v[4 * q + 1] = f.y;
            v[4 * q + 2] = f.z;
            v[4 * q + 3] = f.w;
        }
    } else if constexpr (E == 2) {
        const float2 f = *reinterpret_cast<const float2 *>(p);
        v[0] = f.x;
        v[1] = f.y;
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = p[e];
    }
}

// v[e] for a wave-uniform slot e (a select chain; for narrow rows).
template <int E>
__device__ __forceinline__ float pick_slot(const float (&v)[E], int e) {
    float r = v[0];
#pragma unroll
    for (int q = 1; q < E; ++q) r = e == q ? v[q] : r;
    return r;
}

// Encodes signal `sig` (column s of the tile) with one wave.
//
// Batch-OMP with alpha = alpha0 - G_I gamma.  The least-squares solve is
// carried by the inverse Cholesky factor Li = L^-1 of G_II (G_II = L L^T),
// bordered each time an atom j joins: with g = G[I, j] and w = Li g,
//   l2 = G_jj - w.w  (the new diagonal of L, squared),
//   c_j = alpha_j / sqrt(l2)  (alpha_j the current correlation of j),
//   new row of Li = (-(w^T Li), 1) / sqrt(l2),
//   gamma += c_j * (new row of Li),   ||r||^2 -= c_j^2,
// so gamma = Li^T c is current after every step with O(1) work per lane per
// atom already selected, and no serial substitution.  Lane u holds row u and
// column u of Li and gamma_u; the broadcasts each step (g, w, the new row,
// gamma) go through this signal's alpha0 row in LDS, which is free once
// alpha0 is in registers.  The extreme diagonal values of L decide the FP64
// refit.
// RCQ: the Gram rows of the atoms of the first RCQ steps are kept in
// registers (RCQ * E VGPRs).  The row of the newest atom is fetched as soon
// as the atom is chosen and held for the next step; older rows are re-read
// kRowBatch at a time whenever alpha is formed.
// The code goes to oidx / ocoef (k slots each) and *ocount; the residual to
// p.resid[sig].
template <int E, int KMAX, int T, int RCQ>
__device__ __forceinline__ void omp_pursuit(const DictDev &dict, const OmpParams &p, int64_t sig, int s,
                                            const float *__restrict__ Xt, float *__restrict__ A0, int lane,
                                            int32_t *oidx, float *ocoef, int32_t *ocount, OmpTally &tally) {
    constexpr int Kp = 64 * E;
    constexpr int RC = RCQ < KMAX ? RCQ : KMAX;
    constexpr int kRowBatch = RCQ > 0 ? 1 : (KMAX >= 16 ? 2 : 3);   // within 128 VGPRs (4 waves per SIMD)
    constexpr int NL = KMAX <= 16 ? 16 : 32;                          // lanes that hold selected atoms
    // steps whose broadcasts are lane reads instead of LDS round trips (measured:
    // faster for the wide rows of K > 256, slower for K <= 256; 5 steps by a
    // hair over 4 and 6 at K = 512)
    constexpr int kLaneBcast = E >= 8 ? 5 : 0;
    const int d = dict.d, K = dict.K;
    // k and the lane index are re-read as opaque values per signal, so the
    // per-step tests against them are made where they are used rather than
    // hoisted out of the signal loop (twelve hoisted masks would be spilled)
    int k = p.k;
    asm volatile("" : "+s"(k));
    int lane_t = lane;   // the lane index for the per-step lane tests, likewise opaque
    asm volatile("" : "+v"(lane_t));
    const float *__restrict__ G = dict.G;
    const float *__restrict__ Dg = dict.D;
    const float xv = lane < d ? Xt[lane * xt_stride(T) + s] : 0.f;
    const int dl = lane < d ? lane : d - 1;   // in-bounds row offset for the idle lanes
    if (ballot(lane < d && !isfinite(xv)) != 0) {   // status -1, padded slots
        if (lane < k) {
            oidx[lane] = -1;
            ocoef[lane] = 0.f;
        }
        if (lane == 0) {
            *ocount = -1;
            if (p.resid) p.resid[sig] = __builtin_nanf("");
        }
        return;
    }
    const float xx = wave_sum(xv * xv);
    const float xnorm = __builtin_amdgcn_sqrtf(xx);
    const float eps_abs = p.relative ? p.eps * xnorm : p.eps;
    const float eps2 = eps_abs * eps_abs;
    const float band = 1e-5f * xx;     // FP32 uncertainty of the tracked ||r||^2
    const float brk = 1e-6f * xnorm;   // residual orthogonal to every atom
    // |alpha| <= brk compared on the bit patterns (both non-negative), in scalar registers
    const uint32_t brk_bits = (uint32_t)__builtin_amdgcn_readfirstlane((int)__float_as_uint(brk));

    // Key bit 31 marks an atom still selectable: any such key beats every
    // retired or padding atom, whatever their magnitude bits.
    // alpha0 of the padding atoms (j >= K) is zero (their dictionary columns are)
    float a0[E];
    uint32_t kid[E];
    load_row<E>(A0 + s * a0_stride(Kp) + lane * E, a0);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int j = lane * E + e;
        kid[e] = (j < K ? kKeyLive : 0u) | (kKeyIdx - (uint32_t)j);
    }
    // broadcast buffer: [0, 64) gamma, g and the new row of Li, [32, 64) w;
    // [0, Kp) alpha while the atom is chosen (E >= 4)
    float *bc = A0 + s * a0_stride(Kp);
    // lane u: row u and column u of Li.  Entry t of both is written whole
    // (every lane) at step t and read only by later steps, so neither needs
    // clearing; lanes past the atoms selected hold zeros in them.
    float LR[KMAX], LC[KMAX];
    float gam = 0.f;   // lane t: gamma_t
    int selv = 0;      // lane t: atom of step t
    float rc[RC > 0 ? RC : 1][E];   // G rows of the atoms of steps t < RC
    float nrow[E];                  // G row of the newest atom (step >= RC; loaded before it is read)
    float rr = xx, rr_expl = 0.f;
    // extreme squared diagonals of L, as bit patterns (every l2 taken is positive)
    uint32_t l2max = 0u, l2min = 0x7F7FFFFFu;
    int n = 0;
    bool active = xx > 0.f, expl_done = false;

    // ||x - D_I gamma||^2 with the current gamma (lane i < d holds x_i)
    auto resid2 = [&](int nn) {
        float r = xv;
        nn = __builtin_amdgcn_readfirstlane(nn);
#pragma unroll
        for (int t0 = 0; t0 < KMAX; t0 += 4) {
            if (t0 < nn) {
                float dv[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int jt = readlane_i(selv, t0 + q);
                    dv[q] = Dg[(uint32_t)(jt * d + dl)];   // K d < 2^32: 32-bit offsets
                }
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (t0 + q < nn) r = fmaf(-dv[q], readlane_f(gam, t0 + q), r);
            }
        }
        return wave_sum(lane < d ? r * r : 0.f);
    };

    // Unrolled over the sparsity cap so the per-step arrays stay in
    // registers; `active` skips the remaining steps uniformly.
#pragma unroll
    for (int it = 0; it < KMAX; ++it) {
        if (!active) continue;
        if (it >= k) {
            active = false;
            continue;
        }
        // ---- stop test before the selection ----
        if (eps2 > 0.f) {
            if (rr <= eps2 - band) {
                active = false;
                continue;
            }
            if (rr <= eps2 + band) {   // too close to call on the tracked value
                const float re = resid2(it);
                if (re <= eps2) {
                    expl_done = true;
                    rr_expl = re;
                    active = false;
                    continue;
                }
            }
        }
        // ---- correlations of the residual (gamma_t read from bc) and the selection ----
        float al[E];
#pragma unroll
        for (int e = 0; e < E; ++e) al[e] = a0[e];
        // gamma_t: from lane t at the first steps (a few lane reads beat an
        // LDS round trip), from the broadcast row later
        auto gamma_at = [&](int t) { return it <= kLaneBcast ? readlane_f(gam, t) : bc[t]; };
#pragma unroll
        for (int t = 0; t < (it < RC ? it : RC); ++t) {
            const float gt = gamma_at(t);
#pragma unroll
            for (int e = 0; e < E; ++e) al[e] = fmaf(-gt, rc[t][e], al[e]);
        }
        // rows RC .. it-2 from L2: the first kRowBatch with their loads in
        // flight together, later ones (long supports only) one or two at a
        // time in a real loop, whose trip count is kept opaque to the
        // optimiser so that it does not unroll it and hold every row at once;
        // row it-1 is nrow
#pragma unroll
        for (int t0 = RC; t0 < (it - 1 < RC + kRowBatch ? it - 1 : RC + kRowBatch); t0 += kRowBatch) {
            float gr[kRowBatch][E];
#pragma unroll
            for (int q = 0; q < kRowBatch; ++q)
                if (t0 + q < it - 1) load_row<E>(G + (size_t)readlane_i(selv, t0 + q) * Kp + lane * E, gr[q]);
#pragma unroll
            for (int q = 0; q < kRowBatch; ++q) {
                if (t0 + q < it - 1) {
                    const float gt = gamma_at(t0 + q);
#pragma unroll
                    for (int e = 0; e < E; ++e) al[e] = fmaf(-gt, gr[q][e], al[e]);
                }
            }
        }
        if (it - 1 > RC + kRowBatch) {
            const int tend = (it - 1) | (k >> 16);   // k <= 32: the value is it - 1
            int t = RC + kRowBatch;
            if constexpr (E <= 4) {   // rows in pairs, both loads in flight (registers to spare here)
                for (; t + 1 < tend; t += 2) {
                    float g0[E], g1[E];
                    load_row<E>(G + (size_t)readlane_i(selv, t) * Kp + lane * E, g0);
                    load_row<E>(G + (size_t)readlane_i(selv, t + 1) * Kp + lane * E, g1);
                    const float gt0 = gamma_at(t), gt1 = gamma_at(t + 1);
#pragma unroll
                    for (int e = 0; e < E; ++e) al[e] = fmaf(-gt0, g0[e], al[e]);
#pragma unroll
                    for (int e = 0; e < E; ++e) al[e] = fmaf(-gt1, g1[e], al[e]);
                }
            }
            for (; t < tend; ++t) {
                float gr[E];
                load_row<E>(G + (size_t)readlane_i(selv, t) * Kp + lane * E, gr);
                // from the row only past the lane-read steps: up to step
                // kLaneBcast the row holds this step's alpha, not gamma
                const float gt = gamma_at(t);
#pragma unroll
                for (int e = 0; e < E; ++e) al[e] = fmaf(-gt, gr[e], al[e]);
            }
        }
        if (it - 1 >= RC) {
            const float gt = gamma_at(it - 1);
#pragma unroll
            for (int e = 0; e < E; ++e) al[e] = fmaf(-gt, nrow[e], al[e]);
        }
        if constexpr (E >= 4) {   // alpha to this signal's LDS row (gamma there is consumed), for alpha_j below
#pragma unroll
            for (int e = 0; e < E; e += 4)
                *reinterpret_cast<floatx4 *>(bc + lane * E + e) = floatx4{al[e], al[e + 1], al[e + 2], al[e + 3]};
        }
        uint32_t best = 0u;
#pragma unroll
        for (int e = 0; e < E; ++e) best = max(best, (__float_as_uint(al[e]) & kKeyMag) | kid[e]);
        uint32_t kb = wave_max_u32(best);
        if ((kb & kKeyMag) <= brk_bits) {
            active = false;
            continue;
        }
        // A selected atom keeps its live bit: its correlation with the
        // residual is zero up to rounding, so it wins only when every live
        // atom's correlation is as small.  Then the choice is made again with
        // every selected atom masked (rare), which equals masking them all
        // along; the per-lane key words stay unchanged.
        if (it > 0 && (ballot(selv == (int)(kKeyIdx - (kb & kKeyIdx))) & ((1ull << it) - 1ull)) != 0) {
            uint32_t dead = 0u;   // bit e: this lane's atom e is selected
#pragma unroll
            for (int t = 0; t < it; ++t) {
                const int st = readlane_i(selv, t);
                dead |= st / E == lane ? 1u << (st % E) : 0u;
            }
            best = 0u;
#pragma unroll
            for (int e = 0; e < E; ++e)
                best = max(best, ((dead >> e) & 1u) ? 0u : (__float_as_uint(al[e]) & kKeyMag) | kid[e]);
            kb = wave_max_u32(best);
            if ((kb & kKeyMag) <= brk_bits || !(kb & kKeyLive)) {
                active = false;
                continue;
            }
        }
        const uint32_t kbi = kb & kKeyIdx;
        const int j = (int)(kKeyIdx - kbi);
        if (it < RC)
            load_row<E>(G + (size_t)j * Kp + lane * E, rc[it < RC ? it : 0]);
        else
            load_row<E>(G + (size_t)j * Kp + lane * E, nrow);
        // the signed correlation of atom j, from the lane that holds it
        const int lj = j / E, ej = j - lj * E;   // owner lane and slot (E need not be a power of 2)
        float aj;
        if constexpr (E >= 4) {
            aj = bc[j];
        } else {   // a select over E registers and one lane read
            aj = readlane_f(pick_slot<E>(al, ej), lj);
        }
        // ---- new row of Li: w = Li G[I, j], l2 = G_jj - w.w ----
        const float gjj = G[(size_t)j * Kp + j];
        float wsum = 0.f, acc = 0.f;
        if (it > 0) {
            // lane t < it: G[I_t, j] (K Kp < 2^32: a 32-bit offset)
            const float g = lane_t < it ? G[(uint32_t)(selv * Kp + j)] : 0.f;
            float w = 0.f;
            if (it <= kLaneBcast) {
#pragma unroll
                for (int t = 0; t < it; ++t) w = fmaf(LR[t], readlane_f(g, t), w);
#pragma unroll
                for (int t = 0; t < it; ++t) acc = fmaf(readlane_f(w, t), LC[t], acc);   // (w^T Li)_u
            } else {
                bc[lane] = g;
#pragma unroll
                for (int t = 0; t < it; ++t) w = fmaf(LR[t], bc[t], w);
                if (lane < 32) bc[32 + lane] = w;
#pragma unroll
                for (int t = 0; t < it; ++t) acc = fmaf(bc[32 + t], LC[t], acc);   // (w^T Li)_u
            }
            wsum = lanes_sum<NL>(w * w);
        }
        const float l2 = gjj - wsum;
        if (!(l2 > 1e-9f * gjj)) {   // numerically dependent on the selected atoms
            active = false;
            continue;
        }
        const float il = __builtin_amdgcn_rsqf(l2);   // 1 / L_jj
        const float cj = aj * il;
        rr = readfirstlane_f(fmaf(-cj, cj, rr));
        l2max = max(l2max, __float_as_uint(l2));
        l2min = min(l2min, __float_as_uint(l2));
        const float nu = lane_t == it ? il : -il * acc;   // lane u: Li[it][u] (zero past lane it)
        if (it > 0 && it <= kLaneBcast) {
            // nu made opaque first: in the select below the compiler would
            // otherwise read nu's definition under lane == it (nu = il there)
            // into the lane reads of the other lanes
            float nu_o = nu;
            asm volatile("" : "+v"(nu_o));
#pragma unroll
            for (int u = 0; u < it; ++u) {
                const float nv = readlane_f(nu_o, u);
                LR[u] = lane_t == it ? nv : LR[u];
            }
        } else if (it > 0) {
            bc[lane] = nu;
#pragma unroll
            for (int u = 0; u < it; ++u) LR[u] = lane_t == it ? bc[u] : LR[u];
        }
        LR[it] = lane_t == it ? il : 0.f;
        LC[it] = nu;
        gam = fmaf(cj, nu, gam);
        if (it + 1 > kLaneBcast) bc[lane] = gam;   // the next step reads gamma from the row
        selv = writelane_i(j, it, selv);
        n = it + 1;
    }

    // ---- coefficients, residual, outputs ----
    bool refit = false;
    if (n > 0 && p.fp64_refit) refit = __uint_as_float(l2max) > p.kappa_max * __uint_as_float(l2min);
    float re = 0.f;
    if (!refit) re = expl_done ? rr_expl : resid2(n);
    if (lane < k) {
        oidx[lane] = lane < n ? selv : -1;
        ocoef[lane] = lane < n ? gam : 0.f;
    }
    if (lane == 0) {
        *ocount = refit ? -(2 + n) : n;
        if (p.resid) p.resid[sig] = refit ? 0.f : __builtin_amdgcn_sqrtf(re);
    }
    tally.sig += 1;
    tally.atoms += n;
}

// Codes staged in LDS instead of written to p.idx / p.coef / p.count: slot
// s of the tile at idx[s k ..], coef[s k ..], cnt[s].
struct CodeStage {
    int32_t *idx;
    float *coef;
    int32_t *cnt;
};

// One tile of T signals: load, alpha0 by `mode` (A0_VALU or A0_MFMA_F32; or
// A0_MFMA_BF16X6 when kSplitOK and the LDS holds the split parts),
// then each wave encodes its signals (into `stage` when given).
template <int E, int KMAX, int T, bool kSplitOK, int RCQ, int NW = kOmpWaves>
__device__ __forceinline__ void omp_tile(const DictDev &dict, const OmpParams &p, int mode, int64_t s0, int nt,
                                         unsigned char *smem, int tid, OmpTally &tally,
                                         const CodeStage *stage = nullptr) {
    constexpr int Kp = 64 * E;
    float *A0 = reinterpret_cast<float *>(smem);
    float *Xt = A0 + T * a0_stride(Kp);
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: the signal loop below is per wave
    __syncthreads();   // the previous tile is done with Xt and A0
    load_tile<T, NW>(p, dict.d, s0, nt, Xt, tid);
    __syncthreads();
    bool done = false;
    if constexpr (MfmaF32Split<E, T, NW>::ok) {
        if (mode == A0_MFMA_F32) {
            alpha0_mfma_f32<E, T, NW>(dict.Dr, dict.dpad, Xt, A0, wave, lane);
            done = true;
        }
    }
    if constexpr (kSplitOK && MfmaF32Split<E, T, NW>::ok) {
        if (mode == A0_MFMA_BF16X6) {
            // signal parts [3][T][kXhs]: x = xh + xm + xl in BF16
            uint16_t *Xh = split_in_a0(T, Kp) ? reinterpret_cast<uint16_t *>(A0)
                                              : reinterpret_cast<uint16_t *>(Xt + 64 * xt_stride(T));
            for (int q = tid; q < T * 64; q += 64 * NW) {
                const int s = q >> 6, f = q & 63;
                const float v = Xt[f * xt_stride(T) + s];
                const uint16_t hi = bf16_bits(v);
                const float r1 = v - bf16_to_f32(hi);
                const uint16_t mid = bf16_bits(r1);
                Xh[s * kXhs + f] = hi;
                Xh[(T + s) * kXhs + f] = mid;
                Xh[(2 * T + s) * kXhs + f] = bf16_bits(r1 - bf16_to_f32(mid));
            }
            __syncthreads();
            alpha0_mfma_bf16x6<E, T, NW>(dict.Dbf, dict.Dlo, dict.Dl2, Xh, A0, wave, lane);
            done = true;
        }
    }
    if (!done) alpha0_valu<E, T, NW>(dict.DT, dict.d, Xt, A0, tid);
    __syncthreads();
    for (int s = wave; s < nt; s += NW) {
        const int64_t sig = p.rows ? (int64_t)p.rows[s0 + s] : s0 + s;
        if (p.rows && (uint64_t)sig >= (uint64_t)p.N) continue;   // out-of-range list entry: skipped
        if (stage)
            omp_pursuit<E, KMAX, T, RCQ>(dict, p, sig, s, Xt, A0, lane, stage->idx + s * p.k, stage->coef + s * p.k,
                                         stage->cnt + s, tally);
        else
            omp_pursuit<E, KMAX, T, RCQ>(dict, p, sig, s, Xt, A0, lane, p.idx + sig * p.k, p.coef + sig * p.k,
                                         p.count + sig, tally);
    }
}

// ---------------------------------------------------------------------------
// FP64 refit of flagged supports
// ---------------------------------------------------------------------------

constexpr int kRefitMax = 32;

struct RefitScratch {
    int sel[kRefitMax];
    double z[kRefitMax];
    double Gd[kRefitMax * (kRefitMax + 1) / 2];   // lower triangle, row-packed
    float Di[kRefitMax * 64];                     // the selected atoms, row t at 64 t
    float xs[64];
};

__device__ __forceinline__ int tri(int t, int u) { return t * (t + 1) / 2 + u; }   // u <= t

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// G_II gamma = D_I^T x with G_II and D_I^T x summed in FP64 and solved by a
// Cholesky factorisation, all lane-parallel in LDS: G_II is gathered from the
// dictionary's FP64 Gram (row t by lanes u <= t), the selected atoms are
// staged once for D_I^T x and the residual, and each factorisation /
// substitution step updates its trailing entries in parallel.  The n atoms
// are read from sel_in, gamma is written to coef_out; returns the explicit
// ||x - D_I gamma||^2 (on every lane).
__device__ __forceinline__ double refit_codes(const DictDev &dict, const float *__restrict__ x,
                                              const int32_t *sel_in, float *coef_out, int n, RefitScratch &ws,
                                              int lane) {
    const int d = dict.d;
    const float *__restrict__ D = dict.D;
    if (lane < n) ws.sel[lane] = sel_in[lane];
    if (lane < d) ws.xs[lane] = x[lane];
    wave_lds_sync();
    for (int q = lane; q < n * d; q += 64) {
        const int t = q / d, i = q - t * d;
        ws.Di[t * 64 + i] = D[(size_t)ws.sel[t] * d + i];
    }
    wave_lds_sync();
    {
        const double *__restrict__ G64 = dict.G64;
        const size_t su = lane < n ? (size_t)ws.sel[lane] : 0;
#pragma unroll 4
        for (int t = 0; t < n; ++t)
            if (lane <= t) ws.Gd[tri(t, lane)] = G64[(size_t)ws.sel[t] * dict.K + su];
    }
    if (lane < n) {
        double s = 0.0;
        for (int i = 0; i < d; ++i) s += (double)ws.Di[lane * 64 + i] * (double)ws.xs[i];
        ws.z[lane] = s;
    }
    wave_lds_sync();
    double *Gd = ws.Gd, *z = ws.z;
    for (int j = 0; j < n; ++j) {   // right-looking: G = R R^T, R lower, in place
        const double v = Gd[tri(j, j)];
        const double rjj = sqrt(fmax(v, 1e-300));
        wave_lds_sync();
        if (lane == 0) Gd[tri(j, j)] = rjj;
        if (j + 1 + lane < n) Gd[tri(j + 1 + lane, j)] /= rjj;
        wave_lds_sync();
        const int m = n - j - 1;
        for (int q = lane; q < m * (m + 1) / 2; q += 64) {
            int a = (int)((sqrtf(8.f * (float)q + 1.f) - 1.f) * 0.5f);
            while (tri(a + 1, 0) <= q) ++a;
            while (tri(a, 0) > q) --a;
            const int i = j + 1 + a, c = j + 1 + (q - tri(a, 0));
            Gd[tri(i, c)] -= Gd[tri(i, j)] * Gd[tri(c, j)];
        }
        wave_lds_sync();
    }
    for (int t = 0; t < n; ++t) {   // R y = z
        const double yt = z[t] / Gd[tri(t, t)];
        wave_lds_sync();
        if (lane == 0) z[t] = yt;
        if (t + 1 + lane < n) z[t + 1 + lane] -= Gd[tri(t + 1 + lane, t)] * yt;
        wave_lds_sync();
    }
    for (int t = n - 1; t >= 0; --t) {   // R^T gamma = y
        const double gt = z[t] / Gd[tri(t, t)];
        wave_lds_sync();
        if (lane == 0) z[t] = gt;
        if (lane < t) z[lane] -= Gd[tri(t, lane)] * gt;
        wave_lds_sync();
    }
    double r = 0.0;
    if (lane < d) {
        r = (double)ws.xs[lane];
        for (int t = 0; t < n; ++t) r -= z[t] * (double)ws.Di[t * 64 + lane];
    }
    const double r2 = wave_sum_d(lane < d ? r * r : 0.0);
    if (lane < n) coef_out[lane] = (float)z[lane];
    __builtin_amdgcn_wave_barrier();
    return r2;
}

// FP64 refit of a flagged padded code: gamma, the explicit residual and count = n.
__device__ __forceinline__ void refit_one(const DictDev &dict, const OmpParams &p, int64_t sig, int n,
                                          RefitScratch &ws, int lane) {
    const double r2 = refit_codes(dict, p.X + sig * dict.d, p.idx + sig * p.k, p.coef + sig * p.k, n, ws, lane);
    if (lane == 0) {
        p.count[sig] = n;
        if (p.resid) p.resid[sig] = (float)sqrt(r2);
    }
}

// Scans the call's signals in chunks of 64 (wave `gw` of `nw` waves) and
// refits those flagged with count = -(2 + n).  Returns the number refit.
__device__ __forceinline__ unsigned long long refit_scan(const DictDev &dict, const OmpParams &p, int64_t gw,
                                                         int64_t nw, RefitScratch &ws, int lane) {
    int64_t Nsig = p.N;
    if (p.rows) Nsig = min<int64_t>(Nsig, (int64_t)*p.nrows);
    const int64_t nchunks = (Nsig + 63) / 64;
    unsigned long long nref = 0;
    for (int64_t c = gw; c < nchunks; c += nw) {
        const int64_t i = c * 64 + lane;
        int64_t sig = 0;
        int cnt = 0;
        if (i < Nsig) {
            sig = p.rows ? (int64_t)p.rows[i] : i;
            if ((uint64_t)sig < (uint64_t)p.N) cnt = p.count[sig];   // out-of-range list entries are skipped
        }
        uint64_t flagged = ballot(cnt < -1);
        while (flagged) {
            const int l = __ffsll((unsigned long long)flagged) - 1;
            flagged &= flagged - 1;
            const int lo = __builtin_amdgcn_readlane((int)(sig & 0xFFFFFFFF), l);
            const int hi = __builtin_amdgcn_readlane((int)(sig >> 32), l);
            const int64_t sg = (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
            const int nn = -__builtin_amdgcn_readlane(cnt, l) - 2;
            refit_one(dict, p, sg, nn, ws, lane);
            nref += 1;
        }
    }
    return nref;
}

}  // namespace sc
