// Learned support proposer, inference: a 3-layer MLP d -> 256 -> 256 -> K
// (GELU, BF16 weights and activations, FP32 accumulation on MFMA) fused with
// the exact selection of each signal's n_cand largest logits.
//
// Workgroup = 8 waves, tile = 64 signals.  The layers are computed as
// Z^T = W H^T with v_mfma_f32_32x32x16_bf16: the A operand is a 32 x 16 block
// of the weight matrix read from global memory (L2-resident), the B operand
// comes from the activation tile in LDS.  Each wave owns whole 32-row blocks
// of W for both 32-signal halves of the tile, so every weight is read once
// per tile.  The weights are stored in MFMA operand order (the 64 lanes' 16-byte
// pieces of one block and k-step are 1 KB contiguous), so an A-operand read is
// eight whole cache lines instead of 32 partial ones, and the A operands are
// kept 8 (layers 1-2) or 3 (layer 3) k-steps ahead, the B operands one.  In the
// MFMA output layout a lane holds 16 outputs of one signal per block, so the
// selection needs no transpose:
//   1. each lane takes maxima of groups of K/64 of its logits: 64 group
//      maxima per signal;
//   2. theta = the n_cand-th largest group maximum (eight lanes per signal,
//      bitwise search with group-summed counts) is a safe lower bound of the
//      n_cand-th largest logit, since n_cand groups reach it;
//   3. each writer lane appends its logits >= theta to a private slot list,
//      as keys that order like the logit with the atom index in the low bits
//      (unique keys, lower index wins a tie) -- about n_cand + 5 survivors;
//   4. eight lanes per signal (eight signals per wave at once) pack the
//      survivors into a dense list and keep each survivor that fewer than
//      n_cand others exceed (when some signal of the wave has more than 64
//      survivors: delete the smallest until n_cand remain), mark the chosen
//      atoms in a bit mask and write them in increasing atom index.
// A signal whose slot lists overflow (many logits tied at the threshold) or
// whose input is not finite gets candidate list {-1, ...}: the encoder then
// sends it straight to the full-OMP fallback.  Keys keep the top 32 - IB bits
// of the order-preserving FP32 key (IB = 7, 8, 9 index bits for K = 128, 256,
// 512), so logits closer than ~2^(IB-23) relative count as ties.
#include "mfma.h"
#include "sc_internal.h"
#include "wave.h"

namespace sc {

constexpr int kPT = 64;        // signals per tile
constexpr int kPWaves = 8;
constexpr int kPThreads = 64 * kPWaves;
constexpr int kPH = 256;       // hidden width
constexpr int kXS = 72;        // LDS row stride (bf16) of the input tile
constexpr int kHS = 264;       // LDS row stride (bf16) of a hidden tile
constexpr int kNG = 64;        // group maxima per signal
constexpr int kRankPer = 8;    // survivors ranked per selection lane (rank path: <= 64 per signal)
constexpr int kThetaLowBit = 17;   // lowest key bit the threshold search resolves
constexpr int kPFHidden = 8;       // A-operand k-steps in flight, hidden layers
constexpr int kPFOut = 3;          // A-operand k-steps in flight, output layer

constexpr int kXBytes = kPT * kXS * 2;        //  9216
constexpr int kHBytes = kPT * kHS * 2;        // 33792
constexpr int kPropLds = kXBytes + 2 * kHBytes + kPT * 4;

// Sum over the 8 lanes of a group (lanes 8q .. 8q+7).
__device__ __forceinline__ int grp8_sum(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, SC_DPP_QP1032, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, SC_DPP_QP2301, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, SC_DPP_HMIRROR, 0xF, 0xF, false);
    return v;
}

__device__ __forceinline__ uint32_t grp8_min(uint32_t v) {
    v = min(v, dpp_u<SC_DPP_QP1032>(v));
    v = min(v, dpp_u<SC_DPP_QP2301>(v));
    v = min(v, dpp_u<SC_DPP_HMIRROR>(v));
    return v;
}

__device__ __forceinline__ uint32_t grp8_max(uint32_t v) {
    v = max(v, dpp_u<SC_DPP_QP1032>(v));
    v = max(v, dpp_u<SC_DPP_QP2301>(v));
    v = max(v, dpp_u<SC_DPP_HMIRROR>(v));
    return v;
}

// A operand of 32-row block mb, k-step s, for this lane, from a weight matrix
// of ldw columns stored in MFMA operand order: block-major, then k-step, then
// the 64 lanes' 8 consecutive BF16 values (row 32 mb + lane % 32, columns
// 16 s + 8 (lane / 32) .. + 7).
__device__ __forceinline__ bf16x8 ld_a_op(const uint16_t *W, int ldw, int mb, int s, int lane) {
    return ld_bf16x8(W + (((size_t)mb * (ldw / 16) + s) * 64 + lane) * 8);
}

// One hidden layer for the 64-signal tile: Hout = GELU(W Hin^T + b)^T (BF16),
// 256 outputs.  Wave w computes the 32-neuron block w for both signal halves.
// Each k-step group (next B operands, two MFMAs, the A operand kPFHidden
// steps ahead) is fenced from the scheduler, which otherwise sinks the loads
// to their first use.
template <int KS>
__device__ __forceinline__ void dense_layer(const uint16_t *__restrict__ W, int ldw,
                                            const float *__restrict__ bias, const uint16_t *__restrict__ Hin, int ldh,
                                            uint16_t *__restrict__ Hout, int wave, int lane) {
    const int lr = lane & 31, lk = 8 * (lane >> 5);
    constexpr int PF = KS < kPFHidden ? KS : kPFHidden;
    bf16x8 a[PF];
#pragma unroll
    for (int s = 0; s < PF; ++s) a[s] = ld_a_op(W, ldw, wave, s, lane);
    bf16x8 b[2][2];
#pragma unroll
    for (int n = 0; n < 2; ++n) b[0][n] = ld_bf16x8(Hin + (32 * n + lr) * ldh + lk);
    // the accumulators start from the bias (both signal halves)
    floatx16 acc[2];
    {
        floatx16 bacc;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const float4 bb = *reinterpret_cast<const float4 *>(bias + 32 * wave + 8 * g + 4 * (lane >> 5));
            bacc[4 * g] = bb.x, bacc[4 * g + 1] = bb.y, bacc[4 * g + 2] = bb.z, bacc[4 * g + 3] = bb.w;
        }
        acc[0] = bacc;
        acc[1] = bacc;
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        if (s + 1 < KS) {
#pragma unroll
            for (int n = 0; n < 2; ++n) b[(s + 1) & 1][n] = ld_bf16x8(Hin + (32 * n + lr) * ldh + 16 * (s + 1) + lk);
        }
#pragma unroll
        for (int n = 0; n < 2; ++n) acc[n] = mfma32(a[s % PF], b[s & 1][n], acc[n]);
        if (s + PF < KS) a[s % PF] = ld_a_op(W, ldw, wave, s + PF, lane);
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int n = 0; n < 2; ++n) {
        const int j = 32 * n + lr;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int i0 = 32 * wave + 8 * g + 4 * (lane >> 5);
            uint2 pk;
            pk.x = bf16_pack2(gelu_f(acc[n][4 * g + 0]), gelu_f(acc[n][4 * g + 1]));
            pk.y = bf16_pack2(gelu_f(acc[n][4 * g + 2]), gelu_f(acc[n][4 * g + 3]));
            *reinterpret_cast<uint2 *>(Hout + j * kHS + i0) = pk;
        }
    }
}

// SCREEN: correlation screening instead of the MLP -- the "logits" are
// |D^T x / ||x|||| from one BF16 MFMA layer with W3 = bf16(D) (K x 64).
template <int KT, bool SCREEN>
__global__ __launch_bounds__(kPThreads) __attribute__((amdgpu_waves_per_eu(4))) void proposer_topk_kernel(
    PropDev P, const float *__restrict__ X, int64_t N, int n_cand, int32_t *__restrict__ cand,
    float *__restrict__ logits) {
    constexpr int K = 128 * KT;                 // outputs (= dictionary atoms)
    constexpr int MT3 = 4 * KT;                 // 32-row blocks of W3
    constexpr int NPW = MT3 >= kPWaves ? 2 : 1; // signal halves per wave in layer 3
    constexpr int MPW = MT3 >= kPWaves ? MT3 / kPWaves : 1;   // W3 blocks per wave
    constexpr int NWR = MT3 >= kPWaves ? 16 : 8;              // writer lanes per signal
    constexpr int GS = K / kNG;                 // logits per group maximum
    constexpr int VL = 16 * MPW;                // logits per lane and signal
    constexpr int IB = KT == 1 ? 7 : (KT == 2 ? 8 : 9);   // index bits in a key
    constexpr uint32_t IMASK = (1u << IB) - 1u;
    constexpr int MW = K / 32;                  // mask words per signal
    constexpr int WPL = NWR / 8;                // writers handled per selection lane
    constexpr int kSlots = VL < 16 ? VL : 16;   // candidate slots per writer lane and signal
    // per-signal strides of the group maxima and of the slot regions: 4 words
    // past a multiple of 64, so rows of consecutive signals start on different
    // bank groups (the lanes of a wave touch up to 32 signals at once)
    constexpr int kGS = kNG + 4;
    constexpr int kSS = NWR * kSlots + 4;
                                                // (= VL for K <= 256: no overflow possible)
    extern __shared__ __align__(16) unsigned char lds[];
    uint16_t *Xh = reinterpret_cast<uint16_t *>(lds);
    uint16_t *H1 = reinterpret_cast<uint16_t *>(lds + kXBytes);
    uint16_t *H2 = reinterpret_cast<uint16_t *>(lds + kXBytes + kHBytes);
    int *bad = reinterpret_cast<int *>(lds + kXBytes + 2 * kHBytes);
    // reused once layer 3 is done (Xh, H1 and H2 are dead then); the group
    // maxima are dead once theta is known, so the slots overlay them
    uint32_t *theta = reinterpret_cast<uint32_t *>(lds);                       // [64] threshold keys
    uint32_t *mask = theta + kPT;                                               // [64][MW]
    uint8_t *wcnt = reinterpret_cast<uint8_t *>(mask + kPT * MW);              // [64][NWR]
    float *gmax = reinterpret_cast<float *>(wcnt + kPT * NWR);                 // [64][kGS]
    uint32_t *slots = reinterpret_cast<uint32_t *>(gmax);                      // [64][kSS]: [NWR][kSlots] + pad
    static_assert(kPT * 4 + kPT * MW * 4 + kPT * NWR + (kGS > kSS ? kGS : kSS) * kPT * 4 <= kPropLds &&
                      (kPT * 4 + kPT * MW * 4 + kPT * NWR) % 16 == 0,
                  "selection scratch must fit in the tile's LDS");

    const int d = P.d;
    const int64_t ntiles = (N + kPT - 1) / kPT;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        // lane-derived addresses are recomputed per tile (cheap) rather than
        // kept live across the whole loop, which would spill
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
        const int lr = lane & 31, lk = 8 * (lane >> 5);
        const int64_t s0 = tile * kPT;
        const int nt_sig = (int)min<int64_t>(kPT, N - s0);
        __syncthreads();
        // ---- input tile: x / ||x|| in BF16, zero padded to 64 features ----
        {
            const int s = tid >> 3, q = tid & 7;
            float xv[8];
            float ss = 0.f;
            bool fin = true;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const int f = q + 8 * m;
                float v = 0.f;
                if (s < nt_sig && f < d) v = X[(s0 + s) * d + f];
                fin &= isfinite(v);
                xv[m] = v;
                ss = fmaf(v, v, ss);
            }
            ss += dpp_f<SC_DPP_QP1032>(ss);
            ss += dpp_f<SC_DPP_QP2301>(ss);
            ss += dpp_f<SC_DPP_HMIRROR>(ss);
            int nf = fin ? 0 : 1;
            nf |= __builtin_amdgcn_update_dpp(0, nf, SC_DPP_QP1032, 0xF, 0xF, false);
            nf |= __builtin_amdgcn_update_dpp(0, nf, SC_DPP_QP2301, 0xF, 0xF, false);
            nf |= __builtin_amdgcn_update_dpp(0, nf, SC_DPP_HMIRROR, 0xF, 0xF, false);
            const float nrm = sqrtf(ss);
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const int f = q + 8 * m;
                const float v = (nrm > 0.f && !nf) ? xv[m] / nrm : 0.f;
                Xh[s * kXS + f] = bf16_bits(v);
            }
            if (q == 0) bad[s] = (s >= nt_sig) || nf;
        }
        __syncthreads();
        if constexpr (!SCREEN) {
            dense_layer<4>(P.W1b, 64, P.b1, Xh, kXS, H1, wave, lane);
            __syncthreads();
            dense_layer<16>(P.W2b, kPH, P.b2, H1, kHS, H2, wave, lane);
            __syncthreads();
        }
        // layer-3 input: the second hidden tile, or the signal tile when screening
        constexpr int KIN = SCREEN ? 64 : kPH;
        const uint16_t *Hin = SCREEN ? Xh : H2;
        constexpr int LDH = SCREEN ? kXS : kHS;
        // ---- layer 3: logits; wave owns W3 blocks mb(q) for NPW signal halves ----
        auto mblk = [&](int q) { return MT3 >= kPWaves ? wave + kPWaves * q : (wave & (MT3 - 1)); };
        const int n0 = MT3 >= kPWaves ? 0 : wave / MT3;   // first signal half of the wave
        floatx16 acc[MPW][NPW];
#pragma unroll
        for (int q = 0; q < MPW; ++q) {   // the MLP's accumulators start from the bias
            floatx16 bacc = floatx16{};
            if constexpr (!SCREEN) {
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const float4 bb = *reinterpret_cast<const float4 *>(P.b3 + 32 * mblk(q) + 8 * g + 4 * (lane >> 5));
                    bacc[4 * g] = bb.x, bacc[4 * g + 1] = bb.y, bacc[4 * g + 2] = bb.z, bacc[4 * g + 3] = bb.w;
                }
            }
#pragma unroll
            for (int n = 0; n < NPW; ++n) acc[q][n] = bacc;
        }
        {
            constexpr int PF = kPFOut;
            bf16x8 a[PF][MPW];
#pragma unroll
            for (int s = 0; s < PF; ++s)
#pragma unroll
                for (int q = 0; q < MPW; ++q) a[s][q] = ld_a_op(P.W3b, KIN, mblk(q), s, lane);
            bf16x8 b[2][NPW];
#pragma unroll
            for (int n = 0; n < NPW; ++n) b[0][n] = ld_bf16x8(Hin + (32 * (n0 + n) + lr) * LDH + lk);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int s = 0; s < KIN / 16; ++s) {
                if (s + 1 < KIN / 16) {
#pragma unroll
                    for (int n = 0; n < NPW; ++n)
                        b[(s + 1) & 1][n] = ld_bf16x8(Hin + (32 * (n0 + n) + lr) * LDH + 16 * (s + 1) + lk);
                }
#pragma unroll
                for (int n = 0; n < NPW; ++n)
#pragma unroll
                    for (int q = 0; q < MPW; ++q) acc[q][n] = mfma32(a[s % PF][q], b[s & 1][n], acc[q][n]);
                if (s + PF < KIN / 16) {
#pragma unroll
                    for (int q = 0; q < MPW; ++q) a[s % PF][q] = ld_a_op(P.W3b, KIN, mblk(q), s + PF, lane);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        __syncthreads();   // every wave is done reading the layer-3 input before the scratch overlays it
        // writer index of this lane for its signals, and the signals
        const int wr = (MT3 >= kPWaves ? 2 * wave : 2 * (wave & (MT3 - 1))) + (lane >> 5);
        // optional logits, group maxima
#pragma unroll
        for (int n = 0; n < NPW; ++n) {
            const int j = 32 * (n0 + n) + lr;
#pragma unroll
            for (int q = 0; q < MPW; ++q) {
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int i0 = 32 * mblk(q) + 8 * g + 4 * (lane >> 5);
                    if constexpr (SCREEN) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) acc[q][n][4 * g + r] = fabsf(acc[q][n][4 * g + r]);
                    }
                    if (logits && j < nt_sig) {
                        float4 o = {acc[q][n][4 * g], acc[q][n][4 * g + 1], acc[q][n][4 * g + 2],
                                    acc[q][n][4 * g + 3]};
                        *reinterpret_cast<float4 *>(logits + (s0 + j) * K + i0) = o;
                    }
                }
            }
            // VL logits of signal j in this lane -> VL / GS group maxima
#pragma unroll
            for (int gg = 0; gg < VL / GS; ++gg) {
                float mx = -__builtin_inff();
#pragma unroll
                for (int r = 0; r < GS; ++r) mx = fmaxf(mx, acc[(gg * GS + r) / 16][n][(gg * GS + r) % 16]);
                gmax[j * kGS + wr * (VL / GS) + gg] = mx;
            }
        }
        __syncthreads();
        // ---- threshold: the n_cand-th largest of the 64 group maxima ----
        {
            const int g = lane & 7, s = 8 * wave + (lane >> 3);
            uint32_t gk[8];
            const float4 ga = *reinterpret_cast<const float4 *>(gmax + s * kGS + 8 * g);
            const float4 gb = *reinterpret_cast<const float4 *>(gmax + s * kGS + 8 * g + 4);
            gk[0] = order_key(ga.x), gk[1] = order_key(ga.y), gk[2] = order_key(ga.z), gk[3] = order_key(ga.w);
            gk[4] = order_key(gb.x), gk[5] = order_key(gb.y), gk[6] = order_key(gb.z), gk[7] = order_key(gb.w);
            uint32_t lo = gk[0], hi = gk[0];
#pragma unroll
            for (int m = 1; m < 8; ++m) {
                lo = min(lo, gk[m]);
                hi = max(hi, gk[m]);
            }
            lo = grp8_min(lo);
            hi = grp8_max(hi);
            // keys share the bits above the highest bit where lo and hi differ
            const int hb = lo == hi ? -1 : 31 - __clz(lo ^ hi);
            uint32_t tau = hb < 0 ? lo : (hb == 31 ? 0u : hi & ~((2u << hb) - 1u));
            const int hbw = (int)wave_max_u32((uint32_t)(hb + 1)) - 1;
            // largest tau with >= n_cand maxima at or above it, resolved down to
            // bit kThetaLowBit (the low mantissa bits left at zero only lower
            // tau by < 2^-6 relative: a still-safe bound, at most a few more
            // survivors, and fewer search steps)
            for (int bit = hbw; bit >= kThetaLowBit; --bit) {
                const uint32_t t2 = tau | (1u << bit);
                int c = 0;
#pragma unroll
                for (int m = 0; m < 8; ++m) c += gk[m] >= t2 ? 1 : 0;
                c = grp8_sum(c);
                tau = c >= n_cand ? t2 : tau;
            }
            if (g == 0) theta[s] = bad[s] ? 0xFFFFFFFFu : tau;
        }
        __syncthreads();
        // ---- candidates above the threshold, into private slots ----
#pragma unroll
        for (int n = 0; n < NPW; ++n) {
            const int j = 32 * (n0 + n) + lr;
            const uint32_t thk = theta[j];
            uint32_t *myslots = slots + j * kSS + wr * kSlots;
            int cnt = 0;
#pragma unroll
            for (int q = 0; q < MPW; ++q)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const uint32_t zk = order_key(acc[q][n][r]);
                    if (zk >= thk) {
                        const int i = 32 * mblk(q) + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                        if (cnt < kSlots) myslots[cnt] = (zk & ~IMASK) | (IMASK - (uint32_t)i);
                        ++cnt;
                    }
                }
            wcnt[j * NWR + wr] = (uint8_t)min(cnt, 255);
        }
        __syncthreads();
        // ---- exact top-n_cand: 8 lanes per signal, 8 signals per wave ----
        {
            const int g = lane & 7, s = 8 * wave + (lane >> 3);
            int over = 0, have = 0, cw[WPL];
            uint32_t lim[WPL];   // wave-wide bound on the filled slots of writer block w
#pragma unroll
            for (int w = 0; w < WPL; ++w) {
                const int c = wcnt[s * NWR + g + 8 * w];
                cw[w] = min(c, kSlots);
                over |= c > kSlots;
                have += cw[w];
                lim[w] = wave_max_u32((uint32_t)cw[w]);
            }
            over = grp8_sum(over);
            have = grp8_sum(have);
            const bool skip = s >= nt_sig || bad[s] || over || have < n_cand;
            uint32_t *mw = mask + s * MW;
            for (int w = g; w < MW; w += 8) mw[w] = 0u;
            const int hv = skip ? 0 : have;
            const uint32_t maxS = wave_max_u32((uint32_t)hv);
            if (maxS <= 8 * kRankPer) {
                // Rank selection: the signal's survivors are packed into a dense
                // list (its own slot region), and a survivor is kept iff fewer
                // than n_cand survivors exceed it (keys are unique).  The work is
                // survivors^2 / 8 compares per lane, whatever the excess.
                int m = 0;
#pragma unroll
                for (int w = 0; w < WPL; ++w) m += cw[w];
                int base = m;   // exclusive prefix of m over the 8 lanes of the group
#pragma unroll
                for (int sh = 1; sh < 8; sh <<= 1) {
                    const int t = __shfl_up(base, sh, 8);
                    if (g >= sh) base += t;
                }
                base -= m;
                uint32_t *lst = slots + s * kSS;
                // one writer block per phase: every lane reads its block's keys,
                // then writes them packed; all destinations lie below 64, under
                // the second block's sources (writers 8..15 start at 8 kSlots)
                int j = base;
#pragma unroll
                for (int w = 0; w < WPL; ++w) {
                    uint32_t kk[kSlots];
                    const uint32_t *src = slots + s * kSS + (g + 8 * w) * kSlots;
#pragma unroll
                    for (int e = 0; e < kSlots; ++e) kk[e] = ((uint32_t)e < lim[w] && e < cw[w]) ? src[e] : 0u;
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
                    for (int e = 0; e < kSlots; ++e)
                        if ((uint32_t)e < lim[w] && e < cw[w]) lst[j++] = kk[e];
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                }
                // the list is zero-filled up to a multiple of 16 entries (0 is
                // below every key, so no entry bound is needed); each lane ranks
                // its own survivors g, g + 8, ... against the whole list, 16
                // entries (four 16-byte reads in flight) at a time
                const int nrnd = (int)((maxS + 15u) & ~15u);
                for (int u = hv + g; u < nrnd; u += 8) lst[u] = 0u;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                uint32_t v[kRankPer];
                int r[kRankPer];
#pragma unroll
                for (int i = 0; i < kRankPer; ++i) {
                    const int q = g + 8 * i;
                    v[i] = ((uint32_t)(8 * i) < maxS && q < hv) ? lst[q] : 0u;
                    r[i] = 0;
                }
                for (int u0 = 0; u0 < nrnd; u0 += 16) {
                    uint4 x[4];
#pragma unroll
                    for (int c = 0; c < 4; ++c) x[c] = *reinterpret_cast<const uint4 *>(lst + u0 + 4 * c);
#pragma unroll
                    for (int i = 0; i < kRankPer; ++i) {
                        if ((uint32_t)(8 * i) < maxS) {
#pragma unroll
                            for (int c = 0; c < 4; ++c)
                                r[i] += (x[c].x > v[i] ? 1 : 0) + (x[c].y > v[i] ? 1 : 0) + (x[c].z > v[i] ? 1 : 0) +
                                        (x[c].w > v[i] ? 1 : 0);
                        }
                    }
                }
#pragma unroll
                for (int i = 0; i < kRankPer; ++i) {
                    const int q = g + 8 * i;
                    if ((uint32_t)(8 * i) < maxS && q < hv && r[i] < n_cand) {
                        const uint32_t at = IMASK - (v[i] & IMASK);
                        atomicOr(&mw[at >> 5], 1u << (at & 31));
                    }
                }
            } else {
                // many survivors somewhere in the wave: delete the smallest
                // until n_cand remain (an empty slot holds 0, i.e. ~0 after the
                // shift below)
                uint32_t key[WPL * kSlots];
#pragma unroll
                for (int w = 0; w < WPL; ++w)
#pragma unroll
                    for (int e = 0; e < kSlots; ++e)
                        key[w * kSlots + e] = e < cw[w] ? slots[s * kSS + (g + 8 * w) * kSlots + e] : 0u;
                int excess = skip ? 0 : have - n_cand;
                while (__ballot(excess > 0) != 0) {
                    uint32_t mn = 0xFFFFFFFFu;
#pragma unroll
                    for (int w = 0; w < WPL; ++w)
#pragma unroll
                        for (int e = 0; e < kSlots; ++e)
                            if ((uint32_t)e < lim[w]) mn = min(mn, key[w * kSlots + e] - 1u);
                    mn = grp8_min(mn);
                    if (excess > 0) {
#pragma unroll
                        for (int w = 0; w < WPL; ++w)
#pragma unroll
                            for (int e = 0; e < kSlots; ++e)
                                if ((uint32_t)e < lim[w] && key[w * kSlots + e] - 1u == mn) key[w * kSlots + e] = 0u;
                        --excess;
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                if (!skip) {
#pragma unroll
                    for (int e = 0; e < WPL * kSlots; ++e)
                        if (key[e] != 0u) {
                            const uint32_t i = IMASK - (key[e] & IMASK);
                            atomicOr(&mw[i >> 5], 1u << (i & 31));
                        }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (s < nt_sig) {
                int32_t *out = cand + (s0 + s) * n_cand;
                if (skip) {
                    for (int t = g; t < n_cand; t += 8) out[t] = -1;
                } else {
                    for (int w = g; w < MW; w += 8) {
                        int pos = 0;
                        for (int v = 0; v < w; ++v) pos += __popc(mw[v]);
                        uint32_t word = mw[w];
                        while (word) {
                            const int bpos = __ffs(word) - 1;
                            out[pos++] = 32 * w + bpos;
                            word &= word - 1u;
                        }
                    }
                }
            }
        }
    }
}

// FP32 master parameters -> BF16 copies: row-major W1 (padded to 64 inputs),
// W2, W3 and transposed W2, W3 for the training products (their reduction
// index is then contiguous), and W1, W2, W3 in MFMA operand order for the
// inference kernel.
__global__ void proposer_pack_kernel(const float *__restrict__ params, int d, int H, int K, uint16_t *__restrict__ W1b,
                                     uint16_t *__restrict__ W2b, uint16_t *__restrict__ W3b,
                                     uint16_t *__restrict__ W2bT, uint16_t *__restrict__ W3bT,
                                     uint16_t *__restrict__ W1o, uint16_t *__restrict__ W2o,
                                     uint16_t *__restrict__ W3o) {
    const int64_t n1 = (int64_t)H * 64, n2 = (int64_t)H * H, n3 = (int64_t)K * H;
    const float *W1 = params;
    const float *W2 = W1 + (size_t)H * d + H;
    const float *W3 = W2 + (size_t)H * H + H;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n1 + 2 * (n2 + n3);
         t += (int64_t)gridDim.x * blockDim.x) {
        if (t < n1) {
            const int i = (int)(t / 64), f = (int)(t % 64);
            const uint16_t v = bf16_bits(f < d ? W1[(size_t)i * d + f] : 0.f);
            W1b[t] = v;
            W1o[op_order_index(i, f, 64)] = v;
        } else if (t < n1 + n2) {
            const int64_t q = t - n1;
            const uint16_t v = bf16_bits(W2[q]);
            W2b[q] = v;
            W2o[op_order_index((int)(q / H), (int)(q % H), H)] = v;
        } else if (t < n1 + n2 + n3) {
            const int64_t q = t - n1 - n2;
            const uint16_t v = bf16_bits(W3[q]);
            W3b[q] = v;
            W3o[op_order_index((int)(q / H), (int)(q % H), H)] = v;
        } else if (t < n1 + 2 * n2 + n3) {
            const int64_t q = t - n1 - n2 - n3;   // W2bT[j][i] = W2[i][j]
            const int64_t j = q / H, i = q - j * H;
            if (W2bT) W2bT[q] = bf16_bits(W2[i * H + j]);
        } else {
            const int64_t q = t - n1 - 2 * n2 - n3;   // W3bT[j][i] = W3[i][j], i < K, j < H
            const int64_t j = q / K, i = q - j * K;
            if (W3bT) W3bT[q] = bf16_bits(W3[i * H + j]);
        }
    }
}

hipError_t launch_proposer_pack(const float *params, int d, int H, int K, uint16_t *W1b, uint16_t *W2b,
                                uint16_t *W3b, uint16_t *W2bT, uint16_t *W3bT, uint16_t *W1o, uint16_t *W2o,
                                uint16_t *W3o, hipStream_t st) {
    if (H % 32 != 0 || K % 32 != 0) return hipErrorInvalidValue;
    proposer_pack_kernel<<<1024, 256, 0, st>>>(params, d, H, K, W1b, W2b, W3b, W2bT, W3bT, W1o, W2o, W3o);
    return hipGetLastError();
}

template <int KT, bool SCREEN>
static hipError_t launch_topk_t(const PropDev &P, const float *X, int64_t N, int n_cand, int32_t *cand,
                                float *logits, hipStream_t st) {
    auto kern = proposer_topk_kernel<KT, SCREEN>;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, kPropLds);
        if (e != hipSuccess) return e;
        attr = true;
    }
    int dev = 0, ncu = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t ntiles = (N + kPT - 1) / kPT;
    const int64_t grid = std::min<int64_t>(ntiles, (int64_t)ncu * 2);   // two 77 KB tiles per CU
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(kPThreads), kPropLds, st, P, X, N, n_cand, cand, logits);
    return hipGetLastError();
}

hipError_t launch_proposer_topk(const PropDev &P, const float *X, int64_t N, int n_cand, int32_t *cand,
                                float *logits, hipStream_t st) {
    if (P.H != kPH || P.d > 64 || n_cand < 1 || n_cand > kNG) return hipErrorInvalidValue;
    switch (P.K) {
        case 128: return launch_topk_t<1, false>(P, X, N, n_cand, cand, logits, st);
        case 256: return launch_topk_t<2, false>(P, X, N, n_cand, cand, logits, st);
        case 512: return launch_topk_t<4, false>(P, X, N, n_cand, cand, logits, st);
        default: return hipErrorInvalidValue;
    }
}

// Correlation screening: the n_cand atoms of largest |<a_j, x>| by one BF16
// MFMA product with the dictionary's BF16 copy in MFMA operand order (Kp x 64,
// features padded).
hipError_t launch_screen_topk(const uint16_t *Dbfo, int d, int K, const float *X, int64_t N, int n_cand,
                              int32_t *cand, hipStream_t st) {
    if (d > 64 || n_cand < 1 || n_cand > kNG) return hipErrorInvalidValue;
    PropDev P{d, kPH, K, nullptr, nullptr, nullptr, nullptr, Dbfo, nullptr};
    switch (K) {
        case 128: return launch_topk_t<1, true>(P, X, N, n_cand, cand, nullptr, st);
        case 256: return launch_topk_t<2, true>(P, X, N, n_cand, cand, nullptr, st);
        case 512: return launch_topk_t<4, true>(P, X, N, n_cand, cand, nullptr, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace sc
