// Internal declarations shared by the host entry points and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sc.h"

namespace sc {

// Entries of the correlation vector held per lane by the one-wave-per-signal
// encoders: the dictionary is padded to Kp = 64 * E atoms.
constexpr int kEChoices[] = {1, 2, 4, 8, 12, 16};

inline int pick_E(int K) {
    for (int e : kEChoices)
        if (64 * e >= K) return e;
    return -1;
}

// Sparsity caps with a compiled kernel; k is rounded up to the next one.
constexpr int kKmaxChoices[] = {4, 8, 12, 16, 24, 32};

inline int pick_kmax(int k) {
    for (int c : kKmaxChoices)
        if (c >= k) return c;
    return -1;
}

// Rows of the feature-major dictionary DT: d rounded up to 4, plus one
// further k-step of 4 zero rows (the correlation stage reads a k-step ahead).
inline int dt_rows(int d) { return ((d + 3) & ~3) + 4; }

// Position of element (i, f) of a row-major matrix of C columns (C a multiple
// of 16, rows a multiple of 32) in MFMA operand order: the A operand of
// v_mfma_f32_32x32x16_bf16 for 32-row block i / 32 and k-step f / 16 is 64
// lanes x 8 consecutive values, lane = 32 ((f / 8) % 2) + i % 32.
__host__ __device__ inline size_t op_order_index(int i, int f, int C) {
    return ((((size_t)(i >> 5) * (C >> 4) + (f >> 4)) * 64 + 32 * ((f >> 3) & 1) + (i & 31)) << 3) + (f & 7);
}

// Position of element (atom a, feature f) of a Kp x dpad FP32 dictionary in
// the operand order of v_mfma_f32_16x16x4_f32 over 16-feature chunks: per
// 16-atom block a / 16 and chunk f / 16, 64 lanes x 4 floats, lane
// 16 ((f / 4) % 4) + a % 16 holding features 4 ((f / 4) % 4) .. + 3.
__host__ __device__ inline size_t op_order_f32(int a, int f, int dpad) {
    return ((((size_t)(a >> 4) * (dpad >> 4) + (f >> 4)) * 64 + 16 * ((f >> 2) & 3) + (a & 15)) << 2) + (f & 3);
}

// Position of element (atom a, feature f < 64) of a Kp x 64 BF16 dictionary
// part in the operand order of v_mfma_f32_16x16x32_bf16: per 16-atom block
// a / 16 and 32-feature k-step f / 32, 64 lanes x 8 values, lane
// 16 ((f / 8) % 4) + a % 16 holding features 8 ((f / 8) % 4) .. + 7.
__host__ __device__ inline size_t op_order_bf16x32(int a, int f) {
    return ((((size_t)(a >> 4) * 2 + (f >> 5)) * 64 + 16 * ((f >> 3) & 3) + (a & 15)) << 3) + (f & 7);
}

struct DictDev {
    int d, K, Kp, E;
    const float *D;    // K x d atom-major FP32
    const float *DT;   // dt_rows(d) x Kp feature-major FP32, zero padded atoms and rows >= d
    const float *G;    // K x Kp FP32 Gram rows, zero padded columns
    // split-BF16 parts of D, Kp x 64 each in op_order_bf16x32, zero padded:
    const uint16_t *Dbf;  // bf16(D)
    const uint16_t *Dlo;  // bf16(D - Dbf)
    const uint16_t *Dl2;  // bf16(D - Dbf - Dlo)
    const float *D48;     // K x 48 FP32 atom-major, features zero padded (d <= 48)
    const double *G64;    // K x K Gram, exact products summed in FP64 (not rounded)
    const float *Dr;      // Kp x dpad FP32 in MFMA operand order (op_order_f32), zero padded
    int dpad;             // d rounded up to 16
};

// How the correlation tile alpha0 = D^T X is computed by the batch encoder.
enum { A0_VALU = 0, A0_MFMA_F32 = 1, A0_MFMA_BF16X6 = 2 };

struct OmpParams {
    const float *X;
    int64_t N;
    const int32_t *rows;    // optional: encode rows[0..*nrows) of X (a fallback list)
    const int32_t *nrows;   // device count of rows (read by the kernel)
    int k;
    float eps;
    int relative;
    int fp64_refit;
    float kappa_max;   // condition-estimate threshold for the FP64 refit
    int32_t *idx;
    float *coef;
    int32_t *count;
    float *resid;
    unsigned long long *stats;  // 4 counters (see sc_omp_stats)
};

struct RompParams {
    const float *X;
    int64_t N;
    int k;
    float eps;
    int relative;
    int fp64_refit;
    float kappa_max;
    int kcap;                 // at most kcap restricted steps (<= k); a signal still above eps is a miss
    const int32_t *cand;      // N x n_cand candidate atoms sorted by index; row {-1,...} = none
    int n_cand;
    int32_t *idx;
    float *coef;
    int32_t *count;
    float *resid;
    int32_t *miss_rows;       // signals whose restricted code misses eps are appended here
    int32_t *miss_count;
    unsigned long long *stats;
};

struct PropDev {
    int d, H, K;
    // The weight copies read by the inference kernel are in MFMA operand order
    // (op_order_index below): W1 H x 64 (inputs zero padded), W2 H x H, W3 K x H.
    const uint16_t *W1b;
    const float *b1;
    const uint16_t *W2b;
    const float *b2;
    const uint16_t *W3b;
    const float *b3;
};

// Launchers (return hipError_t of the launch).
hipError_t launch_dict_check(const float *D, int d, int K, int normalize, float *Dcopy, int *status,
                             hipStream_t st);
hipError_t launch_dict_layouts(const float *Dcopy, int d, int K, int Kp, float *DT, uint16_t *Dbf, uint16_t *Dlo,
                               uint16_t *Dl2, float *D48, float *Dr, int dpad, uint16_t *Dbfo, hipStream_t st);
hipError_t launch_gram(const float *Dcopy, int d, int K, int Kp, float *G, double *G64, hipStream_t st);
hipError_t launch_omp_batch(const DictDev &dict, const OmpParams &p, int kmax, int a0mode, int row_cache,
                            hipStream_t st);
hipError_t launch_omp_batch_valu(const DictDev &dict, const OmpParams &p, int kmax, int row_cache, hipStream_t st);
hipError_t launch_omp_batch_mfma(const DictDev &dict, const OmpParams &p, int kmax, int row_cache, hipStream_t st);
hipError_t launch_omp_batch_bf16(const DictDev &dict, const OmpParams &p, int kmax, int row_cache, hipStream_t st);
hipError_t launch_omp_refit(const DictDev &dict, const OmpParams &p, hipStream_t st);
// One-pass encoder into CSC (p.idx / p.coef / p.count unused); ws holds
// csc_encode_workspace_bytes(N) bytes whose first 256 bytes and descriptors
// are zero.
size_t csc_encode_workspace_bytes(int64_t N);
hipError_t launch_omp_csc(const DictDev &dict, const OmpParams &p, int kmax, int a0mode, int row_cache,
                          int64_t *colptr, int32_t *rows, float *vals, int64_t cap, void *ws, hipStream_t st);
hipError_t launch_omp_multi(const sc_scene *scenes, const int *order, int n, int a0mode, int tile, int row_cache,
                            int wg_per_cu, int *counter, hipStream_t st);
hipError_t launch_omp_restricted(const DictDev &dict, const float *D48, const RompParams &p, int kmax,
                                 hipStream_t st);
hipError_t launch_proposer_pack(const float *params, int d, int H, int K, uint16_t *W1b, uint16_t *W2b,
                                uint16_t *W3b, uint16_t *W2bT, uint16_t *W3bT, uint16_t *W1o, uint16_t *W2o,
                                uint16_t *W3o, hipStream_t st);
hipError_t launch_screen_topk(const uint16_t *Dbfo, int d, int K, const float *X, int64_t N, int n_cand,
                              int32_t *cand, hipStream_t st);
hipError_t launch_proposer_topk(const PropDev &P, const float *X, int64_t N, int n_cand, int32_t *cand,
                                float *logits, hipStream_t st);
enum { EPI_STORE = 0, EPI_GELU = 1, EPI_DGELU = 2 };  // GEMM epilogues (train.hip)

struct GemmArgs {
    int M, N, K;
    const void *A;
    int64_t sam, sak;      // A(i, k) = A[i * sam + k * sak]
    const void *B;
    int64_t sbk, sbn;      // B(k, j) = B[k * sbk + j * sbn]
    int epi;
    int Nvalid;            // columns >= Nvalid are not written
    const float *bias;     // [N] or NULL
    const float *aux;      // saved pre-activation for DGELU, row stride ldc
    float *Cf;             // FP32 output (row stride ldc) or NULL
    int64_t ldc;
    void *Ch;              // activation output (BF16 or FP32 by mode, row stride ldh) or NULL
    int64_t ldh;
    float *Cpre;           // GELU: pre-activation output (row stride ldc)
    float *part;           // split-K partial tiles (gemm_splits(M, N, K) * M * N floats) or NULL
};

// Number of K-slices of a STORE-epilogue product with few output tiles
// (weight gradients); 1 = no split.
// Zero nwords 32-bit words at p (a kernel, not hipMemsetAsync).
hipError_t launch_zero_words(void *p, int64_t nwords, hipStream_t st);

int gemm_splits(int M, int N, int K);
hipError_t launch_gemm(const GemmArgs &g, bool f32, hipStream_t st);
hipError_t launch_train_prep(const float *X, const int32_t *rows, int64_t B, int d, void *xh, bool f32,
                             hipStream_t st);
hipError_t launch_bce_grad(const float *Z, int64_t B, int K, const int32_t *rows, const int32_t *sup,
                           const int32_t *cnt, int kcap, float pos_weight, void *dz, float *loss, bool f32,
                           hipStream_t st);
hipError_t launch_colsum(const void *A, int64_t M, int N, int64_t ld, float *out, bool f32, hipStream_t st);
hipError_t launch_adam(float *p, float *m, float *v, const float *g, int64_t n, float lr_t, float beta1, float beta2,
                       float eps_hat, hipStream_t st);
size_t mod_workspace_bytes(int d, int K);
hipError_t launch_mod_update(const float *X, int64_t N, int d, int K, const int32_t *idx, const float *coef,
                             const int32_t *count, int k, const float *resid, float *Dout, int *n_replaced, void *ws,
                             hipStream_t st);
int64_t csc_workspace_blocks(int64_t N);
hipError_t launch_csc_colptr(const int32_t *count, int64_t N, int64_t *colptr, int64_t *bsum, hipStream_t st);
hipError_t launch_csc_fill(const int32_t *idx, const float *coef, const int32_t *count, int64_t N, int k,
                           const int64_t *colptr, int32_t *rows, float *vals, hipStream_t st);
hipError_t launch_csc_eval(const DictDev &dict, const int64_t *colptr, const int32_t *rows, const float *vals,
                           int64_t N, const float *dirs, int64_t M, int shared, const float *pos, const float *dc,
                           const float *cam, float *rgb, hipStream_t st);
hipError_t launch_sh_eval(const DictDev &dict, const int32_t *idx, const float *coef, const int32_t *count,
                          int64_t N, int k, const float *dirs, int64_t M, int shared, float *rgb,
                          hipStream_t st);

}  // namespace sc

struct sc_dict_s {
    sc::DictDev dev;
    int device;
    float *D = nullptr;
    float *DT = nullptr;
    float *G = nullptr;
    uint16_t *Dbf = nullptr;
    uint16_t *Dbfo = nullptr;   // Dbf in MFMA operand order (the screening product)
    uint16_t *Dlo = nullptr;
    uint16_t *Dl2 = nullptr;
    float *Dr = nullptr;    // Kp x dpad FP32 in MFMA operand order (op_order_f32)
    float *D48 = nullptr;   // K x 48 FP32, atoms padded to 16-byte rows
    double *G64 = nullptr;  // K x K FP64 Gram (the FP64 refit's entries)
    int *status = nullptr;
    unsigned long long *stats = nullptr;
    int a0_fp32 = sc::A0_VALU;       // alpha0 stage of the FP32 encoder (tunable)
    int row_cache = 0;               // Gram rows kept in registers by the encoder (tunable: 0 or 4)
    int row_cache_bf16 = 0;          // the same for the split-BF16 encoder
    sc::DictDev *ddev = nullptr;     // device copy of `dev`
    int restricted_cap = 0;          // restricted-OMP step cap of the learned encoder (0 = k; tunable)
};

struct sc_proposer_s {
    int d, H, K;
    int64_t nparams;
    float *params = nullptr;     // FP32 master: W1 (H x d), b1, W2 (H x H), b2, W3 (K x H), b3
    float *m = nullptr;          // Adam first moment
    float *v = nullptr;          // Adam second moment
    float *grads = nullptr;      // gradient buffer (same layout)
    uint16_t *W1b = nullptr, *W2b = nullptr, *W3b = nullptr;
    uint16_t *W2bT = nullptr, *W3bT = nullptr;   // transposed copies for the backward products
    uint16_t *W1o = nullptr, *W2o = nullptr, *W3o = nullptr;   // MFMA operand-order copies (inference)
    int64_t step = 0;
    sc::PropDev dev() const {
        const float *b1 = params + (size_t)H * d;
        const float *b2 = b1 + H + (size_t)H * H;
        const float *b3 = b2 + H + (size_t)K * H;
        return sc::PropDev{d, H, K, W1o, b1, W2o, b2, W3o, b3};
    }
};
