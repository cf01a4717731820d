// C-ABI entry points: argument validation, handle ownership, launches.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <utility>

#include "sc_internal.h"

namespace {

thread_local char g_last_error[512] = "";
constexpr float kKappaMax = 1e3f;   // Cholesky condition estimate above which supports are refit in FP64
constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int set_dev_error(const char *what, hipError_t e) {
    snprintf(g_last_error, sizeof(g_last_error), "%s: %s", what, hipGetErrorString(e));
    return SC_EDEVICE;
}

#define SC_HIP(call, what)                                  \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return set_dev_error(what, e_); \
    } while (0)

// Is the current device a gfx950?  (The kernels are built for it only.)
int check_device(int *dev) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
        snprintf(g_last_error, sizeof(g_last_error), "no HIP device");
        return SC_ENODEV;
    }
    if (hipGetDevice(dev) != hipSuccess) return SC_ENODEV;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, *dev) != hipSuccess) return SC_ENODEV;
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        snprintf(g_last_error, sizeof(g_last_error), "device %s is not gfx950", prop.gcnArchName);
        return SC_ENODEV;
    }
    return SC_OK;
}

void free_dict(sc_dict h) {
    if (!h) return;
    hipFree(h->D);
    hipFree(h->DT);
    hipFree(h->G);
    hipFree(h->Dbf);
    hipFree(h->Dbfo);
    hipFree(h->Dlo);
    hipFree(h->Dl2);
    hipFree(h->Dr);
    hipFree(h->D48);
    hipFree(h->G64);
    hipFree(h->status);
    hipFree(h->stats);
    hipFree(h->ddev);
    delete h;
}

// Row-cache setting of the encoder that `flags` selects (FP32 or split BF16).
int row_cache_for(const sc_dict_s *h, int flags) {
    return (flags & SC_PREC_BF16) ? h->row_cache_bf16 : h->row_cache;
}

}  // namespace

extern "C" {

const char *sc_strerror(int code) {
    switch (code) {
        case SC_OK: return "ok";
        case SC_EINVAL: return "invalid argument";
        case SC_ENORM: return "dictionary atom is not unit-norm";
        case SC_ENONFINITE: return "non-finite value in dictionary or weights";
        case SC_EDEVICE: return "HIP device error";
        case SC_ENOMEM: return "out of device memory or workspace too small";
        case SC_ENODEV: return "no usable gfx950 device";
        default: return "unknown error code";
    }
}

const char *sc_last_error(void) { return g_last_error; }

int sc_gram_precompute(const float *D, int d, int K, int flags, void *stream, sc_dict *out) {
    if (!D || !out || d < 1 || d > 64 || K < 1 || K > 1024) return SC_EINVAL;
    if (flags & ~SC_NORMALIZE) return SC_EINVAL;
    const int E = sc::pick_E(K);
    if (E < 0) return SC_EINVAL;
    int dev = 0;
    int rc = check_device(&dev);
    if (rc != SC_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    sc_dict h = new sc_dict_s();
    h->device = dev;
    const int Kp = 64 * E;
    const int dpad = (d + 15) / 16 * 16;
    bool ok = hipMalloc(&h->D, sizeof(float) * (size_t)K * d) == hipSuccess &&
              hipMalloc(&h->DT, sizeof(float) * (size_t)sc::dt_rows(d) * Kp) == hipSuccess &&
              hipMalloc(&h->G, sizeof(float) * (size_t)K * Kp) == hipSuccess &&
              hipMalloc(&h->Dbf, sizeof(uint16_t) * (size_t)Kp * 64) == hipSuccess &&
              hipMalloc(&h->Dbfo, sizeof(uint16_t) * (size_t)Kp * 64) == hipSuccess &&
              hipMalloc(&h->Dlo, sizeof(uint16_t) * (size_t)Kp * 64) == hipSuccess &&
              hipMalloc(&h->Dl2, sizeof(uint16_t) * (size_t)Kp * 64) == hipSuccess &&
              hipMalloc(&h->Dr, sizeof(float) * (size_t)Kp * dpad) == hipSuccess &&
              hipMalloc(&h->D48, sizeof(float) * (size_t)K * 48) == hipSuccess &&
              hipMalloc(&h->G64, sizeof(double) * (size_t)K * K) == hipSuccess &&
              hipMalloc(&h->status, sizeof(int) * 4) == hipSuccess &&
              hipMalloc(&h->stats, sizeof(unsigned long long) * 4) == hipSuccess;
    if (!ok) {
        free_dict(h);
        snprintf(g_last_error, sizeof(g_last_error), "hipMalloc failed in sc_gram_precompute");
        return SC_ENOMEM;
    }
    hipError_t e;
    int status[4] = {0, 0, 0, 0};
    if ((e = hipMemsetAsync(h->status, 0, sizeof(int) * 4, st)) != hipSuccess ||
        (e = hipMemsetAsync(h->stats, 0, sizeof(unsigned long long) * 4, st)) != hipSuccess ||
        (e = sc::launch_dict_check(D, d, K, flags & SC_NORMALIZE, h->D, h->status, st)) != hipSuccess ||
        (e = hipMemcpyAsync(status, h->status, sizeof(int) * 4, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess) {
        free_dict(h);
        return set_dev_error("sc_gram_precompute", e);
    }
    if (status[0] & 1) {
        free_dict(h);
        return SC_ENONFINITE;
    }
    if (status[0] & 2) {
        free_dict(h);
        return SC_ENORM;
    }
    if ((e = hipMemsetAsync(h->DT, 0, sizeof(float) * (size_t)sc::dt_rows(d) * Kp, st)) != hipSuccess ||
        (e = sc::launch_dict_layouts(h->D, d, K, Kp, h->DT, h->Dbf, h->Dlo, h->Dl2, h->D48, h->Dr, dpad, h->Dbfo,
                                     st)) != hipSuccess ||
        (e = sc::launch_gram(h->D, d, K, Kp, h->G, h->G64, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess) {
        free_dict(h);
        return set_dev_error("sc_gram_precompute", e);
    }
    h->dev = sc::DictDev{d, K, Kp, E, h->D, h->DT, h->G, h->Dbf, h->Dlo, h->Dl2, h->D48, h->G64, h->Dr, dpad};
    h->row_cache = E <= 4 ? 4 : 0;
    h->row_cache_bf16 = h->row_cache;
    // device copy of the layout descriptor, read by the multi-scene encoder
    if ((e = hipMalloc(&h->ddev, sizeof(sc::DictDev))) != hipSuccess ||
        (e = hipMemcpy(h->ddev, &h->dev, sizeof(sc::DictDev), hipMemcpyHostToDevice)) != hipSuccess) {
        free_dict(h);
        return set_dev_error("sc_gram_precompute", e);
    }
    *out = h;
    return SC_OK;
}

int sc_dict_destroy(sc_dict h) {
    if (!h) return SC_OK;
    hipDeviceSynchronize();
    free_dict(h);
    return SC_OK;
}

int sc_dict_dims(sc_dict h, int *d, int *K) {
    if (!h || !d || !K) return SC_EINVAL;
    *d = h->dev.d;
    *K = h->dev.K;
    return SC_OK;
}

int sc_dict_gram(sc_dict h, float *G_out, void *stream) {
    if (!h || !G_out) return SC_EINVAL;
    const int K = h->dev.K;
    SC_HIP(hipMemcpy2DAsync(G_out, sizeof(float) * K, h->G, sizeof(float) * h->dev.Kp, sizeof(float) * K, K,
                            hipMemcpyDeviceToDevice, (hipStream_t)stream),
           "sc_dict_gram");
    return SC_OK;
}

int sc_omp_encode(sc_dict h, const float *X, int64_t N, int k, float eps, int flags, int32_t *idx, float *coef,
                  int32_t *count, float *resid, void *stream) {
    if (!h || N < 0) return SC_EINVAL;
    const int d = h->dev.d, K = h->dev.K;
    if (k < 1 || k > std::min(std::min(K, d), 32)) return SC_EINVAL;
    if (!(eps >= 0.f) || !isfinite(eps)) return SC_EINVAL;
    if (flags & ~(SC_EPS_RELATIVE | SC_PREC_BF16 | SC_NO_FP64_REFIT)) return SC_EINVAL;
    if (N == 0) return SC_OK;   // empty input: arrays may be NULL
    if (!X || !idx || !coef || !count) return SC_EINVAL;
    const int kmax = sc::pick_kmax(k);
    sc::OmpParams p{X, N, nullptr, nullptr, k, eps, (flags & SC_EPS_RELATIVE) ? 1 : 0,
                    (flags & SC_NO_FP64_REFIT) ? 0 : 1, kKappaMax, idx, coef, count, resid, h->stats};
    hipStream_t st = (hipStream_t)stream;
    const int a0 = (flags & SC_PREC_BF16) ? sc::A0_MFMA_BF16X6 : h->a0_fp32;
    hipError_t e = sc::launch_omp_batch(h->dev, p, kmax, a0, row_cache_for(h, flags), st);
    if (e == hipErrorInvalidValue) {
        snprintf(g_last_error, sizeof(g_last_error), "no compiled encoder for K=%d (Kp=%d) with k=%d", K,
                 h->dev.Kp, k);
        return SC_EINVAL;
    }
    if (e != hipSuccess) return set_dev_error("sc_omp_encode", e);
    return SC_OK;
}

int sc_dict_set_tuning(sc_dict h, int key, int value) {
    if (!h) return SC_EINVAL;
    if (key == SC_TUNE_FP32_CORRELATION) {
        if (value != SC_CORR_VALU && value != SC_CORR_MFMA) return SC_EINVAL;
        h->a0_fp32 = value == SC_CORR_VALU ? sc::A0_VALU : sc::A0_MFMA_F32;
        return SC_OK;
    }
    if (key == SC_TUNE_ROW_CACHE || key == SC_TUNE_ROW_CACHE_BF16) {
        if (value != 0 && value != 4) return SC_EINVAL;
        (key == SC_TUNE_ROW_CACHE ? h->row_cache : h->row_cache_bf16) = value;
        return SC_OK;
    }
    if (key == SC_TUNE_RESTRICTED_CAP) {
        if (value < 0 || value > 32) return SC_EINVAL;
        h->restricted_cap = value;
        return SC_OK;
    }
    return SC_EINVAL;
}

int sc_dict_get_tuning(sc_dict h, int key, int *value) {
    if (!h || !value) return SC_EINVAL;
    if (key == SC_TUNE_FP32_CORRELATION) {
        *value = h->a0_fp32 == sc::A0_VALU ? SC_CORR_VALU : SC_CORR_MFMA;
        return SC_OK;
    }
    if (key == SC_TUNE_ROW_CACHE || key == SC_TUNE_ROW_CACHE_BF16) {
        *value = key == SC_TUNE_ROW_CACHE ? h->row_cache : h->row_cache_bf16;
        return SC_OK;
    }
    if (key == SC_TUNE_RESTRICTED_CAP) {
        *value = h->restricted_cap;
        return SC_OK;
    }
    return SC_EINVAL;
}

int sc_omp_stats(sc_dict h, int64_t stats[4], int reset, void *stream) {
    if (!h || !stats) return SC_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    unsigned long long v[4];
    SC_HIP(hipMemcpyAsync(v, h->stats, sizeof(v), hipMemcpyDeviceToHost, st), "sc_omp_stats");
    SC_HIP(hipStreamSynchronize(st), "sc_omp_stats");
    for (int i = 0; i < 4; ++i) stats[i] = (int64_t)v[i];
    if (reset) SC_HIP(hipMemsetAsync(h->stats, 0, sizeof(v), st), "sc_omp_stats");
    return SC_OK;
}

int sc_sh_eval_sparse(sc_dict h, const int32_t *idx, const float *coef, const int32_t *count, int64_t N, int k,
                      const float *dirs, int64_t M, int dir_mode, float *rgb, void *stream) {
    if (!h || N < 0 || k < 1 || k > 1024) return SC_EINVAL;
    const int d = h->dev.d;
    if (d != 9 && d != 24 && d != 45) return SC_EINVAL;
    if (dir_mode == SC_DIRS_PER_SIGNAL) {
        if (M != N) return SC_EINVAL;
    } else if (dir_mode == SC_DIRS_SHARED) {
        if (M < 1) return SC_EINVAL;
    } else {
        return SC_EINVAL;
    }
    if (N == 0) return SC_OK;   // empty input: arrays may be NULL
    if (!idx || !coef || !count || !dirs || !rgb) return SC_EINVAL;
    hipError_t e = sc::launch_sh_eval(h->dev, idx, coef, count, N, k, dirs, M, dir_mode == SC_DIRS_SHARED ? 1 : 0,
                                      rgb, (hipStream_t)stream);
    if (e != hipSuccess) return set_dev_error("sc_sh_eval_sparse", e);
    return SC_OK;
}

/* ------------------------------------------------------------------ */
/* dictionary update                                                    */
/* ------------------------------------------------------------------ */

size_t sc_mod_workspace(int d, int K) {
    if (d < 1 || d > 64 || K < 1 || K > 1024) return 0;
    return sc::mod_workspace_bytes(d, K);
}

int sc_mod_update(const float *X, int64_t N, int d, int K, const int32_t *idx, const float *coef,
                  const int32_t *count, int k, const float *resid, float *D_out, int *n_replaced, void *workspace,
                  size_t ws_bytes, void *stream) {
    if (N < 1 || d < 1 || d > 64 || K < 1 || K > 1024 || k < 1 || k > 32) return SC_EINVAL;
    if (!X || !idx || !coef || !count || !resid || !D_out || !workspace) return SC_EINVAL;
    if (ws_bytes < sc_mod_workspace(d, K)) return SC_ENOMEM;
    int dev = 0;
    int rc = check_device(&dev);
    if (rc != SC_OK) return rc;
    SC_HIP(sc::launch_mod_update(X, N, d, K, idx, coef, count, k, resid, D_out, n_replaced, workspace,
                                 (hipStream_t)stream),
           "sc_mod_update");
    return SC_OK;
}

/* ------------------------------------------------------------------ */
/* CSC storage and its consumers                                        */
/* ------------------------------------------------------------------ */

size_t sc_csc_workspace(int64_t N) {
    if (N < 0) return 0;
    return align_up(sizeof(int64_t) * (size_t)(sc::csc_workspace_blocks(N) + 1));
}

int sc_csc_colptr(const int32_t *count, int64_t N, int64_t *colptr, void *workspace, size_t ws_bytes, void *stream) {
    if (N < 0 || !colptr) return SC_EINVAL;
    if (N > 0 && !count) return SC_EINVAL;
    if (!workspace) return SC_EINVAL;
    if (ws_bytes < sc_csc_workspace(N)) return SC_ENOMEM;
    SC_HIP(sc::launch_csc_colptr(count, N, colptr, (int64_t *)workspace, (hipStream_t)stream), "sc_csc_colptr");
    return SC_OK;
}

int sc_csc_fill(const int32_t *idx, const float *coef, const int32_t *count, int64_t N, int k, const int64_t *colptr,
                int32_t *rows, float *vals, void *stream) {
    if (N < 0 || k < 1 || k > 1024) return SC_EINVAL;
    if (N == 0) return SC_OK;
    if (!idx || !coef || !count || !colptr || !rows || !vals) return SC_EINVAL;
    SC_HIP(sc::launch_csc_fill(idx, coef, count, N, k, colptr, rows, vals, (hipStream_t)stream), "sc_csc_fill");
    return SC_OK;
}

size_t sc_omp_encode_csc_workspace(int64_t N, int k) {
    if (N < 0 || k < 1 || k > 32) return 0;
    return align_up(sc::csc_encode_workspace_bytes(N));
}

int sc_omp_encode_csc(sc_dict h, const float *X, int64_t N, int k, float eps, int flags, int64_t *colptr,
                      int32_t *rows, float *vals, int64_t cap, int64_t *nnz_out, float *resid, void *workspace,
                      size_t ws_bytes, void *stream) {
    if (!h || N < 0 || cap < 0 || !colptr || !nnz_out) return SC_EINVAL;
    if (k < 1 || k > std::min(std::min(h->dev.K, h->dev.d), 32)) return SC_EINVAL;
    if (!(eps >= 0.f) || !isfinite(eps)) return SC_EINVAL;
    if (flags & ~(SC_EPS_RELATIVE | SC_PREC_BF16 | SC_NO_FP64_REFIT)) return SC_EINVAL;
    if (!workspace) return SC_EINVAL;
    if (ws_bytes < sc_omp_encode_csc_workspace(N, k)) return SC_ENOMEM;
    if (N > 0 && !X) return SC_EINVAL;
    if (cap > 0 && (!rows || !vals)) return SC_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const size_t wsz = sc::csc_encode_workspace_bytes(N);
    SC_HIP(sc::launch_zero_words(workspace, (int64_t)(wsz / 4), st), "sc_omp_encode_csc");
    if (N == 0) {
        SC_HIP(sc::launch_zero_words(colptr, 2, st), "sc_omp_encode_csc");
    } else {
        sc::OmpParams p{X, N, nullptr, nullptr, k, eps, (flags & SC_EPS_RELATIVE) ? 1 : 0,
                        (flags & SC_NO_FP64_REFIT) ? 0 : 1, kKappaMax, nullptr, nullptr, nullptr, resid, h->stats};
        const int a0 = (flags & SC_PREC_BF16) ? sc::A0_MFMA_BF16X6 : h->a0_fp32;
        hipError_t e = sc::launch_omp_csc(h->dev, p, sc::pick_kmax(k), a0, row_cache_for(h, flags), colptr, rows, vals,
                                          cap, workspace, st);
        if (e == hipErrorInvalidValue) {
            snprintf(g_last_error, sizeof(g_last_error), "no compiled CSC encoder for K=%d with k=%d", h->dev.K, k);
            return SC_EINVAL;
        }
        if (e != hipSuccess) return set_dev_error("sc_omp_encode_csc", e);
    }
    int64_t nnz = 0;
    int err = 0;
    SC_HIP(hipMemcpyAsync(&nnz, colptr + N, sizeof(int64_t), hipMemcpyDeviceToHost, st), "sc_omp_encode_csc");
    SC_HIP(hipMemcpyAsync(&err, (unsigned char *)workspace + sizeof(int), sizeof(int), hipMemcpyDeviceToHost, st),
           "sc_omp_encode_csc");
    SC_HIP(hipStreamSynchronize(st), "sc_omp_encode_csc");
    *nnz_out = nnz;
    if (err) {
        snprintf(g_last_error, sizeof(g_last_error), "sc_omp_encode_csc: a column-offset wait exceeded its bound");
        return SC_EDEVICE;
    }
    return nnz > cap ? SC_ENOMEM : SC_OK;
}

int sc_sh_eval_csc(sc_dict h, const int64_t *colptr, const int32_t *rows, const float *vals, int64_t N,
                   const float *dirs, int64_t M, int dir_mode, float *rgb, void *stream) {
    if (!h || N < 0) return SC_EINVAL;
    const int d = h->dev.d;
    if (d != 9 && d != 24 && d != 45) return SC_EINVAL;
    if (dir_mode == SC_DIRS_PER_SIGNAL) {
        if (M != N) return SC_EINVAL;
    } else if (dir_mode == SC_DIRS_SHARED) {
        if (M < 1) return SC_EINVAL;
    } else {
        return SC_EINVAL;
    }
    if (N == 0) return SC_OK;
    if (!colptr || !rows || !vals || !dirs || !rgb) return SC_EINVAL;
    SC_HIP(sc::launch_csc_eval(h->dev, colptr, rows, vals, N, dirs, M, dir_mode == SC_DIRS_SHARED ? 1 : 0, nullptr,
                               nullptr, nullptr, rgb, (hipStream_t)stream),
           "sc_sh_eval_csc");
    return SC_OK;
}

int sc_gaussian_rgb_csc(sc_dict h, const int64_t *colptr, const int32_t *rows, const float *vals, int64_t N,
                        const float *pos, const float *dc, const float cam[3], float *rgb, void *stream) {
    if (!h || N < 0 || !cam) return SC_EINVAL;
    const int d = h->dev.d;
    if (d != 9 && d != 24 && d != 45) return SC_EINVAL;
    if (!isfinite(cam[0]) || !isfinite(cam[1]) || !isfinite(cam[2])) return SC_EINVAL;
    if (N == 0) return SC_OK;
    if (!colptr || !rows || !vals || !pos || !dc || !rgb) return SC_EINVAL;
    SC_HIP(sc::launch_csc_eval(h->dev, colptr, rows, vals, N, nullptr, N, 0, pos, dc, cam, rgb, (hipStream_t)stream),
           "sc_gaussian_rgb_csc");
    return SC_OK;
}

/* ------------------------------------------------------------------ */
/* learned support proposer                                             */
/* ------------------------------------------------------------------ */

int64_t sc_proposer_num_params(int d, int H, int K) {
    if (d < 1 || d > 64 || H < 1 || K < 1) return SC_EINVAL;
    return (int64_t)H * d + H + (int64_t)H * H + H + (int64_t)K * H + K;
}

static void free_proposer(sc_proposer p) {
    if (!p) return;
    hipFree(p->params);
    hipFree(p->m);
    hipFree(p->v);
    hipFree(p->grads);
    hipFree(p->W1b);
    hipFree(p->W2b);
    hipFree(p->W3b);
    hipFree(p->W2bT);
    hipFree(p->W3bT);
    hipFree(p->W1o);
    hipFree(p->W2o);
    hipFree(p->W3o);
    delete p;
}

int sc_proposer_create(int d, int H, int K, sc_proposer *out) {
    if (!out || d < 1 || d > 48 || H != 256 || (K != 128 && K != 256 && K != 512)) return SC_EINVAL;
    int dev = 0;
    int rc = check_device(&dev);
    if (rc != SC_OK) return rc;
    sc_proposer p = new sc_proposer_s();
    p->d = d;
    p->H = H;
    p->K = K;
    p->nparams = sc_proposer_num_params(d, H, K);
    const size_t pb = sizeof(float) * (size_t)p->nparams;
    bool ok = hipMalloc(&p->params, pb) == hipSuccess && hipMalloc(&p->m, pb) == hipSuccess &&
              hipMalloc(&p->v, pb) == hipSuccess && hipMalloc(&p->grads, pb) == hipSuccess &&
              hipMalloc(&p->W1b, sizeof(uint16_t) * (size_t)H * 64) == hipSuccess &&
              hipMalloc(&p->W2b, sizeof(uint16_t) * (size_t)H * H) == hipSuccess &&
              hipMalloc(&p->W3b, sizeof(uint16_t) * (size_t)K * H) == hipSuccess &&
              hipMalloc(&p->W2bT, sizeof(uint16_t) * (size_t)H * H) == hipSuccess &&
              hipMalloc(&p->W3bT, sizeof(uint16_t) * (size_t)K * H) == hipSuccess &&
              hipMalloc(&p->W1o, sizeof(uint16_t) * (size_t)H * 64) == hipSuccess &&
              hipMalloc(&p->W2o, sizeof(uint16_t) * (size_t)H * H) == hipSuccess &&
              hipMalloc(&p->W3o, sizeof(uint16_t) * (size_t)K * H) == hipSuccess;
    if (!ok ||
        hipMemset(p->params, 0, pb) != hipSuccess || hipMemset(p->m, 0, pb) != hipSuccess ||
        hipMemset(p->v, 0, pb) != hipSuccess || hipMemset(p->grads, 0, pb) != hipSuccess) {
        free_proposer(p);
        snprintf(g_last_error, sizeof(g_last_error), "hipMalloc failed in sc_proposer_create");
        return SC_ENOMEM;
    }
    *out = p;
    return SC_OK;
}

int sc_proposer_destroy(sc_proposer p) {
    if (!p) return SC_OK;
    hipDeviceSynchronize();
    free_proposer(p);
    return SC_OK;
}

int sc_proposer_dims(sc_proposer p, int *d, int *H, int *K, int64_t *nparams) {
    if (!p || !d || !H || !K || !nparams) return SC_EINVAL;
    *d = p->d;
    *H = p->H;
    *K = p->K;
    *nparams = p->nparams;
    return SC_OK;
}

int sc_proposer_set_params(sc_proposer p, const float *params, void *stream) {
    if (!p || !params) return SC_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const size_t pb = sizeof(float) * (size_t)p->nparams;
    SC_HIP(hipMemcpyAsync(p->params, params, pb, hipMemcpyDeviceToDevice, st), "sc_proposer_set_params");
    SC_HIP(hipMemsetAsync(p->m, 0, pb, st), "sc_proposer_set_params");
    SC_HIP(hipMemsetAsync(p->v, 0, pb, st), "sc_proposer_set_params");
    p->step = 0;
    SC_HIP(sc::launch_proposer_pack(p->params, p->d, p->H, p->K, p->W1b, p->W2b, p->W3b, p->W2bT, p->W3bT, p->W1o,
                                    p->W2o, p->W3o, st),
           "sc_proposer_set_params");
    return SC_OK;
}

int sc_proposer_get_params(sc_proposer p, float *params, void *stream) {
    if (!p || !params) return SC_EINVAL;
    SC_HIP(hipMemcpyAsync(params, p->params, sizeof(float) * (size_t)p->nparams, hipMemcpyDeviceToDevice,
                          (hipStream_t)stream),
           "sc_proposer_get_params");
    return SC_OK;
}

int sc_proposer_forward(sc_proposer p, const float *X, int64_t N, int n_cand, int32_t *cand, float *logits,
                        void *stream) {
    if (!p || N < 0 || n_cand < 1 || n_cand > 32 || n_cand > p->K) return SC_EINVAL;
    if (N == 0) return SC_OK;
    if (!X || !cand) return SC_EINVAL;
    hipError_t e = sc::launch_proposer_topk(p->dev(), X, N, n_cand, cand, logits, (hipStream_t)stream);
    if (e != hipSuccess) return set_dev_error("sc_proposer_forward", e);
    return SC_OK;
}

int sc_screen_topk(sc_dict h, const float *X, int64_t N, int n_cand, int32_t *cand, void *stream) {
    if (!h || N < 0 || n_cand < 1 || n_cand > 32 || n_cand > h->dev.K) return SC_EINVAL;
    const int K = h->dev.K;
    if (K != 128 && K != 256 && K != 512) return SC_EINVAL;
    if (N == 0) return SC_OK;
    if (!X || !cand) return SC_EINVAL;
    hipError_t e = sc::launch_screen_topk(h->Dbfo, h->dev.d, K, X, N, n_cand, cand, (hipStream_t)stream);
    if (e != hipSuccess) return set_dev_error("sc_screen_topk", e);
    return SC_OK;
}

size_t sc_omp_encode_learned_workspace(int64_t N, int n_cand) {
    if (N < 0 || n_cand < 1) return 0;
    return align_up(sizeof(int32_t) * (size_t)N * n_cand) + align_up(sizeof(int32_t) * (size_t)N) + kAlign;
}

int sc_omp_encode_learned(sc_dict h, sc_proposer p, const float *X, int64_t N, int k, float eps, int flags,
                          int n_cand, int32_t *idx, float *coef, int32_t *count, float *resid, void *workspace,
                          size_t ws_bytes, void *stream) {
    if (!h || !p || N < 0) return SC_EINVAL;
    const int d = h->dev.d, K = h->dev.K;
    if (p->K != K || p->d != d || d > 48) return SC_EINVAL;
    if (k < 1 || k > std::min(std::min(K, d), 16)) return SC_EINVAL;
    if (n_cand < k || n_cand > 32 || n_cand > K) return SC_EINVAL;
    if (!(eps >= 0.f) || !isfinite(eps)) return SC_EINVAL;
    if (flags & ~(SC_EPS_RELATIVE | SC_NO_FP64_REFIT | SC_PREC_BF16)) return SC_EINVAL;
    if (N == 0) return SC_OK;
    if (!X || !idx || !coef || !count || !workspace) return SC_EINVAL;
    if (ws_bytes < sc_omp_encode_learned_workspace(N, n_cand)) return SC_ENOMEM;
    hipStream_t st = (hipStream_t)stream;
    unsigned char *w = (unsigned char *)workspace;
    int32_t *cand = (int32_t *)w;
    int32_t *miss_rows = (int32_t *)(w + align_up(sizeof(int32_t) * (size_t)N * n_cand));
    int32_t *miss_count = (int32_t *)((unsigned char *)miss_rows + align_up(sizeof(int32_t) * (size_t)N));
    const int kmax = sc::pick_kmax(k);
    const int rel = (flags & SC_EPS_RELATIVE) ? 1 : 0;
    const int refit = (flags & SC_NO_FP64_REFIT) ? 0 : 1;
    SC_HIP(sc::launch_zero_words(miss_count, 1, st), "sc_omp_encode_learned");
    SC_HIP(sc::launch_proposer_topk(p->dev(), X, N, n_cand, cand, nullptr, st), "sc_omp_encode_learned (proposer)");
    const int kcap = h->restricted_cap > 0 ? std::min(h->restricted_cap, k) : k;
    sc::RompParams rp{X, N, k, eps, rel, refit, kKappaMax, kcap, cand, n_cand, idx, coef, count, resid, miss_rows,
                      miss_count, h->stats};
    // the restricted pursuit never takes more than kcap steps: size its registers for that
    SC_HIP(sc::launch_omp_restricted(h->dev, h->D48, rp, sc::pick_kmax(kcap), st), "sc_omp_encode_learned (restricted)");
    sc::OmpParams fp{X, N, miss_rows, miss_count, k, eps, rel, refit, kKappaMax, idx, coef, count, resid, h->stats};
    const int a0 = (flags & SC_PREC_BF16) ? sc::A0_MFMA_BF16X6 : h->a0_fp32;
    SC_HIP(sc::launch_omp_batch(h->dev, fp, kmax, a0, row_cache_for(h, flags), st), "sc_omp_encode_learned (fallback)");
    return SC_OK;
}

}  // extern "C"

/* ------------------------------------------------------------------ */
/* the learned encoder without allocation                               */
/* ------------------------------------------------------------------ */

// Device scratch of sc_omp_encode_learned_noalloc: every GPU the library runs
// on holds its own copy (at its own address) until the process ends.  In
// host code `scratch` is only a stand-in for the symbol: the kernels get the
// device address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[SC_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device `dev` (the current device), resolved
// on the first call for that device.
int scratch_address(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices) return SC_ENODEV;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return set_dev_error("sc_omp_encode_learned_noalloc (scratch address)", e);
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return SC_OK;
}

}  // namespace

extern "C" {

int sc_omp_encode_learned_noalloc(sc_dict h, sc_proposer p, const float *X, int64_t N, int k, float eps, int flags,
                                  int n_cand, int32_t *idx, float *coef, int32_t *count, float *resid,
                                  void *stream) {
    if (!h || !p || N < 0 || n_cand < 1 || n_cand > 32) return SC_EINVAL;
    const size_t need = sc_omp_encode_learned_workspace(N, n_cand);
    if (need > (size_t)SC_STATIC_SCRATCH_BYTES) {
        snprintf(g_last_error, sizeof(g_last_error),
                 "sc_omp_encode_learned_noalloc: N=%lld with n_cand=%d needs %zu bytes of scratch; the static "
                 "scratch holds %zu",
                 (long long)N, n_cand, need, (size_t)SC_STATIC_SCRATCH_BYTES);
        return SC_ENOMEM;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != h->device) {
        snprintf(g_last_error, sizeof(g_last_error),
                 "sc_omp_encode_learned_noalloc: the dictionary lives on device %d, the current device is %d",
                 h->device, dev);
        return SC_EINVAL;
    }
    void *ws = nullptr;
    const int rc = scratch_address(dev, &ws);
    if (rc != SC_OK) return rc;
    return sc_omp_encode_learned(h, p, X, N, k, eps, flags, n_cand, idx, coef, count, resid, ws,
                                 (size_t)SC_STATIC_SCRATCH_BYTES, stream);
}

int sc_omp_encode_restricted(sc_dict h, const float *X, int64_t N, int k, float eps, int flags, const int32_t *cand,
                             int n_cand, int32_t *idx, float *coef, int32_t *count, float *resid, int32_t *miss_rows,
                             int32_t *miss_count, void *stream) {
    if (!h || N < 0) return SC_EINVAL;
    const int d = h->dev.d, K = h->dev.K;
    if (d > 48 || k < 1 || k > std::min(std::min(K, d), 16)) return SC_EINVAL;
    if (n_cand < k || n_cand > 32 || n_cand > K) return SC_EINVAL;
    if (!(eps >= 0.f) || !isfinite(eps)) return SC_EINVAL;
    if (flags & ~(SC_EPS_RELATIVE | SC_NO_FP64_REFIT)) return SC_EINVAL;
    if (!miss_count) return SC_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    SC_HIP(sc::launch_zero_words(miss_count, 1, st), "sc_omp_encode_restricted");
    if (N == 0) return SC_OK;
    if (!X || !cand || !idx || !coef || !count || !miss_rows) return SC_EINVAL;
    const int kcap = h->restricted_cap > 0 ? std::min(h->restricted_cap, k) : k;
    sc::RompParams rp{X, N, k, eps, (flags & SC_EPS_RELATIVE) ? 1 : 0, (flags & SC_NO_FP64_REFIT) ? 0 : 1, kKappaMax,
                      kcap, cand, n_cand, idx, coef, count, resid, miss_rows, miss_count, h->stats};
    SC_HIP(sc::launch_omp_restricted(h->dev, h->D48, rp, sc::pick_kmax(kcap), st), "sc_omp_encode_restricted");
    return SC_OK;
}

int sc_omp_encode_rows(sc_dict h, const float *X, const int32_t *rows, const int32_t *nrows, int64_t max_rows, int k,
                       float eps, int flags, int32_t *idx, float *coef, int32_t *count, float *resid, void *stream) {
    if (!h || max_rows < 0) return SC_EINVAL;
    const int d = h->dev.d, K = h->dev.K;
    if (k < 1 || k > std::min(std::min(K, d), 32)) return SC_EINVAL;
    if (!(eps >= 0.f) || !isfinite(eps)) return SC_EINVAL;
    if (flags & ~(SC_EPS_RELATIVE | SC_NO_FP64_REFIT | SC_PREC_BF16)) return SC_EINVAL;
    if (max_rows == 0) return SC_OK;
    if (!X || !rows || !nrows || !idx || !coef || !count) return SC_EINVAL;
    sc::OmpParams p{X, max_rows, rows, nrows, k, eps, (flags & SC_EPS_RELATIVE) ? 1 : 0,
                    (flags & SC_NO_FP64_REFIT) ? 0 : 1, kKappaMax, idx, coef, count, resid, h->stats};
    const int a0 = (flags & SC_PREC_BF16) ? sc::A0_MFMA_BF16X6 : h->a0_fp32;
    hipError_t e = sc::launch_omp_batch(h->dev, p, sc::pick_kmax(k), a0, row_cache_for(h, flags), (hipStream_t)stream);
    if (e == hipErrorInvalidValue) return SC_EINVAL;
    if (e != hipSuccess) return set_dev_error("sc_omp_encode_rows", e);
    return SC_OK;
}

/* ------------------------------------------------------------------ */
/* many scenes in one launch                                            */
/* ------------------------------------------------------------------ */

namespace {

constexpr size_t kBatchWorkspace = 256;

int validate_scenes(const sc_scene *scenes, int n) {
    if (!scenes || n < 1 || n > SC_MAX_SCENES) return SC_EINVAL;
    int dev = -1;
    for (int q = 0; q < n; ++q) {
        const sc_scene &s = scenes[q];
        const sc_dict h = s.dict;
        if (!h || s.N < 0) return SC_EINVAL;
        if (dev < 0) dev = h->device;
        if (h->device != dev) return SC_EINVAL;
        const int d = h->dev.d, K = h->dev.K;
        if (h->dev.E > 8 || s.k < 1 || s.k > std::min(std::min(K, d), 16)) return SC_EINVAL;
        if (!(s.eps >= 0.f) || !isfinite(s.eps)) return SC_EINVAL;
        if (s.flags & ~(SC_EPS_RELATIVE | SC_NO_FP64_REFIT)) return SC_EINVAL;
        if (s.N > 0 && (!s.X || !s.idx || !s.coef || !s.count)) return SC_EINVAL;
    }
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess || cur != dev) return SC_EINVAL;
    return SC_OK;
}

int validate_tuning(const sc_batch_tuning *t, int n) {
    if (!t) return SC_OK;
    if (t->tile != 0 && t->tile != 16 && t->tile != 32) return SC_EINVAL;
    if (t->row_cache != 0 && t->row_cache != 4) return SC_EINVAL;
    if (t->wg_per_cu < 0 || t->wg_per_cu > 64) return SC_EINVAL;
    if (t->order != SC_ORDER_COST && t->order != SC_ORDER_GIVEN) return SC_EINVAL;
    if (t->corr != SC_CORR_VALU && t->corr != SC_CORR_MFMA) return SC_EINVAL;
    (void)n;
    return SC_OK;
}

sc_batch_tuning default_tuning() {
    sc_batch_tuning t;
    t.tile = 16;
    t.row_cache = 0;
    t.wg_per_cu = 0;
    t.order = SC_ORDER_COST;
    t.corr = SC_CORR_VALU;
    return t;
}

// Launch on validated arguments.
int encode_batched(const sc_scene *scenes, int n, const sc_batch_tuning &t, int *counter, hipStream_t st) {
    int order[SC_MAX_SCENES];
    double cost[SC_MAX_SCENES];
    int m = 0;
    for (int q = 0; q < n; ++q) {
        const sc_dict h = scenes[q].dict;
        // work of a tile: the correlations (Kp d) and the pursuit (~Kp per step)
        cost[q] = (double)h->dev.Kp * (h->dev.d + 4.0 * std::min(scenes[q].k, 8));
        if (scenes[q].N > 0) order[m++] = q;
    }
    if (m == 0) return SC_OK;
    if (t.order == SC_ORDER_COST)
        std::stable_sort(order, order + m, [&](int a, int b) { return cost[a] > cost[b]; });
    hipError_t e = sc::launch_omp_multi(scenes, order, m, t.corr == SC_CORR_MFMA ? sc::A0_MFMA_F32 : sc::A0_VALU,
                                        t.tile == 32 ? 32 : 16, t.row_cache, t.wg_per_cu, counter, st);
    if (e != hipSuccess) return set_dev_error("sc_omp_encode_batched", e);
    return SC_OK;
}

}  // namespace

size_t sc_omp_encode_batched_workspace(void) { return kBatchWorkspace; }

int sc_omp_encode_batched(const sc_scene *scenes, int n_scenes, const sc_batch_tuning *tuning, void *workspace,
                          size_t ws_bytes, void *stream) {
    int rc = validate_scenes(scenes, n_scenes);
    if (rc != SC_OK) return rc;
    if ((rc = validate_tuning(tuning, n_scenes)) != SC_OK) return rc;
    if (!workspace) return SC_EINVAL;
    if (ws_bytes < kBatchWorkspace) return SC_ENOMEM;
    return encode_batched(scenes, n_scenes, tuning ? *tuning : default_tuning(), (int *)workspace,
                          (hipStream_t)stream);
}

int sc_batch_autotune(const sc_scene *scenes, int n_scenes, int64_t sample, void *workspace, size_t ws_bytes,
                      sc_batch_tuning *best, float *best_ms, void *stream) {
    int rc = validate_scenes(scenes, n_scenes);
    if (rc != SC_OK) return rc;
    if (!workspace || !best || sample < 1) return SC_EINVAL;
    if (ws_bytes < kBatchWorkspace) return SC_ENOMEM;
    hipStream_t st = (hipStream_t)stream;
    int *counter = (int *)workspace;
    sc_scene tr[SC_MAX_SCENES];
    for (int q = 0; q < n_scenes; ++q) {
        tr[q] = scenes[q];
        tr[q].N = std::min<int64_t>(scenes[q].N, sample);
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return set_dev_error("sc_batch_autotune", hipErrorUnknown);
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return set_dev_error("sc_batch_autotune", hipErrorUnknown);
    }
    int err = SC_OK;
    // best of 2 timed launches after a warm-up; +inf on failure
    auto timeit = [&](const sc_scene *sc_, int n, const sc_batch_tuning &t) -> float {
        float bestt = 3.4e38f;
        for (int r = 0; r < 3 && err == SC_OK; ++r) {
            if (hipEventRecord(e0, st) != hipSuccess) err = SC_EDEVICE;
            if (err == SC_OK) err = encode_batched(sc_, n, t, counter, st);
            if (err == SC_OK && hipEventRecord(e1, st) != hipSuccess) err = SC_EDEVICE;
            if (err == SC_OK && hipEventSynchronize(e1) != hipSuccess) err = SC_EDEVICE;
            float ms = 0.f;
            if (err == SC_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) err = SC_EDEVICE;
            if (err == SC_OK && r > 0) bestt = std::min(bestt, ms);
        }
        return bestt;
    };
    sc_batch_tuning bt = default_tuning();
    float bms = 3.4e38f;
    const int corrs[2] = {SC_CORR_VALU, SC_CORR_MFMA}, tiles[2] = {16, 32}, rcs[2] = {0, 4}, wgs[3] = {0, 1, 2},
              orders[2] = {SC_ORDER_COST, SC_ORDER_GIVEN};
    for (int m = 0; m < 2; ++m)
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int c = 0; c < 3; ++c)
                    for (int o = 0; o < 2 && err == SC_OK; ++o) {
                        sc_batch_tuning t = default_tuning();
                        t.corr = corrs[m];
                        t.tile = tiles[a];
                        t.row_cache = rcs[b];
                        t.wg_per_cu = wgs[c];
                        t.order = orders[o];
                        const float ms = timeit(tr, n_scenes, t);
                        if (ms < bms) {
                            bms = ms;
                            bt = t;
                        }
                    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (err != SC_OK) return err;
    *best = bt;
    if (best_ms) *best_ms = bms;
    return SC_OK;
}

/* ------------------------------------------------------------------ */
/* proposer training                                                    */
/* ------------------------------------------------------------------ */

namespace {
struct TrainLayout {
    size_t xh, a1, h1, a2, h2, z, dz, da2, da1, loss, part, total;
};
TrainLayout train_layout(int64_t B, int K) {
    TrainLayout t;
    size_t o = 0;
    auto take = [&](size_t n) {
        size_t r = o;
        o = align_up(o + n);
        return r;
    };
    const size_t e = 4;   // bytes per element (FP32 upper bound)
    t.xh = take(e * B * 64);
    t.a1 = take(e * B * 256);
    t.h1 = take(e * B * 256);
    t.a2 = take(e * B * 256);
    t.h2 = take(e * B * 256);
    t.z = take(e * B * K);
    t.dz = take(e * B * K);
    t.da2 = take(e * B * 256);
    t.da1 = take(e * B * 256);
    t.loss = take(sizeof(float));
    // split-K partial tiles of the three weight-gradient products (reused in turn)
    const int Bi = (int)B;
    size_t np = 0;
    for (const auto &mn : {std::pair<int, int>{K, 256}, {256, 256}, {256, 64}})
        np = std::max(np, (size_t)sc::gemm_splits(mn.first, mn.second, Bi) * mn.first * mn.second);
    t.part = take(sizeof(float) * np);
    t.total = o;
    return t;
}
}  // namespace

size_t sc_proposer_train_workspace(sc_proposer p, int64_t B) {
    if (!p || B < 1) return 0;
    return train_layout(B, p->K).total;
}

int sc_proposer_train_step(sc_proposer p, const float *X, const int32_t *rows, int64_t B, const int32_t *sup_idx,
                           const int32_t *sup_count, int kcap, float lr, float beta1, float beta2, float adam_eps,
                           float pos_weight, int flags, float *loss_out, float *grads_out, void *workspace,
                           size_t ws_bytes, void *stream) {
    if (!p || !X || !sup_idx || !sup_count || !workspace || B < 32 || B % 32 || kcap < 1 || kcap > 64)
        return SC_EINVAL;
    if (flags & ~(SC_TRAIN_FP32 | SC_TRAIN_GRAD_ONLY)) return SC_EINVAL;
    if (!(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(adam_eps > 0.f) ||
        !(pos_weight > 0.f))
        return SC_EINVAL;
    const TrainLayout L = train_layout(B, p->K);
    if (ws_bytes < L.total) return SC_ENOMEM;
    const bool f32 = (flags & SC_TRAIN_FP32) != 0;
    hipStream_t st = (hipStream_t)stream;
    unsigned char *w = (unsigned char *)workspace;
    void *xh = w + L.xh, *h1 = w + L.h1, *h2 = w + L.h2, *dz = w + L.dz, *da2 = w + L.da2, *da1 = w + L.da1;
    float *a1 = (float *)(w + L.a1), *a2 = (float *)(w + L.a2), *z = (float *)(w + L.z);
    float *loss = (float *)(w + L.loss);
    float *part = (float *)(w + L.part);
    const int d = p->d, H = p->H, K = p->K;
    // parameter and gradient views
    const float *W1 = p->params, *b1 = W1 + (size_t)H * d, *W2 = b1 + H, *b2 = W2 + (size_t)H * H, *W3 = b2 + H;
    const float *b3 = W3 + (size_t)K * H;
    float *gW1 = p->grads, *gb1 = gW1 + (size_t)H * d, *gW2 = gb1 + H, *gb2 = gW2 + (size_t)H * H, *gW3 = gb2 + H;
    float *gb3 = gW3 + (size_t)K * H;
    const void *Wb1 = f32 ? (const void *)W1 : (const void *)p->W1b;
    const void *Wb2 = f32 ? (const void *)W2 : (const void *)p->W2b;
    const void *Wb3 = f32 ? (const void *)W3 : (const void *)p->W3b;
    const int64_t ld1 = f32 ? d : 64;
    const char *fn = "sc_proposer_train_step";
    using sc::GemmArgs;
    SC_HIP(sc::launch_zero_words(loss, 1, st), fn);
    SC_HIP(sc::launch_train_prep(X, rows, B, d, xh, f32, st), fn);
    // forward
    GemmArgs g1{(int)B, H, 48, xh, 64, 1, Wb1, 1, ld1, sc::EPI_GELU, H, b1, nullptr, nullptr, H, h1, H, a1};
    SC_HIP(sc::launch_gemm(g1, f32, st), fn);
    GemmArgs g2{(int)B, H, H, h1, H, 1, Wb2, 1, H, sc::EPI_GELU, H, b2, nullptr, nullptr, H, h2, H, a2};
    SC_HIP(sc::launch_gemm(g2, f32, st), fn);
    GemmArgs g3{(int)B, K, H, h2, H, 1, Wb3, 1, H, sc::EPI_STORE, K, b3, nullptr, z, K, nullptr, 0, nullptr};
    SC_HIP(sc::launch_gemm(g3, f32, st), fn);
    SC_HIP(sc::launch_bce_grad(z, B, K, rows, sup_idx, sup_count, kcap, pos_weight, dz, loss, f32, st), fn);
    // backward
    GemmArgs gw3{K, H, (int)B, dz, 1, K, h2, H, 1, sc::EPI_STORE, H, nullptr, nullptr, gW3, H, nullptr, 0, nullptr, part};
    SC_HIP(sc::launch_gemm(gw3, f32, st), fn);
    SC_HIP(sc::launch_colsum(dz, B, K, K, gb3, f32, st), fn);
    // B(k, j) = W3[k][j]: the transposed BF16 copy makes k contiguous (vector loads)
    GemmArgs gd2 = f32 ? GemmArgs{(int)B, H, K, dz, K, 1, Wb3, H, 1, sc::EPI_DGELU, H, nullptr, a2, nullptr, H, da2, H,
                                  nullptr}
                       : GemmArgs{(int)B, H, K, dz, K, 1, p->W3bT, 1, K, sc::EPI_DGELU, H, nullptr, a2, nullptr, H,
                                  da2, H, nullptr};
    SC_HIP(sc::launch_gemm(gd2, f32, st), fn);
    GemmArgs gw2{H, H, (int)B, da2, 1, H, h1, H, 1, sc::EPI_STORE, H, nullptr, nullptr, gW2, H, nullptr, 0, nullptr, part};
    SC_HIP(sc::launch_gemm(gw2, f32, st), fn);
    SC_HIP(sc::launch_colsum(da2, B, H, H, gb2, f32, st), fn);
    GemmArgs gd1 = f32 ? GemmArgs{(int)B, H, H, da2, H, 1, Wb2, H, 1, sc::EPI_DGELU, H, nullptr, a1, nullptr, H, da1, H,
                                  nullptr}
                       : GemmArgs{(int)B, H, H, da2, H, 1, p->W2bT, 1, H, sc::EPI_DGELU, H, nullptr, a1, nullptr, H,
                                  da1, H, nullptr};
    SC_HIP(sc::launch_gemm(gd1, f32, st), fn);
    GemmArgs gw1{H, 64, (int)B, da1, 1, H, xh, 64, 1, sc::EPI_STORE, d, nullptr, nullptr, gW1, d, nullptr, 0, nullptr, part};
    SC_HIP(sc::launch_gemm(gw1, f32, st), fn);
    SC_HIP(sc::launch_colsum(da1, B, H, H, gb1, f32, st), fn);
    if (grads_out)
        SC_HIP(hipMemcpyAsync(grads_out, p->grads, sizeof(float) * (size_t)p->nparams, hipMemcpyDeviceToDevice, st), fn);
    if (loss_out) SC_HIP(hipMemcpyAsync(loss_out, loss, sizeof(float), hipMemcpyDeviceToDevice, st), fn);
    if (!(flags & SC_TRAIN_GRAD_ONLY)) {
        p->step += 1;
        const double bc1 = 1.0 - pow((double)beta1, (double)p->step);
        const double bc2 = 1.0 - pow((double)beta2, (double)p->step);
        const float lr_t = (float)(lr * sqrt(bc2) / bc1);
        const float eps_hat = (float)(adam_eps * sqrt(bc2));
        SC_HIP(sc::launch_adam(p->params, p->m, p->v, p->grads, p->nparams, lr_t, beta1, beta2, eps_hat, st), fn);
        SC_HIP(sc::launch_proposer_pack(p->params, d, H, K, p->W1b, p->W2b, p->W3b, p->W2bT, p->W3bT, p->W1o, p->W2o,
                                        p->W3o, st),
               fn);
    }
    return SC_OK;
}

}  // extern "C"
