// C-ABI entry points: argument validation, handle ownership, launches.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>

#include "sc_internal.h"

namespace {

thread_local char g_last_error[512] = "";

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
    hipFree(h->status);
    hipFree(h->stats);
    delete h;
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
    bool ok = hipMalloc(&h->D, sizeof(float) * (size_t)K * d) == hipSuccess &&
              hipMalloc(&h->DT, sizeof(float) * (size_t)d * Kp) == hipSuccess &&
              hipMalloc(&h->G, sizeof(float) * (size_t)K * Kp) == hipSuccess &&
              hipMalloc(&h->Dbf, sizeof(uint16_t) * (size_t)Kp * 64) == hipSuccess &&
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
    if ((e = sc::launch_dict_layouts(h->D, d, K, Kp, h->DT, h->Dbf, st)) != hipSuccess ||
        (e = sc::launch_gram(h->D, d, K, Kp, h->G, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess) {
        free_dict(h);
        return set_dev_error("sc_gram_precompute", e);
    }
    h->dev = sc::DictDev{d, K, Kp, E, h->D, h->DT, h->G, h->Dbf};
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
    sc::OmpParams p{X, N, k, eps, (flags & SC_EPS_RELATIVE) ? 1 : 0, (flags & SC_NO_FP64_REFIT) ? 0 : 1, 1e3f,
                    idx, coef, count, resid, h->stats};
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = sc::launch_omp_fp32(h->dev, p, kmax, st);
    if (e == hipErrorInvalidValue) {
        snprintf(g_last_error, sizeof(g_last_error), "no compiled encoder for K=%d (Kp=%d) with k=%d", K,
                 h->dev.Kp, k);
        return SC_EINVAL;
    }
    if (e != hipSuccess) return set_dev_error("sc_omp_encode", e);
    return SC_OK;
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

}  // extern "C"
