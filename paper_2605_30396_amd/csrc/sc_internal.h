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

struct DictDev {
    int d, K, Kp, E;
    const float *D;    // K x d atom-major FP32
    const float *DT;   // d x Kp feature-major FP32, zero padded atoms
    const float *G;    // K x Kp FP32 Gram rows, zero padded columns
    const uint16_t *Dbf;  // Kp x 64 BF16 atom-major, features and atoms zero padded
};

struct OmpParams {
    const float *X;
    int64_t N;
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

// Launchers (return hipError_t of the launch).
hipError_t launch_dict_check(const float *D, int d, int K, int normalize, float *Dcopy, int *status,
                             hipStream_t st);
hipError_t launch_dict_layouts(const float *Dcopy, int d, int K, int Kp, float *DT, uint16_t *Dbf,
                               hipStream_t st);
hipError_t launch_gram(const float *Dcopy, int d, int K, int Kp, float *G, hipStream_t st);
hipError_t launch_omp_fp32(const DictDev &dict, const OmpParams &p, int kmax, hipStream_t st);
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
    int *status = nullptr;
    unsigned long long *stats = nullptr;
};
