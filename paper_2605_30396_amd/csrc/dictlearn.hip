// Dictionary update from fixed sparse codes (Sec. 2.1: Eq. (1) is minimised
// by alternating between the codes, from the encoder, and the dictionary).
// The dictionary step is the Method of Optimal Directions:
//
//   D = X A^T (A A^T + ridge I)^-1,   ridge = 1e-10 tr(A A^T) / K
//
// with A the K x N code matrix.  Both products are accumulated in FP64 from
// the padded codes (one wave per signal, FP64 atomics into L2), the K x K
// system is solved by an FP64 Cholesky factorisation in one workgroup, atoms
// that no signal uses are replaced by the worst-represented signals (largest
// residual first, ties to the lower signal index), and every atom is scaled
// to unit norm (the constraint of Eq. (1)).
#include <algorithm>

#include "sc_internal.h"

namespace sc {

struct ModWork {
    double *XAt;    // K x d   (row j: sum_i a_ji x_i)
    double *AAt;    // K x K, then its Cholesky factor (lower)
    double *Y;      // K x d   solution
    int *flags;     // K: 1 = atom unused
    int *nbad;      // count of unused atoms, then the list
    unsigned long long *key;   // argmax scratch
};

// XAt[j_t] += gamma_t x and AAt[j_t][j_u] += gamma_t gamma_u, accumulated in
// LDS: workgroup (b, s) owns rows [b R, b R + R) of both products (R (K + d)
// FP64 values, at most 64 KB) and the s-th slice of the signals.  One
// wave takes one signal at a time; only steps whose atom falls in the block
// touch LDS (FP64 LDS atomics), and the block is added to the global
// products once, at the end, so global atomics scale with the blocks rather
// than with the n (d + n) updates of every signal.
constexpr int kModLdsDoubles = 8192;   // 64 KB of FP64 per workgroup
__host__ __device__ inline int mod_rows(int K, int d) { return max(1, kModLdsDoubles / (K + d)); }

__global__ __launch_bounds__(1024) void mod_accum_kernel(const float *__restrict__ X, int64_t N, int d, int K,
                                                        const int32_t *__restrict__ idx,
                                                        const float *__restrict__ coef,
                                                        const int32_t *__restrict__ count, int k, int nslices,
                                                        ModWork w) {
    extern __shared__ __align__(16) double sAcc[];
    const int R = mod_rows(K, d);
    const int blk = blockIdx.x / nslices, slice = blockIdx.x - blk * nslices;
    const int r0 = blk * R, r1 = min(K, r0 + R), nr = r1 - r0;
    double *sA = sAcc;                 // nr x K
    double *sX = sAcc + (size_t)R * K; // nr x d
    for (int q = threadIdx.x; q < R * K + R * d; q += blockDim.x) sAcc[q] = 0.0;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t per = (N + nslices - 1) / nslices;
    const int64_t i0 = (int64_t)slice * per, i1 = min<int64_t>(N, i0 + per);
    for (int64_t i = i0 + (threadIdx.x >> 6); i < i1; i += blockDim.x >> 6) {
        int n = count[i];
        const int jr = lane < k ? idx[i * k + lane] : -1;   // issued with the count, not after it
        n = n < 0 ? 0 : (n > k ? k : n);
        const int jl = lane < n ? jr : -1;
        const bool mine = jl >= r0 && jl < r1;
        if (__ballot(mine) == 0) continue;   // no step of this signal falls in the block
        const double xv = lane < d ? (double)X[i * d + lane] : 0.0;
        const double gl = lane < n ? (double)coef[i * k + lane] : 0.0;
        const bool okl = jl >= 0 && jl < K;
        uint64_t own = __ballot(mine);
        while (own) {
            const int t = __ffsll((unsigned long long)own) - 1;
            own &= own - 1;
            const int jt = __shfl(jl, t, 64) - r0;
            const double gt = __shfl(gl, t, 64);
            if (lane < d) atomicAdd(&sX[(size_t)jt * d + lane], gt * xv);
            if (lane < n && okl) atomicAdd(&sA[(size_t)jt * K + jl], gt * gl);
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < nr * K; q += blockDim.x) {
        const double v = sA[q];
        if (v != 0.0) atomicAdd(&w.AAt[(size_t)r0 * K + q], v);
    }
    for (int q = threadIdx.x; q < nr * d; q += blockDim.x) {
        const double v = sX[q];
        if (v != 0.0) atomicAdd(&w.XAt[(size_t)r0 * d + q], v);
    }
}

__device__ __forceinline__ double block_sum_d(double v, double *red) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int q = 0; q < nw; ++q) s += red[q];
    return s;
}

// One workgroup: ridge, Cholesky of A A^T + ridge I, two triangular solves
// for the d right-hand sides, unused-atom flags.  YL: the right-hand sides
// are solved in LDS (K d <= kModSolveLds doubles), else in place in w.Y.
constexpr int kModSolveLds = 12288;   // 96 KB
template <bool YL>
__global__ __launch_bounds__(1024) void mod_solve_kernel(int d, int K, ModWork w) {
    extern __shared__ __align__(16) double sY[];
    __shared__ double red[16];
    __shared__ double diag_sh;
    double *A = w.AAt;
    // unused atoms and the trace
    double tr = 0.0;
    for (int j = threadIdx.x; j < K; j += blockDim.x) {
        const double a = A[(size_t)j * K + j];
        tr += a;
        w.flags[j] = a > 0.0 ? 0 : 1;
    }
    tr = block_sum_d(tr, red);
    const double ridge = 1e-10 * tr / K;
    for (int j = threadIdx.x; j < K; j += blockDim.x) A[(size_t)j * K + j] += ridge;
    __syncthreads();
    // right-looking Cholesky, A = L L^T in the lower triangle: for each column,
    // the pivot, the scaled column (also kept in LDS), then the trailing lower
    // triangle updated by 32 x 32 threads (thread rows over i, lanes over
    // consecutive c, so each row's update is one coalesced run)
    __shared__ double colj[1024];   // K <= 1024
    const int tr_i = threadIdx.x >> 5, tr_c = threadIdx.x & 31;
    for (int j = 0; j < K; ++j) {
        if (threadIdx.x == 0) {
            const double v = A[(size_t)j * K + j];
            diag_sh = sqrt(v > 1e-300 ? v : 1e-300);
            A[(size_t)j * K + j] = diag_sh;
        }
        __syncthreads();
        const double rl = 1.0 / diag_sh;
        for (int i = j + 1 + threadIdx.x; i < K; i += blockDim.x) {
            const double v = A[(size_t)i * K + j] * rl;
            A[(size_t)i * K + j] = v;
            colj[i] = v;
        }
        __syncthreads();
        for (int i = j + 1 + tr_i; i < K; i += 32) {
            const double li = colj[i];
            double *Ai = A + (size_t)i * K;
            for (int c = j + 1 + tr_c; c <= i; c += 32) Ai[c] -= li * colj[c];
        }
        __syncthreads();
    }
    // L Z = XAt, then L^T Y = Z, column-oriented: each step finishes one row of
    // the d right-hand sides (d <= 64: lane = right-hand side, the 16 waves
    // over rows) and updates the remaining rows in parallel
    double *Y = YL ? sY : w.Y;
    for (int q = threadIdx.x; q < K * d; q += blockDim.x) Y[q] = w.XAt[q];
    __syncthreads();
    const int sc_c = threadIdx.x & 63, sc_r = threadIdx.x >> 6, nrw = blockDim.x >> 6;
    for (int p = 0; p < K; ++p) {
        const double rl = 1.0 / A[(size_t)p * K + p];
        if (threadIdx.x < d) Y[(size_t)p * d + threadIdx.x] *= rl;
        __syncthreads();
        if (sc_c < d) {
            const double yp = Y[(size_t)p * d + sc_c];
            for (int i = p + 1 + sc_r; i < K; i += nrw) Y[(size_t)i * d + sc_c] -= A[(size_t)i * K + p] * yp;
        }
        __syncthreads();
    }
    for (int p = K - 1; p >= 0; --p) {
        const double rl = 1.0 / A[(size_t)p * K + p];
        if (threadIdx.x < d) Y[(size_t)p * d + threadIdx.x] *= rl;
        __syncthreads();
        if (sc_c < d) {
            const double yp = Y[(size_t)p * d + sc_c];
            for (int i = sc_r; i < p; i += nrw) Y[(size_t)i * d + sc_c] -= A[(size_t)p * K + i] * yp;
        }
        __syncthreads();
    }
    if (YL) {
        for (int q = threadIdx.x; q < K * d; q += blockDim.x) w.Y[q] = sY[q];
        __syncthreads();
    }
    // atoms with a vanishing solution count as unused too
    for (int j = threadIdx.x; j < K; j += blockDim.x) {
        double s = 0.0;
        for (int c = 0; c < d; ++c) s += Y[(size_t)j * d + c] * Y[(size_t)j * d + c];
        if (!(sqrt(s) > 1e-12)) w.flags[j] = 1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int nb = 0;
        for (int j = 0; j < K; ++j)
            if (w.flags[j]) w.nbad[1 + nb++] = j;
        w.nbad[0] = nb;
    }
}

// Largest residual with key below *prev (keys: residual order bits high,
// ~index low, so equal residuals resolve to the lower index).
__global__ __launch_bounds__(256) void mod_worst_kernel(const float *__restrict__ resid, int64_t N,
                                                        unsigned long long prev, unsigned long long *key) {
    unsigned long long best = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        const float r = resid[i];
        const uint32_t u = __float_as_uint(isfinite(r) ? r : 0.f);
        const uint32_t ok = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
        const unsigned long long kk = ((unsigned long long)ok << 32) | (0xFFFFFFFFull - (unsigned long long)i);
        if (kk < prev && kk > best) best = kk;
    }
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long o = __shfl_xor(best, off, 64);
        best = o > best ? o : best;
    }
    if ((threadIdx.x & 63) == 0 && best) atomicMax(key, best);
}

__global__ void mod_zero_key_kernel(unsigned long long *key) {
    if (threadIdx.x == 0) *key = 0;
}

// Row `slot` of the unused-atom list takes signal X[index of *key].
__global__ void mod_replace_kernel(const float *__restrict__ X, int d, int slot, ModWork w) {
    const int j = w.nbad[1 + slot];
    const int64_t i = (int64_t)(0xFFFFFFFFull - (*w.key & 0xFFFFFFFFull));
    for (int c = threadIdx.x; c < d; c += blockDim.x) w.Y[(size_t)j * d + c] = (double)X[i * d + c];
}

__global__ void mod_normalise_kernel(int d, int K, ModWork w, float *__restrict__ Dout) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= K) return;
    double s = 0.0;
    for (int c = 0; c < d; ++c) s += w.Y[(size_t)j * d + c] * w.Y[(size_t)j * d + c];
    const double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
    for (int c = 0; c < d; ++c) Dout[(size_t)j * d + c] = (float)(w.Y[(size_t)j * d + c] * inv);
}

static size_t al256(size_t v) { return (v + 255) / 256 * 256; }

size_t mod_workspace_bytes(int d, int K) {
    return al256(sizeof(double) * (size_t)K * d) * 2 + al256(sizeof(double) * (size_t)K * K) +
           al256(sizeof(int) * (size_t)K) + al256(sizeof(int) * (size_t)(K + 1)) + al256(sizeof(unsigned long long));
}

static ModWork mod_layout(void *ws, int d, int K) {
    unsigned char *p = (unsigned char *)ws;
    ModWork w;
    w.XAt = (double *)p;
    p += al256(sizeof(double) * (size_t)K * d);
    w.AAt = (double *)p;
    p += al256(sizeof(double) * (size_t)K * K);
    w.Y = (double *)p;
    p += al256(sizeof(double) * (size_t)K * d);
    w.flags = (int *)p;
    p += al256(sizeof(int) * (size_t)K);
    w.nbad = (int *)p;
    p += al256(sizeof(int) * (size_t)(K + 1));
    w.key = (unsigned long long *)p;
    return w;
}

// Stream-ordered except for one read of the unused-atom count.
hipError_t launch_mod_update(const float *X, int64_t N, int d, int K, const int32_t *idx, const float *coef,
                             const int32_t *count, int k, const float *resid, float *Dout, int *n_replaced, void *ws,
                             hipStream_t st) {
    ModWork w = mod_layout(ws, d, K);
    hipError_t e;
    if ((e = launch_zero_words(w.XAt, 2 * (int64_t)K * d, st)) != hipSuccess) return e;
    if ((e = launch_zero_words(w.AAt, 2 * (int64_t)K * K, st)) != hipSuccess) return e;
    int dev = 0, ncu = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    const int R = mod_rows(K, d), nblk = (K + R - 1) / R;
    const int nslices = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)ncu * 2 / nblk + 1, (N + 63) / 64));
    const size_t smem = sizeof(double) * ((size_t)R * K + (size_t)R * d);
    static bool attr = false;
    if (!attr) {
        if ((e = hipFuncSetAttribute((const void *)mod_accum_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)(sizeof(double) * kModLdsDoubles))) != hipSuccess)
            return e;
        attr = true;
    }
    hipLaunchKernelGGL(mod_accum_kernel, dim3((unsigned)(nblk * nslices)), dim3(1024), smem, st, X, N, d, K, idx,
                       coef, count, k, nslices, w);
    if (K * d <= kModSolveLds) {
        static bool sattr = false;
        if (!sattr) {
            if ((e = hipFuncSetAttribute((const void *)mod_solve_kernel<true>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)(sizeof(double) * kModSolveLds))) != hipSuccess)
                return e;
            sattr = true;
        }
        hipLaunchKernelGGL(mod_solve_kernel<true>, dim3(1), dim3(1024), sizeof(double) * (size_t)K * d, st, d, K, w);
    } else {
        hipLaunchKernelGGL(mod_solve_kernel<false>, dim3(1), dim3(1024), 0, st, d, K, w);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    int nb = 0;
    if ((e = hipMemcpyAsync(&nb, w.nbad, sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    unsigned long long prev = ~0ull;
    for (int s = 0; s < nb; ++s) {
        hipLaunchKernelGGL(mod_zero_key_kernel, dim3(1), dim3(64), 0, st, w.key);
        const int64_t g2 = std::max<int64_t>(1, std::min<int64_t>((N + 255) / 256, (int64_t)ncu * 4));
        hipLaunchKernelGGL(mod_worst_kernel, dim3((unsigned)g2), dim3(256), 0, st, resid, N, prev, w.key);
        hipLaunchKernelGGL(mod_replace_kernel, dim3(1), dim3(64), 0, st, X, d, s, w);
        if ((e = hipMemcpyAsync(&prev, w.key, sizeof(prev), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(mod_normalise_kernel, dim3((K + 255) / 256), dim3(256), 0, st, d, K, w, Dout);
    if (n_replaced) *n_replaced = nb;
    return hipGetLastError();
}

}  // namespace sc
