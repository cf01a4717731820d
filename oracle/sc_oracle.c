/*
 * FP64 CPU oracle for the sparse-coding hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * HIP path is checked against.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product library neither
 * links nor calls it, and it shares no code, header or table with the HIP
 * sources.
 *
 * What it computes, and where the paper defines it:
 *   orc_omp       Orthogonal Matching Pursuit (Sec. 2.1, the paragraph after
 *                 Eq. (1)): greedy atom selection by largest |<a_j, r>|,
 *                 least-squares refit of x on the selected atoms, stop when
 *                 the sparsity k is reached or the residual norm is within the
 *                 tolerance.  Written in its textbook residual form; the
 *                 least-squares step is a Householder QR solve recomputed from
 *                 scratch at every step (no Gram matrix, no Cholesky).
 *   orc_sh_basis  real spherical harmonics of degree 1..3 (the non-DC SH
 *                 functions whose coefficients Sec. 2.2 compresses), from the
 *                 associated Legendre functions with the Condon-Shortley
 *                 phase, ordered m = -l..l inside each band.
 *   orc_radiance  the view-dependent radiance of Sec. 2.2: reconstruct the
 *                 dense SH rest vector x = D_I gamma, then sum each channel's
 *                 15 coefficients against the SH basis at the view direction.
 *
 * Readings where the paper is silent (each is listed with its reason in the
 * design notes): eps bounds the absolute L2 residual (or eps*||x|| when
 * `relative` is set); the stop test runs before every selection, so a signal
 * with ||x|| <= eps gets no atom; argmax ties go to the lowest atom index;
 * selected atoms are excluded from later selection; a step whose best
 * correlation is <= 1e-14 ||x|| ends the pursuit (residual orthogonal to every
 * atom); a signal with a non-finite entry gets count -1, padded slots and a
 * NaN residual.
 *
 * Build: gcc -O2 -fPIC -shared -pthread sc_oracle.c -lm -o libsc_oracle.so
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------- least squares by Householder QR ---------------------- */

/* Solve min_g || x - A g ||_2 for A given as n columns of length d (each
 * column contiguous), n <= d.  W (d*n) and b (d) are scratch. Returns 0, or
 * -1 if a column is exactly dependent on the previous ones. */
static int lsq_householder(const double *A, int d, int n, const double *x, double *g,
                           double *W, double *b, double *rdiag)
{
    memcpy(W, A, sizeof(double) * (size_t)d * n);
    memcpy(b, x, sizeof(double) * d);
    for (int j = 0; j < n; ++j) {
        double *col = W + (size_t)j * d;
        double s = 0.0;
        for (int i = j; i < d; ++i) s += col[i] * col[i];
        double nrm = sqrt(s);
        if (nrm == 0.0) return -1;
        double alpha = col[j] > 0.0 ? -nrm : nrm;     /* avoids cancellation */
        double v0 = col[j] - alpha;
        double vtv = s - col[j] * col[j] + v0 * v0;   /* |v|^2, v = col - alpha e_j */
        col[j] = v0;
        for (int c = j + 1; c < n; ++c) {
            double *y = W + (size_t)c * d;
            double t = 0.0;
            for (int i = j; i < d; ++i) t += col[i] * y[i];
            double f = 2.0 * t / vtv;
            for (int i = j; i < d; ++i) y[i] -= f * col[i];
        }
        double t = 0.0;
        for (int i = j; i < d; ++i) t += col[i] * b[i];
        double f = 2.0 * t / vtv;
        for (int i = j; i < d; ++i) b[i] -= f * col[i];
        rdiag[j] = alpha;
    }
    /* R g = (Q^T x)[0..n): R[i][c] sits in W[c*d + i] above the diagonal */
    for (int i = n - 1; i >= 0; --i) {
        double s = b[i];
        for (int c = i + 1; c < n; ++c) s -= W[(size_t)c * d + i] * g[c];
        g[i] = s / rdiag[i];
    }
    return 0;
}

/* ---------------- OMP on one signal -------------------------------------- */

typedef struct {
    const double *D;      /* K x d, atom-major, fp64 copy */
    int d, K, k;
    double eps;
    int relative;
    const float *X;
    const int32_t *cand;  /* N x n_cand candidate atoms, or NULL for all */
    int n_cand;
    int32_t *idx;
    double *coef;
    int32_t *count;
    double *resid;
    double *margin;       /* optional: min over steps of (|c|_(1)-|c|_(2))/||r|| */
    double *rpath;        /* optional N x (k+1): ||r|| after 0..count atoms, NaN after */
    double *gap;          /* optional: min over steps of |c|_(1) - |c|_(2) (absolute) */
    double *mpath;        /* optional N x k: step t's (|c|_(1)-|c|_(2))/||r||, NaN past the end */
    double *gpath;        /* optional N x k: step t's |c|_(1) - |c|_(2), NaN past the end */
    int64_t lo, hi;
} omp_job;

static void omp_one(const omp_job *J, int64_t s, double *ws, unsigned char *used)
{
    const int d = J->d, k = J->k;
    double *x = ws, *r = x + d, *A = r + d, *W = A + (size_t)d * k, *b = W + (size_t)d * k;
    double *g = b + d, *rdiag = g + k;
    int32_t *I = (int32_t *)(rdiag + k);
    int32_t *oidx = J->idx + s * k;
    double *ocoef = J->coef + s * k;
    for (int t = 0; t < k; ++t) { oidx[t] = -1; ocoef[t] = 0.0; }

    int finite = 1;
    for (int i = 0; i < d; ++i) {
        x[i] = (double)J->X[s * d + i];
        if (!isfinite(x[i])) finite = 0;
    }
    double *path = J->rpath ? J->rpath + s * (k + 1) : NULL;
    if (path)
        for (int t = 0; t <= k; ++t) path[t] = NAN;
    double *mp = J->mpath ? J->mpath + s * k : NULL, *gp = J->gpath ? J->gpath + s * k : NULL;
    for (int t = 0; t < k; ++t) {
        if (mp) mp[t] = NAN;
        if (gp) gp[t] = NAN;
    }
    if (!finite) {
        J->count[s] = -1;
        J->resid[s] = NAN;
        if (J->margin) J->margin[s] = NAN;
        if (J->gap) J->gap[s] = NAN;
        return;
    }
    double xn = 0.0;
    for (int i = 0; i < d; ++i) xn += x[i] * x[i];
    xn = sqrt(xn);
    const double eps_abs = J->relative ? J->eps * xn : J->eps;
    const int32_t *cl = J->cand ? J->cand + s * J->n_cand : NULL;
    const int ncl = J->cand ? J->n_cand : J->K;

    memcpy(r, x, sizeof(double) * d);
    memset(used, 0, (size_t)J->K);
    int n = 0;
    double marg = INFINITY, gmin = INFINITY;
    for (;;) {
        double rn = 0.0;
        for (int i = 0; i < d; ++i) rn += r[i] * r[i];
        rn = sqrt(rn);
        if (path) path[n] = rn;
        if (n >= k || rn <= eps_abs) break;
        int best = -1;
        double bv = -1.0, sv = 0.0;
        for (int q = 0; q < ncl; ++q) {
            int j = cl ? cl[q] : q;
            if (j < 0 || j >= J->K || used[j]) continue;
            const double *a = J->D + (size_t)j * d;
            double c = 0.0;
            for (int i = 0; i < d; ++i) c += a[i] * r[i];
            c = fabs(c);
            if (c > bv || (c == bv && j < best)) {
                if (best >= 0) sv = bv > sv ? bv : sv;
                bv = c;
                best = j;
            } else if (c > sv) {
                sv = c;
            }
        }
        if (best < 0 || bv <= 1e-14 * xn) break;
        double m = (bv - sv) / rn;
        if (m < marg) marg = m;
        if (bv - sv < gmin) gmin = bv - sv;
        if (mp) mp[n] = m;
        if (gp) gp[n] = bv - sv;
        used[best] = 1;
        I[n] = best;
        memcpy(A + (size_t)n * d, J->D + (size_t)best * d, sizeof(double) * d);
        ++n;
        if (lsq_householder(A, d, n, x, g, W, b, rdiag) != 0) { --n; break; }
        for (int i = 0; i < d; ++i) {
            double v = x[i];
            for (int t = 0; t < n; ++t) v -= A[(size_t)t * d + i] * g[t];
            r[i] = v;
        }
    }
    /* final coefficients of the chosen support (recomputed: n may have
     * dropped back after a dependent atom) */
    if (n > 0) lsq_householder(A, d, n, x, g, W, b, rdiag);
    double rr = 0.0;
    for (int i = 0; i < d; ++i) {
        double v = x[i];
        for (int t = 0; t < n; ++t) v -= A[(size_t)t * d + i] * g[t];
        rr += v * v;
    }
    for (int t = 0; t < n; ++t) { oidx[t] = I[t]; ocoef[t] = g[t]; }
    J->count[s] = n;
    J->resid[s] = sqrt(rr);
    if (J->margin) J->margin[s] = marg;
    if (J->gap) J->gap[s] = gmin;
}

static void *omp_worker(void *arg)
{
    omp_job *J = (omp_job *)arg;
    const int d = J->d, k = J->k;
    size_t nws = (size_t)2 * d + 2 * (size_t)d * k + d + 2 * (size_t)k + (size_t)k;
    double *ws = (double *)malloc(sizeof(double) * (nws + 8));
    unsigned char *used = (unsigned char *)malloc((size_t)J->K);
    for (int64_t s = J->lo; s < J->hi; ++s) omp_one(J, s, ws, used);
    free(used);
    free(ws);
    return NULL;
}

/*
 * OMP over N signals.  D_atoms: K x d float32 (atom-major), X: N x d float32.
 * cand: optional N x n_cand int32 candidate lists (restricted pursuit over the
 * listed atoms only), NULL for the whole dictionary.
 * Outputs: idx N x k (selection order, -1 padded), coef N x k (0 padded),
 * count N, resid N (explicit ||x - D_I gamma||), margin N (optional, may be
 * NULL), rpath N x (k+1) (optional: the residual norm before each selection
 * and at the end, NaN past the end), gap N (optional: min over steps of the
 * absolute gap between the two largest |correlations|), mpath and gpath
 * N x k (optional: the relative margin and the absolute gap of each step,
 * NaN past the end).  Returns 0, or -1 on bad arguments.
 */
int orc_omp(const float *D_atoms, int d, int K, const float *X, int64_t N, int k, double eps,
            int relative, const int32_t *cand, int n_cand, int32_t *idx, double *coef,
            int32_t *count, double *resid, double *margin, double *rpath, double *gap,
            double *mpath, double *gpath, int nthreads)
{
    if (d <= 0 || K <= 0 || k <= 0 || k > d || N < 0 || !(eps >= 0.0)) return -1;
    if (cand && n_cand <= 0) return -1;
    double *Dd = (double *)malloc(sizeof(double) * (size_t)K * d);
    for (size_t i = 0; i < (size_t)K * d; ++i) Dd[i] = (double)D_atoms[i];
    if (nthreads < 1) nthreads = 1;
    if ((int64_t)nthreads > N) nthreads = N > 0 ? (int)N : 1;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * nthreads);
    omp_job *jobs = (omp_job *)malloc(sizeof(omp_job) * nthreads);
    for (int t = 0; t < nthreads; ++t) {
        omp_job J = {Dd, d, K, k, eps, relative, X, cand, n_cand, idx, coef, count, resid, margin,
                     rpath, gap, mpath, gpath, N * t / nthreads, N * (t + 1) / nthreads};
        jobs[t] = J;
        pthread_create(&th[t], NULL, omp_worker, &jobs[t]);
    }
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    free(jobs);
    free(th);
    free(Dd);
    return 0;
}

/* ---------------- real spherical harmonics ------------------------------ */

/* Associated Legendre P_l^m(t), m >= 0, with the Condon-Shortley phase
 * (-1)^m, by the standard three-term recurrence in l. */
static double legendre_p(int l, int m, double t)
{
    double somx2 = sqrt((1.0 - t) * (1.0 + t));
    double pmm = 1.0, fact = 1.0;
    for (int i = 1; i <= m; ++i) { pmm *= -fact * somx2; fact += 2.0; }
    if (l == m) return pmm;
    double pmmp1 = t * (2.0 * m + 1.0) * pmm;
    if (l == m + 1) return pmmp1;
    double pll = 0.0;
    for (int ll = m + 2; ll <= l; ++ll) {
        pll = ((2.0 * ll - 1.0) * t * pmmp1 - (ll + m - 1.0) * pmm) / (ll - m);
        pmm = pmmp1;
        pmmp1 = pll;
    }
    return pll;
}

static double factorial(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

/* Y[M x ((L+1)^2 - 1)]: for l = 1..L and m = -l..l,
 *   Y_lm = sqrt(2) K_l^|m| P_l^|m|(cos th) * (cos(m ph) if m > 0, sin(|m| ph) if m < 0)
 *   Y_l0 = K_l^0 P_l^0(cos th),  K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!).
 * dirs need not be normalised (the direction is what matters). */
void orc_sh_basis(const double *dirs, int64_t M, int L, double *Y)
{
    const int nb = (L + 1) * (L + 1) - 1;
    for (int64_t p = 0; p < M; ++p) {
        double x = dirs[3 * p], y = dirs[3 * p + 1], z = dirs[3 * p + 2];
        double rn = sqrt(x * x + y * y + z * z);
        double ct = z / rn;
        if (ct > 1.0) ct = 1.0;
        if (ct < -1.0) ct = -1.0;
        double ph = atan2(y, x);
        for (int l = 1; l <= L; ++l) {
            for (int m = -l; m <= l; ++m) {
                int am = m < 0 ? -m : m;
                double Kl = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * factorial(l - am) / factorial(l + am));
                double P = legendre_p(l, am, ct);
                double v;
                if (m > 0) v = sqrt(2.0) * Kl * P * cos(m * ph);
                else if (m < 0) v = sqrt(2.0) * Kl * P * sin(am * ph);
                else v = Kl * P;
                Y[p * nb + (l * l - 1) + (m + l)] = v;
            }
        }
    }
}

/* ---------------- radiance from sparse codes ---------------------------- */

/*
 * rgb_c(w) = sum_j Y_j(w) * xhat[c*nb + j],  xhat = sum_{t<count} coef_t a_{idx_t}.
 * d = 3 * nb, nb = (L+1)^2 - 1 with L in {1,2,3}.
 * shared_dirs = 0: one direction per signal (M == N), rgb N x 3.
 * shared_dirs = 1: M directions for every signal, rgb N x M x 3.
 * Signals with count < 0 get NaN radiance.  Returns 0 or -1.
 */
int orc_radiance(const float *D_atoms, int d, int K, const int32_t *idx, const float *coef,
                 const int32_t *count, int64_t N, int kcap, const float *dirs, int64_t M,
                 int shared_dirs, double *rgb)
{
    int nb = d / 3, L = 0;
    for (int l = 1; l <= 3; ++l)
        if ((l + 1) * (l + 1) - 1 == nb) L = l;
    if (d % 3 != 0 || L == 0) return -1;
    if (!shared_dirs && M != N) return -1;
    double *dd = (double *)malloc(sizeof(double) * 3 * (size_t)M);
    for (int64_t i = 0; i < 3 * M; ++i) dd[i] = (double)dirs[i];
    double *Y = (double *)malloc(sizeof(double) * (size_t)M * nb);
    orc_sh_basis(dd, M, L, Y);
    double *xh = (double *)malloc(sizeof(double) * d);
    for (int64_t s = 0; s < N; ++s) {
        int cnt = count[s];
        int64_t m0 = shared_dirs ? 0 : s, m1 = shared_dirs ? M : s + 1;
        if (cnt < 0) {
            for (int64_t m = m0; m < m1; ++m)
                for (int c = 0; c < 3; ++c)
                    rgb[(shared_dirs ? (s * M + m) : s) * 3 + c] = NAN;
            continue;
        }
        for (int i = 0; i < d; ++i) xh[i] = 0.0;
        for (int t = 0; t < cnt && t < kcap; ++t) {
            int j = idx[s * kcap + t];
            if (j < 0 || j >= K) continue;
            double cf = (double)coef[s * kcap + t];
            for (int i = 0; i < d; ++i) xh[i] += cf * (double)D_atoms[(size_t)j * d + i];
        }
        for (int64_t m = m0; m < m1; ++m) {
            const double *y = Y + m * nb;
            for (int c = 0; c < 3; ++c) {
                double v = 0.0;
                for (int j = 0; j < nb; ++j) v += y[j] * xh[c * nb + j];
                rgb[(shared_dirs ? (s * M + m) : s) * 3 + c] = v;
            }
        }
    }
    free(xh);
    free(Y);
    free(dd);
    return 0;
}
