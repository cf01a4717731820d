/*
 * sc.h -- C ABI of the MI355X (gfx950) sparse-coding hot path for
 * post-training 3DGS compression ("Smaller and Faster 3DGS via Post-Training
 * Dictionary Learning").
 *
 * The paper compresses each Gaussian's 45 view-dependent SH coefficients
 * (the 48 SH values minus the 3 DC terms, Sec. 2.2) into a sparse code over a
 * shared dictionary D of unit-norm atoms (Eq. (1)), found by Orthogonal
 * Matching Pursuit that stops at sparsity k and/or residual tolerance eps
 * (Sec. 2.1), and renders radiance directly from the codes (Sec. 2.2,
 * Eq. (2)-(3)).  This library exposes that path:
 *
 *   sc_gram_precompute   dictionary set-up: checks, layouts, Gram matrix
 *   sc_omp_encode        OMP of N signals (Batch-OMP on the GPU)
 *   sc_sh_eval_sparse    radiance straight from (index, coefficient) codes
 * and three additions around it: a learned support proposer (sc_proposer_*,
 * sc_omp_encode_learned), a BF16/FP32/FP64 precision policy (flags of
 * sc_omp_encode) and a batched persistent launch over many dictionaries
 * (sc_omp_encode_batched).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Every array argument is a DEVICE pointer owned by the caller; the
 *    library never frees it.  Handles own their own device memory.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Every call is
 *    stream-ordered and asynchronous unless its comment says it synchronises.
 *  - Return value: SC_OK (0) or a negative SC_E* code.  Argument errors are
 *    detected on the host before any device work, so the outputs are then
 *    untouched.  SC_EDEVICE means a HIP call failed; sc_last_error() gives
 *    the HIP message.
 *  - Layouts (row-major, 0-based):
 *      D     K x d float32, atom-major: the paper's d x K matrix stored column
 *            by column, each atom's d values contiguous.
 *      X     N x d float32, one Gaussian per row, channel-major
 *            [R_1..R_15, G_1..G_15, B_1..B_15] for d = 45.
 *      idx   N x k int32, selected atoms in selection order, -1 padded.
 *      coef  N x k float32, the least-squares coefficients, 0 padded.
 *      count N int32, number of atoms used; -1 for a signal with a
 *            non-finite entry (a per-signal status, not a call failure).
 *      resid N float32, explicit ||x - D_I coef||_2 (NaN when count = -1).
 *  - Limits: 1 <= d <= 64, 1 <= K <= 1024, 1 <= k <= min(K, d, 32).
 */
#ifndef SC_H
#define SC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---- */
#define SC_OK          0
#define SC_EINVAL     -1   /* null pointer, bad size or range, unknown flag      */
#define SC_ENORM      -2   /* an atom with | ||a_j|| - 1 | > 1e-4 (Eq. (1))       */
#define SC_ENONFINITE -3   /* NaN/Inf in the dictionary or the proposer weights  */
#define SC_EDEVICE    -4   /* a HIP runtime call or kernel launch failed         */
#define SC_ENOMEM     -5   /* device allocation failed, or workspace too small   */
#define SC_ENODEV     -6   /* no usable gfx950 device                            */

/* ---- flags ---- */
#define SC_EPS_RELATIVE  0x1  /* stop when ||r|| <= eps * ||x|| instead of eps     */
#define SC_PREC_BF16     0x2  /* correlations on BF16 MFMA (FP32 otherwise)        */
#define SC_NO_FP64_REFIT 0x4  /* never refit ill-conditioned supports in FP64      */
#define SC_NORMALIZE     0x8  /* sc_gram_precompute: scale atoms to unit norm
                                 instead of rejecting them                         */

/* ---- radiance direction modes ---- */
#define SC_DIRS_PER_SIGNAL 0  /* dirs is N x 3, rgb is N x 3                      */
#define SC_DIRS_SHARED     1  /* dirs is M x 3 for every signal, rgb N x M x 3    */

typedef struct sc_dict_s *sc_dict;
typedef struct sc_proposer_s *sc_proposer;

/* Human-readable text of an error code (static storage). */
const char *sc_strerror(int code);
/* Message of the last SC_EDEVICE failure on this thread (static storage). */
const char *sc_last_error(void);

/*
 * sc_gram_precompute -- set up a dictionary D for encoding and rendering.
 *
 * Sec. 2.1 (Eq. (1)) requires unit-norm atoms; Batch-OMP precomputes the
 * Gram matrix G = D^T D (K x K) once per dictionary.  The handle keeps, in
 * device memory it owns: a copy of D (FP32), D feature-major and padded for
 * the correlation stage, D in BF16 for MFMA, and G in FP32.
 *
 *   D      device, K x d float32 atom-major (caller-owned, read only here)
 *   d, K   1 <= d <= 64, 1 <= K <= 1024
 *   flags  0 or SC_NORMALIZE
 *   out    receives the new handle (set only on success)
 *
 * Checks every atom (finite, unit norm within 1e-4 unless SC_NORMALIZE); this
 * reads a status word back, so the call SYNCHRONISES with `stream`.
 * Errors: SC_EINVAL, SC_ENONFINITE, SC_ENORM, SC_ENOMEM, SC_EDEVICE, SC_ENODEV.
 */
int sc_gram_precompute(const float *D, int d, int K, int flags, void *stream, sc_dict *out);

/* Release a dictionary handle (waits for the device).  NULL is accepted. */
int sc_dict_destroy(sc_dict h);

/* Dimensions of a dictionary handle. */
int sc_dict_dims(sc_dict h, int *d, int *K);

/* Copy the handle's FP32 Gram matrix G = D^T D into G_out (device, K x K
 * row-major, caller-owned).  Stream-ordered.  For inspection and tests. */
int sc_dict_gram(sc_dict h, float *G_out, void *stream);

/*
 * sc_omp_encode -- sparse-code N signals with OMP (Sec. 2.1).
 *
 * Greedy selection of the atom with the largest |correlation| to the
 * residual (ties to the lowest index, selected atoms excluded), least-squares
 * coefficients on the selected atoms, stop before a selection when the
 * residual norm is <= eps (or eps*||x|| with SC_EPS_RELATIVE) or k atoms are
 * in use.  eps = 0 means "k atoms".  The GPU runs Batch-OMP: correlations
 * alpha0 = D^T x once; per step the Gram-column update
 * alpha = alpha0 - G_I gamma, the selection, and one new row of the inverse
 * Cholesky factor L^-1 of G_II (G_II = L L^T), from which the least-squares
 * coefficients gamma = L^-T L^-1 D_I^T x and the residual norm are updated
 * in place.
 *
 * Precision (flags): FP32 throughout by default.  SC_PREC_BF16 forms
 * alpha0 = D^T x on BF16 matrix cores with FP32 accumulation: D and x are
 * each split into three BF16 parts (every part the rounding of what the
 * previous ones leave) and the six products of scale >= 2^-16 are summed in
 * FP32 (Dm xm + Dl xh + Dh xl + Dm xh + Dh xm + Dh xh).  The products left
 * out and the parts' own rounding add <= 4 * 2^-27 ||x|| per unit atom, so
 * the correlations have the accuracy of FP32 dot products, at half the
 * matrix-core time of FP32 operands (32-signal tiles on eight waves when
 * 64 < K <= 512, else 16-signal tiles).  The Gram-form update, the factor,
 * the stop test and the coefficients are FP32 as in the default path.
 * Supports whose Cholesky condition estimate (max l_ii / min l_ii)^2 exceeds
 * 1e3 are refit in FP64 unless SC_NO_FP64_REFIT.
 *
 *   X      device N x d float32          idx   device N x k int32 (out)
 *   N      >= 0 (0: no device work, the  coef  device N x k float32 (out)
 *          arrays may then be NULL)
 *   k      1 <= k <= min(K, d, 32)       count device N int32 (out)
 *   eps    >= 0, finite                  resid device N float32 (out, may be NULL)
 * Errors: SC_EINVAL, SC_EDEVICE.
 */
int sc_omp_encode(sc_dict h, const float *X, int64_t N, int k, float eps, int flags, int32_t *idx,
                  float *coef, int32_t *count, float *resid, void *stream);

/*
 * Tuning of a dictionary handle (chosen by the autotuner; results do not
 * depend on it beyond FP32 rounding order):
 *   SC_TUNE_FP32_CORRELATION  how the FP32 encoder computes alpha0 = D^T x for
 *     a tile of signals: SC_CORR_VALU (FP32 FMAs over 16-signal tiles,
 *     default) or SC_CORR_MFMA (FP32 matrix cores; 32-signal tiles on eight
 *     waves when 64 < K <= 512, else 16-signal tiles).
 *   SC_TUNE_ROW_CACHE  Gram rows of the first selected atoms kept in
 *     registers by the encoder: 0 (default for K > 256: every row re-read
 *     from cache memory when the correlations are formed) or 4 (applies to
 *     K <= 512 here; the batched encoder has its own row_cache setting, see
 *     sc_batch_tuning).
 *   SC_TUNE_ROW_CACHE_BF16  the same choice for the split-BF16 form
 *     (SC_PREC_BF16), whose encoder holds more registers, so its best value
 *     can differ.
 *   SC_TUNE_RESTRICTED_CAP  at most this many restricted-OMP steps in
 *     sc_omp_encode_learned / _restricted (0 = k, default).  A signal whose
 *     candidate code is still above eps after the cap goes to the full-OMP
 *     fallback, so every code still meets the tolerance; only the split of
 *     signals between the two paths (and the speed) changes.
 */
#define SC_TUNE_FP32_CORRELATION 1
#define SC_TUNE_ROW_CACHE 2
#define SC_TUNE_RESTRICTED_CAP 3
#define SC_TUNE_ROW_CACHE_BF16 4
#define SC_CORR_VALU 0
#define SC_CORR_MFMA 1
int sc_dict_set_tuning(sc_dict h, int key, int value);
int sc_dict_get_tuning(sc_dict h, int key, int *value);

/*
 * sc_omp_stats -- counters accumulated by the encoders of this handle since
 * the last reset: stats[0] = signals encoded, stats[1] = total atoms
 * selected, stats[2] = supports refit in FP64, stats[3] = signals sent to the
 * full-OMP fallback by sc_omp_encode_learned.  Synchronises with `stream`
 * when reading; reset = 1 clears them afterwards.
 */
int sc_omp_stats(sc_dict h, int64_t stats[4], int reset, void *stream);

/*
 * sc_sh_eval_sparse -- view-dependent radiance from sparse codes (Sec. 2.2).
 *
 * For each signal and view direction w:
 *   rgb_c(w) = sum_{t < count} coef_t * sum_{j=1..nb} D[idx_t][c*nb + j] * Y_j(w)
 * with Y_j the real SH basis of degree 1..L (Condon-Shortley phase, m = -l..l
 * within each band l), nb = (L+1)^2 - 1 and d = 3 nb, so d in {9, 24, 45}.
 * Only the linear view-dependent part is returned (no DC term, offset or
 * clamp).  Signals with count < 0 give NaN.  Indices outside [0, K) are
 * skipped.
 *
 *   idx, coef   device N x k codes (as written by sc_omp_encode)
 *   count       device N int32
 *   dirs        device float32 unit vectors: N x 3 (SC_DIRS_PER_SIGNAL, M = N)
 *               or M x 3 (SC_DIRS_SHARED)
 *   rgb         device float32 out: N x 3 or N x M x 3
 * Errors: SC_EINVAL, SC_EDEVICE.
 */
int sc_sh_eval_sparse(sc_dict h, const int32_t *idx, const float *coef, const int32_t *count,
                      int64_t N, int k, const float *dirs, int64_t M, int dir_mode, float *rgb,
                      void *stream);

/* ------------------------------------------------------------------ */
/* Learned support proposer (an addition to the paper's method)         */
/* ------------------------------------------------------------------ */
/*
 * A small MLP proposes, for each signal, the candidate atoms among which OMP
 * is then run; the full OMP of Sec. 2.1 stays the fallback whenever the
 * restricted code's residual exceeds eps, so the result always meets the
 * paper's stop rule or equals the plain encoder's.  Network:
 *   xh = x / ||x|| (0 for x = 0),  h1 = GELU(W1 xh + b1),  h2 = GELU(W2 h1 + b2),
 *   z = W3 h2 + b3  (one logit per atom),  GELU(t) = t Phi(t) (exact, erf form),
 * BF16 weights and activations with FP32 accumulation on MFMA.
 * Parameters are one FP32 vector (the master copy), in this order:
 *   W1 (H x d row-major), b1 (H), W2 (H x H), b2 (H), W3 (K x H), b3 (K).
 * Supported shapes: d <= 48, H = 256, K in {128, 256, 512}.
 */

/* Number of FP32 parameters of a d -> H -> H -> K proposer (negative on bad sizes). */
int64_t sc_proposer_num_params(int d, int H, int K);

/* Create a proposer; parameters start at zero (set them before use).
 * Errors: SC_EINVAL, SC_ENOMEM, SC_ENODEV. */
int sc_proposer_create(int d, int H, int K, sc_proposer *out);

/* Release a proposer (waits for the device).  NULL is accepted. */
int sc_proposer_destroy(sc_proposer p);

/* Dimensions and parameter count of a proposer. */
int sc_proposer_dims(sc_proposer p, int *d, int *H, int *K, int64_t *nparams);

/* Copy nparams FP32 parameters from device memory into the proposer, refresh
 * its BF16 copies and reset the optimiser state.  Stream-ordered. */
int sc_proposer_set_params(sc_proposer p, const float *params, void *stream);

/* Copy the FP32 master parameters out to device memory.  Stream-ordered. */
int sc_proposer_get_params(sc_proposer p, float *params, void *stream);

/*
 * sc_proposer_forward -- candidates of N signals.
 *   X       device N x d float32
 *   n_cand  1 <= n_cand <= min(32, K)
 *   cand    device N x n_cand int32 out: the n_cand atoms with the largest
 *           logits (ties to the lower index), listed in increasing atom
 *           index; a row of -1 when the input is not finite or when more than
 *           64 logits tie at the selection threshold (no candidates: the
 *           learned encoder then uses the full OMP for that signal)
 *   logits  device N x K float32 out, or NULL (the FP32 logits, for tests)
 */
int sc_proposer_forward(sc_proposer p, const float *X, int64_t N, int n_cand, int32_t *cand, float *logits,
                        void *stream);

/* Bytes of device workspace sc_omp_encode_learned needs for N signals. */
size_t sc_omp_encode_learned_workspace(int64_t N, int n_cand);

/*
 * sc_omp_encode_learned -- proposer-guided OMP with the full OMP as fallback.
 *
 * 1. candidates = the proposer's n_cand largest logits per signal;
 * 2. Batch-OMP restricted to the candidates, same stop rule as sc_omp_encode;
 * 3. explicit FP32 residual ||x - D_I coef||: accepted if <= eps (or
 *    eps ||x|| with SC_EPS_RELATIVE), else the signal is re-encoded by the
 *    plain FP32 encoder of sc_omp_encode (counted in sc_omp_stats[3]).
 * Outputs and per-signal status as sc_omp_encode.  eps = 0 sends every
 * signal that is not represented exactly to the fallback.
 *   k        1 <= k <= min(K, d, 16);  n_cand: k <= n_cand <= min(32, K)
 *   flags    SC_EPS_RELATIVE, SC_NO_FP64_REFIT, SC_PREC_BF16 (the fallback
 *            encoder then runs in the BF16 precision form)
 *   workspace  device, >= sc_omp_encode_learned_workspace(N, n_cand) bytes,
 *              caller-owned, contents overwritten
 * Requires the proposer's d and K to match the dictionary, d <= 48.
 * Errors: SC_EINVAL, SC_ENOMEM (workspace too small), SC_EDEVICE.
 */
int sc_omp_encode_learned(sc_dict h, sc_proposer p, const float *X, int64_t N, int k, float eps, int flags,
                          int n_cand, int32_t *idx, float *coef, int32_t *count, float *resid, void *workspace,
                          size_t ws_bytes, void *stream);

/*
 * sc_omp_encode_learned_noalloc -- sc_omp_encode_learned for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same computation, with the
 * library's static device scratch in place of the caller's workspace.
 *
 * The scratch is one array of SC_STATIC_SCRATCH_BYTES per GPU, held until the
 * process ends and shared by every call on that GPU, so calls that overlap in
 * time on one GPU (on different streams, or from different threads) race and
 * must be serialised by the caller.  Each call clears what must start at zero.
 *   N, n_cand  sc_omp_encode_learned_workspace(N, n_cand) must not exceed
 *              SC_STATIC_SCRATCH_BYTES (N <= 335,541 at n_cand = 24);
 *              larger sizes return SC_ENOMEM before any device work, with the
 *              sizes in sc_last_error()
 *   h          must live on the current device (SC_EINVAL otherwise)
 * Other arguments, outputs and errors as sc_omp_encode_learned.  No
 * hipMalloc, hipFree or allocating library call is made.
 */
#define SC_STATIC_SCRATCH_BYTES (32u << 20)
int sc_omp_encode_learned_noalloc(sc_dict h, sc_proposer p, const float *X, int64_t N, int k, float eps, int flags,
                                  int n_cand, int32_t *idx, float *coef, int32_t *count, float *resid,
                                  void *stream);

/*
 * sc_screen_topk -- correlation screening, the proposer-free baseline of the
 * learned encoder: for each signal the n_cand atoms of largest |<a_j, x>|
 * (one BF16 MFMA product with the dictionary, FP32 accumulation; exact
 * top-n_cand of those values, ties to the lower index), written as sc_
 * proposer_forward writes them (sorted by atom index, -1 row for a signal
 * that is not finite).  Feed the list to sc_omp_encode_restricted and
 * sc_omp_encode_rows to run the screened encoder.
 *   K in {128, 256, 512}, d <= 64, 1 <= n_cand <= min(32, K)
 *   cand  device N x n_cand int32 (out)
 * Errors: SC_EINVAL, SC_EDEVICE.
 */
int sc_screen_topk(sc_dict h, const float *X, int64_t N, int n_cand, int32_t *cand, void *stream);

/*
 * sc_omp_encode_restricted -- step 2 and 3 of sc_omp_encode_learned on their
 * own: Batch-OMP of each signal restricted to its candidate atoms (cand,
 * N x n_cand, sorted by atom index, a row starting with -1 = no candidates),
 * explicit-residual acceptance.  A candidate entry outside [0, K) is read as
 * -1 (no candidate), so a row whose first entry is out of range takes the
 * fallback like a row of -1.  Accepted codes are written to idx/coef/
 * count/resid, the other signals' indices are appended to miss_rows
 * (device int32[N]) and counted in *miss_count (device int32, zeroed by the
 * call).  The order of miss_rows varies from call to call (rows are appended
 * as workgroups finish); the set does not.  The restricted pursuit takes at
 * most the handle's restricted-step cap (SC_TUNE_RESTRICTED_CAP, 0 = k)
 * steps.  Same limits as sc_omp_encode_learned.
 */
int sc_omp_encode_restricted(sc_dict h, const float *X, int64_t N, int k, float eps, int flags, const int32_t *cand,
                             int n_cand, int32_t *idx, float *coef, int32_t *count, float *resid, int32_t *miss_rows,
                             int32_t *miss_count, void *stream);

/*
 * sc_omp_encode_rows -- the plain FP32 encoder of sc_omp_encode applied to
 * the rows listed in rows[0 .. *nrows) of X (nrows is a DEVICE int32, read by
 * the kernel, so the list can come from sc_omp_encode_restricted without a
 * host round trip); outputs are written at those rows.  max_rows bounds
 * *nrows (it sizes the launch), and the call requires max_rows <= the number
 * of rows of X (it is the number of rows whose outputs may be written).  A
 * list entry outside [0, max_rows) is skipped (nothing is read or written
 * for it).
 */
int sc_omp_encode_rows(sc_dict h, const float *X, const int32_t *rows, const int32_t *nrows, int64_t max_rows, int k,
                       float eps, int flags, int32_t *idx, float *coef, int32_t *count, float *resid, void *stream);

/* ---- proposer training ---- */
#define SC_TRAIN_FP32      0x1  /* FP32 operands on FP32 MFMA (gradient checks); BF16 otherwise */
#define SC_TRAIN_GRAD_ONLY 0x2  /* compute the gradients, do not update the parameters        */

/* Bytes of device workspace one training step with batch B needs. */
size_t sc_proposer_train_workspace(sc_proposer p, int64_t B);

/*
 * sc_proposer_train_step -- one Adam step on a batch of (signal, OMP support)
 * pairs.
 *
 * Loss: the mean over the B x K entries of the binary cross-entropy on
 * logits, w y softplus(-z) + (1 - y) softplus(z), with y the multi-hot
 * indicator of the signal's support (the atoms OMP selected) and w =
 * pos_weight.  Backpropagation through the three layers (GELU' exact), then
 * Adam with bias correction (step counter kept in the handle, reset by
 * sc_proposer_set_params), then the BF16 copies are refreshed.
 *
 *   X          device N x d float32 training signals
 *   rows       device int32[B]: the batch is X[rows[b]] (NULL: rows 0..B-1)
 *   B          batch size, a positive multiple of 32
 *   sup_idx    device N x kcap int32 supports (as written by sc_omp_encode)
 *   sup_count  device int32[N] support sizes (entries < 0 count as empty)
 *   lr, beta1, beta2, adam_eps   Adam hyper-parameters
 *   flags      SC_TRAIN_FP32, SC_TRAIN_GRAD_ONLY
 *   loss_out   device float, or NULL: the batch loss (before the update)
 *   grads_out  device float[nparams], or NULL: the gradient (parameter order)
 *   workspace  device, >= sc_proposer_train_workspace(p, B) bytes
 * Stream-ordered; no allocation.
 * Errors: SC_EINVAL, SC_ENOMEM (workspace too small), SC_EDEVICE.
 */
int sc_proposer_train_step(sc_proposer p, const float *X, const int32_t *rows, int64_t B, const int32_t *sup_idx,
                           const int32_t *sup_count, int kcap, float lr, float beta1, float beta2, float adam_eps,
                           float pos_weight, int flags, float *loss_out, float *grads_out, void *workspace,
                           size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------ */
/* Dictionary learning (Sec. 2.1)                                       */
/* ------------------------------------------------------------------ */

/*
 * sc_mod_update -- the dictionary half of the alternating minimisation of
 * Eq. (1) (Sec. 2.1), with the codes fixed: the Method of Optimal Directions
 *   D = X A^T (A A^T + ridge I)^-1,  ridge = 1e-10 tr(A A^T) / K,
 * where A (K x N) holds the codes idx/coef/count (as sc_omp_encode writes
 * them; count < 0 counts as no atom).  Products are accumulated and solved in
 * FP64.  Atoms no signal uses (or whose solution vanishes) are replaced by
 * the signals with the largest resid (ties to the lower signal index), then
 * every atom is scaled to unit norm.  Alternate with sc_gram_precompute +
 * sc_omp_encode for the full learning loop.
 *   X          device N x d float32 training signals (N >= 1, d <= 64)
 *   K          atoms (<= 1024); k: code width (<= 32)
 *   resid      device float32[N], the codes' residual norms
 *   D_out      device K x d float32 (out), atom-major, unit-norm atoms
 *   n_replaced host int (out, may be NULL): atoms replaced
 *   workspace  device, >= sc_mod_workspace(d, K) bytes
 * Synchronises `stream` once (to read the number of unused atoms).
 * Errors: SC_EINVAL, SC_ENOMEM (workspace too small), SC_ENODEV, SC_EDEVICE.
 */
size_t sc_mod_workspace(int d, int K);
int sc_mod_update(const float *X, int64_t N, int d, int K, const int32_t *idx, const float *coef,
                  const int32_t *count, int k, const float *resid, float *D_out, int *n_replaced, void *workspace,
                  size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------ */
/* CSC storage of the codes (Sec. 2.2) and its consumers                */
/* ------------------------------------------------------------------ */

/*
 * The paper stores each Gaussian's non-zero coefficients and their atom
 * indices in Compressed-Sparse-Column form, since the codes differ in length
 * (Sec. 2.2).  Column i (Gaussian i) is rows/vals[colptr[i] .. colptr[i+1]),
 * in selection order; a code with count <= 0 (including status -1) is an
 * empty column.
 *
 * sc_csc_colptr -- colptr[i] = sum_{g<i} max(count[g], 0) for i = 0..N
 * (device int64[N+1]; colptr[N] = number of non-zeros).  workspace: device,
 * >= sc_csc_workspace(N) bytes.  Read colptr[N] (stream-ordered) to size
 * rows/vals before sc_csc_fill.
 * sc_csc_fill -- scatters idx/coef (N x k, padded, as sc_omp_encode writes
 * them) into rows (int32) / vals (float32) at colptr.
 * Errors: SC_EINVAL, SC_ENOMEM (workspace too small), SC_EDEVICE.
 */
size_t sc_csc_workspace(int64_t N);
int sc_csc_colptr(const int32_t *count, int64_t N, int64_t *colptr, void *workspace, size_t ws_bytes, void *stream);
int sc_csc_fill(const int32_t *idx, const float *coef, const int32_t *count, int64_t N, int k, const int64_t *colptr,
                int32_t *rows, float *vals, void *stream);

/*
 * sc_omp_encode_csc -- the tolerance-controlled encoder writing CSC (Sec. 2.2
 * with the eps-controlled sparsity of Sec. 3.2) in one pass: no padded
 * N x k codes exist anywhere.  Workgroups take 16-signal tiles in increasing
 * order, encode them (same pursuit and results as sc_omp_encode), and find
 * each tile's column offset from the counts of the tiles before it; the
 * columns are written straight to colptr (device int64[N+1]) / rows / vals,
 * in selection order.  Supports refit in FP64 (unless SC_NO_FP64_REFIT) get
 * their coefficients solved again in place by a second pass.
 *   cap       capacity of rows / vals (entries); they may be NULL when cap = 0
 *   *nnz_out  (host) the number of non-zeros.  If it exceeds cap the call
 *             returns SC_ENOMEM after writing colptr completely (rows / vals
 *             hold the entries below cap), so the caller can size the arrays
 *             (cap = N * k always suffices) and call again.
 *   resid     device float32[N] or NULL
 *   workspace device, >= sc_omp_encode_csc_workspace(N, k) bytes (8 bytes per
 *             16 signals, plus 256); calls sharing it must not overlap
 *   flags     SC_EPS_RELATIVE, SC_PREC_BF16, SC_NO_FP64_REFIT
 * Synchronises `stream` once (to read the non-zero count).  Errors: SC_EINVAL,
 * SC_ENOMEM, SC_EDEVICE (including a column-offset wait that exceeded its
 * bound, reported in sc_last_error()).
 */
size_t sc_omp_encode_csc_workspace(int64_t N, int k);
int sc_omp_encode_csc(sc_dict h, const float *X, int64_t N, int k, float eps, int flags, int64_t *colptr,
                      int32_t *rows, float *vals, int64_t cap, int64_t *nnz_out, float *resid, void *workspace,
                      size_t ws_bytes, void *stream);

/*
 * sc_sh_eval_csc -- sc_sh_eval_sparse for codes in CSC form (same sum,
 * same directions and layouts; an empty column gives rgb = 0).
 */
int sc_sh_eval_csc(sc_dict h, const int64_t *colptr, const int32_t *rows, const float *vals, int64_t N,
                   const float *dirs, int64_t M, int dir_mode, float *rgb, void *stream);

/*
 * sc_gaussian_rgb_csc -- the renderer's per-Gaussian colour with the
 * compressed SH (Sec. 2.2, the step Eq. (2)-(3) model): view direction
 * w = (pos_i - cam) / ||pos_i - cam||, then
 *   rgb_c = max(0, C0 * dc_ic + sum_t vals_t sum_j D[c*nb + j, rows_t] Y_j(w) + 0.5),
 * C0 = 1 / (2 sqrt(pi)) (the degree-0 SH constant).
 *   pos, dc  device N x 3 float32 (Gaussian centres, DC SH coefficients)
 *   cam      HOST float[3], camera centre
 *   rgb      device N x 3 float32 (out)
 */
int sc_gaussian_rgb_csc(sc_dict h, const int64_t *colptr, const int32_t *rows, const float *vals, int64_t N,
                        const float *pos, const float *dc, const float cam[3], float *rgb, void *stream);

/* ------------------------------------------------------------------ */
/* Many scenes in one launch                                            */
/* ------------------------------------------------------------------ */

/*
 * Compression is applied per trained scene (Sec. 3: each scene has its own
 * learned dictionary), so a batch of scenes of uneven size, each with its
 * own dictionary D_s, sparsity cap k_s and tolerance eps_s, is encoded by one
 * persistent launch: every scene's codes are those sc_omp_encode(D_s, X_s,
 * k_s, eps_s, flags_s) returns (same support, coefficients up to FP32
 * rounding order).
 *
 * sc_scene: one scene.  dict: handle with K <= 512 on the current device;
 * X: device N x d float32; k: 1 <= k <= min(K, d, 16); eps >= 0 finite;
 * flags: SC_EPS_RELATIVE, SC_NO_FP64_REFIT; outputs as sc_omp_encode (resid
 * may be NULL; with N = 0 the pointers may be NULL).  Caller-owned.
 */
#define SC_MAX_SCENES 32
typedef struct {
    sc_dict dict;
    const float *X;
    int64_t N;
    int k;
    float eps;
    int flags;
    int32_t *idx;
    float *coef;
    int32_t *count;
    float *resid;
} sc_scene;

/*
 * sc_batch_tuning: launch shape of the batched encoder (results do not
 * depend on it beyond FP32 rounding order).
 *   tile       signals per workgroup tile: 16 or 32 (0 = 16)
 *   row_cache  Gram rows kept in registers: 0 or 4 (4 applies to the
 *              scenes with K <= 256; scenes of K > 256 keep 2 when k <= 12
 *              and re-read every row when k > 12, which keeps the merged
 *              kernel within 128 registers)
 *   wg_per_cu  persistent workgroups per compute unit, 0 = as many as fit
 *   order      SC_ORDER_COST: scenes taken most expensive tile first;
 *              SC_ORDER_GIVEN: in the order of the array
 *   corr       correlation stage of every scene: SC_CORR_VALU or SC_CORR_MFMA
 */
#define SC_ORDER_COST 0
#define SC_ORDER_GIVEN 1
typedef struct {
    int tile;
    int row_cache;
    int wg_per_cu;
    int order;
    int corr;
} sc_batch_tuning;

/* Device workspace bytes the batched encoder needs (a work counter). */
size_t sc_omp_encode_batched_workspace(void);

/*
 * sc_omp_encode_batched -- encode n_scenes (1..SC_MAX_SCENES) scenes in one
 * stream-ordered launch (plus an FP64-refit scan when a scene allows it).
 *   tuning     NULL: tile 16, row_cache 0, all workgroups that fit, cost
 *              order, VALU correlations
 *   workspace  device, >= sc_omp_encode_batched_workspace() bytes; calls
 *              sharing a workspace must not overlap in time
 * No allocation.  Errors: SC_EINVAL (a scene or the tuning out of range, or
 * dictionaries on different devices), SC_ENOMEM (workspace too small),
 * SC_EDEVICE.
 */
int sc_omp_encode_batched(const sc_scene *scenes, int n_scenes, const sc_batch_tuning *tuning, void *workspace,
                          size_t ws_bytes, void *stream);

/*
 * sc_batch_autotune -- the project's autotuner for sc_omp_encode_batched:
 * runs the batched encoder on the first min(N_s, sample) signals of every
 * scene (writing those outputs) and times each launch shape with HIP events
 * on `stream`: every combination of corr x tile x row_cache x wg_per_cu
 * (0, 1, 2) x order.  Writes the fastest shape to *best and its time (ms,
 * best of 2 after a warm-up launch) to *best_ms.  Synchronises the stream.
 * Errors: as sc_omp_encode_batched; sample must be >= 1.
 */
int sc_batch_autotune(const sc_scene *scenes, int n_scenes, int64_t sample, void *workspace, size_t ws_bytes,
                      sc_batch_tuning *best, float *best_ms, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SC_H */
