"""Shared helpers of the GPU parity tests: the comparison rules of the HIP
encoder against the FP64 oracle.

Where several results are correct (near-ties in the argmax, a stop decision
within rounding of eps, ill-conditioned supports), only what is unique is
compared exactly; the rest is checked for validity.  A selection step of the
oracle's FP64 run is "unique" when
  * it won by a relative margin (|c|_(1) - |c|_(2)) / ||r|| >= margin_min,
  * the residual before it does not lie within 1e-3 relative of eps, and
  * the atoms selected before it have a Gram submatrix of condition number
    <= 1e3.
A signal is "well separated" when all of its steps are unique: its support,
count and coefficients are compared.  On every signal, the selections up to
its first non-unique step are compared in order (the greedy choice is then
the same on both sides, step by step).

The same rule holds the BF16 precision form: its six-product split-BF16
correlations have the accuracy of FP32 dot products (error <= 4 * 2^-27
||x|| from the products left out, plus FP32 accumulation), far below the
margins compared.
"""
import numpy as np

import oracle

COEF_RTOL = 1e-4      # norm-wise per signal, on matched supports
RESID_AGG_RTOL = 1e-2


def unique_prefix(D, X, ref, eps, relative=False, margin_min=1e-3):
    """Number of leading selections of each signal that are unique (see the
    module docstring); 0 for signals with status -1."""
    N, k = ref["idx"].shape
    xn = np.linalg.norm(X.astype(np.float64), axis=1)
    with np.errstate(invalid="ignore"):
        ok = ref["mpath"] >= margin_min
        if eps > 0:
            tol = eps * xn if relative else np.full(N, eps)
            near = np.abs(ref["rpath"][:, :k] - tol[:, None]) <= 1e-3 * tol[:, None]
            ok &= ~np.nan_to_num(near, nan=False).astype(bool)
    cnt = np.maximum(ref["count"], 0)
    ok &= np.arange(k)[None, :] < cnt[:, None]
    m = np.where(ok.all(axis=1), k, np.argmin(ok, axis=1))
    m = np.minimum(m, cnt)
    Dd = D.astype(np.float64)
    for i in np.nonzero(m >= 3)[0]:
        S = ref["idx"][i, :m[i]]
        G = Dd[S] @ Dd[S].T
        for t in range(2, m[i]):   # step t is taken with the first t atoms selected
            if np.linalg.cond(G[:t, :t]) > 1e3:
                m[i] = t
                break
    return m


def well_separated(D, X, ref, eps, relative=False, margin_min=1e-3):
    k = ref["idx"].shape[1]
    sep = ref["margin"] > margin_min
    xn = np.linalg.norm(X.astype(np.float64), axis=1)
    tol = eps * xn if relative else np.full(len(X), eps)
    if eps > 0:
        rp = ref["rpath"]
        with np.errstate(invalid="ignore"):
            near = np.abs(rp - tol[:, None]) <= 1e-3 * tol[:, None]
        sep &= ~np.nan_to_num(near, nan=False).any(axis=1)
    Dd = D.astype(np.float64)
    for i in np.nonzero(sep)[0]:
        n = ref["count"][i]
        if n >= 2:
            S = ref["idx"][i, :n]
            if np.linalg.cond(Dd[S] @ Dd[S].T) > 1e3:
                sep[i] = False
    sep &= ref["count"] >= 0
    return sep


def oracle_run(D, X, k, eps, relative=False):
    return oracle.omp(D, X, k, eps, relative, with_margin=True, with_path=True)


def compare_codes(D, X, k, eps, gpu, ref=None, relative=False, margin_min=1e-3, min_sep_frac=0.5,
                  min_step_frac=0.5):
    """gpu: dict of numpy idx, coef, count, resid.  Asserts the parity bar and
    returns a dict of statistics.  min_sep_frac: least share of well-separated
    signals; min_step_frac: least share of all the oracle's selections that
    fall in unique prefixes (each of them is compared)."""
    if ref is None:
        ref = oracle_run(D, X, k, eps, relative)
    sep = well_separated(D, X, ref, eps, relative, margin_min)
    N = len(X)
    assert sep.sum() >= min_sep_frac * N, f"too few well-separated signals: {sep.sum()} of {N}"
    # selections in order, up to each signal's first non-unique step
    pre = unique_prefix(D, X, ref, eps, relative, margin_min)
    steps_total = int(np.maximum(ref["count"], 0).sum())
    steps_cmp = int(pre.sum())
    cols = np.arange(k)[None, :] < pre[:, None]
    diff = np.nonzero(np.any((gpu["idx"] != ref["idx"]) & cols, axis=1))[0]
    assert diff.size == 0, (f"{diff.size} signals select another atom within their unique prefix; first "
                            f"signal {diff[0]}: gpu {gpu['idx'][diff[0]]} oracle {ref['idx'][diff[0]]} "
                            f"prefix {pre[diff[0]]}")
    assert steps_cmp >= min_step_frac * steps_total, \
        f"too few unique selections compared: {steps_cmp} of {steps_total}"
    # per-signal status and padding are exact everywhere
    np.testing.assert_array_equal(gpu["count"] == -1, ref["count"] == -1)
    for i in range(0, N, max(1, N // 512)):
        n = gpu["count"][i]
        if n >= 0:
            assert np.all(gpu["idx"][i, n:] == -1) and np.all(gpu["coef"][i, n:] == 0)
    # supports: bit-exact, in selection order, on well-separated signals
    bad = np.nonzero(np.any(gpu["idx"][sep] != ref["idx"][sep], axis=1))[0]
    assert bad.size == 0, (f"{bad.size} support mismatches among {sep.sum()} separated signals; "
                           f"first signal {np.nonzero(sep)[0][bad[0]]}")
    np.testing.assert_array_equal(gpu["count"][sep], ref["count"][sep])
    # coefficients: 1e-4 relative, norm-wise
    gc = gpu["coef"][sep].astype(np.float64)
    rc = ref["coef"][sep]
    rn = np.linalg.norm(rc, axis=1)
    err = np.linalg.norm(gc - rc, axis=1) / np.where(rn > 0, rn, 1.0)
    assert err.max(initial=0) <= COEF_RTOL, f"coef rel err {err.max()}"
    # residual: aggregate within 1% over all valid signals, and the reported
    # residual equals ||x - D_I coef|| of the GPU's own code
    ok = ref["count"] >= 0
    agg_g = np.sqrt(np.sum(gpu["resid"][ok].astype(np.float64) ** 2))
    agg_r = np.sqrt(np.sum(ref["resid"][ok] ** 2))
    assert abs(agg_g - agg_r) <= RESID_AGG_RTOL * agg_r + 1e-12, (agg_g, agg_r)
    Dd, Xd = D.astype(np.float64), X.astype(np.float64)
    ls_err = 0.0
    for i in np.nonzero(ok)[0][:: max(1, ok.sum() // 256)]:
        n = gpu["count"][i]
        S = gpu["idx"][i, :n]
        r = Xd[i] - gpu["coef"][i, :n].astype(np.float64) @ Dd[S]
        assert abs(np.linalg.norm(r) - gpu["resid"][i]) <= 1e-5 * (np.linalg.norm(Xd[i]) + 1e-30)
        # whatever the support, the coefficients are its least-squares fit
        if n > 0 and np.linalg.cond(Dd[S] @ Dd[S].T) <= 1e3:
            g = np.linalg.lstsq(Dd[S].T, Xd[i], rcond=None)[0]
            e = np.linalg.norm(gpu["coef"][i, :n] - g) / max(np.linalg.norm(g), 1e-30)
            ls_err = max(ls_err, e)
    assert ls_err <= COEF_RTOL, f"coefficients are not the least-squares fit: {ls_err}"
    return dict(n=N, separated=int(sep.sum()), steps_compared=steps_cmp, steps_total=steps_total,
                coef_err=float(err.max(initial=0)), resid_gpu=agg_g,
                resid_ref=agg_r, resid_gap=float((agg_g - agg_r) / agg_r) if agg_r > 0 else 0.0,
                support_mismatch=float(np.mean(np.any(gpu["idx"][ok] != ref["idx"][ok], axis=1))))
