"""Pins of the FP64 OMP oracle against what mathematics fixes (no GPU).

OMP is defined in Sec. 2.1 (after Eq. (1)): greedy selection of the atom most
correlated with the residual, least-squares refit, stop at sparsity k or
tolerance eps.  The paper prints no worked example, so every pin below comes
from a closed form, a theorem or brute force:
  * k = 1 equals exhaustive search over single atoms (unit-norm atoms);
  * for k = 2 on tiny dictionaries the exhaustive best pair is never worse;
  * exact recovery under Tropp's exact-recovery condition (ERC);
  * orthonormal dictionaries reduce OMP to hard thresholding;
  * the residual is orthogonal to the selected atoms and never increases;
  * least-squares agreement with LAPACK, scale and permutation equivariance.
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_2605_30396_amd import inputs as I


def _unit_rows(rng, K, d):
    A = rng.standard_normal((K, d))
    return (A / np.linalg.norm(A, axis=1, keepdims=True)).astype(np.float32)


def _ls_resid(A, x):
    g, *_ = np.linalg.lstsq(A.T, x, rcond=None)
    return np.linalg.norm(x - A.T @ g), g


def test_k1_equals_exhaustive_search():
    rng = I.rng_for(11)
    D = _unit_rows(rng, 40, 12)
    X = rng.standard_normal((300, 12)).astype(np.float32)
    r = oracle.omp(D, X, 1)
    Dd, Xd = D.astype(np.float64), X.astype(np.float64)
    for i in range(X.shape[0]):
        res = [np.linalg.norm(Xd[i] - (Dd[j] @ Xd[i]) / (Dd[j] @ Dd[j]) * Dd[j]) for j in range(40)]
        j = int(np.argmin(res))
        assert r["idx"][i, 0] == j
        assert abs(r["resid"][i] - res[j]) < 1e-12
        assert abs(r["coef"][i, 0] - (Dd[j] @ Xd[i]) / (Dd[j] @ Dd[j])) < 1e-12


def test_k2_never_beats_exhaustive_pair():
    rng = I.rng_for(12)
    D = _unit_rows(rng, 12, 8)
    X = rng.standard_normal((200, 8)).astype(np.float32)
    r = oracle.omp(D, X, 2)
    Dd = D.astype(np.float64)
    for i in range(X.shape[0]):
        x = X[i].astype(np.float64)
        best = min(_ls_resid(Dd[[a, b]], x)[0] for a, b in itertools.combinations(range(12), 2))
        assert best <= r["resid"][i] + 1e-12
        # OMP's own pair is a least-squares fit: its residual is that pair's LS residual
        own = _ls_resid(Dd[r["idx"][i]], x)[0]
        assert abs(own - r["resid"][i]) < 1e-12


def _hadamard(n):
    H = np.array([[1.0]])
    while H.shape[0] < n:
        H = np.block([[H, H], [H, -H]])
    return H


def test_k2_recovers_exact_pairs_under_low_coherence():
    """Identity + normalised Hadamard in R^32: mutual coherence 1/sqrt(32) < 1/3,
    so every exactly 2-sparse signal is recovered (Tropp 2004, mu < 1/(2k-1))."""
    d = 32
    D = np.vstack([np.eye(d), _hadamard(d) / np.sqrt(d)]).astype(np.float32)
    G = D.astype(np.float64) @ D.T.astype(np.float64)
    assert np.max(np.abs(G - np.eye(2 * d))) < 1 / 3
    rng = I.rng_for(13)
    N = 400
    sup = np.array([rng.choice(2 * d, 2, replace=False) for _ in range(N)])
    cf = rng.uniform(0.2, 1.0, (N, 2)) * rng.choice([-1, 1], (N, 2))
    X = np.einsum("ns,nsd->nd", cf, D.astype(np.float64)[sup]).astype(np.float32)
    r = oracle.omp(D, X, 2)
    Xd = X.astype(np.float64)
    for i in range(N):
        assert set(r["idx"][i]) == set(sup[i])
        assert r["resid"][i] < 1e-12 * np.linalg.norm(Xd[i]) + 1e-15


def _erc(Dd, S):
    """Tropp's exact recovery certificate max_{j not in S} ||pinv(D_S) a_j||_1."""
    P = np.linalg.pinv(Dd[S].T)
    rest = np.setdiff1d(np.arange(Dd.shape[0]), S)
    return np.max(np.abs(P @ Dd[rest].T).sum(axis=0))


def test_exact_recovery_under_erc():
    rng = I.rng_for(14)
    D = I.random_dictionary(rng, 64)             # 45 x 64 Gaussian, unit atoms
    Dd = D.astype(np.float64)
    checked = 0
    for trial in range(400):
        s = int(rng.integers(1, 5))
        S = rng.choice(64, s, replace=False)
        if _erc(Dd, S) >= 1.0:
            continue
        c = rng.uniform(0.1, 1.0, s) * rng.choice([-1, 1], s)
        x = (c @ Dd[S])
        # use the float32 signal exactly as the oracle sees it
        x32 = x.astype(np.float32)
        r = oracle.omp(D, x32[None], s)
        assert set(r["idx"][0]) == set(S)
        g_true = np.linalg.lstsq(Dd[S].T, x32.astype(np.float64), rcond=None)[0]
        pos = {j: t for t, j in enumerate(r["idx"][0])}
        got = np.array([r["coef"][0][pos[j]] for j in S])
        assert np.max(np.abs(got - g_true)) < 1e-12
        assert np.max(np.abs(g_true - c)) < 1e-6          # float32 rounding of x only
        checked += 1
    assert checked > 100


def test_orthonormal_dictionary_is_hard_thresholding():
    rng = I.rng_for(15)
    d, K, k = 20, 16, 5
    Q, _ = np.linalg.qr(rng.standard_normal((d, d)))
    D = Q[:K].astype(np.float32)                     # K orthonormal atoms (rows)
    X = rng.standard_normal((300, d)).astype(np.float32)
    r = oracle.omp(D, X, k)
    c = X.astype(np.float64) @ D.astype(np.float64).T
    for i in range(X.shape[0]):
        order = np.lexsort((np.arange(K), -np.abs(c[i])))[:k]
        assert list(r["idx"][i]) == list(order)
        np.testing.assert_allclose(r["coef"][i], c[i, order], atol=1e-6)  # D is float32-rounded


def test_tie_break_lowest_index():
    """D = I: correlations are the signal's entries; equal magnitudes must be
    taken in increasing index order."""
    D = np.eye(6, dtype=np.float32)
    x = np.array([[0.5, -1.0, 1.0, 0.25, -1.0, 0.5]], np.float32)
    r = oracle.omp(D, x, 5)
    assert list(r["idx"][0]) == [1, 2, 4, 0, 5]
    np.testing.assert_array_equal(r["coef"][0], [-1.0, 1.0, -1.0, 0.5, 0.5])


def test_invariants_residual_orthogonal_and_monotone():
    rng = I.rng_for(16)
    D = I.random_dictionary(rng, 128)
    X, _, _ = I.sparse_signals(rng, D, 300, 6, 1e-2)
    Dd, Xd = D.astype(np.float64), X.astype(np.float64)
    prev = np.linalg.norm(Xd, axis=1)
    prev_idx = None
    for k in range(1, 11):
        r = oracle.omp(D, X, k)
        for i in range(X.shape[0]):
            n = r["count"][i]
            S = r["idx"][i, :n]
            res = Xd[i] - r["coef"][i, :n] @ Dd[S]
            assert abs(np.linalg.norm(res) - r["resid"][i]) < 1e-12
            assert np.max(np.abs(Dd[S] @ res)) <= 1e-12 * np.linalg.norm(Xd[i])
            # Batch-OMP identity: ||r||^2 = ||x||^2 - (D_I^T x)^T gamma
            a0 = Dd[S] @ Xd[i]
            assert abs(r["resid"][i] ** 2 - (Xd[i] @ Xd[i] - a0 @ r["coef"][i, :n])) < 1e-12
        assert np.all(r["resid"] <= prev + 1e-13)
        # greedy: the support for k-1 is a prefix of the support for k
        if prev_idx is not None:
            np.testing.assert_array_equal(r["idx"][:, : k - 1], prev_idx)
        prev, prev_idx = r["resid"], r["idx"].copy()


def test_least_squares_matches_lapack():
    rng = I.rng_for(17)
    D = I.random_dictionary(rng, 90)
    X = rng.standard_normal((200, 45)).astype(np.float32)
    r = oracle.omp(D, X, 12)
    Dd = D.astype(np.float64)
    for i in range(X.shape[0]):
        res, g = _ls_resid(Dd[r["idx"][i]], X[i].astype(np.float64))
        np.testing.assert_allclose(r["coef"][i], g, rtol=0, atol=1e-12)
        assert abs(res - r["resid"][i]) < 1e-12


def test_scale_and_permutation_equivariance():
    rng = I.rng_for(18)
    D = I.random_dictionary(rng, 64)
    X, _, _ = I.sparse_signals(rng, D, 200, 4, 1e-3)
    r = oracle.omp(D, X, 4, with_margin=True)
    ok = r["margin"] > 1e-6
    r2 = oracle.omp(D, (X * np.float32(4.0)), 4)            # power-of-two: exact scaling
    np.testing.assert_array_equal(r2["idx"][ok], r["idx"][ok])
    np.testing.assert_allclose(r2["coef"][ok], 4.0 * r["coef"][ok], rtol=1e-12, atol=1e-13)
    perm = rng.permutation(64)
    r3 = oracle.omp(D[perm], X, 4)
    np.testing.assert_array_equal(perm[r3["idx"][ok]], r["idx"][ok])
    np.testing.assert_allclose(r3["coef"][ok], r["coef"][ok], rtol=1e-10, atol=1e-12)


def test_stop_rules():
    rng = I.rng_for(19)
    D = I.random_dictionary(rng, 64)
    X, _, _ = I.sparse_signals(rng, D, 300, 4, 1e-3)
    X[0] = 0.0
    X[1, 3] = np.nan
    X[2] = X[2] * np.float32(1e-3)               # tiny signal: below the tolerance
    eps = 2e-2
    r = oracle.omp(D, X, 12, eps)
    assert r["count"][0] == 0 and r["resid"][0] == 0.0 and np.all(r["idx"][0] == -1)
    assert r["count"][1] == -1 and np.isnan(r["resid"][1]) and np.all(r["idx"][1] == -1)
    assert r["count"][2] == 0
    good = r["count"] >= 0
    # stopped early only because the residual reached eps; at k the residual may exceed eps
    early = good & (r["count"] < 12)
    assert np.all(r["resid"][early] <= eps)
    # one step fewer would not have met the tolerance (stop test before each selection)
    r_prev = oracle.omp(D, X, 12, 0.0)
    for i in np.nonzero(good & (r["count"] > 0))[0][:100]:
        n = r["count"][i]
        if n >= 2:
            rp = oracle.omp(D, X[i : i + 1], n - 1)
            assert rp["resid"][0] > eps
    # relative tolerance: ||r|| <= eps * ||x||; eps < 1 always admits the first atom
    rr = oracle.omp(D, X[3:], 12, 0.5, relative=True)
    xn = np.linalg.norm(X[3:].astype(np.float64), axis=1)
    assert np.all(rr["count"] >= 1)
    early = rr["count"] < 12
    assert np.all(rr["resid"][early] <= 0.5 * xn[early])
    assert r_prev["count"][3:].min() == 12


def test_restricted_pursuit_over_all_atoms_is_full_pursuit():
    rng = I.rng_for(20)
    D = I.random_dictionary(rng, 64)
    X, _, _ = I.sparse_signals(rng, D, 100, 4, 1e-3)
    full = oracle.omp(D, X, 6, 1e-2)
    cand = np.tile(rng.permutation(64).astype(np.int32), (100, 1))
    res = oracle.omp(D, X, 6, 1e-2, cand=cand)
    for key in ("idx", "count"):
        np.testing.assert_array_equal(res[key], full[key])
    np.testing.assert_allclose(res["coef"], full["coef"], atol=1e-14)
    # a candidate list holding the full pursuit's support gives the same codes
    extra = rng.integers(0, 64, (100, 8)).astype(np.int32)
    cand2 = np.concatenate([np.where(full["idx"] >= 0, full["idx"], extra[:, :6]), extra], axis=1)
    res2 = oracle.omp(D, X, 6, 1e-2, cand=cand2)
    same = full["count"] > 0
    np.testing.assert_array_equal(res2["idx"][same], full["idx"][same])


def test_ill_conditioned_pair():
    """a1 = e1, a2 = normalise(e1 + 1e-3 e2), a3 = e3, x = e2: OMP takes a2 then
    a1 and must represent e2 exactly, with coefficients of size ~1e3."""
    a2 = np.array([1.0, 1e-3, 0.0]) / np.sqrt(1 + 1e-6)
    D = np.array([[1, 0, 0], a2, [0, 0, 1]], np.float32)
    x = np.array([[0, 1, 0]], np.float32)
    r = oracle.omp(D, x, 2)
    assert list(r["idx"][0]) == [1, 0]
    Dd = D.astype(np.float64)
    g = np.linalg.solve(Dd[[1, 0]][:, :2].T, np.array([0.0, 1.0]))
    np.testing.assert_allclose(r["coef"][0], g, rtol=1e-9)
    assert r["resid"][0] < 1e-9
    assert np.linalg.cond(Dd[[1, 0]] @ Dd[[1, 0]].T) > 1e5
