"""Pins of the MOD dictionary-update oracle (no GPU).

* planted dictionary: if X = A^T D_true exactly and the codes are the
  planted ones, the least-squares update returns D_true (its atoms already
  have unit norm, so the normalisation is the identity);
* unused atoms: an atom no code uses is replaced by the worst-fit signal
  (largest residual first, ties to the lower signal index), normalised;
* the fitted dictionary never increases the fit error of the same codes
  before normalisation (least squares)."""
import numpy as np

import oracle
from paper_2605_30396_amd import inputs as I


def planted(N=300, K=12, d=8, s=3, seed=61):
    rng = np.random.default_rng(seed)
    D = I.random_dictionary(I.rng_for(seed), K, d).astype(np.float64)
    idx = np.full((N, s), -1, np.int32)
    coef = np.zeros((N, s), np.float32)
    for i in range(N):
        idx[i] = rng.choice(K, s, replace=False)
        coef[i] = rng.uniform(0.5, 1.5, s) * rng.choice([-1, 1], s)
    X = np.zeros((N, d))
    for t in range(s):
        X += coef[:, t:t + 1].astype(np.float64) * D[idx[:, t]]
    r = dict(idx=idx, coef=coef, count=np.full(N, s, np.int32), resid=np.zeros(N))
    return D, X, r


def test_planted_dictionary_is_a_fixed_point():
    D, X, r = planted()
    Dn = oracle.mod_step(X, r, D.shape[0])
    np.testing.assert_allclose(Dn, D, atol=1e-9)


def test_unused_atom_takes_the_worst_signal():
    D, X, r = planted(K=12)
    used = r["idx"] != 11
    keep = used.all(axis=1)
    X, r = X[keep], {k: v[keep] for k, v in r.items()}
    resid = np.linspace(0, 1, len(X))
    resid[[5, 9]] = 7.0                        # equal largest residuals: the lower index wins
    r["resid"] = resid
    Dn = oracle.mod_step(X, r, 12)
    np.testing.assert_allclose(Dn[11], X[5] / np.linalg.norm(X[5]), atol=1e-12)
    np.testing.assert_allclose(Dn[:11], D[:11], atol=1e-9)


def test_update_does_not_increase_the_fit_error():
    rng = np.random.default_rng(4)
    D = I.random_dictionary(I.rng_for(62), 20, 10).astype(np.float64)
    X = rng.normal(size=(400, 10))
    r = oracle.omp(D.astype(np.float32), X.astype(np.float32), 3, 0.0)
    A = np.zeros((20, 400))
    for i in range(400):
        A[r["idx"][i, :r["count"][i]], i] = r["coef"][i, :r["count"][i]]
    before = np.linalg.norm(X.T - D.T @ A)
    XAt, AAt = X.T @ A.T, A @ A.T
    Dls = np.linalg.solve(AAt + 1e-10 * np.trace(AAt) / 20 * np.eye(20), XAt.T)
    after = np.linalg.norm(X.T - Dls.T @ A)
    assert after <= before + 1e-9
    # and mod_step is that solution, normalised
    Dn = oracle.mod_step(X, r, 20)
    np.testing.assert_allclose(Dn, Dls / np.linalg.norm(Dls, axis=1, keepdims=True), atol=1e-9)
