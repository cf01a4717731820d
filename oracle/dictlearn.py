"""Dictionary learning by alternating minimisation -- TEST INFRASTRUCTURE.

Eq. (1) of the paper is solved approximately by updating the sparse codes with
the dictionary fixed and then the dictionary with the codes fixed (Sec. 2.1).
The paper does not name the dictionary step; this oracle uses the Method of
Optimal Directions: with the codes A (K x N) fixed, the least-squares
dictionary is X A^T (A A^T)^-1, after which every atom is scaled back to unit
norm (the constraint of Eq. (1)).  An atom that no signal uses is replaced by
the currently worst-represented signal, normalised.
"""
from __future__ import annotations

import numpy as np

from .core import omp


def mod_step(X, r, K):
    """One dictionary update from fixed codes r (dict of idx, coef, count,
    resid as omp returns them): D = X A^T (A A^T + ridge I)^-1 with ridge =
    1e-10 tr(A A^T) / K, atoms used by no signal replaced by the worst-fit
    signals (largest residual first), every atom scaled to unit norm.
    Returns the (K, d) float64 atom-major dictionary."""
    Xd = np.asarray(X, np.float64)
    N, d = Xd.shape
    k = r["idx"].shape[1]
    cnt = np.maximum(r["count"], 0)
    rows = np.repeat(np.arange(N), cnt)
    sel = np.arange(k)[None, :] < cnt[:, None]
    cols = r["idx"][sel]
    vals = r["coef"][sel].astype(np.float64)
    # A is K x N with A[cols, rows] = vals
    XAt = np.zeros((d, K))
    np.add.at(XAt.T, cols, vals[:, None] * Xd[rows])
    AAt = np.zeros((K, K))
    # per-signal outer products of its nonzero coefficients
    for t1 in range(k):
        m1 = cnt > t1
        for t2 in range(k):
            m = m1 & (cnt > t2)
            np.add.at(AAt, (r["idx"][m, t1], r["idx"][m, t2]),
                      r["coef"][m, t1].astype(np.float64) * r["coef"][m, t2].astype(np.float64))
    ridge = 1e-10 * np.trace(AAt) / K
    Dn = np.linalg.solve(AAt + ridge * np.eye(K), XAt.T)      # (K, d) = (X A^T (AA^T)^-1)^T
    norms = np.linalg.norm(Dn, axis=1)
    used = np.diag(AAt) > 0
    bad = np.nonzero(~used | (norms <= 1e-12))[0]
    if bad.size:
        worst = np.argsort(-np.asarray(r["resid"], np.float64), kind="stable")[: bad.size]
        Dn[bad] = Xd[worst]
        norms[bad] = np.linalg.norm(Dn[bad], axis=1)
    return Dn / norms[:, None]


def mod_learn(X, K, k, eps, passes=10, seed=0, nthreads=None, init_atoms=None):
    """X: (N, d) float32 training signals.  Returns the (K, d) float32 atom-major
    dictionary after `passes` code/dictionary updates, and the per-pass mean
    squared residual (measured with the codes of that pass)."""
    X = np.ascontiguousarray(X, np.float32)
    Xd = X.astype(np.float64)
    N, d = X.shape
    rng = np.random.Generator(np.random.PCG64(seed))
    if init_atoms is None:
        nz = np.nonzero(np.linalg.norm(Xd, axis=1) > 0)[0]
        pick = nz[rng.choice(nz.size, size=K, replace=False)]
        D = Xd[pick].copy()
    else:
        D = np.asarray(init_atoms, np.float64).copy()
    D /= np.linalg.norm(D, axis=1, keepdims=True)
    history = []
    for _ in range(passes):
        D32 = D.astype(np.float32)
        r = omp(D32, X, k, eps, nthreads=nthreads)
        history.append(float(np.mean(r["resid"] ** 2)))
        D = mod_step(Xd, r, K)
    return D.astype(np.float32), history
