"""Oracle of the proposer-guided encoder -- TEST INFRASTRUCTURE.

Steps, in order: proposer logits for every signal; keep the n_cand atoms
with the largest logits; OMP restricted to those atoms; wherever the
restricted pursuit ends with an explicit residual above the tolerance, run the
full OMP over the whole dictionary instead.
"""
from __future__ import annotations

import numpy as np

from .core import omp
from .mlp import mlp_forward, topk_lowest_index


def learned_encode(D, X, params, k, eps, n_cand=24, relative=False, bf16=True, nthreads=None, cap=None):
    """cap: at most this many restricted steps (None = k); a restricted code
    that has not reached eps by then is a miss and takes the full OMP."""
    X = np.ascontiguousarray(X, np.float32)
    z = mlp_forward(params, X, bf16=bf16)
    cand = topk_lowest_index(z, n_cand)
    kr = k if not cap else min(int(cap), k)
    res = omp(D, X, kr, eps, relative, nthreads, cand=cand)
    if kr < k:   # widen the restricted codes to k columns (-1 / 0 padding)
        for key, fill in (("idx", -1), ("coef", 0.0)):
            wide = np.full((X.shape[0], k), fill, res[key].dtype)
            wide[:, :kr] = res[key]
            res[key] = wide
    xn = np.linalg.norm(X.astype(np.float64), axis=1)
    tol = eps * xn if relative else np.full(X.shape[0], eps)
    miss = ~(res["resid"] <= tol)
    miss &= res["count"] >= 0
    if miss.any():
        full = omp(D, X[miss], k, eps, relative, nthreads)
        for key in ("idx", "coef", "count", "resid"):
            res[key][miss] = full[key]
    res["fallback"] = miss
    res["cand"] = cand
    res["logits"] = z
    return res
