"""Dictionary learning on the GPU (Sec. 2.1): alternate the encoder (codes
with the dictionary fixed) and the MOD update (dictionary with the codes
fixed), both in this library's kernels."""
from __future__ import annotations

import numpy as np
import torch

from . import sc


def init_indices(X: np.ndarray, K: int, seed: int) -> np.ndarray:
    """Seeded choice of K distinct non-zero signals as the starting atoms."""
    nz = np.nonzero(np.linalg.norm(np.asarray(X, np.float64), axis=1) > 0)[0]
    rng = np.random.Generator(np.random.PCG64(seed))
    return nz[rng.choice(nz.size, size=K, replace=False)]


def learn(X, K, k, eps, passes=10, init_atoms=None, flags=0):
    """X: (N, d) float32 CUDA tensor.  init_atoms: (K, d) starting atoms (any
    norm).  Returns the (K, d) float32 unit-atom dictionary (CUDA tensor) and
    the per-pass mean squared residual of that pass's codes."""
    D = init_atoms.to(X.device, torch.float32)
    D = D / torch.linalg.vector_norm(D.double(), dim=1, keepdim=True).float()
    N, d = X.shape
    ws = torch.empty(max(int(sc.load().sc_mod_workspace(d, K)), 1), dtype=torch.uint8, device=X.device)
    out = (torch.empty((N, k), dtype=torch.int32, device=X.device),
           torch.empty((N, k), dtype=torch.float32, device=X.device),
           torch.empty((N,), dtype=torch.int32, device=X.device),
           torch.empty((N,), dtype=torch.float32, device=X.device))
    hist = []
    for _ in range(passes):
        h = sc.gram_precompute(D.contiguous(), sc.NORMALIZE)
        idx, coef, count, resid = sc.omp_encode(h, X, k, eps, flags, out=out)
        hist.append(float((resid.double() ** 2).mean().item()))
        D, _ = sc.mod_update(X, idx, coef, count, resid, K, workspace=ws)
        h.destroy()
    return D, hist
