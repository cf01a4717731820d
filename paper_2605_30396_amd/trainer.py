"""Training driver of the support proposer: labels from the FP32 GPU encoder,
then epochs of GPU training steps (sc_proposer_train_step) over seeded
shuffles of the training set.  Only the batching order is decided here; all
arithmetic runs in the library's kernels."""
from __future__ import annotations

import time

import numpy as np
import torch

from . import sc


def omp_labels(h: sc.Dictionary, X, k, eps):
    """Supports of the training signals from the plain FP32 encoder."""
    idx, coef, count, resid = sc.omp_encode(h, X, k, eps)
    return idx, count


def train(p: sc.Proposer, X, sup_idx, sup_count, epochs=2, batch=4096, lr=1e-3, pos_weight=1.0, seed=0,
          beta1=0.9, beta2=0.999, adam_eps=1e-8, verbose=False):
    """Run `epochs` passes over X (device, N x d) in seeded random order.
    Returns a dict with the per-epoch mean loss and the wall time."""
    N = X.shape[0]
    nb = N // batch
    if nb < 1:
        raise ValueError("training set smaller than one batch")
    ws = torch.empty(sc.train_workspace_bytes(p, batch), dtype=torch.uint8, device=X.device)
    losses = torch.zeros(nb, dtype=torch.float32, device=X.device)
    rng = np.random.Generator(np.random.PCG64(seed))
    hist = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(N)[: nb * batch].astype(np.int32)).to(X.device)
        for b in range(nb):
            sc.proposer_train_step(p, X, sup_idx, sup_count, batch, rows=perm[b * batch:(b + 1) * batch], lr=lr,
                                   beta1=beta1, beta2=beta2, adam_eps=adam_eps, pos_weight=pos_weight,
                                   loss=losses[b:b + 1], workspace=ws)
        hist.append(float(losses.mean().item()))
        if verbose:
            print(f"epoch {ep}: mean loss {hist[-1]:.6f}", flush=True)
    torch.cuda.synchronize()
    return dict(loss=hist, seconds=time.perf_counter() - t0, steps=epochs * nb, batch=batch)


def candidate_recall(cand, sup_idx, sup_count):
    """Fraction of signals whose whole OMP support is among their candidate
    list (cand: N x n_cand device int32, -1 for no candidate)."""
    c = cand.cpu().numpy()
    s = sup_idx.cpu().numpy()
    n = sup_count.cpu().numpy()
    hit = (s[:, :, None] == c[:, None, :]).any(-1)
    valid = np.arange(s.shape[1])[None, :] < n[:, None]
    return float(np.mean(np.all(hit | ~valid, axis=1)))


def support_recall(p: sc.Proposer, X, sup_idx, sup_count, n_cand=24):
    """Fraction of signals whose whole OMP support is among the proposer's
    n_cand candidates (host-side evaluation)."""
    cand, _ = sc.proposer_forward(p, X, n_cand)
    return candidate_recall(cand, sup_idx, sup_count)
