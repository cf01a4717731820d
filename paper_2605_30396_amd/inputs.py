"""Seeded synthetic inputs shared by the HIP path's tests/bench and the oracle.

This module only draws random numbers and lays them out; it performs none of
the sparse-coding or radiance arithmetic.  Every generator uses NumPy's PCG64
bit generator with an explicit seed and draws in a fixed order, so the same
(seed, sizes) always give the same arrays.

Layouts (all float32 unless stated):
  * dictionary ``D``: shape (K, d) -- atom-major, i.e. the d x K matrix of the
    paper's Eq. (1) stored column by column, each atom's d values contiguous.
  * signals ``X``: shape (N, d), one Gaussian's SH "rest" vector per row,
    channel-major [R_1..R_15, G_1..G_15, B_1..B_15] (Sec. 2.2: the DC term of
    each channel is excluded, leaving 45 of the 48 coefficients).
  * directions: shape (M, 3), unit vectors.
"""
from __future__ import annotations

import math

import numpy as np

D_SH = 45  # 3 channels x 15 non-DC real SH functions of degree <= 3 (Sec. 2.2)
_CHUNK = 1 << 20  # fixed chunk size: keeps the draw order independent of N


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def random_dictionary(rng: np.random.Generator, K: int, d: int = D_SH) -> np.ndarray:
    """K atoms with i.i.d. N(0,1) entries, each scaled to unit L2 norm (Eq. (1)
    requires unit-norm atoms).  Returns float32 (K, d)."""
    A = rng.standard_normal((K, d))
    A /= np.linalg.norm(A, axis=1, keepdims=True)
    return A.astype(np.float32)


def _distinct_supports(rng: np.random.Generator, N: int, K: int, s: int) -> np.ndarray:
    """Uniform random s-subsets of range(K), one per row (rows with a repeated
    atom are redrawn until all rows are distinct)."""
    if s > K:
        raise ValueError("support size exceeds dictionary size")
    idx = rng.integers(0, K, size=(N, s))
    while True:
        srt = np.sort(idx, axis=1)
        bad = np.nonzero((srt[:, 1:] == srt[:, :-1]).any(axis=1))[0] if s > 1 else np.zeros(0, np.int64)
        if bad.size == 0:
            return idx
        idx[bad] = rng.integers(0, K, size=(bad.size, s))


def sparse_signals(rng: np.random.Generator, D: np.ndarray, N: int, s: int,
                   noise_sigma: float = 1e-3, coef_range: float = 1.0):
    """Generator G1: each signal is an exact s-sparse combination of atoms of D
    (uniform random support, coefficients U[-coef_range, coef_range]) plus
    i.i.d. N(0, noise_sigma^2) noise.  Returns (X float32 (N,d), support int64
    (N,s), coefficients float64 (N,s))."""
    K, d = D.shape
    sup = _distinct_supports(rng, N, K, s)
    cf = rng.uniform(-coef_range, coef_range, size=(N, s))
    Dd = D.astype(np.float64)
    X = np.empty((N, d), np.float32)
    for a in range(0, N, _CHUNK):
        b = min(N, a + _CHUNK)
        blk = np.einsum("ns,nsd->nd", cf[a:b], Dd[sup[a:b]])
        if noise_sigma > 0:
            blk += noise_sigma * rng.standard_normal((b - a, d))
        X[a:b] = blk
    return X, sup, cf


def add_near_duplicates(rng: np.random.Generator, X: np.ndarray, frac: float,
                        sigma: float = 1e-4) -> np.ndarray:
    """Overwrite a fraction `frac` of the rows of X with copies of other
    (unmodified) rows plus N(0, sigma^2) noise.  Returns the overwritten row
    indices.  X is modified in place."""
    N, d = X.shape
    n_dup = int(round(frac * N))
    if n_dup == 0:
        return np.zeros(0, np.int64)
    dup = np.sort(rng.choice(N, size=n_dup, replace=False))
    keep = np.setdiff1d(np.arange(N), dup, assume_unique=True)
    src = keep[rng.integers(0, keep.size, size=n_dup)]
    X[dup] = (X[src].astype(np.float64) + sigma * rng.standard_normal((n_dup, d))).astype(np.float32)
    return dup


def sh_like_signals(rng: np.random.Generator, N: int, rho: float = 0.8,
                    base_scale: float = 0.3) -> np.ndarray:
    """Generator G2: SH-like rest coefficients.  For every Gaussian and every
    non-DC basis function j of band l (l = 1, 2, 3 holding 3, 5, 7 functions),
    draw a shared term s and per-channel terms e_R, e_G, e_B i.i.d.
    Laplace(0, base_scale * 2**-l), and set x_{c,j} = sqrt(rho) s + sqrt(1-rho) e_c.
    The channel correlation is exactly rho.  Returns float32 (N, 45)."""
    band = np.repeat(np.arange(1, 4), [3, 5, 7])          # band of j = 1..15
    scale = base_scale * np.power(2.0, -band)             # (15,)
    X = np.empty((N, 45), np.float32)
    a_, b_ = math.sqrt(rho), math.sqrt(1.0 - rho)
    for a in range(0, N, _CHUNK):
        b = min(N, a + _CHUNK)
        sh = rng.laplace(0.0, 1.0, size=(b - a, 15)) * scale
        e = rng.laplace(0.0, 1.0, size=(b - a, 3, 15)) * scale
        X[a:b] = (a_ * sh[:, None, :] + b_ * e).reshape(b - a, 45)
    return X


def unit_directions(rng: np.random.Generator, M: int) -> np.ndarray:
    """M directions uniform on the sphere (normalised N(0, I_3)).  float32 (M,3)."""
    v = rng.standard_normal((M, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v.astype(np.float32)


# --------------------------------------------------------------------------
# Workload recipes (sizes and seeds of the synthetic stand-ins for trained
# 3DGS scenes; the paper's datasets are not available).
# --------------------------------------------------------------------------

def workload_plain_small(N: int = 4096, K: int = 64, s: int = 4, M: int = 64, seed: int = 1,
                         dir_seed: int = 101):
    """Plain OMP case: K=64 Gaussian dictionary, exactly 4-sparse signals with
    coefficients U[-1,1] plus N(0,(1e-3)^2) noise, k=4, eps=0, 64 shared
    view directions."""
    rng = rng_for(seed)
    D = random_dictionary(rng, K)
    X, sup, cf = sparse_signals(rng, D, N, s, 1e-3)
    dirs = unit_directions(rng_for(dir_seed), M)
    return dict(D=D, X=X, support=sup, coef=cf, dirs=dirs, k=4, eps=0.0)


def workload_sh_like(N: int = 1_000_000, seed: int = 2, dir_seed: int = 102):
    """SH-like case: Laplace band-scaled, RGB-correlated coefficients; the
    K=256 dictionary is learned from the first 100k signals (stored fixture);
    k=8, eps=1e-3; one view direction per Gaussian."""
    X = sh_like_signals(rng_for(seed), N)
    dirs = unit_directions(rng_for(dir_seed), N)
    return dict(X=X, dirs=dirs, k=8, eps=1e-3)


def workload_precision(N: int = 3_000_000, K: int = 512, s: int = 4, seed: int = 3,
                       dup_frac: float = 0.05):
    """Precision case: K=512 Gaussian dictionary, 4-sparse signals with 5%
    near-duplicate rows; k=12, eps=0."""
    rng = rng_for(seed)
    D = random_dictionary(rng, K)
    X, sup, cf = sparse_signals(rng, D, N, s, 1e-3)
    dup = add_near_duplicates(rng, X, dup_frac)
    return dict(D=D, X=X, support=sup, coef=cf, dup_rows=dup, k=12, eps=0.0)


def scene_batch_specs(n_scenes: int = 16, seed: int = 4, n_min: float = 5e4, n_max: float = 6e6):
    """Batched case: per-scene sizes log-uniform in [n_min, n_max], K in
    {128, 256, 512}, k in {4, 8, 12, 16}.  Returns a list of dicts with the
    scene's N, K, k and its own generator seed."""
    rng = rng_for(seed)
    logN = rng.uniform(math.log(n_min), math.log(n_max), size=n_scenes)
    Ks = rng.choice(np.array([128, 256, 512]), size=n_scenes)
    ks = rng.choice(np.array([4, 8, 12, 16]), size=n_scenes)
    sub = rng.integers(0, 2**31 - 1, size=n_scenes)
    return [dict(N=int(round(math.exp(logN[i]))), K=int(Ks[i]), k=int(ks[i]), seed=int(sub[i]))
            for i in range(n_scenes)]


def scene_inputs(spec: dict, s: int = 4, N_override: int | None = None):
    rng = rng_for(spec["seed"])
    D = random_dictionary(rng, spec["K"])
    X, sup, cf = sparse_signals(rng, D, spec["N"] if N_override is None else N_override, s, 1e-3)
    return D, X


def learned_dictionary(K: int = 512, seed: int = 5):
    """Dictionary of the learned-proposer case (drawn first from seed 5)."""
    return random_dictionary(rng_for(seed), K)


def learned_train_signals(D: np.ndarray, N: int = 2_000_000, s: int = 4, seed: int = 5):
    rng = rng_for(seed)
    random_dictionary(rng, D.shape[0], D.shape[1])  # advance past the dictionary draw
    X, sup, cf = sparse_signals(rng, D, N, s, 1e-3)
    return X


def learned_eval_signals(D: np.ndarray, N: int = 6_000_000, s: int = 4, seed: int = 55):
    X, sup, cf = sparse_signals(rng_for(seed), D, N, s, 1e-3)
    return X


def mlp_init(rng: np.random.Generator, d: int, H: int, K: int):
    """Seeded initial weights for the support-proposer MLP d->H->H->K:
    uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) for weights and biases.
    Returns a dict of float32 arrays W1 (H,d), b1 (H,), W2 (H,H), b2 (H,),
    W3 (K,H), b3 (K,)."""
    out = {}
    for name, (o, i) in (("1", (H, d)), ("2", (H, H)), ("3", (K, H))):
        bnd = 1.0 / math.sqrt(i)
        out["W" + name] = rng.uniform(-bnd, bnd, size=(o, i)).astype(np.float32)
        out["b" + name] = rng.uniform(-bnd, bnd, size=(o,)).astype(np.float32)
    return out
