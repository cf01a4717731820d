"""FP64 NumPy oracle of the support-proposer network -- TEST INFRASTRUCTURE.

The network maps a signal's direction x/||x|| (x = 0 maps to 0) through
  a1 = W1 xh + b1,  h1 = GELU(a1)
  a2 = W2 h1 + b2,  h2 = GELU(a2)
  z  = W3 h2 + b3                       (one logit per dictionary atom)
with the exact GELU(t) = t * Phi(t) = t/2 (1 + erf(t/sqrt 2)).  It is trained
with binary cross-entropy on logits against the multi-hot indicator of the
atoms OMP selected, and Adam.  Nothing of this is in the paper: the proposer
is an addition, specified only by its layer sizes, the GELU activation and
BF16 weights with FP32 accumulation.

`bf16=True` rounds, exactly where the GPU kernels do, the network input, the
weights and the two hidden activations to bfloat16 (round to nearest even),
while all sums stay in FP64; this is the precision in which the kernels take
their top-k decision.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

_SQRT2 = math.sqrt(2.0)
_INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even), via float32.  Returns
    float64 holding bf16-representable values."""
    f = np.ascontiguousarray(a, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    out = r.view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if nan.any():
        out[nan] = np.nan
    return out


def gelu(t):
    t = np.asarray(t, np.float64)
    return 0.5 * t * (1.0 + erf(t / _SQRT2))


def gelu_grad(t):
    """d/dt [t Phi(t)] = Phi(t) + t phi(t)."""
    t = np.asarray(t, np.float64)
    return 0.5 * (1.0 + erf(t / _SQRT2)) + t * _INV_SQRT_2PI * np.exp(-0.5 * t * t)


def normalise_input(X):
    X = np.asarray(X, np.float64)
    n = np.linalg.norm(X, axis=1, keepdims=True)
    return np.divide(X, n, out=np.zeros_like(X), where=n > 0)


def mlp_forward(params, X, bf16=False, keep=False):
    """Logits z (N, K) in FP64.  params: dict W1 (H,d), b1, W2 (H,H), b2,
    W3 (K,H), b3.  With keep=True also returns the intermediates."""
    r = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    W1, W2, W3 = r(params["W1"]), r(params["W2"]), r(params["W3"])
    b1, b2, b3 = (np.asarray(params[n], np.float64) for n in ("b1", "b2", "b3"))
    xh = r(normalise_input(X))
    a1 = xh @ W1.T + b1
    h1 = r(gelu(a1))
    a2 = h1 @ W2.T + b2
    h2 = r(gelu(a2))
    z = h2 @ W3.T + b3
    if keep:
        return z, dict(xh=xh, a1=a1, h1=h1, a2=a2, h2=h2, W1=W1, W2=W2, W3=W3)
    return z


def multi_hot(idx, count, K):
    """(N, K) float64 indicator of each row's first count[i] indices."""
    N, kcap = idx.shape
    Y = np.zeros((N, K), np.float64)
    for t in range(kcap):
        sel = (count > t) & (idx[:, t] >= 0)
        Y[np.nonzero(sel)[0], idx[sel, t]] = 1.0
    return Y


def bce_with_logits(z, Y, pos_weight=1.0):
    """Mean over all N*K entries of  w y softplus(-z) + (1-y) softplus(z),
    and its gradient with respect to z."""
    z = np.asarray(z, np.float64)
    sp_pos = np.maximum(z, 0) + np.log1p(np.exp(-np.abs(z)))   # softplus(z)
    sp_neg = sp_pos - z                                          # softplus(-z)
    n = z.size
    loss = float(np.sum(pos_weight * Y * sp_neg + (1.0 - Y) * sp_pos) / n)
    sig = 0.5 * (1.0 + np.tanh(0.5 * z))                         # logistic(z)
    dz = (pos_weight * Y * (sig - 1.0) + (1.0 - Y) * sig) / n
    return loss, dz


def mlp_loss_and_grads(params, X, Y, pos_weight=1.0, bf16=False):
    """Loss and gradients of every parameter (backpropagation written out
    layer by layer)."""
    z, c = mlp_forward(params, X, bf16=bf16, keep=True)
    loss, dz = bce_with_logits(z, Y, pos_weight)
    g = {}
    g["W3"] = dz.T @ c["h2"]
    g["b3"] = dz.sum(0)
    dh2 = dz @ c["W3"]
    da2 = dh2 * gelu_grad(c["a2"])
    g["W2"] = da2.T @ c["h1"]
    g["b2"] = da2.sum(0)
    dh1 = da2 @ c["W2"]
    da1 = dh1 * gelu_grad(c["a1"])
    g["W1"] = da1.T @ c["xh"]
    g["b1"] = da1.sum(0)
    return loss, g


def adam_step(params, grads, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected, step number t >= 1), in place on
    float64 copies; returns the new params dict."""
    out = {}
    for n in params:
        p = np.asarray(params[n], np.float64)
        gr = grads[n]
        m[n] = beta1 * m[n] + (1 - beta1) * gr
        v[n] = beta2 * v[n] + (1 - beta2) * gr * gr
        mh = m[n] / (1 - beta1 ** t)
        vh = v[n] / (1 - beta2 ** t)
        out[n] = p - lr * mh / (np.sqrt(vh) + eps)
    return out


def topk_lowest_index(z, n):
    """Indices of the n largest entries of every row, ordered by value
    descending and, among equal values, by index ascending."""
    z = np.asarray(z)
    N, K = z.shape
    order = np.lexsort((np.broadcast_to(np.arange(K), (N, K)), -z), axis=1)
    return order[:, :n].astype(np.int32)
