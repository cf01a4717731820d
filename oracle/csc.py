"""CSC storage of sparse codes and the per-Gaussian colour -- TEST
INFRASTRUCTURE (only tests, the smoke check and the benchmark's CPU-baseline
leg use it; the product library never does).

pack_csc / unpack_csc: Sec. 2.2 stores, for every Gaussian, only the non-zero
  coefficients of its code and their atom indices, column after column
  (Compressed-Sparse-Column), because the codes have different lengths.
  Column i holds the code's entries in selection order; a code with count <= 0
  (no atom, or the non-finite status -1) is an empty column.
gaussian_rgb: the colour the 3DGS renderer computes from SH coefficients,
  with the view-dependent part taken from the sparse codes (Sec. 2.2):
  w = (pos - cam) / ||pos - cam||,
  rgb = max(0, C0 * dc + radiance(codes, w) + 0.5), C0 = Y_0^0 = 1 / (2 sqrt(pi)).
"""
from __future__ import annotations

import math

import numpy as np

from .core import radiance

SH_C0 = 1.0 / (2.0 * math.sqrt(math.pi))


def pack_csc(idx, coef, count):
    """Padded codes (N x k) -> colptr int64[N+1], rows int32[nnz], vals float32[nnz]."""
    idx = np.asarray(idx)
    coef = np.asarray(coef)
    n = np.clip(np.asarray(count, np.int64), 0, idx.shape[1])
    colptr = np.zeros(len(n) + 1, np.int64)
    rows, vals = [], []
    for i in range(len(n)):
        colptr[i + 1] = colptr[i] + n[i]
        rows.append(idx[i, :n[i]])
        vals.append(coef[i, :n[i]])
    rows = np.concatenate(rows).astype(np.int32) if rows else np.zeros(0, np.int32)
    vals = np.concatenate(vals).astype(np.float32) if vals else np.zeros(0, np.float32)
    return colptr, rows, vals


def unpack_csc(colptr, rows, vals, k):
    """Inverse of pack_csc: padded codes (idx -1 / coef 0 padding)."""
    N = len(colptr) - 1
    idx = np.full((N, k), -1, np.int32)
    coef = np.zeros((N, k), np.float32)
    count = np.zeros(N, np.int32)
    for i in range(N):
        a, b = colptr[i], colptr[i + 1]
        count[i] = b - a
        idx[i, :b - a] = rows[a:b]
        coef[i, :b - a] = vals[a:b]
    return idx, coef, count


def gaussian_rgb(D, idx, coef, count, pos, dc, cam):
    """float64 (N, 3) colours; status -1 codes count as empty."""
    w = np.asarray(pos, np.float64) - np.asarray(cam, np.float64)[None, :]
    nrm = np.linalg.norm(w, axis=1, keepdims=True)
    w = np.where(nrm > 0, w / np.where(nrm > 0, nrm, 1.0), 0.0)
    cnt = np.maximum(np.asarray(count, np.int32), 0)
    rest = radiance(D, idx, coef, cnt, w.astype(np.float32), False)
    return np.maximum(SH_C0 * np.asarray(dc, np.float64) + rest + 0.5, 0.0)
