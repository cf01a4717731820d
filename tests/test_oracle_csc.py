"""Pins of the CSC storage oracle, the per-Gaussian colour oracle and the
storage accounting (no GPU)."""
import math

import numpy as np
import scipy.special

import oracle
from paper_2605_30396_amd import inputs as I
from paper_2605_30396_amd import storage


def test_pack_roundtrip_and_pointer_structure():
    rng = np.random.default_rng(3)
    N, k = 57, 6
    count = rng.integers(-1, k + 1, size=N).astype(np.int32)
    idx = np.full((N, k), -1, np.int32)
    coef = np.zeros((N, k), np.float32)
    for i in range(N):
        n = max(count[i], 0)
        idx[i, :n] = rng.choice(90, n, replace=False)
        coef[i, :n] = rng.normal(size=n)
    colptr, rows, vals = oracle.pack_csc(idx, coef, count)
    assert colptr[0] == 0 and colptr[-1] == np.maximum(count, 0).sum() == len(rows) == len(vals)
    assert np.all(np.diff(colptr) == np.maximum(count, 0))
    i2, c2, n2 = oracle.unpack_csc(colptr, rows, vals, k)
    np.testing.assert_array_equal(n2, np.maximum(count, 0))
    ok = count >= 0
    np.testing.assert_array_equal(i2[ok], idx[ok])
    np.testing.assert_array_equal(c2[ok], coef[ok])
    # an empty input packs to the single pointer 0
    c0, r0, v0 = oracle.pack_csc(np.zeros((0, 3), np.int32), np.zeros((0, 3), np.float32), np.zeros(0, np.int32))
    assert list(c0) == [0] and len(r0) == 0 and len(v0) == 0


def test_degree0_constant():
    assert abs(oracle.SH_C0 - 0.28209479177387814) < 1e-16
    y00 = scipy.special.sph_harm_y(0, 0, 0.3, 1.1)
    assert abs(float(np.real(y00)) - oracle.SH_C0) < 1e-15


def test_colour_with_identity_dictionary_is_the_dense_formula():
    """With D = I (45 atoms), a full code is the dense rest vector, so the
    colour is the plain 3DGS evaluation: C0 dc + sum_j x_cj Y_j(w) + 0.5,
    clamped at 0, with w the unit vector from the camera to the Gaussian."""
    rng = np.random.default_rng(5)
    N = 40
    X = rng.normal(scale=0.3, size=(N, 45)).astype(np.float32)
    D = np.eye(45, dtype=np.float32)
    idx = np.tile(np.arange(45, dtype=np.int32), (N, 1))
    pos = rng.normal(size=(N, 3)).astype(np.float32)
    dc = rng.normal(size=(N, 3)).astype(np.float32)
    cam = np.array([0.2, -0.1, 3.0])
    got = oracle.gaussian_rgb(D, idx, X, np.full(N, 45, np.int32), pos, dc, cam)
    w = pos.astype(np.float64) - cam
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    Y = oracle.sh_basis(w)
    rest = np.stack([(X[:, c * 15:(c + 1) * 15].astype(np.float64) * Y).sum(1) for c in range(3)], axis=1)
    ref = np.maximum(0.28209479177387814 * dc.astype(np.float64) + rest + 0.5, 0.0)
    np.testing.assert_allclose(got, ref, atol=1e-7)   # directions enter as FP32
    assert (ref == 0).any()   # the clamp is exercised


def test_colour_of_an_empty_code_is_the_dc_term():
    D = I.random_dictionary(I.rng_for(7), 64)
    N = 5
    dc = np.linspace(-3, 3, 3 * N).reshape(N, 3).astype(np.float32)
    got = oracle.gaussian_rgb(D, np.full((N, 4), -1, np.int32), np.zeros((N, 4), np.float32),
                              np.array([0, 0, -1, 0, 0], np.int32), np.ones((N, 3), np.float32), dc, [0, 0, 0])
    np.testing.assert_allclose(got, np.maximum(oracle.SH_C0 * dc.astype(np.float64) + 0.5, 0.0), atol=1e-15)


def test_compression_ratio_by_hand():
    # 1000 Gaussians, 11.7 non-zeros each, K = 90: 180 kB dense against
    # 11700 * 8 + 1001 * 4 + 90 * 45 * 4 bytes
    r = storage.compression_ratio(1000, 11700, 90)
    assert math.isclose(r, 180000 / (93600 + 4004 + 16200))
    assert storage.csc_bytes(0, 0) == 4
