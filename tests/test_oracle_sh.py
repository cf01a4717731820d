"""Pins of the SH basis and radiance oracle (no GPU).

Sec. 2.2 evaluates radiance directly from the sparse codes: each channel's 15
non-DC SH coefficients (degree 1..3) are summed against the real SH basis at
the view direction.  The paper fixes no SH convention; the reading used is the
real orthonormal basis with the Condon-Shortley phase, m = -l..l per band (the
one of the 3DGS renderer the paper builds on).  Pins: Cartesian closed forms,
the addition theorem, exact quadrature orthonormality, SciPy's complex
harmonics, and the structure of the radiance sum.
"""
import math

import numpy as np
import scipy.special as sp

import oracle
from paper_2605_30396_amd import inputs as I


def test_degree1_closed_form_and_axes():
    c1 = math.sqrt(3.0 / (4.0 * math.pi))
    dirs = I.unit_directions(I.rng_for(30), 50).astype(np.float64)
    Y = oracle.sh_basis(dirs, 1)
    x, y, z = dirs.T
    np.testing.assert_allclose(Y, np.stack([-c1 * y, c1 * z, -c1 * x], 1), atol=1e-14)
    # +z axis: only the m = 0 function of every band is non-zero, equal to sqrt((2l+1)/4pi)
    Yz = oracle.sh_basis(np.array([[0.0, 0.0, 1.0]]), 3)[0]
    for l in (1, 2, 3):
        band = Yz[l * l - 1 : (l + 1) ** 2 - 1]
        np.testing.assert_allclose(band[l], math.sqrt((2 * l + 1) / (4 * math.pi)), rtol=1e-14)
        assert np.all(np.abs(np.delete(band, l)) < 1e-14)
    # -z axis: m = 0 functions pick up (-1)^l
    Ymz = oracle.sh_basis(np.array([[0.0, 0.0, -1.0]]), 3)[0]
    for l in (1, 2, 3):
        np.testing.assert_allclose(Ymz[l * l - 1 + l], (-1) ** l * math.sqrt((2 * l + 1) / (4 * math.pi)),
                                   rtol=1e-14)


def test_degree2_closed_form():
    dirs = I.unit_directions(I.rng_for(31), 50).astype(np.float64)
    x, y, z = dirs.T
    a = math.sqrt(15 / (4 * math.pi))
    b = math.sqrt(5 / (16 * math.pi))
    c = math.sqrt(15 / (16 * math.pi))
    ref = np.stack([a * x * y, -a * y * z, b * (2 * z * z - x * x - y * y), -a * x * z, c * (x * x - y * y)], 1)
    np.testing.assert_allclose(oracle.sh_basis(dirs, 2)[:, 3:8], ref, atol=1e-14)


def test_addition_theorem():
    dirs = I.unit_directions(I.rng_for(32), 200).astype(np.float64)
    Y = oracle.sh_basis(dirs, 3)
    for l in (1, 2, 3):
        band = Y[:, l * l - 1 : (l + 1) ** 2 - 1]
        np.testing.assert_allclose((band ** 2).sum(1), (2 * l + 1) / (4 * math.pi), rtol=1e-13)


def test_orthonormal_by_exact_quadrature():
    """Gauss-Legendre in cos(theta) (6 nodes) x 8 uniform azimuths integrates
    products of degree <= 6 exactly."""
    t, w = np.polynomial.legendre.leggauss(6)
    ph = 2 * np.pi * np.arange(8) / 8
    T, P = np.meshgrid(t, ph, indexing="ij")
    st = np.sqrt(1 - T * T)
    dirs = np.stack([st * np.cos(P), st * np.sin(P), T], -1).reshape(-1, 3)
    wts = (w[:, None] * np.full(8, 2 * np.pi / 8)[None, :]).reshape(-1)
    Y = oracle.sh_basis(dirs, 3)
    Gm = (Y * wts[:, None]).T @ Y
    np.testing.assert_allclose(Gm, np.eye(15), atol=1e-13)


def test_matches_scipy_complex_harmonics():
    dirs = I.unit_directions(I.rng_for(33), 100).astype(np.float64)
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    theta = np.arccos(np.clip(dirs[:, 2], -1, 1))
    phi = np.mod(np.arctan2(dirs[:, 1], dirs[:, 0]), 2 * np.pi)  # SciPy wants [0, 2pi]
    Y = oracle.sh_basis(dirs, 3)
    for l in (1, 2, 3):
        for m in range(-l, l + 1):
            Ylm = sp.sph_harm_y(l, abs(m), theta, phi)
            if m > 0:
                ref = math.sqrt(2) * Ylm.real
            elif m < 0:
                ref = math.sqrt(2) * Ylm.imag
            else:
                ref = Ylm.real
            np.testing.assert_allclose(Y[:, l * l - 1 + m + l], ref, atol=1e-13)


def _codes(rng, N, K, kcap):
    cnt = rng.integers(0, kcap + 1, N).astype(np.int32)
    idx = np.full((N, kcap), -1, np.int32)
    cf = np.zeros((N, kcap), np.float32)
    for i in range(N):
        idx[i, : cnt[i]] = rng.choice(K, cnt[i], replace=False)
        cf[i, : cnt[i]] = rng.uniform(-1, 1, cnt[i])
    return idx, cf, cnt


def test_radiance_structure():
    rng = I.rng_for(34)
    D = I.random_dictionary(rng, 90)
    N, kcap = 64, 12
    idx, cf, cnt = _codes(rng, N, 90, kcap)
    dirs = I.unit_directions(rng, N)
    rgb = oracle.radiance(D, idx, cf, cnt, dirs, shared_dirs=False)
    Y = oracle.sh_basis(dirs.astype(np.float64), 3)
    Dd = D.astype(np.float64)
    for i in range(N):
        # per-atom form: sum_t coef_t * (a_t restricted to channel c) . Y
        v = np.zeros(3)
        for t in range(cnt[i]):
            a = Dd[idx[i, t]].reshape(3, 15)
            v += float(cf[i, t]) * (a @ Y[i])
        np.testing.assert_allclose(rgb[i], v, atol=1e-13)
    # linear in the coefficients
    rgb2 = oracle.radiance(D, idx, cf * np.float32(2.0), cnt, dirs, shared_dirs=False)
    np.testing.assert_allclose(rgb2, 2 * rgb, atol=1e-13)
    # shared directions: M views of every signal
    M = 7
    sd = I.unit_directions(rng, M)
    rs = oracle.radiance(D, idx, cf, cnt, sd, shared_dirs=True)
    assert rs.shape == (N, M, 3)
    for m in range(M):
        one = oracle.radiance(D, idx, cf, cnt, np.repeat(sd[m : m + 1], N, 0), shared_dirs=False)
        np.testing.assert_allclose(rs[:, m], one, atol=1e-14)


def test_identity_dictionary_is_plain_sh_evaluation():
    rng = I.rng_for(35)
    D = np.eye(45, dtype=np.float32)
    N = 20
    x = rng.standard_normal((N, 45)).astype(np.float32)
    idx = np.tile(np.arange(45, dtype=np.int32), (N, 1))
    cnt = np.full(N, 45, np.int32)
    dirs = I.unit_directions(rng, N)
    rgb = oracle.radiance(D, idx, x, cnt, dirs, shared_dirs=False)
    Y = oracle.sh_basis(dirs.astype(np.float64), 3)
    ref = np.einsum("ncj,nj->nc", x.astype(np.float64).reshape(N, 3, 15), Y)
    np.testing.assert_allclose(rgb, ref, atol=1e-13)


def test_lower_degrees_and_bad_codes():
    rng = I.rng_for(36)
    for L, d in ((1, 9), (2, 24)):
        D = I.random_dictionary(rng, 20, d)
        idx, cf, cnt = _codes(rng, 10, 20, 4)
        dirs = I.unit_directions(rng, 10)
        rgb = oracle.radiance(D, idx, cf, cnt, dirs, shared_dirs=False)
        Y = oracle.sh_basis(dirs.astype(np.float64), L)
        xh = np.zeros((10, d))
        for i in range(10):
            for t in range(cnt[i]):
                xh[i] += cf[i, t] * D[idx[i, t]].astype(np.float64)
        ref = np.einsum("ncj,nj->nc", xh.reshape(10, 3, d // 3), Y)
        np.testing.assert_allclose(rgb, ref, atol=1e-13)
    D = I.random_dictionary(rng, 20)
    idx, cf, cnt = _codes(rng, 5, 20, 4)
    cnt[2] = -1
    rgb = oracle.radiance(D, idx, cf, cnt, I.unit_directions(rng, 5), shared_dirs=False)
    assert np.all(np.isnan(rgb[2])) and np.all(np.isfinite(np.delete(rgb, 2, 0)))
