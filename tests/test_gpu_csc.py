"""GPU parity of the CSC storage (sc_csc_colptr / sc_csc_fill), the radiance
from CSC columns (sc_sh_eval_csc) and the per-Gaussian colour step
(sc_gaussian_rgb_csc), through the C ABI.

Packing is index and byte work: colptr, rows and vals must equal the
oracle's packing of the same codes bit for bit.  Radiance and colour are
FP32 sums: within 1e-4 absolute of the FP64 oracle; the CSC radiance runs
the padded-code kernel's arithmetic in the same order, so the two agree
exactly wherever the padded kernel returns a number."""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2605_30396_amd import inputs as I
from paper_2605_30396_amd import sc

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def codes(N, K, k, seed, eps=0.0, bad=()):
    rng = I.rng_for(seed)
    D = I.random_dictionary(rng, K)
    X, _, _ = I.sparse_signals(rng, D, N, 4, 1e-3)
    for i in bad:
        X[i, 2] = np.nan
    h = sc.gram_precompute(torch.from_numpy(D).to(DEV))
    out = sc.omp_encode(h, torch.from_numpy(X).to(DEV), k, eps)
    return D, X, h, out


@pytest.mark.parametrize("N", [0, 1, 4095, 4096, 4097, 20011])
def test_pack_matches_oracle_bit_for_bit(N):
    bad = (0,) if N > 0 else ()
    D, X, h, (idx, coef, count, resid) = codes(N, 128, 8, 500 + N, eps=2e-2, bad=bad)
    colptr, rows, vals = sc.pack_csc(idx, coef, count)
    torch.cuda.synchronize()
    rc, rr, rv = oracle.pack_csc(idx.cpu().numpy(), coef.cpu().numpy(), count.cpu().numpy())
    np.testing.assert_array_equal(colptr.cpu().numpy(), rc)
    np.testing.assert_array_equal(rows.cpu().numpy(), rr)
    np.testing.assert_array_equal(vals.cpu().numpy().view(np.uint32), rv.view(np.uint32))
    h.destroy()


def test_pack_large_scan_spans_many_blocks():
    """3M codes: 733 scan blocks, counts from 0 to 12 (eps stops some early)."""
    N, k = 3_000_000, 12
    rng = np.random.default_rng(9)
    cnt = rng.integers(-1, k + 1, size=N).astype(np.int32)
    idx = np.where(np.arange(k)[None, :] < np.maximum(cnt, 0)[:, None],
                   rng.integers(0, 512, size=(N, k)), -1).astype(np.int32)
    coef = np.where(idx >= 0, rng.normal(size=(N, k)), 0).astype(np.float32)
    colptr, rows, vals = sc.pack_csc(torch.from_numpy(idx).to(DEV), torch.from_numpy(coef).to(DEV),
                                     torch.from_numpy(cnt).to(DEV))
    ref_ptr = np.concatenate([[0], np.cumsum(np.maximum(cnt, 0))])
    np.testing.assert_array_equal(colptr.cpu().numpy(), ref_ptr)
    m = idx >= 0
    np.testing.assert_array_equal(rows.cpu().numpy(), idx[m])
    np.testing.assert_array_equal(vals.cpu().numpy(), coef[m])


def test_csc_radiance_equals_padded_radiance_and_oracle():
    N, K, k = 3000, 256, 8
    D, X, h, (idx, coef, count, resid) = codes(N, K, k, 510, bad=(7,))
    dirs = torch.from_numpy(I.unit_directions(I.rng_for(511), N)).to(DEV)
    colptr, rows, vals = sc.pack_csc(idx, coef, count)
    a = sc.sh_eval_csc(h, colptr, rows, vals, dirs).cpu().numpy()
    b = sc.sh_eval_sparse(h, idx, coef, count, dirs).cpu().numpy()
    ok = count.cpu().numpy() >= 0
    np.testing.assert_array_equal(a[ok], b[ok])
    np.testing.assert_array_equal(a[~ok], 0.0)          # status -1 packs as an empty column
    ref = oracle.radiance(D, idx.cpu().numpy(), coef.cpu().numpy(), np.maximum(count.cpu().numpy(), 0),
                          dirs.cpu().numpy(), False)
    assert np.abs(a - ref).max() <= 1e-4
    # shared directions
    sd = torch.from_numpy(I.unit_directions(I.rng_for(512), 9)).to(DEV)
    a2 = sc.sh_eval_csc(h, colptr, rows, vals, sd, sc.DIRS_SHARED).cpu().numpy()
    ref2 = oracle.radiance(D, idx.cpu().numpy(), coef.cpu().numpy(), np.maximum(count.cpu().numpy(), 0),
                           sd.cpu().numpy(), True)
    assert np.abs(a2 - ref2).max() <= 1e-4
    h.destroy()


@pytest.mark.parametrize("K", [90, 256, 630, 640, 1000])
def test_gaussian_colour_step(K):
    """The fused colour: camera-to-Gaussian direction, C0 DC term, compressed
    SH, +0.5, clamp at 0 (K = 640 and 1000 read D from global memory, not LDS)."""
    N = 2500
    D, X, h, (idx, coef, count, resid) = codes(N, K, 12, 520 + K, eps=1e-2, bad=(3,))
    rng = np.random.default_rng(K)
    pos = rng.normal(scale=2.0, size=(N, 3)).astype(np.float32)
    dc = rng.normal(scale=1.5, size=(N, 3)).astype(np.float32)
    cam = np.array([0.3, -1.2, 5.0], np.float32)
    colptr, rows, vals = sc.pack_csc(idx, coef, count)
    got = sc.gaussian_rgb_csc(h, colptr, rows, vals, torch.from_numpy(pos).to(DEV), torch.from_numpy(dc).to(DEV),
                              cam).cpu().numpy()
    ref = oracle.gaussian_rgb(D, idx.cpu().numpy(), coef.cpu().numpy(), count.cpu().numpy(), pos, dc, cam)
    assert np.abs(got - ref).max() <= 1e-4
    assert (ref == 0).any() and (ref > 0).any()
    h.destroy()


def test_csc_argument_errors():
    D, X, h, (idx, coef, count, resid) = codes(100, 128, 4, 530)
    lib = sc.load()
    colptr = torch.empty(101, dtype=torch.int64, device=DEV)
    ws = torch.empty(8, dtype=torch.uint8, device=DEV)
    assert lib.sc_csc_colptr(sc._ptr(count), 100, sc._ptr(colptr), sc._ptr(ws), 0, None) == sc.SC_ENOMEM
    assert lib.sc_csc_colptr(sc._ptr(count), -1, sc._ptr(colptr), sc._ptr(ws), 8, None) == sc.SC_EINVAL
    assert lib.sc_csc_fill(None, sc._ptr(coef), sc._ptr(count), 100, 4, sc._ptr(colptr), None, None,
                           None) == sc.SC_EINVAL
    c = (sc.C.c_float * 3)(0.0, float("nan"), 0.0)
    assert lib.sc_gaussian_rgb_csc(h.handle, sc._ptr(colptr), None, None, 100, None, None, c, None,
                                   None) == sc.SC_EINVAL
    h.destroy()


def test_encode_straight_to_csc():
    """eps-controlled encode written as CSC equals encode-then-pack; a too
    small capacity reports the needed size."""
    N, K, k, tol = 5001, 256, 32, 0.1
    X = I.sh_like_signals(I.rng_for(540), N)
    D = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sh_like_dict_K256.npy"))
    h = sc.gram_precompute(torch.from_numpy(D).to(DEV))
    Xg = torch.from_numpy(X).to(DEV)
    colptr, rows, vals, resid = sc.omp_encode_csc(h, Xg, k, tol, sc.EPS_RELATIVE)
    idx, coef, count, resid2 = sc.omp_encode(h, Xg, k, tol, sc.EPS_RELATIVE)
    c2, r2, v2 = sc.pack_csc(idx, coef, count)
    np.testing.assert_array_equal(colptr.cpu().numpy(), c2.cpu().numpy())
    np.testing.assert_array_equal(rows.cpu().numpy(), r2.cpu().numpy())
    np.testing.assert_array_equal(vals.cpu().numpy(), v2.cpu().numpy())
    np.testing.assert_array_equal(resid.cpu().numpy(), resid2.cpu().numpy())
    xn = np.linalg.norm(X.astype(np.float64), axis=1)
    above = resid.cpu().numpy() > tol * xn * (1 + 1e-5) + 1e-7
    assert np.all(np.diff(colptr.cpu().numpy())[above] == k)   # only codes that hit the cap miss the tolerance
    nnz = int(colptr[-1].item())
    with pytest.raises(sc.ScError) as e:
        sc.omp_encode_csc(h, Xg, k, tol, sc.EPS_RELATIVE, cap=nnz - 1)
    assert e.value.code == sc.SC_ENOMEM
    h.destroy()


def _csc_columns_against_oracle(D, X, k, eps, relative, colptr, rows, vals, resid):
    """Column by column against the oracle's OMP packed by the oracle's CSC
    packing: exact on signals whose greedy path is unique, valid everywhere
    (least-squares fit on the column's own support, residual reported)."""
    from parity import oracle_run, unique_prefix, well_separated
    ref = oracle_run(D, X, k, eps, relative)
    rc, rr, rv = oracle.pack_csc(ref["idx"], ref["coef"], ref["count"])
    sep = well_separated(D, X, ref, eps, relative)
    pre = unique_prefix(D, X, ref, eps, relative)
    assert colptr[0] == 0 and np.all(np.diff(colptr) >= 0)
    cnt = np.diff(colptr)
    np.testing.assert_array_equal(cnt[sep], np.diff(rc)[sep])
    Dd, Xd = D.astype(np.float64), X.astype(np.float64)
    worst = 0.0
    for i in range(len(X)):
        a, b = colptr[i], colptr[i + 1]
        S, c = rows[a:b], vals[a:b].astype(np.float64)
        # selections in order up to the first non-unique step
        np.testing.assert_array_equal(S[:pre[i]], rr[rc[i]:rc[i] + pre[i]], err_msg=f"column {i} prefix")
        if sep[i]:
            np.testing.assert_array_equal(S, rr[rc[i]:rc[i + 1]], err_msg=f"column {i}")
            ro = rv[rc[i]:rc[i + 1]].astype(np.float64)
            worst = max(worst, np.linalg.norm(c - ro) / max(np.linalg.norm(ro), 1e-30))
        if ref["count"][i] < 0:
            assert b == a and np.isnan(resid[i])
            continue
        if b > a:
            r = Xd[i] - c @ Dd[S]
            assert abs(np.linalg.norm(r) - resid[i]) <= 1e-5 * (np.linalg.norm(Xd[i]) + 1e-30)
            if np.linalg.cond(Dd[S] @ Dd[S].T) <= 1e3:
                g = np.linalg.lstsq(Dd[S].T, Xd[i], rcond=None)[0]
                assert np.linalg.norm(c - g) <= 1e-4 * max(np.linalg.norm(g), 1e-30), i
    assert worst <= 1e-4, worst
    return sep, pre.sum() / max(int(np.maximum(ref["count"], 0).sum()), 1)


@pytest.mark.parametrize("N", [1, 16, 4097])
def test_one_pass_csc_encoder_against_oracle(N):
    """sc_omp_encode_csc at a relative tolerance (the codes' length varies),
    k = 32, SH-like signals over the K = 256 MOD dictionary: every column
    equals the oracle's OMP packed by the oracle's CSC packing on signals
    whose greedy path is unique, and is a valid code elsewhere; a NaN signal
    is an empty column."""
    K, k, tol = 256, 32, 0.1
    X = I.sh_like_signals(I.rng_for(560 + N), N)
    if N > 16:
        X[5, 3] = np.nan
    D = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sh_like_dict_K256.npy"))
    h = sc.gram_precompute(torch.from_numpy(D).to(DEV))
    colptr, rows, vals, resid = (t.cpu().numpy() for t in sc.omp_encode_csc(h, torch.from_numpy(X).to(DEV), k,
                                                                            tol, sc.EPS_RELATIVE))
    sep, steps = _csc_columns_against_oracle(D, X, k, tol, True, colptr, rows, vals, resid)
    assert N <= 16 or (sep.mean() > 0.1 and steps > 0.5), (sep.mean(), steps)   # 16% and 60% here
    lens = np.diff(colptr)
    assert N < 16 or lens.min() < lens.max()   # variable-length columns
    h.destroy()


@pytest.mark.parametrize("K,k", [(512, 24), (1000, 16)])
def test_one_pass_csc_encoder_long_caps_large_dictionaries(K, k):
    """8-sparse signals over K > 256 dictionaries at eps = 1e-2 with caps of
    16 and 24: pursuits of about eight steps, past the steps whose
    broadcasts are lane reads, with every Gram row re-read from the cache
    (no row cache at these shapes); columns against the oracle."""
    rng = I.rng_for(580 + K + k)
    D = I.random_dictionary(rng, K)
    X, _, _ = I.sparse_signals(rng, D, 2100, 8, 1e-3)
    h = sc.gram_precompute(torch.from_numpy(D).to(DEV))
    colptr, rows, vals, resid = (t.cpu().numpy() for t in sc.omp_encode_csc(h, torch.from_numpy(X).to(DEV), k,
                                                                            1e-2))
    sep, steps = _csc_columns_against_oracle(D, X, k, 1e-2, False, colptr, rows, vals, resid)
    print(K, k, sep.mean(), steps)
    assert sep.mean() > 0.4 and steps > 0.6, (sep.mean(), steps)
    assert np.diff(colptr).max() > 4   # the pursuits run past step 4
    h.destroy()


def test_one_pass_csc_encoder_sparse_and_refit():
    """4-sparse signals over a K = 512 dictionary at eps = 1e-2 (columns of
    about four atoms, 200 tiles), plus a support refit in FP64 inside the
    same call (its column pointer is restored and its coefficients are the
    FP64 fit); a second call with too small a capacity reports the size and
    leaves colptr whole."""
    K, k, eps = 512, 12, 1e-2
    rng = I.rng_for(570)
    D = I.random_dictionary(rng, K)
    X, _, _ = I.sparse_signals(rng, D, 3200, 4, 1e-3)
    h = sc.gram_precompute(torch.from_numpy(D).to(DEV))
    Xg = torch.from_numpy(X).to(DEV)
    colptr, rows, vals, resid = (t.cpu().numpy() for t in sc.omp_encode_csc(h, Xg, k, eps))
    _csc_columns_against_oracle(D, X, k, eps, False, colptr, rows, vals, resid)
    nnz = int(colptr[-1])
    with pytest.raises(sc.ScError) as e:
        sc.omp_encode_csc(h, Xg, k, eps, cap=nnz // 2)
    assert e.value.code == sc.SC_ENOMEM
    h.destroy()
    # ill-conditioned support: a1 = e1, a2 = normalise(e1 + 1e-3 e2), a3 = e3; x = e2
    a2 = np.array([1.0, 1e-3, 0.0]) / np.sqrt(1 + 1e-6)
    Dill = np.array([[1, 0, 0], a2, [0, 0, 1]], np.float32)
    Xill = np.tile(np.array([[0, 1, 0]], np.float32), (40, 1))
    h = sc.gram_precompute(torch.from_numpy(Dill).to(DEV))
    sc.omp_stats(h, reset=True)
    colptr, rows, vals, resid = (t.cpu().numpy() for t in sc.omp_encode_csc(h, torch.from_numpy(Xill).to(DEV), 2, 0.0))
    assert sc.omp_stats(h)["fp64_refits"] == 40
    ref = oracle.omp(Dill, Xill[:1], 2)
    assert np.all(colptr == 2 * np.arange(41))
    for i in range(40):
        np.testing.assert_array_equal(rows[2 * i:2 * i + 2], ref["idx"][0])
        err = np.linalg.norm(vals[2 * i:2 * i + 2] - ref["coef"][0]) / np.linalg.norm(ref["coef"][0])
        assert err <= 1e-4, (i, err)
    h.destroy()
