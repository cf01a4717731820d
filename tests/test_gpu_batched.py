"""GPU parity of the batched multi-scene encoder (sc_omp_encode_batched) and
its autotuner (sc_batch_autotune), through the C ABI.

The batched launch runs the same tile body as sc_omp_encode, so with the
same correlation stage and row cache every scene's codes equal the
single-dictionary encoder's bit for bit; against the FP64 oracle they meet
the same bar as sc_omp_encode (exact supports on well-separated signals,
1e-4 coefficients, 1% aggregate residual)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2605_30396_amd import inputs as I
from paper_2605_30396_amd import sc
from parity import compare_codes

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def make_scene(K, k, eps, N, seed, s=4):
    rng = I.rng_for(seed)
    D = I.random_dictionary(rng, K)
    X, _, _ = I.sparse_signals(rng, D, N, min(s, k), 1e-3)
    return D, X


def to_np(out):
    idx, coef, count, resid = out
    return dict(idx=idx.cpu().numpy(), coef=coef.cpu().numpy(), count=count.cpu().numpy(),
                resid=resid.cpu().numpy())


def single(h, X, k, eps, corr, rc):
    h.set_tuning(sc.TUNE_FP32_CORRELATION, corr)
    h.set_tuning(sc.TUNE_ROW_CACHE, rc)
    return to_np(sc.omp_encode(h, X, k, eps))


# (K, k, eps, N): every class of the launch (E = 1, 2, 4, 8; KMAX = 4..16),
# empty and one-signal scenes, ragged tails; at K = 512 the caps whose bodies
# keep 2 Gram rows (KMAX <= 12) and none (KMAX = 16) when the row cache is on
SCENES = [(512, 12, 1e-2, 4133), (256, 16, 0.0, 1000), (128, 4, 0.0, 37), (64, 8, 0.0, 777), (512, 4, 0.0, 0),
          (300, 12, 0.0, 1), (200, 8, 1e-2, 2049), (90, 16, 0.0, 513), (512, 8, 0.0, 333), (512, 16, 0.0, 701)]

TUNINGS = [None,
           dict(tile=32, row_cache=4, wg_per_cu=1, order=sc.ORDER_GIVEN, corr=sc.CORR_MFMA),
           dict(tile=16, row_cache=4, wg_per_cu=2, order=sc.ORDER_COST, corr=sc.CORR_VALU),
           dict(tile=32, row_cache=0, wg_per_cu=0, order=sc.ORDER_COST, corr=sc.CORR_MFMA),
           dict(tile=16, row_cache=4, wg_per_cu=0, order=sc.ORDER_GIVEN, corr=sc.CORR_MFMA)]


@pytest.mark.parametrize("tuning", TUNINGS)
def test_batched_equals_single_dictionary(tuning):
    hs, scenes, data = [], [], []
    for q, (K, k, eps, N) in enumerate(SCENES):
        D, X = make_scene(K, k, eps, N, 400 + q)
        h = sc.gram_precompute(torch.from_numpy(D).to(DEV))
        Xg = torch.from_numpy(X).to(DEV)
        hs.append(h)
        scenes.append(dict(dict=h, X=Xg, k=k, eps=eps))
        data.append((D, X))
    outs = sc.omp_encode_batched(scenes, tuning)
    torch.cuda.synchronize()
    t = tuning or dict(row_cache=0, corr=sc.CORR_VALU)
    for q, (K, k, eps, N) in enumerate(SCENES):
        g = to_np(outs[q])
        ref = single(hs[q], scenes[q]["X"], k, eps, t["corr"], t["row_cache"])
        for key in ("idx", "count", "coef", "resid"):
            np.testing.assert_array_equal(g[key], ref[key], err_msg=f"scene {q} {key}")
    for h in hs:
        h.destroy()


def test_thirty_two_small_scenes_in_one_launch():
    """The most scenes a launch takes (32): 0..97 signals each over six
    dictionaries of every class (several scenes share a handle), caps 4..16,
    eps 0 or 1e-2; workgroups switch scenes many times and fetch each next
    tile number while encoding the current tile.  Every scene's codes equal
    the single-dictionary encoder's with the same correlation stage and row
    cache, bit for bit."""
    Ks = [64, 128, 256, 512, 90, 300]
    hs, Ds = [], []
    for i, K in enumerate(Ks):
        D = I.random_dictionary(I.rng_for(700 + i), K)
        Ds.append(D)
        hs.append(sc.gram_precompute(torch.from_numpy(D).to(DEV)))
    sizes = I.rng_for(710).integers(0, 98, size=32)
    scenes, which = [], []
    for q in range(32):
        hi, k = q % len(Ks), (4, 8, 12, 16)[(q // len(Ks)) % 4]
        X, _, _ = I.sparse_signals(I.rng_for(720 + q), Ds[hi], int(sizes[q]), min(4, k), 1e-3)
        scenes.append(dict(dict=hs[hi], X=torch.from_numpy(X).to(DEV), k=k, eps=1e-2 if q % 3 == 0 else 0.0))
        which.append(hi)
    for t in (dict(tile=32, row_cache=4, wg_per_cu=1, order=sc.ORDER_GIVEN, corr=sc.CORR_MFMA),
              dict(tile=16, row_cache=0, wg_per_cu=0, order=sc.ORDER_COST, corr=sc.CORR_VALU)):
        outs = sc.omp_encode_batched(scenes, t)
        torch.cuda.synchronize()
        for q, s in enumerate(scenes):
            g = to_np(outs[q])
            ref = single(hs[which[q]], s["X"], s["k"], s["eps"], t["corr"], t["row_cache"])
            for key in ("idx", "count", "coef", "resid"):
                np.testing.assert_array_equal(g[key], ref[key], err_msg=f"tuning {t} scene {q} {key}")
    for h in hs:
        h.destroy()


def test_sixteen_scene_batch_against_oracle():
    """The 16-scene batch (sizes log-uniform in 50k..6M, K in {128, 256, 512},
    k in {4, 8, 12, 16}, eps = 0) with each scene cut to 20,000 signals; all
    scenes in one launch, 300 signals per scene checked by the oracle."""
    specs = I.scene_batch_specs()
    hs, scenes, data = [], [], []
    for sp in specs:
        D, X = I.scene_inputs(sp, N_override=min(sp["N"], 20000))
        h = sc.gram_precompute(torch.from_numpy(D).to(DEV))
        hs.append(h)
        scenes.append(dict(dict=h, X=torch.from_numpy(X).to(DEV), k=sp["k"], eps=0.0))
        data.append((D, X))
    outs = sc.omp_encode_batched(scenes)
    torch.cuda.synchronize()
    rs = np.random.Generator(np.random.PCG64(41))
    for q, sp in enumerate(specs):
        D, X = data[q]
        g = to_np(outs[q])
        sel = rs.choice(len(X), 300, replace=False)
        r = compare_codes(D, X[sel], sp["k"], 0.0, {k_: v[sel] for k_, v in g.items()}, min_sep_frac=0.2)
        assert sc.omp_stats(hs[q])["signals"] == len(X)
        print(q, sp, r["separated"], r["resid_gap"])
    for h in hs:
        h.destroy()


def test_fp64_refit_inside_a_batch():
    a2 = np.array([1.0, 1e-3, 0.0]) / np.sqrt(1 + 1e-6)
    Dill = np.array([[1, 0, 0], a2, [0, 0, 1]], np.float32)
    Xill = np.tile(np.array([[0, 1, 0]], np.float32), (70, 1))
    D2, X2 = make_scene(256, 8, 0.0, 500, 431)
    h1 = sc.gram_precompute(torch.from_numpy(Dill).to(DEV))
    h2 = sc.gram_precompute(torch.from_numpy(D2).to(DEV))
    scenes = [dict(dict=h2, X=torch.from_numpy(X2).to(DEV), k=8, eps=0.0),
              dict(dict=h1, X=torch.from_numpy(Xill).to(DEV), k=2, eps=0.0)]
    outs = sc.omp_encode_batched(scenes)
    torch.cuda.synchronize()
    g = to_np(outs[1])
    ref = oracle.omp(Dill, Xill, 2)
    np.testing.assert_array_equal(g["idx"], ref["idx"])
    np.testing.assert_array_equal(g["count"], ref["count"])
    err = np.linalg.norm(g["coef"] - ref["coef"], axis=1) / np.linalg.norm(ref["coef"], axis=1)
    assert err.max() <= 1e-4
    assert sc.omp_stats(h1)["fp64_refits"] == 70
    # the same scene without the refit keeps the FP32 coefficients
    scenes[1]["flags"] = sc.NO_FP64_REFIT
    sc.omp_stats(h1, reset=True)
    sc.omp_encode_batched(scenes)
    assert sc.omp_stats(h1)["fp64_refits"] == 0
    h1.destroy()
    h2.destroy()


def test_batched_argument_errors():
    D, X = make_scene(128, 4, 0.0, 64, 450)
    h = sc.gram_precompute(torch.from_numpy(D).to(DEV))
    Xg = torch.from_numpy(X).to(DEV)
    ok = dict(dict=h, X=Xg, k=4, eps=0.0)
    with pytest.raises(ValueError):
        sc.omp_encode_batched([ok] * 33)
    for bad in (dict(ok, k=0), dict(ok, k=17), dict(ok, eps=-1.0), dict(ok, eps=float("nan")),
                dict(ok, flags=sc.PREC_BF16)):
        with pytest.raises(sc.ScError) as e:
            sc.omp_encode_batched([ok, bad])
        assert e.value.code == sc.SC_EINVAL
    Dbig = I.random_dictionary(I.rng_for(451), 600)
    hb = sc.gram_precompute(torch.from_numpy(Dbig).to(DEV))
    with pytest.raises(sc.ScError):
        sc.omp_encode_batched([dict(dict=hb, X=Xg, k=4, eps=0.0)])
    for t in (dict(tile=8, row_cache=0, wg_per_cu=0, order=0, corr=0),
              dict(tile=16, row_cache=2, wg_per_cu=0, order=0, corr=0),
              dict(tile=16, row_cache=0, wg_per_cu=-1, order=0, corr=0),
              dict(tile=16, row_cache=0, wg_per_cu=0, order=2, corr=0),
              dict(tile=16, row_cache=0, wg_per_cu=0, order=0, corr=5)):
        with pytest.raises(sc.ScError):
            sc.omp_encode_batched([ok], t)
    small = torch.empty(8, dtype=torch.uint8, device=DEV)
    with pytest.raises(sc.ScError) as e:
        sc.omp_encode_batched([ok], workspace=small)
    assert e.value.code == sc.SC_ENOMEM
    hb.destroy()
    h.destroy()


def test_autotuner_picks_a_valid_shape():
    specs = I.scene_batch_specs()[:6]
    hs, scenes = [], []
    for sp in specs:
        D, X = I.scene_inputs(sp, N_override=min(sp["N"], 30000))
        h = sc.gram_precompute(torch.from_numpy(D).to(DEV))
        hs.append(h)
        scenes.append(dict(dict=h, X=torch.from_numpy(X).to(DEV), k=sp["k"], eps=0.0))
    best, ms = sc.batch_autotune(scenes, sample=8192)
    t = best.as_dict()
    assert t["tile"] in (16, 32) and t["row_cache"] in (0, 4) and t["wg_per_cu"] in (0, 1, 2)
    assert t["order"] in (sc.ORDER_COST, sc.ORDER_GIVEN) and t["corr"] in (sc.CORR_VALU, sc.CORR_MFMA)
    assert 0 < ms < 1e4
    outs = sc.omp_encode_batched(scenes, best)
    torch.cuda.synchronize()
    for q, sp in enumerate(specs):
        ref = single(hs[q], scenes[q]["X"], sp["k"], 0.0, t["corr"], t["row_cache"])
        g = to_np(outs[q])
        for key in ("idx", "count", "coef"):
            np.testing.assert_array_equal(g[key], ref[key])
    print("autotuned", t, ms)
    for h in hs:
        h.destroy()
