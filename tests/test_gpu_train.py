"""GPU training of the proposer: gradients of the hand-written kernels
against the FP64 oracle's backpropagation, Adam against the oracle's update,
and what the trained network gains over the untrained one."""
import numpy as np
import pytest
import torch

import oracle
from paper_2605_30396_amd import inputs as I
from paper_2605_30396_amd import sc, trainer

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def problem(K=256, N=256, k=4, seed=300, scale3=4.0):
    rng = I.rng_for(seed)
    D = I.random_dictionary(rng, K)
    X, _, _ = I.sparse_signals(rng, D, N, 4, 1e-3)
    ref = oracle.omp(D, X, k, 1e-2)
    P = I.mlp_init(rng, 45, 256, K)
    P["W3"] = P["W3"] * np.float32(scale3)
    return D, X, ref, P


def gpu_grads(P, X, ref, K, B, flags, pos_weight=1.0, rows=None):
    p = sc.proposer_create(45, 256, K)
    p.set_params(P)
    Xg = torch.from_numpy(X).to(DEV)
    sup = torch.from_numpy(ref["idx"]).to(DEV)
    cnt = torch.from_numpy(ref["count"]).to(DEV)
    loss = torch.zeros(1, device=DEV)
    grads = torch.zeros(p.nparams, device=DEV)
    rg = None if rows is None else torch.from_numpy(rows.astype(np.int32)).to(DEV)
    sc.proposer_train_step(p, Xg, sup, cnt, B, rows=rg, pos_weight=pos_weight, flags=flags | sc.TRAIN_GRAD_ONLY,
                           loss=loss, grads=grads)
    torch.cuda.synchronize()
    g = sc.unpack_params(grads.cpu(), 45, 256, K)
    out = float(loss.item()), {n: v.numpy().astype(np.float64) for n, v in g.items()}
    p.destroy()
    return out


@pytest.mark.parametrize("pos_weight", [1.0, 8.0])
def test_fp32_gradients_match_oracle(pos_weight):
    K, B = 256, 128
    D, X, ref, P = problem(K=K, N=300)
    rows = I.rng_for(301).choice(300, B, replace=False)
    loss, g = gpu_grads(P, X, ref, K, B, sc.TRAIN_FP32, pos_weight, rows)
    Y = oracle.multi_hot(ref["idx"][rows], ref["count"][rows], K)
    lref, gref = oracle.mlp_loss_and_grads(P, X[rows], Y, pos_weight, bf16=False)
    assert abs(loss - lref) <= 1e-5 * abs(lref)
    for n in gref:
        err = np.linalg.norm(g[n] - gref[n]) / np.linalg.norm(gref[n])
        assert err <= 1e-4, (n, err)


def test_bf16_gradients_match_oracle():
    K, B = 512, 256
    D, X, ref, P = problem(K=K, N=B, seed=302)
    loss, g = gpu_grads(P, X, ref, K, B, 0, 1.0)
    Y = oracle.multi_hot(ref["idx"], ref["count"], K)
    lref, gref = oracle.mlp_loss_and_grads(P, X, Y, 1.0, bf16=True)
    assert abs(loss - lref) <= 1e-3 * abs(lref)
    for n in gref:
        err = np.linalg.norm(g[n] - gref[n]) / np.linalg.norm(gref[n])
        assert err <= 2e-2, (n, err)


def test_adam_steps_match_oracle():
    """Three FP32 training steps of the GPU against the oracle's own
    trajectory from the same start: at every step the oracle takes its FP64
    gradients at its own parameters and applies Adam with its moments carried
    over (nothing of the GPU's state enters it).  Step t's update is compared
    on the parameters whose oracle gradient is clear of zero at every step so
    far (there the sign of each moment is fixed), at 2e-3 lr; a bias
    correction stuck at t = 1 or moments overwritten each step change those
    updates by 25-35% from t = 2 on."""
    K, B = 128, 64
    D, X, ref, P = problem(K=K, N=B, seed=303)
    p = sc.proposer_create(45, 256, K)
    p.set_params(P)
    Xg = torch.from_numpy(X).to(DEV)
    sup = torch.from_numpy(ref["idx"]).to(DEV)
    cnt = torch.from_numpy(ref["count"]).to(DEV)
    Y = oracle.multi_hot(ref["idx"], ref["count"], K)
    lr = 1e-4
    pref = {n: np.asarray(v, np.float64) for n, v in P.items()}
    m = {n: np.zeros_like(v) for n, v in pref.items()}
    v = {n: np.zeros_like(x) for n, x in pref.items()}
    clear = {n: np.ones(x.shape, bool) for n, x in pref.items()}
    before = {n: t.numpy().astype(np.float64) for n, t in sc.unpack_params(p.get_params().cpu(), 45, 256, K).items()}
    for step in (1, 2, 3):
        _, gref = oracle.mlp_loss_and_grads(pref, X, Y, 1.0)
        nref = oracle.adam_step(pref, gref, m, v, step, lr=lr)
        sc.proposer_train_step(p, Xg, sup, cnt, B, lr=lr, flags=sc.TRAIN_FP32)
        after = {n: t.numpy().astype(np.float64)
                 for n, t in sc.unpack_params(p.get_params().cpu(), 45, 256, K).items()}
        worst = 0.0
        for n in nref:
            clear[n] &= np.abs(gref[n]) > 1e-2 * np.abs(gref[n]).max()
            assert clear[n].mean() > 0.2, (n, step, clear[n].mean())
            upd_g = (after[n] - before[n])[clear[n]]
            upd_r = (nref[n] - pref[n])[clear[n]]
            err = np.max(np.abs(upd_g - upd_r)) / lr
            worst = max(worst, err)
            assert err <= 2e-3, (n, step, err)
        print(f"step {step}: worst update error {worst:.2e} lr")
        pref, before = nref, after
    p.destroy()


def test_training_gains_over_untrained_network():
    """A short GPU training run (2000 Adam steps) on 4-sparse signals over a
    K=512 dictionary: the loss falls, the share of signals whose whole OMP
    support lies among the 24 candidates rises above the untrained network's
    (which is ~0), and the learned encoder sends fewer signals to the
    full-OMP fallback."""
    D = I.learned_dictionary()
    Xtr = I.learned_train_signals(D, N=1 << 19)
    Xte = I.learned_eval_signals(D, N=8192)
    h = sc.gram_precompute(torch.from_numpy(D).to(DEV))
    Xtr_g, Xte_g = torch.from_numpy(Xtr).to(DEV), torch.from_numpy(Xte).to(DEV)
    sup, cnt = trainer.omp_labels(h, Xtr_g, 12, 1e-2)
    sup_te, cnt_te = trainer.omp_labels(h, Xte_g, 12, 1e-2)
    p = sc.proposer_create(45, 256, 512)
    p.set_params(I.mlp_init(I.rng_for(5), 45, 256, 512))

    def fallbacks():
        sc.omp_stats(h, reset=True)
        sc.omp_encode_learned(h, p, Xte_g, 12, 1e-2)
        return sc.omp_stats(h)["fallbacks"]

    r0, f0 = trainer.support_recall(p, Xte_g, sup_te, cnt_te), fallbacks()
    hist = trainer.train(p, Xtr_g, sup, cnt, epochs=4, batch=1024, lr=3e-3, pos_weight=8.0, seed=312)
    r1, f1 = trainer.support_recall(p, Xte_g, sup_te, cnt_te), fallbacks()
    print("recall@24 untrained", r0, "trained", r1, "fallbacks", f0, f1, "loss", hist["loss"], "s", hist["seconds"])
    assert hist["loss"][-1] < hist["loss"][0]
    assert r1 > r0 + 0.05
    assert f1 < f0 - 0.05 * len(Xte)
    h.destroy()
    p.destroy()
