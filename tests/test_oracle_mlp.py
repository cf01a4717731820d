"""Pins of the proposer-network oracle (no GPU): GELU special values, loss
closed forms, gradients against FP64 central differences, Adam's first step,
top-k tie order, bf16 rounding, and the learned-encoder composition."""
import math

import numpy as np
import pytest

import oracle
from oracle import mlp as M
from paper_2605_30396_amd import inputs as I


def test_gelu_values():
    np.testing.assert_allclose(oracle.gelu([0.0, 1.0, -1.0]), [0.0, 0.8413447460685429, -0.15865525393145707],
                               rtol=1e-15)
    assert oracle.gelu_grad(0.0) == 0.5
    t = np.linspace(-4, 4, 41)
    h = 1e-6
    np.testing.assert_allclose(oracle.gelu_grad(t), (oracle.gelu(t + h) - oracle.gelu(t - h)) / (2 * h),
                               rtol=1e-8, atol=1e-10)


def test_bce_closed_forms():
    z = np.zeros((2, 4))
    Y = np.array([[1, 0, 0, 0], [0, 0, 1, 1]], float)
    loss, dz = oracle.bce_with_logits(z, Y)
    assert abs(loss - math.log(2)) < 1e-15
    np.testing.assert_allclose(dz, (0.5 - Y) / 8, rtol=1e-15)
    loss_w, _ = oracle.bce_with_logits(z, Y, pos_weight=3.0)
    assert abs(loss_w - math.log(2) * (3 * 3 + 5) / 8) < 1e-14
    # large logits stay finite
    l2, d2 = oracle.bce_with_logits(np.array([[800.0, -800.0]]), np.array([[1.0, 0.0]]))
    assert l2 == 0.0 and np.all(d2 == 0.0)


def _small_params(rng, d=6, H=5, K=7):
    return I.mlp_init(rng, d, H, K)


@pytest.mark.parametrize("pos_weight", [1.0, 4.0])
def test_gradients_match_central_differences(pos_weight):
    rng = I.rng_for(40)
    P = {k: v.astype(np.float64) for k, v in _small_params(rng).items()}
    X = rng.standard_normal((9, 6))
    Y = (rng.random((9, 7)) < 0.3).astype(float)
    loss, g = oracle.mlp_loss_and_grads(P, X, Y, pos_weight)
    h = 1e-6
    for name, arr in P.items():
        num = np.zeros_like(arr)
        for ix in np.ndindex(arr.shape):
            a = dict(P)
            a[name] = arr.copy(); a[name][ix] += h
            lp, _ = oracle.mlp_loss_and_grads(a, X, Y, pos_weight)
            a[name] = arr.copy(); a[name][ix] -= h
            lm, _ = oracle.mlp_loss_and_grads(a, X, Y, pos_weight)
            num[ix] = (lp - lm) / (2 * h)
        scale = np.max(np.abs(num)) + 1e-12
        assert np.max(np.abs(num - g[name])) <= 1e-6 * scale, name


def test_forward_input_is_direction():
    rng = I.rng_for(41)
    P = _small_params(rng)
    X = rng.standard_normal((5, 6))
    z1 = oracle.mlp_forward(P, X)
    z2 = oracle.mlp_forward(P, 3.5 * X)
    np.testing.assert_allclose(z1, z2, rtol=1e-13)
    z0 = oracle.mlp_forward(P, np.zeros((1, 6)))
    # x = 0 feeds zeros: z = W3 GELU(W2 GELU(b1) + b2) + b3
    h1 = oracle.gelu(P["b1"].astype(float))
    h2 = oracle.gelu(P["W2"].astype(float) @ h1 + P["b2"])
    np.testing.assert_allclose(z0[0], P["W3"].astype(float) @ h2 + P["b3"], rtol=1e-13)


def test_adam_first_step_is_signed_lr():
    p = {"w": np.array([1.0, -2.0, 3.0])}
    g = {"w": np.array([0.5, -1e-3, 0.0])}
    m = {"w": np.zeros(3)}
    v = {"w": np.zeros(3)}
    out = oracle.adam_step(p, g, m, v, 1, lr=0.1, eps=0.0 + 1e-30)
    np.testing.assert_allclose(out["w"], [0.9, -1.9, 3.0], rtol=1e-12)


def test_adam_constant_gradient_is_signed_lr_at_every_step():
    """With a constant gradient g the moments are m_t = (1 - b1^t) g and
    v_t = (1 - b2^t) g^2, so the bias-corrected ratio is g / |g| at every step
    t: each update is -lr sign(g).  Moments overwritten instead of accumulated,
    or a bias correction stuck at t = 1, give 0.74 lr or 1.34 lr at t = 2."""
    g = {"w": np.array([0.5, -2.0, 1e-3])}
    p = {"w": np.array([1.0, -2.0, 3.0])}
    m = {"w": np.zeros(3)}
    v = {"w": np.zeros(3)}
    for t in range(1, 6):
        new = oracle.adam_step(p, g, m, v, t, lr=0.1, eps=1e-30)
        np.testing.assert_allclose(new["w"] - p["w"], [-0.1, 0.1, -0.1], rtol=1e-12)
        p = new


def test_adam_three_steps_worked_by_hand():
    """b1 = 1/2, b2 = 3/4, lr = 1/10, gradients 1, 3, -2 (eps negligible):
      t = 1: m = 1/2, v = 1/4; m^ = 1, v^ = 1 -> update -1/10
      t = 2: m = 1/4 + 3/2 = 7/4, v = 3/16 + 9/4 = 39/16;
             m^ = (7/4) / (3/4) = 7/3, v^ = (39/16) / (7/16) = 39/7 -> update -(7/3) / sqrt(39/7) / 10
      t = 3: m = 7/8 - 1 = -1/8, v = 117/64 + 1 = 181/64;
             m^ = (-1/8) / (7/8) = -1/7, v^ = (181/64) / (37/64) = 181/37 -> update (1/7) / sqrt(181/37) / 10"""
    p = {"w": np.array([0.0])}
    m = {"w": np.zeros(1)}
    v = {"w": np.zeros(1)}
    expected = [-0.1, -(7 / 3) / np.sqrt(39 / 7) / 10, (1 / 7) / np.sqrt(181 / 37) / 10]
    for t, (gv, de) in enumerate(zip((1.0, 3.0, -2.0), expected), start=1):
        new = oracle.adam_step(p, {"w": np.array([gv])}, m, v, t, lr=0.1, beta1=0.5, beta2=0.75, eps=1e-30)
        np.testing.assert_allclose(new["w"] - p["w"], [de], rtol=1e-13)
        p = new


def test_topk_order_and_ties():
    z = np.array([[0.1, 0.5, 0.5, -1.0, 0.5, 0.2]])
    np.testing.assert_array_equal(oracle.topk_lowest_index(z, 4), [[1, 2, 4, 5]])


def test_bf16_rounding():
    # 8 significant bits: halfway cases go to the even neighbour
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, 1.0 + 2 ** -9, 1.0 + 3 * 2 ** -8, -3.1415926])
    r = M.bf16_round(v)
    np.testing.assert_array_equal(r[:5], [1.0, 1.0, 1.0 + 2 ** -7, 1.0, 1.0 + 2 ** -6])
    assert abs(r[5] + 3.140625) < 1e-12


def test_multi_hot():
    idx = np.array([[3, 1, -1], [0, 2, 2]], np.int32)
    cnt = np.array([2, 1], np.int32)
    Y = oracle.multi_hot(idx, cnt, 5)
    np.testing.assert_array_equal(Y, [[0, 1, 0, 1, 0], [1, 0, 0, 0, 0]])


def test_learned_encode_composition():
    """With every atom a candidate the proposer-guided encoder is plain OMP;
    with few candidates, signals whose restricted pursuit misses eps fall back
    to full OMP, and the result always meets eps or equals full OMP."""
    rng = I.rng_for(42)
    D = I.random_dictionary(rng, 64)
    X, _, _ = I.sparse_signals(rng, D, 200, 4, 1e-3)
    P = I.mlp_init(rng, 45, 32, 64)
    full = oracle.omp(D, X, 8, 1e-2)
    allc = oracle.learned_encode(D, X, P, 8, 1e-2, n_cand=64)
    np.testing.assert_array_equal(allc["idx"], full["idx"])
    assert not allc["fallback"].any()
    few = oracle.learned_encode(D, X, P, 8, 1e-2, n_cand=6)
    assert few["fallback"].any()
    fb = few["fallback"]
    np.testing.assert_array_equal(few["idx"][fb], full["idx"][fb])
    assert np.all(few["resid"][~fb] <= 1e-2)
    # accepted restricted codes use only candidate atoms
    for i in np.nonzero(~fb)[0]:
        assert set(few["idx"][i, : few["count"][i]]) <= set(few["cand"][i])


def test_learned_encode_step_cap():
    """A restricted-step cap c keeps exactly the restricted codes that reach
    eps within c atoms (they equal the uncapped restricted codes of those
    signals); every other signal is the full OMP code, and cap = k changes
    nothing."""
    rng = I.rng_for(43)
    D = I.random_dictionary(rng, 64)
    X2, _, _ = I.sparse_signals(rng, D, 300, 2, 1e-3)
    X4, _, _ = I.sparse_signals(rng, D, 300, 4, 1e-3)
    X = np.concatenate([X2, X4])
    P = I.mlp_init(rng, 45, 32, 64)
    k, eps, nc = 8, 1e-2, 32
    full = oracle.omp(D, X, k, eps)
    base = oracle.learned_encode(D, X, P, k, eps, n_cand=nc)
    same = oracle.learned_encode(D, X, P, k, eps, n_cand=nc, cap=k)
    for key in ("idx", "count", "fallback"):
        np.testing.assert_array_equal(base[key], same[key])
    capped = oracle.learned_encode(D, X, P, k, eps, n_cand=nc, cap=3)
    acc = ~capped["fallback"]
    assert acc.any() and capped["fallback"].any()
    assert np.all(capped["count"][acc] <= 3) and np.all(capped["resid"][acc] <= eps)
    np.testing.assert_array_equal(capped["idx"][acc], base["idx"][acc])          # same restricted path
    np.testing.assert_array_equal(capped["idx"][~acc], full["idx"][~acc])
    # a signal accepted uncapped with more than 3 atoms is a miss under the cap
    long_ok = (~base["fallback"]) & (base["count"] > 3)
    assert long_ok.any() and np.all(capped["fallback"][long_ok])
    assert capped["idx"].shape == (len(X), k)
