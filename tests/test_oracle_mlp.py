"""Pins of the learned q/k head's FP64 oracle (oracle/qk_mlp_oracle.py).

Each check rests on something other than the oracle's own formulas: central
finite differences of the loss, the affine closed form of a network whose
units are all active, invariance under relabelling hidden units, closed-form
Adam steps, and features / labels of hand-made spectra."""
import math

import numpy as np
import pytest

from oracle import qk as O


def _params(seed, scale=0.2):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(O.N_PARAMS) * scale


def _batch(seed, B=7):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1.0, 0.5, size=(B, O.N_IN))
    q = rng.integers(0, O.N_Q, size=B)
    logk = np.log(rng.integers(1, 57, size=B).astype(np.float64))
    return X, q, logk


def test_parameter_count():
    # 64*128 + 128 + 128*128 + 128 + 128*6 + 6
    assert O.N_PARAMS == 25606


def test_gradient_matches_central_differences():
    theta = _params(1)
    X, q, logk = _batch(2)
    _, g = O.loss_and_grad(theta, X, q, logk)
    rng = np.random.default_rng(3)
    # offsets of the six groups; probe several entries in each
    sizes = [128 * 64, 128, 128 * 128, 128, 6 * 128, 6]
    starts = np.cumsum([0] + sizes[:-1])
    h = 1e-6
    for s0, sz in zip(starts, sizes):
        for idx in rng.choice(sz, size=min(sz, 12), replace=False):
            i = int(s0 + idx)
            tp = theta.copy(); tp[i] += h
            tm = theta.copy(); tm[i] -= h
            lp, _ = O.loss_and_grad(tp, X, q, logk)
            lm, _ = O.loss_and_grad(tm, X, q, logk)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[i]) <= 1e-7 + 1e-5 * abs(fd), (i, fd, g[i])


def test_all_active_network_is_the_composed_affine_map():
    rng = np.random.default_rng(4)
    W1 = rng.uniform(0.0, 0.1, (128, 64)); b1 = rng.uniform(0.1, 0.2, 128)
    W2 = rng.uniform(0.0, 0.1, (128, 128)); b2 = rng.uniform(0.1, 0.2, 128)
    W3 = rng.standard_normal((6, 128)); b3 = rng.standard_normal(6)
    theta = O.pack(W1, b1, W2, b2, W3, b3)
    X = rng.uniform(0.0, 1.0, (5, 64))           # every pre-activation > 0
    z, _ = O.forward(theta, X)
    M = W3 @ W2 @ W1                               # composed linear part
    c = W3 @ (W2 @ b1 + b2) + b3                   # composed offset
    assert np.allclose(z, X @ M.T + c, rtol=1e-12, atol=1e-12)


def test_relabelling_hidden_units_leaves_outputs_unchanged():
    theta = _params(5)
    W1, b1, W2, b2, W3, b3 = O.unpack(theta)
    rng = np.random.default_rng(6)
    p1, p2 = rng.permutation(128), rng.permutation(128)
    theta2 = O.pack(W1[p1], b1[p1], W2[p2][:, p1], b2[p2], W3[:, p2], b3)
    X, _, _ = _batch(7)
    assert np.allclose(O.forward(theta, X)[0], O.forward(theta2, X)[0], rtol=1e-12, atol=1e-13)


def test_zero_network_gives_uniform_softmax_loss():
    # all weights zero: logits = b3; with b3 = 0 the cross entropy is ln 5
    theta = np.zeros(O.N_PARAMS)
    X, q, _ = _batch(8)
    loss, g = O.loss_and_grad(theta, X, q, np.zeros(len(q)))
    assert abs(loss - math.log(5.0)) < 1e-14
    # gradient of b3 is the mean of softmax - onehot = 1/5 - frequency of q
    db3 = g[-6:]
    freq = np.bincount(q, minlength=5) / len(q)
    assert np.allclose(db3[:5], 0.2 - freq, atol=1e-15)


def test_large_logits_stay_finite():
    W1, b1, W2, b2, W3, b3 = O.unpack(np.zeros(O.N_PARAMS))
    b3 = np.array([1000.0, -1000.0, 0.0, 0.0, 0.0, 0.0])
    theta = O.pack(W1, b1, W2, b2, W3, b3)
    loss, g = O.loss_and_grad(theta, np.zeros((2, 64)), np.array([0, 1]), np.zeros(2))
    assert math.isfinite(loss) and np.all(np.isfinite(g))
    assert abs(loss - 1000.0) < 1e-9   # sample 0 costs ~0, sample 1 costs 2000


def test_adam_constant_gradient_steps():
    # with bias correction every step of a constant gradient moves by
    # lr * g / (|g| + eps) exactly (m_hat = g and v_hat = g^2 at every t)
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    st = O.AdamState(4)
    th = np.zeros(4)
    lr, eps = 0.01, 1e-8
    for _ in range(3):
        prev = th
        th = O.adam_step(th, g, st, lr)
        assert np.allclose(prev - th, lr * g / (np.abs(g) + eps), rtol=1e-12, atol=0)


def test_adam_sign_flip_second_step():
    # g then -g: m_hat_2 = -(1 - b1) g / (1 + b1), v_hat_2 = g^2
    g = np.array([0.3, -1.5])
    st = O.AdamState(2)
    lr, b1, eps = 0.1, 0.9, 1e-8
    th1 = O.adam_step(np.zeros(2), g, st, lr)
    th2 = O.adam_step(th1, -g, st, lr)
    mhat = -(1 - b1) * g / (1 + b1)
    assert np.allclose(th1 - th2, lr * mhat / (np.abs(g) + eps), rtol=1e-12)


def test_features_of_a_known_diagonal():
    d = np.ones(64)
    d[0] = 2.0
    d[1] = 0.2              # ratio 0.1
    d[2] = 2e-6             # ratio 1e-6: not above the floor
    d[3] = 0.0
    d[4] = np.nan
    d[5] = 4.0              # ratio 2: above L_11
    L = np.diag(d)
    f = O.features(L)
    scale = math.log(1e6)
    assert f[0] == 0.0
    assert abs(f[1] - math.log(0.1) / scale) < 1e-15
    assert f[2] == -1.0 and f[3] == -1.0 and f[4] == -1.0
    assert abs(f[5] - math.log(2.0) / scale) < 1e-15
    assert np.all(O.features(np.zeros((64, 64))) == -1.0)


def test_labels_of_a_step_spectrum():
    # sigma = 1 (x10) then 1e-4 (x90): k* = 10, r_opt(l) closed form
    s = np.concatenate([np.ones(10), np.full(90, 1e-4)])
    assert O.k_star(s, 56) == 10
    l = 18
    assert abs(O.r_opt(s, l) - math.sqrt(82e-8 / (10 + 90e-8))) < 1e-18
    r_best = O.r_opt(s, l)
    assert O.q_star([10 * r_best, 1.06 * r_best, 1.04 * r_best, r_best, r_best], r_best) == 2
    assert O.q_star([2 * r_best] * 5, r_best) == 4
    # no singular value below 1e-3 sigma_1 before the cap
    assert O.k_star(np.linspace(1.0, 0.5, 100), 56) == 56


def test_predict_rounds_and_clamps():
    W1, b1, W2, b2, W3, b3 = O.unpack(np.zeros(O.N_PARAMS))
    b3 = np.array([0.0, 0.5, 0.1, 0.5, 0.0, math.log(12.4)])
    th = O.pack(W1, b1, W2, b2, W3, b3)
    assert O.predict(th, np.zeros(64), 56) == (1, 12)     # first of two equal maxima
    b3[5] = math.log(500.0)
    assert O.predict(O.pack(W1, b1, W2, b2, W3, b3), np.zeros(64), 56) == (1, 56)
