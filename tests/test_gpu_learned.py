"""The learned q/k head on the GPU against its FP64 CPU oracle.

Forward pass, loss, gradient and Adam steps are compared with
oracle/qk_mlp_oracle.py at FP32 tolerances; the probe features with the
oracle's feature map; pbpqlp_factor_auto's choice and fallback with plain
pbpqlp_factor calls (bit for bit)."""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import qk as O
from paper_2103_07245_amd import pbpqlp as B
from paper_2103_07245_amd import train_qk as T

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _batch(seed, n):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1.0, 0.3, size=(n, 64)).astype(np.float32)
    q = rng.integers(0, 5, size=n).astype(np.int32)
    logk = np.log(rng.integers(1, 57, size=n)).astype(np.float32)
    return X, q, logk


def _close(a, b, rtol, what):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    err = np.abs(a - b).max()
    assert err <= rtol * max(1.0, np.abs(b).max()), (what, err)


@pytest.mark.parametrize("batch", [1, 37, 300])
def test_forward_matches_oracle(batch):
    print(f"mlp forward batch={batch}", flush=True)
    theta = synth.mlp_init(11)
    theta[-6:] = np.linspace(-0.5, 0.5, 6)
    X, _, _ = _batch(batch, batch)
    md = B.Model(theta)
    Z = md.forward(X).cpu().numpy()
    Zr, _ = O.forward(theta.astype(np.float64), X.astype(np.float64))
    # FP32 dot products of length <= 128 through three layers
    _close(Z, Zr, 2e-5, "outputs")
    md.close()


@pytest.mark.parametrize("batch", [5, 64, 257])
def test_loss_and_gradient_match_oracle(batch):
    print(f"mlp loss/grad batch={batch}", flush=True)
    theta = synth.mlp_init(12)
    X, q, logk = _batch(100 + batch, batch)
    md = B.Model(theta)
    loss, g = md.loss_grad(X, q, logk)
    lr_, gr = O.loss_and_grad(theta.astype(np.float64), X.astype(np.float64), q, logk.astype(np.float64))
    assert abs(float(loss.item()) - lr_) <= 1e-5 * max(1.0, abs(lr_))
    g = g.cpu().numpy()
    # compare every parameter group at its own scale
    offs = np.cumsum([0, 128 * 64, 128, 128 * 128, 128, 6 * 128, 6])
    for a, b in zip(offs[:-1], offs[1:]):
        _close(g[a:b], gr[a:b], 5e-5, f"grad[{a}:{b}]")
    md.close()


def test_adam_training_steps_match_oracle():
    theta = synth.mlp_init(13)
    md = B.Model(theta)
    st = O.AdamState()
    th = theta.astype(np.float64)
    lrs = [3e-3, 2e-3, 1e-3, 1e-3]
    for i, lr in enumerate(lrs):
        X, q, logk = _batch(200 + i, 48)
        md.train_step(X, q, logk, lr)
        _, g = O.loss_and_grad(th, X.astype(np.float64), q, logk.astype(np.float64))
        th = O.adam_step(th, g, st, lr)
    got = md.params()
    assert md.steps == len(lrs)
    # each step moves a parameter by at most lr; FP32 rounding of the moments
    assert np.abs(got - th).max() <= 2e-5
    assert np.abs(got - theta).max() > 1e-3      # it did move
    md.close()


def test_save_load_resumes_training(tmp_path):
    md = B.Model(synth.mlp_init(14))
    for i in range(3):
        X, q, logk = _batch(300 + i, 32)
        md.train_step(X, q, logk, 1e-3)
    path = tmp_path / "m.bin"
    md.save(str(path))
    md2 = B.Model.load(str(path))
    assert md2.steps == 3
    assert np.array_equal(md.params(), md2.params())
    X, q, logk = _batch(400, 32)
    md.train_step(X, q, logk, 1e-3)
    md2.train_step(X, q, logk, 1e-3)
    assert np.array_equal(md.params(), md2.params())
    md.close(); md2.close()


def test_probe_features_match_oracle():
    spec = synth.qk_spec(0, 42, (300, 300), (260, 260), 200, family="exp")
    A = synth.qk_matrix(spec)
    At = torch.from_numpy(A).to(DEV)
    f, L, info = B.probe(At, spec.seed_omega)
    L = L.cpu().numpy()
    # the kernel's map applied to the GPU's own L
    assert np.abs(f.cpu().numpy() - O.features(L)).max() <= 1e-6
    # and against the oracle probe (FP64 throughout)
    from oracle import pbpqlp as oracle_pbpqlp
    ref = oracle_pbpqlp(A, 56, 8, 0, spec.seed_omega)
    assert np.abs(f.cpu().numpy() - O.features(ref.L)).max() <= 1e-6


def _const_model(q_logits, k):
    W1, b1, W2, b2, W3, b3 = O.unpack(np.zeros(O.N_PARAMS))
    b3 = np.array(list(q_logits) + [math.log(k)])
    return B.Model(O.pack(W1, b1, W2, b2, W3, b3).astype(np.float32))


@pytest.mark.parametrize("tau,expect_fallback", [(1.0, False), (1e-9, True)])
def test_factor_auto_choice_and_fallback(tau, expect_fallback):
    print(f"factor_auto tau={tau}", flush=True)
    spec = synth.qk_spec(1, 43, (400, 400), (300, 300), 200, family="poly")
    At = torch.from_numpy(synth.qk_matrix(spec, np.float32)).to(DEV)
    md = _const_model([0.0, 2.0, 0.5, 0.1, -1.0], 9.4)     # q_hat = 1, k_hat = 9
    Q, L, P, res, info = B.factor_auto(md, At, 8, spec.seed_omega, 40, tau)
    assert res["q_pred"] == 1 and res["k_pred"] == 9
    assert res["fell_back"] == int(expect_fallback)
    q_used = 3 if expect_fallback else 1
    assert res["q_used"] == q_used and res["k_used"] == 9
    Qr, Lr, Pr, infr = B.factor(At, 9, 8, q_used, spec.seed_omega)
    assert torch.equal(Q, Qr) and torch.equal(L, Lr) and torch.equal(P, Pr)
    assert res["resid_final"] == infr.resid_rel_est
    md.close()


def test_factor_auto_prediction_equals_batched_forward():
    spec = synth.qk_spec(2, 44, (500, 500), (420, 420), 200, family="step")
    At = torch.from_numpy(synth.qk_matrix(spec, np.float32)).to(DEV)
    md = B.Model(synth.mlp_init(15))
    f, _, _ = B.probe(At, spec.seed_omega)
    z = md.forward(f[None, :]).cpu().numpy()[0]
    qh = int(np.argmax(z[:5]))
    kh = int(min(40, max(1, math.floor(math.exp(min(float(z[5]), 30.0)) + 0.5))))
    _, _, _, res, _ = B.factor_auto(md, At, 8, spec.seed_omega, 40, 1.0)
    assert (res["q_pred"], res["k_pred"]) == (qh, kh)
    md.close()


def test_label_rules_agree_with_oracle():
    rng = np.random.default_rng(5)
    for i in range(50):
        _, s = synth.spectrum_family(rng, 200)
        assert T.k_star(s) == O.k_star(s, 56)
        l = T.k_star(s) + 8
        assert T.r_opt(s, l) == pytest.approx(O.r_opt(s, l), rel=1e-14)
        rs = sorted(rng.uniform(0.5, 3.0, 5) * O.r_opt(s, l), reverse=True)
        assert T.q_star(rs, O.r_opt(s, l)) == O.q_star(rs, O.r_opt(s, l))
