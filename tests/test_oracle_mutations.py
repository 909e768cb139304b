"""Plausible mistakes planted in the oracle (on the CPU, via monkeypatch) must
be caught by at least one pin.  Each case reruns the pin's check against a
deliberately broken oracle and asserts that it now fails."""
import numpy as np
import pytest

import oracle.pbpqlp_oracle as O
from tests.test_oracle_pbpqlp import _brute_force, _planted_tiny


def _pin_brute_force():
    sig = [3.0, 2.5, 2.0, 1.5, 1.0, 0.7, 0.5, 0.3, 0.2]
    A = _planted_tiny(12, 9, sig, 22)
    Om = O.omega(9, 4, 77)
    r = O.pbpqlp(A, 3, 1, 1, Omega=Om)
    Qb, Lb, Pb, _ = _brute_force(A, Om, 1)
    return (np.allclose(r.Q, Qb, atol=1e-12) and np.allclose(r.L, Lb, atol=1e-12)
            and np.allclose(r.P, Pb, atol=1e-12))


def test_unbroken_oracle_passes():
    assert _pin_brute_force()


def test_dropped_sign_normalization_is_caught(monkeypatch):
    def qr_nosign(M):
        q, r = np.linalg.qr(M)
        return q, r
    monkeypatch.setattr(O, "householder_qr", qr_nosign)
    monkeypatch.setattr(O, "hh_orth", lambda M: qr_nosign(M)[0])
    assert not _pin_brute_force()


def test_missing_power_iteration_is_caught(monkeypatch):
    real = O.pbpqlp

    def one_less(A, k, p, q, seed=None, Omega=None):
        return real(A, k, p, max(q - 1, 0), seed=seed, Omega=Omega)
    monkeypatch.setattr(O, "pbpqlp", one_less)
    assert not _pin_brute_force()


def test_transposed_small_qr_is_caught(monkeypatch):
    # factoring R instead of R^T in the last step
    real_qr = O.householder_qr
    calls = {"n": 0}

    def qr_spy(M):
        calls["n"] += 1
        if M.shape[0] == M.shape[1] and np.allclose(M, np.tril(M)) and not np.allclose(M, np.triu(M)):
            return real_qr(M.T)
        return real_qr(M)
    monkeypatch.setattr(O, "householder_qr", qr_spy)
    assert not _pin_brute_force()


def test_wrong_omega_index_order_is_caught(monkeypatch):
    real = O.omega
    monkeypatch.setattr(O, "omega", lambda n, l, seed: real(l, n, seed).T.copy())
    # the by-hand Box-Muller pin recomputes element t = i*l + j
    from tests.test_oracle_rng import test_omega_box_muller_by_hand
    import tests.test_oracle_rng as R
    monkeypatch.setattr(R, "omega", O.omega)
    with pytest.raises(AssertionError):
        test_omega_box_muller_by_hand()


# ---- the learned q/k head's oracle --------------------------------------
import oracle.qk_mlp_oracle as QK
import tests.test_oracle_mlp as PQ


def _fails(check):
    try:
        check()
    except AssertionError:
        return True
    return False


def test_mlp_pins_pass_unbroken():
    for check in (PQ.test_gradient_matches_central_differences,
                  PQ.test_all_active_network_is_the_composed_affine_map,
                  PQ.test_relabelling_hidden_units_leaves_outputs_unchanged,
                  PQ.test_adam_constant_gradient_steps, PQ.test_adam_sign_flip_second_step):
        assert not _fails(check)


def test_mlp_transposed_hidden_weights_are_caught(monkeypatch):
    real = QK.forward

    def fwd_t(theta, X):
        W1, b1, W2, b2, W3, b3 = QK.unpack(theta)
        return real(QK.pack(W1, b1, W2.T, b2, W3, b3), X)
    monkeypatch.setattr(QK, "forward", fwd_t)
    assert _fails(PQ.test_all_active_network_is_the_composed_affine_map)
    assert _fails(PQ.test_relabelling_hidden_units_leaves_outputs_unchanged)


def test_mlp_missing_relu_mask_in_backward_is_caught(monkeypatch):
    # backward without the ReLU derivative: treat every unit as active
    def grad_linear(theta, X, q, logk):
        W1, b1, W2, b2, W3, b3 = QK.unpack(theta)
        X = np.asarray(X, dtype=np.float64)
        B = X.shape[0]
        z, (h1, h2) = QK.forward(theta, X)
        mx = z[:, :5].max(axis=1, keepdims=True)
        ls = z[:, :5] - mx - np.log(np.exp(z[:, :5] - mx).sum(axis=1, keepdims=True))
        err = z[:, 5] - logk
        loss = float(np.mean(-ls[np.arange(B), q]) + np.mean(err * err))
        dz = np.zeros_like(z)
        dz[:, :5] = np.exp(ls)
        dz[np.arange(B), q] -= 1.0
        dz[:, :5] /= B
        dz[:, 5] = 2.0 * err / B
        dh2 = dz @ W3
        dh1 = dh2 @ W2
        return loss, QK.pack(dh1.T @ X, dh1.sum(0), dh2.T @ h1, dh2.sum(0), dz.T @ h2, dz.sum(0))
    monkeypatch.setattr(QK, "loss_and_grad", grad_linear)
    assert _fails(PQ.test_gradient_matches_central_differences)


def test_adam_without_bias_correction_is_caught(monkeypatch):
    def adam_nobc(theta, g, st, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        st.t += 1
        st.m = beta1 * st.m + (1 - beta1) * g
        st.v = beta2 * st.v + (1 - beta2) * g * g
        return theta - lr * st.m / (np.sqrt(st.v) + eps)
    monkeypatch.setattr(QK, "adam_step", adam_nobc)
    assert _fails(PQ.test_adam_constant_gradient_steps)
