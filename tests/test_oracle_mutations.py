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
