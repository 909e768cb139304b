"""Pins for the oracle's PbP-QLP against the mathematics it must reach.

* brute force: the plain definition evaluated at 50 significant digits with
  mpmath's own QR and Cholesky (no re-orthonormalization needed there);
* a special case with a textbook routine: Q L^T P^T equals the orthogonal
  projection Q Q^T A that the randomized SVD with the same Omega also returns;
* closed forms: L = chol(R R^T), ||A - Ahat||_F^2 = ||A||_F^2 - ||L||_F^2;
* exact recovery when rank(A) <= l, orthonormality, argument rules, and the
  orientation (the spec form is the paper's Algorithm 1 applied to A^T).
"""
import math

import mpmath
import numpy as np
import pytest

import synth
from oracle import (householder_qr, omega, pbpqlp, pbpqlp_alg1, rel_residual,
                    validate_args)


def _planted_tiny(m, n, sig, seed):
    rng = synth.rng_for(seed)
    U = synth.haar_panel(rng, m, len(sig))
    V = synth.haar_panel(rng, n, len(sig))
    return (U * np.asarray(sig)) @ V.T


def _mp_qr_signed(M):
    Q, R = mpmath.qr(M, mode="skinny")
    c = R.cols
    for j in range(c):
        if R[j, j] < 0:
            for i in range(Q.rows):
                Q[i, j] = -Q[i, j]
            for i in range(c):
                R[j, i] = -R[j, i]
    return Q, R


def _brute_force(A, Om, q):
    """Definition: Q = qr((A A^T)^q A Omega), [P, R] = qr(A^T Q),
    L = chol(R R^T), Qtilde = R^T L^-T, output Q Qtilde."""
    mpmath.mp.dps = 50
    Am = mpmath.matrix(A.tolist())
    K = Am * mpmath.matrix(Om.tolist())
    AAt = Am * Am.T
    for _ in range(q):
        K = AAt * K
    Q, _ = _mp_qr_signed(K)
    P, R = _mp_qr_signed(Am.T * Q)
    L = mpmath.cholesky(R * R.T)
    Qt = R.T * (L.T) ** -1
    to = lambda M: np.array(M.tolist(), dtype=np.float64)
    return to(Q * Qt), to(L), to(P), to(R)


@pytest.mark.parametrize("q", [0, 1, 2])
def test_matches_50_digit_brute_force(q):
    sig = [3.0, 2.5, 2.0, 1.5, 1.0, 0.7, 0.5, 0.3, 0.2]
    A = _planted_tiny(12, 9, sig, 21 + q)
    k, p = 3, 1
    Om = omega(9, k + p, 77)
    r = pbpqlp(A, k, p, q, Omega=Om)
    Qb, Lb, Pb, Rb = _brute_force(A, Om, q)
    np.testing.assert_allclose(r.Q, Qb, atol=1e-12)
    np.testing.assert_allclose(r.L, Lb, atol=1e-12)
    np.testing.assert_allclose(r.P, Pb, atol=1e-12)
    np.testing.assert_allclose(r.R, Rb, atol=1e-12)


@pytest.mark.parametrize("q", [0, 1, 3])
def test_equals_randomized_svd_projection(q):
    # The randomized SVD with the same Omega and power scheme returns
    # Ubar Ubar^T A with Ubar = orth((A A^T)^q A Omega); PbP-QLP's Q L^T P^T is
    # the same orthogonal projection (both keep range(Ubar)).
    rng = synth.rng_for(500 + q)
    A = rng.standard_normal((80, 60))
    k, p = 10, 5
    r = pbpqlp(A, k, p, q, seed=4)
    K = A @ r.Omega
    for _ in range(q):
        K = A @ (A.T @ K)
    Ubar, _ = np.linalg.qr(K)
    G = Ubar.T @ A
    Uu, s, Vt = np.linalg.svd(G, full_matrices=False)
    rsvd = (Ubar @ Uu) * s @ Vt
    np.testing.assert_allclose(r.reconstruct(), rsvd, atol=1e-12)


def test_L_is_cholesky_of_R_Rt_and_lower_triangular():
    w = synth.config1()
    r = pbpqlp(w.A, w.k, w.p, w.q, w.seed)
    assert np.array_equal(r.L, np.tril(r.L))
    assert np.all(np.diag(r.L) > 0)
    np.testing.assert_allclose(r.L, np.linalg.cholesky(r.R @ r.R.T), atol=1e-13)
    np.testing.assert_allclose(r.Qtilde @ r.L.T, r.R.T, atol=1e-13)


def test_residual_identity_and_orthonormality_config1():
    w = synth.config1()
    r = pbpqlp(w.A, w.k, w.p, w.q, w.seed)
    l = w.l
    assert np.abs(r.Q.T @ r.Q - np.eye(l)).max() <= 1e-12
    assert np.abs(r.P.T @ r.P - np.eye(l)).max() <= 1e-12
    res = rel_residual(w.A, r.Q, r.L, r.P)
    na2 = float(np.sum(w.A * w.A))
    ident = math.sqrt(max(na2 - float(np.sum(r.L * r.L)), 0.0) / na2)
    assert abs(res - ident) <= 1e-12 * max(1.0, res) + 1e-9 * res
    # close to the optimal rank-l error, which the planted spectrum fixes
    opt = math.sqrt(float(np.sum(w.sigma[l:] ** 2)) / float(np.sum(w.sigma ** 2)))
    assert opt <= res <= 1.01 * opt


@pytest.mark.parametrize("rank,l", [(5, 8), (8, 8), (3, 12)])
def test_exact_recovery_low_rank(rank, l):
    rng = synth.rng_for(700 + rank)
    A = (rng.standard_normal((90, rank)) @ rng.standard_normal((rank, 70)))
    r = pbpqlp(A, l - 2, 2, 1, seed=rank)
    assert rel_residual(A, r.Q, r.L, r.P) <= 1e-13
    assert np.abs(r.Q.T @ r.Q - np.eye(l)).max() <= 1e-12
    assert np.abs(r.P.T @ r.P - np.eye(l)).max() <= 1e-12
    # diag(L) beyond the rank is at rounding level
    assert np.all(np.abs(np.diag(r.L)[rank:]) <= 1e-12 * np.abs(r.L[0, 0]))


def test_full_width_sketch_is_exact():
    rng = synth.rng_for(800)
    A = rng.standard_normal((40, 25))
    r = pbpqlp(A, 20, 5, 0, seed=1)
    assert rel_residual(A, r.Q, r.L, r.P) <= 1e-13


def test_zero_matrix():
    A = np.zeros((30, 20))
    r = pbpqlp(A, 4, 2, 1, seed=3)
    np.testing.assert_array_equal(r.L, np.zeros((6, 6)))
    np.testing.assert_allclose(r.Q.T @ r.Q, np.eye(6), atol=1e-15)
    np.testing.assert_allclose(r.P.T @ r.P, np.eye(6), atol=1e-15)


def test_orientation_is_algorithm1_on_transpose():
    rng = synth.rng_for(900)
    A = rng.standard_normal((50, 35))
    k, p, q = 6, 4, 2
    r = pbpqlp(A, k, p, q, seed=11)
    Qp, Lp, Pp, Rp = pbpqlp_alg1(A.T, r.Omega, q)     # paper notation on A^T
    np.testing.assert_allclose(Qp, r.P, atol=1e-13)    # paper Q  <-> spec P
    np.testing.assert_allclose(Pp, r.Q, atol=1e-13)    # paper P  <-> spec Q Qtilde
    np.testing.assert_allclose(Lp, r.L, atol=1e-13)
    # A^T ~= Qp Lp Pp^T  <=>  A ~= Q L^T P^T
    np.testing.assert_allclose((Qp @ Lp @ Pp.T).T, r.reconstruct(), atol=1e-13)
    # the literal "Q L P^T" is a different, clearly worse matrix on a decaying spectrum
    B = _planted_tiny(50, 35, 0.7 ** np.arange(20), 902)
    rb = pbpqlp(B, k, p, q, seed=11)
    lit = rb.Q @ rb.L @ rb.P.T
    assert np.linalg.norm(B - lit) > 3 * np.linalg.norm(B - rb.reconstruct())


@pytest.mark.parametrize("args", [(0, 5, 1, 0, 0), (5, 5, 0, 0, 0), (5, 5, 3, -1, 0),
                                  (5, 5, 4, 2, 0), (5, 5, 2, 0, -1), (5, 5, 2, 0, 17)])
def test_argument_rules(args):
    with pytest.raises(ValueError):
        validate_args(*args)


def test_sign_normalized_R_diagonal():
    rng = synth.rng_for(901)
    A = rng.standard_normal((60, 40))
    r = pbpqlp(A, 8, 4, 1, seed=2)
    assert np.all(np.diag(r.R) >= 0)
    assert np.all(np.diag(r.L) >= 0)
    Q2, R2 = householder_qr(A.T @ r.Qbasis)
    np.testing.assert_allclose(R2, r.R, atol=1e-13)
