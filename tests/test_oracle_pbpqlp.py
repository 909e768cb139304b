"""Pins for the oracle's PbP-QLP against the mathematics it must reach.

* brute force: the plain definition evaluated at 50 significant digits with
  mpmath's own QR and Cholesky (no re-orthonormalization needed there);
* a special case with a textbook routine: Q L^T P^T equals the orthogonal
  projection Q Q^T A that the randomized SVD with the same Omega also returns;
* closed forms: L = chol(R R^T), ||A - Ahat||_F^2 = ||A||_F^2 - ||L||_F^2;
* exact recovery when rank(A) <= l, orthonormality, argument rules, and the
  paper's own orientation (pbpqlp of A^T) against the defining equations.
"""
import math

import mpmath
import numpy as np
import pytest

import synth
from oracle import (householder_qr, omega, pbpqlp, rel_residual, validate_args)


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


def test_paper_orientation_from_definitions():
    """The paper's orientation (A is n1 x n2, Phi is n1 x d, A ~= Q L P^T) is
    pbpqlp(A.T, Omega=Phi) with the roles (P, L, Q) -> (Q, L, P).  Checked
    against the defining equations of Section III rather than against a
    second implementation:
      Pbar: orthonormal, QR-type basis of (A^T A)^q A^T Phi (eq. (c) and the
            power scheme of Section III-B);
      D = A Pbar = Q R with Q orthonormal, R upper with diag >= 0 (eqs. (D),
            (DQR));
      R^T = Pt Rt, L = Rt^T, P = Pbar Pt: then Q^T A P = L is lower
            triangular and L L^T = R R^T (eq. (R^T = Pt Rt));
      A_hat = Q L P^T = Q Q^T A Pbar Pbar^T (eq. (Ahat))."""
    rng = synth.rng_for(900)
    A = rng.standard_normal((50, 35))          # n1 x n2
    d, q = 10, 2
    Phi = omega(50, d, 11)
    r = pbpqlp(A.T, 6, 4, q, Omega=Phi)
    Pbar, Qp, Lp, Pp, Rp = r.Qbasis, r.P, r.L, r.Q, r.R
    I = np.eye(d)
    # Pbar spans the power sketch, nested like a QR factor of it
    K = A.T @ Phi
    for _ in range(q):
        K = A.T @ (A @ K)
    T = Pbar.T @ K
    np.testing.assert_allclose(Pbar @ T, K, atol=1e-11 * np.abs(K).max())
    np.testing.assert_allclose(np.tril(T, -1), 0.0, atol=1e-11 * np.abs(K).max())
    assert np.all(np.diag(T) > 0)
    np.testing.assert_allclose(Pbar.T @ Pbar, I, atol=1e-13)
    # D = A Pbar = Q R
    np.testing.assert_allclose(Qp @ Rp, A @ Pbar, atol=1e-12)
    np.testing.assert_allclose(Qp.T @ Qp, I, atol=1e-13)
    assert np.all(np.diag(Rp) >= 0) and np.array_equal(np.tril(Rp, -1), np.zeros((d, d)))
    # Q^T A P = L, lower triangular; L L^T = R R^T; P orthonormal in span(Pbar)
    np.testing.assert_allclose(Qp.T @ A @ Pp, Lp, atol=1e-12)
    assert np.array_equal(np.triu(Lp, 1), np.zeros((d, d))) and np.all(np.diag(Lp) >= 0)
    np.testing.assert_allclose(Lp @ Lp.T, Rp @ Rp.T, atol=1e-12)
    np.testing.assert_allclose(Pp.T @ Pp, I, atol=1e-13)
    np.testing.assert_allclose(Pbar @ (Pbar.T @ Pp), Pp, atol=1e-13)
    # A_hat = Q L P^T = Q Q^T A Pbar Pbar^T
    np.testing.assert_allclose(Qp @ Lp @ Pp.T, Qp @ (Qp.T @ A @ Pbar) @ Pbar.T, atol=1e-12)
    # the spec form of A^T: A^T ~= Q' L^T P'^T with (Q', P') = (Pp, Qp)
    np.testing.assert_allclose(r.reconstruct(), (Qp @ Lp @ Pp.T).T, atol=1e-13)
    # the literal "Q L P^T" of the spec outputs is a different, clearly
    # worse matrix on a decaying spectrum
    Bm = _planted_tiny(50, 35, 0.7 ** np.arange(20), 902)
    rb = pbpqlp(Bm, 6, 4, q, seed=11)
    lit = rb.Q @ rb.L @ rb.P.T
    assert np.linalg.norm(Bm - lit) > 3 * np.linalg.norm(Bm - rb.reconstruct())


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
