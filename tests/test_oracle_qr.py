"""Pins for the oracle's unpivoted QR (the paper's qr and packaged-QR orth)
and its Jacobi SVD, against LAPACK through numpy."""
import numpy as np
import pytest

from oracle import householder_qr, hh_orth, jacobi_svd


def _signed_numpy_qr(M):
    q, r = np.linalg.qr(M)
    d = np.sign(np.diag(r))
    d[d == 0] = 1
    return q * d, d[:, None] * r


@pytest.mark.parametrize("shape", [(7, 7), (30, 5), (200, 37), (64, 64), (3, 1)])
def test_householder_matches_lapack(shape):
    rng = np.random.Generator(np.random.Philox(sum(shape)))
    M = rng.standard_normal(shape)
    Q, R = householder_qr(M)
    Qn, Rn = _signed_numpy_qr(M)
    assert np.all(np.diag(R) >= 0)
    assert np.allclose(np.tril(R, -1), 0)
    np.testing.assert_allclose(Q, Qn, atol=1e-13)
    np.testing.assert_allclose(R, Rn, atol=1e-13 * np.abs(Rn).max())
    np.testing.assert_allclose(Q @ R, M, atol=1e-13 * np.abs(M).max())
    np.testing.assert_allclose(Q.T @ Q, np.eye(shape[1]), atol=1e-14)


def test_householder_lower_triangular_input():
    # the second QR of the method factors R^T, a lower-triangular matrix
    rng = np.random.Generator(np.random.Philox(3))
    R = np.triu(rng.standard_normal((25, 25))) + 5 * np.eye(25)
    Q, U = householder_qr(R.T)
    Qn, Un = _signed_numpy_qr(R.T)
    np.testing.assert_allclose(Q, Qn, atol=1e-13)
    np.testing.assert_allclose(U, Un, atol=1e-12)


def test_zero_column_convention():
    # a column already zero at/below the diagonal gets no reflector: e_j in Q, 0 on diag(R)
    M = np.zeros((6, 3))
    Q, R = householder_qr(M)
    np.testing.assert_array_equal(Q, np.eye(6, 3))
    np.testing.assert_array_equal(R, np.zeros((3, 3)))
    M = np.array([[1.0, 2.0, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    Q, R = householder_qr(M)
    np.testing.assert_allclose(Q @ R, M, atol=1e-15)
    np.testing.assert_allclose(Q.T @ Q, np.eye(3), atol=1e-15)


def test_orth_keeps_nested_spans():
    rng = np.random.Generator(np.random.Philox(9))
    M = rng.standard_normal((40, 6))
    T = np.triu(rng.standard_normal((6, 6))) + 3 * np.eye(6)
    # an upper-triangular mixing with positive diagonal does not change orth()
    np.testing.assert_allclose(hh_orth(M @ T), hh_orth(M), atol=1e-13)


@pytest.mark.parametrize("shape", [(6, 4), (9, 9), (12, 5), (4, 7)])
def test_jacobi_svd_matches_lapack(shape):
    rng = np.random.Generator(np.random.Philox(100 + shape[0]))
    M = rng.standard_normal(shape)
    s, V = jacobi_svd(M)
    np.testing.assert_allclose(s, np.linalg.svd(M, compute_uv=False), rtol=1e-13, atol=1e-14)
    if V is not None:
        np.testing.assert_allclose(V.T @ V, np.eye(V.shape[1]), atol=1e-13)
        # M V has orthogonal columns whose norms are the singular values
        MV = M @ V
        np.testing.assert_allclose(MV.T @ MV, np.diag(s ** 2), atol=1e-12)
