"""Sparse A in CSR (Section IV-E: for a sparse A each product with A or A^T
costs O(z d)): pbpqlp_factor_csr against the FP64 oracle run on the same
matrix stored dense (the method's result does not depend on the storage; the
sums differ only in their order).

Tolerances: FP64 elementwise Q, L, P within 1e-10, |dr| <= 1e-12; FP32
|dr| <= 1e-5 with ||Q^T Q - I||, ||P^T P - I|| <= 1e-4.  Inputs: sparse
low-rank-plus-noise matrices (sparse Gaussian factors, sigma_k = 0.9^k, sparse
noise), with uniform and with power-law column degrees (a few nearly dense
columns: long rows of A^T).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import pbpqlp as oracle_pbpqlp, rel_residual
from paper_2103_07245_amd import pbpqlp as B

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _csr_dev(A, dtype):
    return (torch.from_numpy(A.indptr.astype(np.int64)).to(DEV), torch.from_numpy(A.indices.astype(np.int32)).to(DEV),
            torch.from_numpy(A.data.astype(dtype)).to(DEV))


def _np(*xs):
    return [x.cpu().numpy().astype(np.float64) for x in xs]


@pytest.mark.parametrize("m,n,k,p,q,alpha", [(3000, 2000, 30, 10, 1, 0.0), (2500, 3100, 40, 8, 2, 1.1),
                                             (4000, 1500, 280, 20, 1, 0.8)])
def test_sparse_fp64_elementwise(m, n, k, p, q, alpha):
    A, _ = synth.sparse_lowrank(m, n, 60 if k + p < 256 else 320, 0.05, 4, 100 + m, col_alpha=alpha)
    print(f"sparse fp64 {m}x{n} nnz={A.nnz} l={k + p} q={q} alpha={alpha}", flush=True)
    Ad = A.toarray()
    ref = oracle_pbpqlp(Ad, k, p, q, 17)
    Q, L, P, info = B.factor_csr(*_csr_dev(A, np.float64), (m, n), k, p, q, 17)
    torch.cuda.synchronize()
    Q, L, P = _np(Q, L, P)
    assert info.status_flags == 0
    assert np.abs(L - ref.L).max() <= 1e-10
    assert np.abs(Q - ref.Q).max() <= 1e-10
    assert np.abs(P - ref.P).max() <= 1e-10
    r = rel_residual(Ad, Q, L, P)
    assert abs(r - rel_residual(Ad, ref.Q, ref.L, ref.P)) <= 1e-12
    assert abs(info.norm_a_fro2 - float(np.sum(A.data ** 2))) <= 1e-12 * float(np.sum(A.data ** 2))
    assert abs(info.resid_rel_est - r) <= 1e-9


def test_sparse_fp32_against_oracle_and_deterministic():
    A, _ = synth.sparse_lowrank(5000, 3000, 80, 0.03, 6, 7, col_alpha=1.0, dtype=np.float32)
    print(f"sparse fp32 5000x3000 nnz={A.nnz} l=70 q=2", flush=True)
    Ad = A.toarray().astype(np.float64)
    ref = oracle_pbpqlp(Ad, 60, 10, 2, 3)
    csr = _csr_dev(A, np.float32)
    a = B.factor_csr(*csr, (5000, 3000), 60, 10, 2, 3)
    b = B.factor_csr(*csr, (5000, 3000), 60, 10, 2, 3)
    torch.cuda.synchronize()
    assert all(torch.equal(x, y) for x, y in zip(a[:3], b[:3]))
    Q, L, P = _np(*a[:3])
    assert abs(rel_residual(Ad, Q, L, P) - rel_residual(Ad, ref.Q, ref.L, ref.P)) <= 1e-5
    assert np.abs(Q.T @ Q - np.eye(70)).max() <= 1e-4
    assert np.abs(P.T @ P - np.eye(70)).max() <= 1e-4
    # the dense path on the same matrix gives the same factorization up to rounding
    Qd, Ld, Pd, _ = B.factor(torch.from_numpy(A.toarray()).to(DEV), 60, 10, 2, 3)
    Qd, Ld, Pd = _np(Qd, Ld, Pd)
    assert np.abs(np.diag(L) - np.diag(Ld)).max() <= 1e-5 * Ld[0, 0]


def test_sparse_empty_rows_columns_and_zero_matrix():
    import scipy.sparse as sp
    A, _ = synth.sparse_lowrank(1200, 900, 20, 0.02, 0, 5)
    A = sp.lil_matrix(A)
    A[100:300, :] = 0     # empty rows
    A[:, 50:120] = 0      # empty columns
    A = sp.csr_matrix(A)
    A.eliminate_zeros()
    print(f"sparse empty rows/cols 1200x900 nnz={A.nnz} l=25 q=1", flush=True)
    Ad = A.toarray()
    ref = oracle_pbpqlp(Ad, 20, 5, 1, 9)
    Q, L, P, info = B.factor_csr(*_csr_dev(A, np.float64), (1200, 900), 20, 5, 1, 9)
    torch.cuda.synchronize()
    Q, L, P = _np(Q, L, P)
    # rank 20 < l = 25: the first 20 L-values and the residual are determined
    assert abs(rel_residual(Ad, Q, L, P) - rel_residual(Ad, ref.Q, ref.L, ref.P)) <= 1e-12
    assert np.abs(np.diag(L)[:20] - np.diag(ref.L)[:20]).max() <= 1e-10
    assert np.abs(Q.T @ Q - np.eye(25)).max() <= 1e-10
    # nnz = 0: A = 0, L = 0, orthonormal Q and P
    z = (torch.zeros(1201, dtype=torch.int64, device=DEV), torch.zeros(0, dtype=torch.int32, device=DEV),
         torch.zeros(0, dtype=torch.float64, device=DEV))
    Q, L, P, info = B.factor_csr(*z, (1200, 900), 20, 5, 1, 9)
    torch.cuda.synchronize()
    Q, L, P = _np(Q, L, P)
    assert np.abs(L).max() == 0.0 and info.norm_a_fro2 == 0.0
    assert np.abs(Q.T @ Q - np.eye(25)).max() <= 1e-10 and np.abs(P.T @ P - np.eye(25)).max() <= 1e-10


def test_sparse_invalid_indices_are_flagged_and_skipped():
    """A column index outside [0, n) and a row pointer past nnz: the kernels
    clamp them (no out-of-bounds access), skip those entries and flag the
    input; the result is the factorization of the valid entries."""
    A, _ = synth.sparse_lowrank(800, 600, 10, 0.05, 2, 3)
    ip, ix, v = (x.copy() for x in (A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data))
    ix[5] = 600                      # out of range: skipped
    v_ok = v.copy()
    v_ok[5] = 0.0
    print("sparse invalid index 800x600 l=16", flush=True)
    Q, L, P, info = B.factor_csr(torch.from_numpy(ip).to(DEV), torch.from_numpy(ix).to(DEV),
                                 torch.from_numpy(v).to(DEV), (800, 600), 12, 4, 1, 1)
    torch.cuda.synchronize()
    assert info.status_flags & B.FLAG_BADINPUT
    import scipy.sparse as sp
    ix_ok = A.indices.astype(np.int32)
    Ad = sp.csr_matrix((v_ok, ix_ok, ip), shape=(800, 600)).toarray()
    ref = oracle_pbpqlp(Ad, 12, 4, 1, 1)
    L = L.cpu().numpy()
    assert np.abs(L - ref.L).max() <= 1e-10
