"""Sketches wider than 256 columns (the sample sizes d = 0.2 n and 0.3 n of the
paper's runtime experiments, Section V-A, Tables I-III).

Past 256 columns every streaming product runs in launches of 256 columns of
the sketch, the Cholesky of the l x l Gram is blocked by 256 (single-block
factor of each diagonal block, triangular solve of its row, FP64 matrix-core
update of the trailing triangle) and the triangular apply is blocked the same
way.  Compared with the FP64 oracle at the tolerances of the narrow path:
FP64 elementwise 1e-10 on well-conditioned problems; FP32 |dr| <= 1e-5;
mixed |dr| <= 1e-4; ||Q^T Q - I||, ||P^T P - I|| <= 1e-4 (FP32) or 1e-12
(FP64).  A rank-deficient case (rank below l, dependent columns in a later
block) is held to the invariants: exact recovery and orthonormal factors.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import omega as oracle_omega, pbpqlp as oracle_pbpqlp, rel_residual
from paper_2103_07245_amd import pbpqlp as B

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _np(*xs):
    return [x.cpu().numpy().astype(np.float64) for x in xs]


def _decay(m, n, r, rate, seed, dtype, noise=0.0):
    rng = synth.rng_for(seed)
    sigma = rate ** np.arange(r, dtype=np.float64)
    return synth.planted(rng, m, n, sigma, noise, dtype)


@pytest.mark.parametrize("n,l", [(700, 300), (333, 520), (1000, 1000)])
def test_wide_omega_bit_exact(n, l):
    print(f"omega n={n} l={l}", flush=True)
    g = B.omega(n, l, 99, dtype=torch.float64, device=DEV).cpu().numpy()
    assert np.array_equal(g, oracle_omega(n, l, 99))


@pytest.mark.parametrize("m,n,k,p,q", [(1200, 900, 280, 20, 1), (1100, 1000, 500, 20, 0), (900, 1100, 600, 8, 2)])
def test_wide_fp64_elementwise(m, n, k, p, q):
    A = _decay(m, n, min(m, n), 0.995, 31 + m, np.float64)
    print(f"wide fp64 {m}x{n} l={k + p} q={q}", flush=True)
    ref = oracle_pbpqlp(A, k, p, q, 7)
    Q, L, P, info = B.factor(torch.from_numpy(A).to(DEV), k, p, q, 7)
    torch.cuda.synchronize()
    Q, L, P = _np(Q, L, P)
    assert np.abs(L - ref.L).max() <= 1e-10
    assert np.abs(Q - ref.Q).max() <= 1e-10
    assert np.abs(P - ref.P).max() <= 1e-10
    l = k + p
    assert np.abs(Q.T @ Q - np.eye(l)).max() <= 1e-12
    assert np.abs(P.T @ P - np.eye(l)).max() <= 1e-12
    r = rel_residual(A, Q, L, P)
    assert abs(r - rel_residual(A, ref.Q, ref.L, ref.P)) <= 1e-12
    assert abs(info.resid_rel_est - r) <= 1e-9
    assert info.status_flags == 0


@pytest.fixture(scope="module")
def d03n():
    A = _decay(2000, 2000, 1200, 0.996, 77, np.float32, 1e-6)
    print("oracle 2000x2000 l=600 q=2", flush=True)
    return A, oracle_pbpqlp(A, 580, 20, 2, 11)


@pytest.mark.parametrize("plan,tol", [("native", 1e-5), ("mixed", 1e-4), ("bf16x3", 1e-5)])
def test_wide_fp32_against_oracle(d03n, plan, tol):
    """The paper's d = 0.3 n at n = 2000 (l = 600), q = 2, FP32 storage."""
    A, ref = d03n
    print(f"wide fp32 2000x2000 l=600 q=2 plan={plan}", flush=True)
    Q, L, P, info = B.factor(torch.from_numpy(A).to(DEV), 580, 20, 2, 11, plan=plan)
    torch.cuda.synchronize()
    Q, L, P = _np(Q, L, P)
    r = rel_residual(A, Q, L, P)
    assert abs(r - rel_residual(A, ref.Q, ref.L, ref.P)) <= tol
    assert np.abs(Q.T @ Q - np.eye(600)).max() <= 1e-4
    assert np.abs(P.T @ P - np.eye(600)).max() <= 1e-4
    assert np.abs(np.diag(L) - np.diag(ref.L)).max() <= 1e-3 * ref.L[0, 0]


def test_wide_rank_deficient_exact_recovery():
    """rank(A) = 350 < l = 400: the sketch has 50 dependent columns, all in
    the second 256-block; the factorization still recovers A exactly with
    orthonormal factors (the trailing columns are not unique)."""
    A = _decay(1500, 1200, 350, 0.99, 5, np.float64)
    print("wide rank-deficient 1500x1200 rank 350 l=400 q=1", flush=True)
    Q, L, P, info = B.factor(torch.from_numpy(A).to(DEV), 390, 10, 1, 3)
    torch.cuda.synchronize()
    Q, L, P = _np(Q, L, P)
    assert rel_residual(A, Q, L, P) <= 1e-12
    assert np.abs(Q.T @ Q - np.eye(400)).max() <= 1e-10
    assert np.abs(P.T @ P - np.eye(400)).max() <= 1e-10
    assert info.status_flags & B.FLAG_DEPENDENT
    ref = oracle_pbpqlp(A, 390, 10, 1, 3)
    # the leading 350 L-values are determined
    assert np.abs(np.diag(L)[:350] - np.diag(ref.L)[:350]).max() <= 1e-10


def test_wide_host_resident_panels():
    A = _decay(1800, 1000, 900, 0.995, 9, np.float32, 1e-6)
    print("wide host panels 1800x1000 l=300 q=1 panel=512", flush=True)
    ref = oracle_pbpqlp(A, 290, 10, 1, 5)
    Q, L, P, info = B.factor_host(torch.from_numpy(A).pin_memory(), 290, 10, 1, 5, panel_rows=512)
    torch.cuda.synchronize()
    Q, L, P = _np(Q, L, P)
    assert abs(rel_residual(A, Q, L, P) - rel_residual(A, ref.Q, ref.L, ref.P)) <= 1e-5


def test_wide_rr_paper_orientation():
    """The paper's own orientation (sketch A^T Phi, Phi m x l) at l = 300, FP64:
    the oracle runs on A^T with the same Phi."""
    A = _decay(1000, 800, 800, 0.995, 13, np.float64)
    print("wide rr orientation A 1000x800 l=300 q=1", flush=True)
    Q, L, P, R, rank, used, info = B.factor_rr(torch.from_numpy(A).to(DEV), 290, 10, 1, 21, orientation="A")
    torch.cuda.synchronize()
    ref = oracle_pbpqlp(A.T, 290, 10, 1, Omega=oracle_omega(1000, 300, 21))
    Q, L, P, R = _np(Q, L, P, R)
    assert used == "A"
    assert np.abs(L - ref.L).max() <= 1e-10
    assert np.abs(R - ref.R).max() <= 1e-10
    assert np.abs(Q - ref.P).max() <= 1e-10 and np.abs(P - ref.Q).max() <= 1e-10
    res = np.linalg.norm(A - Q @ L @ P.T) / np.linalg.norm(A)
    assert abs(res - rel_residual(A.T, ref.Q, ref.L, ref.P)) <= 1e-12
