"""Batched factorization (pbpqlp_batch_*): many independent uneven-size
problems in one plan.

Each problem of a batch runs exactly the kernels and parameters of
pbpqlp_factor with the per-problem plan the batch reports (one contraction
split, the batch's Gram workgroup target), so its outputs must equal that
single call's bit for bit: with and without the
graph, on repeated runs of one plan, across shape classes (different tile
counts, aligned and unaligned rows) and across launch-sequence classes
(different q).  Against the FP64 oracle the usual FP32 tolerance applies.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import pbpqlp as oracle_pbpqlp, rel_residual
from paper_2103_07245_amd import pbpqlp as B

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _c4_like(count, m_range=(120, 1400), n_range=(90, 800), seed=0):
    """C4-recipe members (U diag(exp(-i/r)) V^T + 1e-5 noise, k=r, p=8) at
    smaller sizes; every third problem gets q = 2 and every fifth an odd n."""
    rng = np.random.default_rng(4242 + seed)
    out = []
    for b in range(count):
        m = int(rng.integers(m_range[0], m_range[1] + 1))
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        if b % 5 == 4:
            n |= 1
        r = int(rng.integers(8, 64 + 1))
        r = min(r, min(m, n) - 8)
        w = synth.config4_matrix(100 + b + 1000 * seed, m, n, r)
        q = 2 if b % 3 == 2 else w.q
        out.append((w.A, w.k, w.p, q, w.seed))
    return out


def _batch(members, plan="native", use_graph=True):
    mats = [torch.from_numpy(np.ascontiguousarray(A)).to(DEV) for A, *_ in members]
    bt = B.Batch(mats, [k for _, k, _, _, _ in members], [p for _, _, p, _, _ in members],
                 [q for _, _, _, q, _ in members], [s for *_, s in members], plan=plan,
                 use_graph=use_graph)
    return bt, mats


def _single(bt, i, At, k, p, q, seed, plan="native"):
    """pbpqlp_factor with the plan the batch chose for problem i."""
    split_k, gram_wg = bt.problem_plan(i)
    return B.factor(At, k, p, q, seed, plan=plan, split_k=split_k, gram_wg=gram_wg)


@pytest.fixture(scope="module")
def members():
    return _c4_like(14)


@pytest.mark.parametrize("plan", ["native", "mixed"])
def test_batch_equals_single_calls_bitwise(members, plan):
    print(f"batch of {len(members)} c4-recipe problems, plan {plan}", flush=True)
    bt, mats = _batch(members, plan=plan)
    bt.run()
    torch.cuda.synchronize()
    for i, (A, k, p, q, seed) in enumerate(members):
        Q, L, P, info = _single(bt, i, mats[i], k, p, q, seed, plan=plan)
        torch.cuda.synchronize()
        assert torch.equal(bt.Q[i], Q), i
        assert torch.equal(bt.L[i], L), i
        assert torch.equal(bt.P[i], P), i
        bi = bt.info(i)
        assert bi.status_flags == info.status_flags and bi.l == info.l and bi.q == info.q
        assert bi.resid_rel_est == info.resid_rel_est
    st = bt.stats()
    # grouped launches: far fewer than the problems' own launches
    assert 0 < st["launches"] < 6 * 60
    bt.close()


def test_graph_replays_and_direct_launches_agree(members):
    bt, _ = _batch(members)
    bt.run()
    torch.cuda.synchronize()
    first = [(q.clone(), l.clone(), p.clone()) for q, l, p in zip(bt.Q, bt.L, bt.P)]
    for use_graph in (True, True, False):
        for t in bt.Q + bt.L + bt.P:
            t.fill_(float("nan"))
        torch.cuda.synchronize()
        bt.use_graph(use_graph)
        bt.run()
        torch.cuda.synchronize()
        for i, (q, l, p) in enumerate(first):
            assert torch.equal(bt.Q[i], q) and torch.equal(bt.L[i], l) and torch.equal(bt.P[i], p), i
    bt.close()


def test_batch_against_oracle(members):
    bt, _ = _batch(members[:5])
    bt.run()
    torch.cuda.synchronize()
    for i, (A, k, p, q, seed) in enumerate(members[:5]):
        A64 = A.astype(np.float64)
        ref = oracle_pbpqlp(A64, k, p, q, seed)
        r_ref = rel_residual(A64, ref.Q, ref.L, ref.P)
        Q, L, P = (t.cpu().numpy().astype(np.float64) for t in (bt.Q[i], bt.L[i], bt.P[i]))
        r = rel_residual(A64, Q, L, P)
        assert abs(r - r_ref) <= 1e-5, (i, r, r_ref)
        l = k + p
        assert np.abs(Q.T @ Q - np.eye(l)).max() <= 1e-4
        assert np.abs(P.T @ P - np.eye(l)).max() <= 1e-4
    bt.close()


def test_fp64_batch_and_padded_rows():
    rng = synth.rng_for(77)
    shapes = [(300, 200, 6, 4), (257, 129, 10, 2), (180, 333, 12, 4)]
    mats, ks, ps, qs, seeds = [], [], [], [], []
    for j, (m, n, k, p) in enumerate(shapes):
        sig = 0.9 ** np.arange(min(m, n))
        A = synth.planted(rng, m, n, sig, 0.0, np.float64)
        big = torch.zeros((m, n + 3), dtype=torch.float64, device=DEV)
        big[:, :n] = torch.from_numpy(A).to(DEV)
        mats.append(big[:, :n])                     # padded leading dimension
        ks.append(k); ps.append(p); qs.append(1 + j % 2); seeds.append(31 + j)
    bt = B.Batch(mats, ks, ps, qs, seeds)
    bt.run()
    torch.cuda.synchronize()
    for i in range(len(shapes)):
        Q, L, P, _ = _single(bt, i, mats[i], ks[i], ps[i], qs[i], seeds[i])
        torch.cuda.synchronize()
        assert torch.equal(bt.Q[i], Q) and torch.equal(bt.L[i], L) and torch.equal(bt.P[i], P), i
        A64 = mats[i].cpu().numpy()
        ref = oracle_pbpqlp(A64, ks[i], ps[i], qs[i], seeds[i])
        assert np.abs(bt.L[i].cpu().numpy() - ref.L).max() <= 1e-9
    bt.close()


def test_batch_full_range_against_oracle():
    """Batched problems at the corners of the C4 ranges (m in [256, 4096],
    n in [256, 2048], rank r in [8, 64], l = r + 8 up to 72), odd sizes
    included, each against the FP64 oracle at the FP32 tolerance."""
    shapes = [(4096, 2048, 64), (4096, 256, 8), (256, 2048, 64), (256, 256, 8), (3001, 1999, 41),
              (4095, 2047, 64), (2222, 1023, 17)]
    members = []
    for b, (m, n, r) in enumerate(shapes):
        w = synth.config4_matrix(500 + b, m, n, r)
        members.append((w.A, w.k, w.p, w.q, w.seed))
    print(f"batch of {len(members)} problems at the C4 range corners", flush=True)
    bt, _ = _batch(members)
    bt.run()
    torch.cuda.synchronize()
    for i, (A, k, p, q, seed) in enumerate(members):
        A64 = A.astype(np.float64)
        ref = oracle_pbpqlp(A64, k, p, q, seed)
        r_ref = rel_residual(A64, ref.Q, ref.L, ref.P)
        Q, L, P = (t.cpu().numpy().astype(np.float64) for t in (bt.Q[i], bt.L[i], bt.P[i]))
        assert abs(rel_residual(A64, Q, L, P) - r_ref) <= 1e-5, (i, shapes[i])
        l = k + p
        assert np.abs(Q.T @ Q - np.eye(l)).max() <= 1e-5, i
        assert np.abs(P.T @ P - np.eye(l)).max() <= 1e-5, i
        assert np.max(np.abs(np.diag(L)[:k] - np.diag(ref.L)[:k])) <= 1e-5 * ref.L[0, 0], i
    bt.close()
