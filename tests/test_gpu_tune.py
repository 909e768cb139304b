"""Autotuner: the tuned plan is what automatic calls then use (bit for bit),
and tuning never changes results beyond the plan's own rounding order."""
import numpy as np
import pytest
import torch

import synth
from oracle import pbpqlp as oracle_pbpqlp, rel_residual
from paper_2103_07245_amd import pbpqlp as B

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def test_tuned_plan_is_used_by_automatic_calls():
    B.tune_clear()
    rng = synth.rng_for(91)
    m, n, k, p, q = 3000, 1400, 40, 8, 1
    A = synth.planted(rng, m, n, 0.95 ** np.arange(200), 1e-6, np.float32)
    At = torch.from_numpy(A).to(DEV)
    plan = B.tune_factor(At, k, p, q, 5)
    print("tuned", plan, flush=True)
    assert plan["ms"] > 0 and (plan["split_k"] == -1 or plan["split_k"] >= 1)
    assert B.tune_lookup(m, n, k, p) == plan
    Qa, La, Pa, _ = B.factor(At, k, p, q, 5)                         # automatic
    Qe, Le, Pe, _ = B.factor(At, k, p, q, 5, split_k=plan["split_k"], gram_wg=plan["gram_wg"])
    assert torch.equal(Qa, Qe) and torch.equal(La, Le) and torch.equal(Pa, Pe)
    ref = oracle_pbpqlp(A.astype(np.float64), k, p, q, 5)
    r_ref = rel_residual(A.astype(np.float64), ref.Q, ref.L, ref.P)
    r = rel_residual(A.astype(np.float64), *(x.cpu().numpy().astype(np.float64) for x in (Qa, La, Pa)))
    assert abs(r - r_ref) <= 1e-5
    B.tune_clear()


def test_tuned_batch_plan_is_used_by_new_batches():
    B.tune_clear()
    mats, ks, ps, qs, seeds = [], [], [], [], []
    for b in range(6):
        w = synth.config4_matrix(500 + b, 300 + 40 * b, 200 + 30 * b, 12)
        mats.append(torch.from_numpy(np.ascontiguousarray(w.A)).to(DEV))
        ks.append(w.k); ps.append(w.p); qs.append(w.q); seeds.append(w.seed)
    bt = B.Batch(mats, ks, ps, qs, seeds)
    plan = bt.tune()
    print("tuned batch", plan, flush=True)
    assert plan["gram_wg"] in (4, 16, 64, 256)
    bt.close()
    bt2 = B.Batch(mats, ks, ps, qs, seeds)
    bt2.run()
    torch.cuda.synchronize()
    for i in range(len(mats)):
        assert bt2.problem_plan(i) == (1, plan["gram_wg"])
        Q, L, P, _ = B.factor(mats[i], ks[i], ps[i], qs[i], seeds[i], split_k=1, gram_wg=plan["gram_wg"])
        assert torch.equal(bt2.Q[i], Q) and torch.equal(bt2.L[i], L) and torch.equal(bt2.P[i], P)
    bt2.close()
    B.tune_clear()
