"""pbpqlp_factor_noalloc (the allocation-free entry point) against
pbpqlp_factor: the same kernels and plan with the workspace taken from the
library's static device array, so the outputs must agree bit for bit.  Two
calls in a row on one GPU, the second smaller than the first, so the second
runs on the array as the first left it."""
import numpy as np
import pytest
import torch

import synth
from paper_2103_07245_amd import pbpqlp as B

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _planted(m, n, seed, dtype):
    rng = synth.rng_for(seed)
    return torch.from_numpy(synth.planted(rng, m, n, 0.9 ** np.arange(min(m, n) // 2), 1e-6, dtype)).to(DEV)


@pytest.mark.parametrize("plan,dtype", [("native", np.float32), ("mixed", np.float32), ("native", np.float64)])
def test_noalloc_equals_factor_twice(plan, dtype):
    cases = [(3000, 2100, 40, 8, 1, 5), (700, 515, 14, 6, 2, 6)]   # second call smaller
    for m, n, k, p, q, seed in cases:
        print(f"noalloc {plan} {dtype.__name__} {m}x{n} k={k} p={p} q={q}", flush=True)
        A = _planted(m, n, 100 + m, dtype)
        Qa, La, Pa, infoa = B.factor_noalloc(A, k, p, q, seed, plan=plan)
        torch.cuda.synchronize()
        Qa, La, Pa, infoa = Qa.clone(), La.clone(), Pa.clone(), infoa.clone()
        Qb, Lb, Pb, infob = B.factor(A, k, p, q, seed, plan=plan)
        torch.cuda.synchronize()
        assert torch.equal(Qa, Qb) and torch.equal(La, Lb) and torch.equal(Pa, Pb)
        ia = B.Info.from_device(infoa)
        assert ia.status_flags == infob.status_flags and ia.resid_rel_est == infob.resid_rel_est
        assert ia.l == k + p and ia.q == q


def test_noalloc_rejects_oversized_problem():
    # the workspace of a 16384 x 16384 problem with l = 256 exceeds the array
    A = torch.empty((8, 8), dtype=torch.float32, device=DEV)
    lib = B.library()
    st = lib.pbpqlp_factor_noalloc(
        __import__("ctypes").c_void_p(A.data_ptr()), 16384, 16384, 16384, B.F32, 200, 56, 1,
        __import__("ctypes").c_uint64(1), __import__("ctypes").c_void_p(A.data_ptr() + 1024), 256,
        __import__("ctypes").c_void_p(A.data_ptr() + 2048), 256,
        __import__("ctypes").c_void_p(A.data_ptr() + 4096), 256, None, None, None)
    assert st == B.EUNSUPPORTED
