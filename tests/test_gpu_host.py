"""A in host memory (Section IV-E: when A is stored externally every product
with A or A^T is one more pass over it, 2q + 2 in all): pbpqlp_factor_host
streams A from host memory in row panels on every pass.

* One panel: the same launches as pbpqlp_factor on a device copy of A, so the
  results are equal bit for bit.
* Several panels (a ragged last one, padded rows, pinned and pageable host
  memory): A X is computed panel by panel with the same kernels; A^T X sums
  every panel's partials in a fixed order, a different order from the device
  path, so the results are compared with the FP64 oracle at the tolerances of
  the device path (FP64: elementwise 1e-10; FP32: |dr| <= 1e-5; mixed: |dr| <=
  1e-4; FP16: |dr| <= 1e-3) and with pbpqlp_factor to rounding level.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import pbpqlp as oracle_pbpqlp, rel_residual
from paper_2103_07245_amd import pbpqlp as B

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _np(*xs):
    return [x.cpu().numpy().astype(np.float64) for x in xs]


@pytest.mark.parametrize("plan", ["native", "mixed"])
def test_single_panel_equals_device_path(plan):
    w = synth.config2(m=2048, n=1536, r=256, k=60, p=10, q=1)
    print(f"host one panel 2048x1536 l=70 plan={plan}", flush=True)
    Ah = torch.from_numpy(w.A).pin_memory()
    Qh, Lh, Ph, ih = B.factor_host(Ah, w.k, w.p, w.q, w.seed, plan=plan, panel_rows=4096)
    Qd, Ld, Pd, idv = B.factor(Ah.to(DEV), w.k, w.p, w.q, w.seed, plan=plan)
    torch.cuda.synchronize()
    assert torch.equal(Qh, Qd) and torch.equal(Lh, Ld) and torch.equal(Ph, Pd)
    assert ih.norm_a_fro2 == idv.norm_a_fro2 and ih.resid_rel_est == idv.resid_rel_est


@pytest.mark.parametrize("pinned", [True, False])
def test_fp64_panels_elementwise_against_oracle(pinned):
    w = synth.config1()
    print(f"host panels 1000x1000 fp64 l=25 q=1 panel=256 pinned={pinned}", flush=True)
    ref = oracle_pbpqlp(w.A, w.k, w.p, w.q, w.seed)
    Ah = torch.from_numpy(w.A)
    Q, L, P, info = B.factor_host(Ah.pin_memory() if pinned else Ah, w.k, w.p, w.q, w.seed, panel_rows=256)
    torch.cuda.synchronize()
    Q, L, P = _np(Q, L, P)
    assert np.abs(Q - ref.Q).max() <= 1e-10
    assert np.abs(L - ref.L).max() <= 1e-10
    assert np.abs(P - ref.P).max() <= 1e-10
    r = rel_residual(w.A, Q, L, P)
    assert abs(r - rel_residual(w.A, ref.Q, ref.L, ref.P)) <= 1e-12
    assert abs(info.norm_a_fro2 - float(np.sum(w.A ** 2))) <= 1e-12 * float(np.sum(w.A ** 2))
    assert abs(info.resid_rel_est - r) <= 1e-9


@pytest.mark.parametrize("plan,tol,panel,pinned", [("native", 1e-5, 512, True), ("native", 1e-5, 256, False),
                                                   ("mixed", 1e-4, 768, True), ("bf16x3", 1e-5, 1280, True)])
def test_fp32_panels_against_oracle(plan, tol, panel, pinned):
    w = synth.config2(m=2000, n=1536, r=256, k=60, p=10, q=2)
    print(f"host panels 2000x1536 l=70 q=2 plan={plan} panel={panel} pinned={pinned}", flush=True)
    ref = oracle_pbpqlp(w.A, w.k, w.p, w.q, w.seed)
    r_ref = rel_residual(w.A, ref.Q, ref.L, ref.P)
    Ah = torch.from_numpy(w.A)
    if pinned:
        Ah = Ah.pin_memory()
    Q, L, P, info = B.factor_host(Ah, w.k, w.p, w.q, w.seed, plan=plan, panel_rows=panel)
    Qd, Ld, Pd, _ = B.factor(Ah.to(DEV), w.k, w.p, w.q, w.seed, plan=plan)
    torch.cuda.synchronize()
    Q, L, P, Qd, Ld, Pd = _np(Q, L, P, Qd, Ld, Pd)
    r = rel_residual(w.A, Q, L, P)
    assert abs(r - r_ref) <= tol, (r, r_ref)
    assert np.abs(Q.T @ Q - np.eye(w.l)).max() <= 1e-4
    assert np.abs(P.T @ P - np.eye(w.l)).max() <= 1e-4
    # the device path on the same matrix: the same factorization up to rounding
    assert abs(r - rel_residual(w.A, Qd, Ld, Pd)) <= 1e-6
    assert np.abs(np.diag(L) - np.diag(Ld)).max() <= 1e-5 * L[0, 0]


def test_padded_rows_and_many_panels():
    """lda > n (a column slice of a wider host matrix) and 16 panels of 128
    rows (rounded up to 256: 8 panels), so the A^T X partials of many panels
    are reduced together."""
    w = synth.config2(m=2000, n=700, r=128, k=30, p=8, q=1)
    wide = np.zeros((2000, 768), dtype=np.float32)
    wide[:, :700] = w.A
    Ah = torch.from_numpy(wide)[:, :700]
    assert Ah.stride(0) == 768
    print("host panels 2000x700 lda=768 l=38 q=1 panel=128", flush=True)
    ref = oracle_pbpqlp(w.A, w.k, w.p, w.q, w.seed)
    Q, L, P, info = B.factor_host(Ah, w.k, w.p, w.q, w.seed, panel_rows=128)
    torch.cuda.synchronize()
    Q, L, P = _np(Q, L, P)
    assert abs(rel_residual(w.A, Q, L, P) - rel_residual(w.A, ref.Q, ref.L, ref.P)) <= 1e-5
    assert info.status_flags == 0


def test_tall_fp16_panels_against_oracle():
    w = synth.config3(m=20000, n=1024, r=64, k=64, p=16, q=1)
    print("host panels 20000x1024 fp16 l=80 q=1 panel=4096", flush=True)
    ref = oracle_pbpqlp(w.A, w.k, w.p, w.q, w.seed)
    Q, L, P, info = B.factor_host(torch.from_numpy(w.A).pin_memory(), w.k, w.p, w.q, w.seed, plan="fp16",
                                  panel_rows=4096)
    torch.cuda.synchronize()
    Q, L, P = _np(Q, L, P)
    assert abs(rel_residual(w.A, Q, L, P) - rel_residual(w.A, ref.Q, ref.L, ref.P)) <= 1e-3


def test_pageable_equals_pinned():
    """Pageable host memory goes through pinned bounce buffers; the device
    sees the same panels, so the results are equal bit for bit."""
    w = synth.config2(m=1800, n=1000, r=128, k=40, p=8, q=1)
    print("host pageable vs pinned 1800x1000 l=48 q=1 panel=512", flush=True)
    Ah = torch.from_numpy(w.A)
    a = B.factor_host(Ah.pin_memory(), w.k, w.p, w.q, w.seed, plan="mixed", panel_rows=512)[:3]
    b = B.factor_host(Ah, w.k, w.p, w.q, w.seed, plan="mixed", panel_rows=512)[:3]
    torch.cuda.synchronize()
    assert all(torch.equal(x, y) for x, y in zip(a, b))
