"""Training data, training and evaluation of the learned q/k head.

    python -m paper_2103_07245_amd.train_qk data  --count 4096 --seed 1 --out qk_data.npz
    python -m paper_2103_07245_amd.train_qk train --data qk_data.npz --epochs 400 --out qk_mlp.bin

Every step of the method and of the network runs in libpbpqlp.so: the probe and
the label runs are pbpqlp_factor calls, the features come from
pbpqlp_probe_features, and training runs pbpqlp_mlp_train_step (the forward,
backward and Adam kernels).  PyTorch holds device memory and builds the
synthetic matrices.

Labels of one matrix with planted singular values sigma (sigma_1 = 1) follow
what pbpqlp_factor_auto returns -- the leading rank-(k + p) part of the l = 64
factorization whose power iterations continue the probe's:
  k* = the smallest k with sigma_{k+1} <= 1e-3 sigma_1, capped at the probe's
       k = 56;
  r(q) = sqrt(||A||^2 - ||L'||^2) / ||A|| for the leading (k* + p) block L' of
       L after q iterations, q = 0..4, in FP64 (the probe, then four
       pbpqlp_factor_sketch continuations with Omega = the previous P: ten
       passes over A in all);
  q* = the smallest q with r(q) <= 1.05 r_opt(k* + p), else 4, where r_opt(l)
       is the best rank-l residual sqrt(sum_{i>l} sigma_i^2) / ||sigma||.
Features come from the probe of the same matrix stored in FP32.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

from . import pbpqlp as B

_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if _ROOT not in sys.path:
    sys.path.insert(0, _ROOT)
import synth  # noqa: E402  (seeded inputs only)

K_REL = 1e-3
Q_SLACK = 1.05
K_MAX = B.PROBE_K
P_OVER = 8
Q_MAX = 4


def _log(*a):
    print(*a, flush=True)


def r_opt(sigma: np.ndarray, l: int) -> float:
    """Best relative Frobenius residual of a rank-l approximation."""
    s2 = np.asarray(sigma, dtype=np.float64) ** 2
    return float(math.sqrt(s2[l:].sum() / s2.sum()))


def k_star(sigma: np.ndarray, k_max: int = K_MAX) -> int:
    s = np.asarray(sigma, dtype=np.float64)
    for k in range(1, min(k_max, s.shape[0] - 1) + 1):
        if s[k] <= K_REL * s[0]:
            return k
    return k_max


def q_star(r_of_q, r_best: float) -> int:
    for q, r in enumerate(r_of_q):
        if r <= Q_SLACK * r_best:
            return q
    return len(r_of_q) - 1


def make_matrix(spec, device) -> torch.Tensor:
    """A = U diag(sigma) V^T in FP64 on the device, U and V from the QR of
    Gaussian panels drawn from the spec's seed."""
    g = torch.Generator(device=device)
    g.manual_seed(int(spec.seed_a))
    r = spec.sigma.shape[0]
    U = torch.linalg.qr(torch.randn(spec.m, r, generator=g, dtype=torch.float64, device=device))[0]
    V = torch.linalg.qr(torch.randn(spec.n, r, generator=g, dtype=torch.float64, device=device))[0]
    sig = torch.as_tensor(spec.sigma, dtype=torch.float64, device=device)
    return (U * sig) @ V.T


def truncated_residual(L: torch.Tensor, norm_a2: float, lt: int) -> float:
    """Residual estimate of the leading rank-lt part of a factorization."""
    Lh = L[:lt, :lt].double().cpu().numpy()
    s2 = float(np.sum(Lh * Lh))
    return math.sqrt(max(norm_a2 - s2, 0.0) / norm_a2) if norm_a2 > 0 else 0.0


def label_matrix(A64: torch.Tensor, sigma: np.ndarray, seed: int, plan="native"):
    """(features, q*, k*, r(q) list, r_opt) of one matrix."""
    A32 = A64.float().contiguous()
    f, _, _ = B.probe(A32, seed, plan)
    ks = k_star(sigma)
    lt = ks + P_OVER
    rs = []
    _, L, P, info = B.factor(A64, B.PROBE_K, B.PROBE_P, 0, seed)
    for q in range(Q_MAX + 1):
        if q > 0:
            _, L, P, info = B.factor_sketch(A64, P, B.PROBE_K, B.PROBE_P, 0)
        rs.append(truncated_residual(L, info.norm_a_fro2, lt))
    rb = r_opt(sigma, lt)
    return f.cpu().numpy(), q_star(rs, rb), ks, rs, rb


def make_dataset(count: int, seed: int, device, m_range=(512, 2048), n_range=(512, 2048),
                 rank_cap: int = 256, log=_log, checkpoint=None):
    X = np.zeros((count, B.MLP_IN), dtype=np.float32)
    qs = np.zeros(count, dtype=np.int32)
    ks = np.zeros(count, dtype=np.int32)
    rq = np.zeros((count, Q_MAX + 1))
    ro = np.zeros(count)
    fams = []
    t0 = time.time()
    for i in range(count):
        spec = synth.qk_spec(i, seed, m_range, n_range, rank_cap)
        A = make_matrix(spec, device)
        X[i], qs[i], ks[i], rq[i], ro[i] = label_matrix(A, spec.sigma, spec.seed_omega)
        fams.append(spec.family)
        del A
        if (i + 1) % 128 == 0 or i + 1 == count:
            log(f"  {i + 1}/{count} matrices labelled ({time.time() - t0:.0f} s); "
                f"q* histogram {np.bincount(qs[:i + 1], minlength=5).tolist()}")
        if checkpoint and ((i + 1) % 1024 == 0):
            checkpoint({"X": X[:i + 1], "q": qs[:i + 1], "k": ks[:i + 1], "r_q": rq[:i + 1],
                        "r_opt": ro[:i + 1], "family": np.array(fams)})
    return {"X": X, "q": qs, "k": ks, "r_q": rq, "r_opt": ro, "family": np.array(fams)}


def evaluate(model: B.Model, X: np.ndarray, q: np.ndarray, k: np.ndarray, device):
    """q accuracy, rate of q_hat >= q*, mean |ln k_hat - ln k*|."""
    Z = model.forward(torch.as_tensor(X, device=device)).cpu().numpy().astype(np.float64)
    qh = np.argmax(Z[:, :5], axis=1)
    kh = np.clip(np.floor(np.exp(np.minimum(Z[:, 5], 30.0)) + 0.5), 1, K_MAX)
    return {"q_acc": float(np.mean(qh == q)), "q_safe": float(np.mean(qh >= q)),
            "logk_mae": float(np.mean(np.abs(np.log(kh) - np.log(k))))}


def expected_passes(q_hat: np.ndarray, q_true: np.ndarray) -> np.ndarray:
    """Passes over A that pbpqlp_factor_auto spends for a prediction, counting
    one residual check per answer: 2 q_hat + 3 when q_hat >= q* or q_hat >= 3
    (no fallback), else 10 (the fallback to q = 3 and a second check)."""
    ok = q_hat >= q_true
    return np.where(ok, 2 * q_hat + 3, np.where(q_hat < 3, 10, 2 * q_hat + 3))


def calibrate(model: B.Model, X: np.ndarray, q: np.ndarray, device, log=_log):
    """Cost-sensitive calibration of the five q logits: offsets d_q added to
    the output biases (so q_hat stays the argmax of the network's logits)
    chosen by coordinate descent to minimize the expected passes on held-out
    samples.  Returns a new model with the shifted biases."""
    Z = model.forward(torch.as_tensor(X, device=device)).cpu().numpy().astype(np.float64)[:, :5]
    d = np.zeros(5)
    cost = lambda dd: float(np.mean(expected_passes(np.argmax(Z + dd, axis=1), q)))
    best = cost(d)
    base = best
    grid = np.linspace(-4.0, 4.0, 81)
    for _ in range(4):
        for c in range(1, 5):
            for g in grid:
                t = d.copy()
                t[c] = g
                v = cost(t)
                if v < best - 1e-12:
                    best, d = v, t
    theta = model.params().astype(np.float64)
    theta[-6:-1] += d
    log(f"  calibration offsets {np.round(d, 2).tolist()}: expected passes {base:.3f} -> {best:.3f}")
    return B.Model(theta.astype(np.float32), device=device), d


def train(data: dict, epochs: int, batch: int, lr: float, seed: int, device, val_frac=0.125,
          log=_log):
    X, q, k = data["X"], data["q"], data["k"]
    n = X.shape[0]
    nval = max(1, int(round(n * val_frac)))
    ntr = n - nval
    model = B.Model(synth.mlp_init(seed), device=device)
    Xd = torch.as_tensor(X[:ntr], device=device)
    qd = torch.as_tensor(q[:ntr].astype(np.int32), device=device)
    lkd = torch.as_tensor(np.log(k[:ntr]).astype(np.float32), device=device)
    rng = np.random.default_rng(seed)
    steps = epochs * ((ntr + batch - 1) // batch)
    step = 0
    hist = []
    for ep in range(epochs):
        perm = torch.as_tensor(rng.permutation(ntr), device=device)
        total, nb = None, 0
        for i in range(0, ntr, batch):
            idx = perm[i:i + batch]
            # cosine decay of the learning rate to 5 % of its start
            a = lr * (0.05 + 0.95 * 0.5 * (1.0 + math.cos(math.pi * step / steps)))
            loss = model.train_step(Xd[idx], qd[idx], lkd[idx], a)
            total = loss if total is None else total + loss
            nb += 1
            step += 1
        if (ep + 1) % max(1, epochs // 10) == 0 or ep + 1 == epochs:
            tr = float(total.item()) / nb
            ev = evaluate(model, X[ntr:], q[ntr:], k[ntr:], device)
            hist.append({"epoch": ep + 1, "train_loss": tr, **ev})
            log(f"  epoch {ep + 1}: train loss {tr:.4f}  val q acc {ev['q_acc']:.3f}  "
                f"q_hat>=q* {ev['q_safe']:.3f}  |dln k| {ev['logk_mae']:.3f}")
    # calibrate on the first half of the held-out samples, report on the second
    half = ntr + nval // 2
    steps_done = model.steps
    model, offs = calibrate(model, X[ntr:half], q[ntr:half], device, log)
    ev = evaluate(model, X[half:], q[half:], k[half:], device)
    Z = model.forward(torch.as_tensor(X[half:], device=device)).cpu().numpy()
    ev["expected_passes"] = float(np.mean(expected_passes(np.argmax(Z[:, :5], axis=1), q[half:])))
    ev["expected_passes_oracle_q"] = float(np.mean(expected_passes(q[half:], q[half:])))
    ev["calibration_offsets"] = offs.tolist()
    ev["adam_steps"] = steps_done
    hist.append({"epoch": "calibrated", **ev})
    log(f"  calibrated: q acc {ev['q_acc']:.3f}  q_hat>=q* {ev['q_safe']:.3f}  expected passes "
        f"{ev['expected_passes']:.3f} (exact q*: {ev['expected_passes_oracle_q']:.3f}, plain q=3: 8)")
    return model, hist


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    d = sub.add_parser("data")
    d.add_argument("--count", type=int, default=4096)
    d.add_argument("--seed", type=int, default=1)
    d.add_argument("--m-min", type=int, default=512)
    d.add_argument("--m-max", type=int, default=2048)
    d.add_argument("--out", required=True)
    t = sub.add_parser("train")
    t.add_argument("--data", required=True, nargs="+")
    t.add_argument("--epochs", type=int, default=400)
    t.add_argument("--batch", type=int, default=256)
    t.add_argument("--lr", type=float, default=2e-3)
    t.add_argument("--seed", type=int, default=3)
    t.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    dev = torch.device("cuda:0")
    if a.cmd == "data":
        t0 = time.time()
        data = make_dataset(a.count, a.seed, dev, (a.m_min, a.m_max), (a.m_min, a.m_max),
                            checkpoint=lambda d: np.savez(a.out, **d))
        np.savez(a.out, **data)
        print(f"wrote {a.count} samples to {a.out} in {time.time() - t0:.0f} s", flush=True)
    else:
        parts = [np.load(f, allow_pickle=False) for f in a.data]
        data = {key: np.concatenate([z[key] for z in parts]) for key in parts[0].files}
        t0 = time.time()
        model, hist = train(data, a.epochs, a.batch, a.lr, a.seed, dev)
        torch.cuda.synchronize()
        model.save(a.out)
        print(f"trained {hist[-1]['adam_steps']} Adam steps on {len(data['q'])} samples in "
              f"{time.time() - t0:.1f} s; wrote {a.out}", flush=True)
        print("final", hist[-1], flush=True)
        with open(a.out + ".json", "w") as fh:
            json.dump({"samples": int(len(data["q"])), "history": hist}, fh, indent=1)


if __name__ == "__main__":
    main()
