"""FP64 CPU oracle of the learned q/k head -- test infrastructure only.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run this module.  It shares
no code with the GPU library.

This part is a project extension; the paper has no learned component.  What
it builds on from the paper: the diagonal of the QLP factor L tracks the
singular values of A (Section III-A, the discussion after eq. (Ahat), and the
bounds of Theorems 3-5), so the diagonal of L from a cheap q = 0 run describes
the spectrum's decay; and the power iterations of Algorithm 1 trade passes
over A for accuracy (Section III-B), which is the choice being learned.

Definitions (each function states the one it follows):

* Probe features: f_i = clip(ln(L_ii / L_11) / ln(1/FLOOR), -1, 1) for the
  64 diagonal entries of the q = 0, l = 64 probe; a ratio that is not above
  FLOOR (including zero, negative or non-finite ones, and every entry when
  L_11 <= 0) gives f_i = -1.
* Network: 64 -> 128 (ReLU) -> 128 (ReLU) -> 6 outputs: five logits for
  q in {0, .., 4} and one regression output for ln k.  Parameters form one
  flat FP32 vector in the order W1 (128 x 64, row j holds the weights into
  hidden unit j), b1, W2 (128 x 128), b2, W3 (6 x 128), b3: 25606 values.
* Loss of a batch of B samples: mean over the batch of the softmax
  cross-entropy of the five logits against q*, plus LAMBDA_K times the mean of
  (output_6 - ln k*)^2.
* Adam (Kingma and Ba, ICLR 2015, Algorithm 1) with bias correction:
  m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
  theta -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
* Labels: r_opt(l) = sqrt(sum_{i > l} sigma_i^2) / sqrt(sum_i sigma_i^2) (the
  best rank-l residual, Eckart-Young); k* = the smallest k with
  sigma_{k+1} <= K_REL * sigma_1, capped at k_max; q* = the smallest q in
  0..4 with r(q) <= Q_SLACK * r_opt(k* + p), else 4.

Pins (tests/test_oracle_mlp.py): central finite differences of the loss for
every parameter group; the closed form of the network where every unit is
active (an affine map computed as one composed matrix); invariance under a
permutation of hidden units; the softmax cross-entropy gradient p - onehot;
Adam's closed-form steps for constant and sign-flipping gradients; features
and labels of hand-made spectra.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "N_IN", "N_HID", "N_OUT", "N_Q", "N_PARAMS", "FLOOR", "LAMBDA_K", "K_REL", "Q_SLACK",
    "unpack", "pack", "features", "forward", "loss_and_grad", "adam_step", "AdamState",
    "r_opt", "k_star", "q_star", "predict",
]

N_IN, N_HID, N_OUT, N_Q = 64, 128, 6, 5
N_PARAMS = N_HID * N_IN + N_HID + N_HID * N_HID + N_HID + N_OUT * N_HID + N_OUT
FLOOR = 1e-6          # smallest ratio L_ii / L_11 the features resolve
LAMBDA_K = 1.0        # weight of the ln k regression term
K_REL = 1e-3          # k*: singular values below K_REL * sigma_1 are noise
Q_SLACK = 1.05        # q*: residual within 5 % of the best rank-l residual


def unpack(theta: np.ndarray):
    """Flat parameter vector -> (W1, b1, W2, b2, W3, b3), in the order above."""
    theta = np.asarray(theta, dtype=np.float64)
    if theta.shape != (N_PARAMS,):
        raise ValueError("expected %d parameters" % N_PARAMS)
    shapes = [(N_HID, N_IN), (N_HID,), (N_HID, N_HID), (N_HID,), (N_OUT, N_HID), (N_OUT,)]
    out, o = [], 0
    for s in shapes:
        size = int(np.prod(s))
        out.append(theta[o:o + size].reshape(s))
        o += size
    return tuple(out)


def pack(W1, b1, W2, b2, W3, b3) -> np.ndarray:
    return np.concatenate([np.ravel(x) for x in (W1, b1, W2, b2, W3, b3)]).astype(np.float64)


def features(L: np.ndarray) -> np.ndarray:
    """Probe features from the l x l factor L (l = 64) of a q = 0 run."""
    d = np.diag(np.asarray(L, dtype=np.float64))[:N_IN]
    if d.shape[0] != N_IN:
        raise ValueError("the probe needs l = 64")
    scale = math.log(1.0 / FLOOR)
    f = np.full(N_IN, -1.0)
    if not (d[0] > 0.0 and math.isfinite(d[0])):
        return f
    for i in range(N_IN):
        t = d[i] / d[0]
        if math.isfinite(t) and t > FLOOR:
            f[i] = min(math.log(t) / scale, 1.0)
    return f


def _relu(x):
    return np.maximum(x, 0.0)


def forward(theta: np.ndarray, X: np.ndarray):
    """Outputs (B x 6) of the network for features X (B x 64), and the hidden
    activations (h1, h2) the gradient needs."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    h1 = _relu(X @ W1.T + b1)
    h2 = _relu(h1 @ W2.T + b2)
    z = h2 @ W3.T + b3
    return z, (h1, h2)


def _log_softmax(z: np.ndarray) -> np.ndarray:
    mx = np.max(z, axis=1, keepdims=True)
    return z - mx - np.log(np.sum(np.exp(z - mx), axis=1, keepdims=True))


def loss_and_grad(theta: np.ndarray, X: np.ndarray, q: np.ndarray, logk: np.ndarray):
    """Batch loss and its gradient with respect to the flat parameters."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    q = np.asarray(q, dtype=np.int64)
    logk = np.asarray(logk, dtype=np.float64)
    B = X.shape[0]
    z, (h1, h2) = forward(theta, X)
    ls = _log_softmax(z[:, :N_Q])
    ce = -ls[np.arange(B), q]
    err = z[:, N_Q] - logk
    loss = float(np.mean(ce) + LAMBDA_K * np.mean(err * err))
    # d loss / d z
    dz = np.zeros_like(z)
    dz[:, :N_Q] = np.exp(ls)
    dz[np.arange(B), q] -= 1.0
    dz[:, :N_Q] /= B
    dz[:, N_Q] = 2.0 * LAMBDA_K * err / B
    # back through the three layers
    dW3 = dz.T @ h2
    db3 = dz.sum(axis=0)
    dh2 = (dz @ W3) * (h2 > 0.0)
    dW2 = dh2.T @ h1
    db2 = dh2.sum(axis=0)
    dh1 = (dh2 @ W2) * (h1 > 0.0)
    dW1 = dh1.T @ X
    db1 = dh1.sum(axis=0)
    return loss, pack(dW1, db1, dW2, db2, dW3, db3)


class AdamState:
    """Adam's moment estimates and step count."""

    def __init__(self, n: int = N_PARAMS):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0


def adam_step(theta: np.ndarray, g: np.ndarray, st: AdamState, lr: float,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> np.ndarray:
    """One Adam update (Kingma and Ba, Algorithm 1); returns the new theta."""
    st.t += 1
    st.m = beta1 * st.m + (1.0 - beta1) * g
    st.v = beta2 * st.v + (1.0 - beta2) * g * g
    mhat = st.m / (1.0 - beta1 ** st.t)
    vhat = st.v / (1.0 - beta2 ** st.t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps)


def predict(theta: np.ndarray, f: np.ndarray, k_max: int):
    """(q_hat, k_hat): the argmax of the five logits (lowest index on ties)
    and exp of the regression output rounded to the nearest integer, clamped
    to [1, k_max]."""
    z, _ = forward(theta, np.asarray(f, dtype=np.float64)[None, :])
    z = z[0]
    qh = int(np.argmax(z[:N_Q]))
    kh = int(math.floor(math.exp(min(z[N_Q], 30.0)) + 0.5))
    return qh, max(1, min(k_max, kh))


def r_opt(sigma: np.ndarray, l: int) -> float:
    """Best relative Frobenius residual of a rank-l approximation."""
    s2 = np.asarray(sigma, dtype=np.float64) ** 2
    return float(math.sqrt(s2[l:].sum() / s2.sum()))


def k_star(sigma: np.ndarray, k_max: int) -> int:
    """Smallest k with sigma_{k+1} <= K_REL sigma_1, capped at k_max."""
    s = np.asarray(sigma, dtype=np.float64)
    for k in range(1, min(k_max, s.shape[0] - 1) + 1):
        if s[k] <= K_REL * s[0]:
            return k
    return k_max


def q_star(r_of_q, r_best: float) -> int:
    """Smallest q with r(q) <= Q_SLACK * r_best; 4 if none does."""
    for q, r in enumerate(r_of_q):
        if r <= Q_SLACK * r_best:
            return q
    return len(r_of_q) - 1
