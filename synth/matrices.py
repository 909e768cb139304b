"""Seeded planted-spectrum matrices for the PbP-QLP workloads.

Every generator draws from ``numpy.random.Generator(numpy.random.Philox(seed))``
so that a (config, batch index) pair always yields the same matrix on any host.
Seeds follow one convention: the matrix of config ``c`` and batch index ``b``
uses ``seed_A = 1_000_000*c + b`` and its sketch uses
``seed_omega = 1_000_000*c + 500_000 + b``.

The workloads restate the paper's synthetic test classes (Section V-B: low-rank
plus noise, fast and slow decay; all built as U*diag(sigma)*V^T with random
orthogonal U, V) at the sizes the benchmark configurations use.  Nothing here
computes any part of the factorization.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

__all__ = [
    "rng_for", "seed_a", "seed_omega", "haar_panel", "planted", "Workload",
    "config1", "config2", "config3", "config4_shapes", "config4_matrix",
    "lowrank_plus_noise", "paper_matrix1", "paper_matrix3", "paper_matrix4",
    "spectrum_family", "gaussian", "sparse_lowrank",
]


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(int(seed)))


def seed_a(config: int, b: int = 0) -> int:
    return 1_000_000 * config + b


def seed_omega(config: int, b: int = 0) -> int:
    return 1_000_000 * config + 500_000 + b


def gaussian(rng: np.random.Generator, shape, dtype=np.float64) -> np.ndarray:
    return rng.standard_normal(shape, dtype=dtype)


def haar_panel(rng: np.random.Generator, n: int, k: int) -> np.ndarray:
    """n x k matrix with orthonormal columns, Haar-distributed.

    QR of an i.i.d. N(0,1) panel with the signs of diag(R) folded into Q
    (Mezzadri, Notices AMS 2007), so the distribution is exactly Haar.
    """
    g = rng.standard_normal((n, k))
    q, r = np.linalg.qr(g)
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d


def planted(rng: np.random.Generator, m: int, n: int, sigma: np.ndarray,
            noise: float = 0.0, dtype=np.float64, block_rows: int = 4096) -> np.ndarray:
    """A = U diag(sigma) V^T + noise * N(0,1), U (m x r), V (n x r) Haar panels.

    The low-rank part is formed in float64; noise is added in float64 and the
    sum is rounded once to ``dtype``.  Rows are produced in blocks to bound
    host memory for the large workloads.
    """
    sigma = np.asarray(sigma, dtype=np.float64)
    r = sigma.shape[0]
    u = haar_panel(rng, m, r)
    v = haar_panel(rng, n, r)
    us = u * sigma
    out = np.empty((m, n), dtype=dtype)
    for r0 in range(0, m, block_rows):
        r1 = min(m, r0 + block_rows)
        blk = us[r0:r1] @ v.T
        if noise != 0.0:
            blk += noise * rng.standard_normal((r1 - r0, n), dtype=np.float32)
        out[r0:r1] = blk
    return out


@dataclass
class Workload:
    """One factorization problem: the matrix and the method's parameters."""
    name: str
    A: np.ndarray
    k: int
    p: int
    q: int
    seed: int
    sigma: Optional[np.ndarray] = None      # planted singular values (noise-free part)
    noise: float = 0.0
    extra: dict = field(default_factory=dict)

    @property
    def l(self) -> int:
        return self.k + self.p


def config1(b: int = 0) -> Workload:
    """1000 x 1000 FP64: Haar U, V (full QR of seeded N(0,1) 1000x1000),
    sigma_i = 1 for i <= 20 and 0.5**(i-20) after; k=20, p=5, q=1."""
    n = 1000
    rng = rng_for(seed_a(1, b))
    i = np.arange(1, n + 1, dtype=np.float64)
    sigma = np.where(i <= 20, 1.0, 0.5 ** (i - 20))
    A = planted(rng, n, n, sigma, 0.0, np.float64)
    return Workload("c1_1000sq_f64", A, 20, 5, 1, seed_omega(1, b), sigma)


def config2(b: int = 0, m: int = 16384, n: int = 16384, r: int = 512,
            k: int = 200, p: int = 20, q: int = 2) -> Workload:
    """16384 x 16384 stored FP32: U, V from QR of seeded Gaussian 16384x512
    panels, sigma_i = 1/i for i <= 512, plus 1e-6 * N(0,1); k=200, p=20, q=2.
    Smaller (m, n, r, k, p) give same-recipe parity cases."""
    rng = rng_for(seed_a(2, b))
    sigma = 1.0 / np.arange(1, r + 1, dtype=np.float64)
    A = planted(rng, m, n, sigma, 1e-6, np.float32)
    return Workload(f"c2_{m}x{n}_f32", A, k, p, q, seed_omega(2, b), sigma, 1e-6)


def lowrank_plus_noise(rng: np.random.Generator, m: int, n: int, r: int, noise: float,
                       dtype=np.float32, block_rows: int = 8192):
    """A = X Y^T + noise * N(0,1) with X (m x r), Y (n x r) entries N(0, 1/r).
    Returns (A, planted singular values of X Y^T)."""
    s = 1.0 / math.sqrt(r)
    X = rng.standard_normal((m, r)) * s
    Y = rng.standard_normal((n, r)) * s
    out = np.empty((m, n), dtype=dtype)
    for r0 in range(0, m, block_rows):
        r1 = min(m, r0 + block_rows)
        blk = X[r0:r1] @ Y.T
        if noise != 0.0:
            blk += noise * rng.standard_normal((r1 - r0, n), dtype=np.float32)
        out[r0:r1] = blk
    # singular values of X Y^T = those of R_X R_Y^T (thin QR of each factor)
    rx = np.linalg.qr(X, mode="r")
    ry = np.linalg.qr(Y, mode="r")
    sig = np.linalg.svd(rx @ ry.T, compute_uv=False)
    return out, sig


def config3(b: int = 0, m: int = 200000, n: int = 4096, r: int = 64,
            k: int = 64, p: int = 16, q: int = 1) -> Workload:
    """200000 x 4096 FP32: X Y^T with entries N(0,1/64), plus 1e-3 * N(0,1);
    k=64, p=16, q=1."""
    rng = rng_for(seed_a(3, b))
    A, sig = lowrank_plus_noise(rng, m, n, r, 1e-3, np.float32)
    return Workload(f"c3_{m}x{n}_f32", A, k, p, q, seed_omega(3, b), sig, 1e-3)


def config4_shapes(count: int = 1024, m_range=(256, 4096), n_range=(256, 2048),
                   r_range=(8, 64)):
    """Shapes of the batched workload: m ~ U[256,4096], n ~ U[256,2048],
    rank r ~ U[8,64] (inclusive integers), drawn from one seeded stream."""
    rng = rng_for(seed_a(4, 999_999))
    m = rng.integers(m_range[0], m_range[1] + 1, size=count)
    n = rng.integers(n_range[0], n_range[1] + 1, size=count)
    r = rng.integers(r_range[0], r_range[1] + 1, size=count)
    return [(int(a), int(b_), int(c)) for a, b_, c in zip(m, n, r)]


def config4_matrix(b: int, m: int, n: int, r: int) -> Workload:
    """Batch member b: U diag(exp(-i/r)) V^T (rank r) + 1e-5 N(0,1), FP32;
    k=r, p=8, q=1."""
    rng = rng_for(seed_a(4, b))
    sigma = np.exp(-np.arange(1, r + 1, dtype=np.float64) / r)
    A = planted(rng, m, n, sigma, 1e-5, np.float32)
    return Workload(f"c4_{b}", A, r, 8, 1, seed_omega(4, b), sigma, 1e-5)


def _square_planted(rng, n, sigma, dtype=np.float64):
    u = haar_panel(rng, n, n)
    v = haar_panel(rng, n, n)
    return ((u * sigma) @ v.T).astype(dtype)


def paper_matrix1(mu: float = 0.005, n: int = 1000, k: int = 20, seed: int = 11) -> Workload:
    """Low-rank plus noise (paper Section V-B, Matrix 1): sigma decreasing
    linearly from 1 towards 1e-25 across n points, kept for i <= k and zero
    after; plus mu * sigma_k * N with N a Gaussian matrix of unit 2-norm.
    mu = 0.005 gives the large-gap case, mu = 0.02 the small-gap case."""
    rng = rng_for(seed)
    full = np.linspace(1.0, 1e-25, n)
    sigma = np.where(np.arange(n) < k, full, 0.0)
    A1 = _square_planted(rng, n, sigma)
    G = rng.standard_normal((n, n))
    N = G / np.linalg.norm(G, 2)
    return Workload(f"paper_m1_mu{mu}", A1 + mu * sigma[k - 1] * N, k, 0, 0, seed + 500_000, sigma)


def paper_matrix3(n: int = 1000, seed: int = 13) -> Workload:
    """Fast decay (paper Matrix 3): sigma_i = exp(-i/6)."""
    rng = rng_for(seed)
    sigma = np.exp(-np.arange(1, n + 1) / 6.0)
    return Workload("paper_m3", _square_planted(rng, n, sigma), 20, 0, 0, seed + 500_000, sigma)


def paper_matrix4(n: int = 1000, seed: int = 14) -> Workload:
    """Slow decay (paper Matrix 4): sigma_i = i^-2."""
    rng = rng_for(seed)
    sigma = np.arange(1, n + 1, dtype=np.float64) ** -2.0
    return Workload("paper_m4", _square_planted(rng, n, sigma), 20, 0, 0, seed + 500_000, sigma)


def spectrum_family(rng: np.random.Generator, length: int, family: Optional[str] = None):
    """Random spectrum from one of three families used for the learned q/k
    predictor: 'step' (1 up to s, then a drop to 10^-U[2,6]), 'poly'
    (i^-a, a ~ U[0.5, 3]) and 'exp' (exp(-i/tau), tau ~ logU[2, 200]).
    Returns (family, sigma) with sigma non-increasing and sigma_1 = 1."""
    fams = ("step", "poly", "exp")
    if family is None:
        family = fams[int(rng.integers(0, 3))]
    i = np.arange(1, length + 1, dtype=np.float64)
    if family == "step":
        s = int(rng.integers(4, 97))
        drop = 10.0 ** (-rng.uniform(2.0, 6.0))
        sigma = np.where(i <= s, 1.0, drop * np.exp(-(i - s) / 50.0))
    elif family == "poly":
        a = rng.uniform(0.5, 3.0)
        sigma = i ** (-a)
    elif family == "exp":
        tau = math.exp(rng.uniform(math.log(2.0), math.log(200.0)))
        sigma = np.exp(-(i - 1) / tau)
    else:
        raise ValueError(family)
    return family, sigma


def sparse_lowrank(m: int, n: int, r: int, density: float, noise_nnz_per_row: float, seed: int,
                   decay: float = 0.9, col_alpha: float = 0.0, dtype=np.float64):
    """Sparse A = sum_k sigma_k u_k v_k^T + sparse noise, in CSR (scipy).

    u_k (m) and v_k (n) are sparse Gaussian vectors with about density * m and
    density * n nonzeros, scaled to unit norm, sigma_k = decay^k; the noise has
    about noise_nnz_per_row entries per row with N(0, 1e-3) values.  With
    col_alpha > 0 the column indices of both parts are drawn with probability
    proportional to (j + 1)^-col_alpha (a power-law column degree
    distribution: a few nearly dense columns, many short ones).  Returns
    (A_csr, sigma)."""
    import scipy.sparse as sp
    rng = rng_for(seed)
    if col_alpha > 0:
        w = (np.arange(n, dtype=np.float64) + 1.0) ** -col_alpha
        col_p = w / w.sum()
    else:
        col_p = None
    sigma = decay ** np.arange(r, dtype=np.float64)
    A = sp.csr_matrix((m, n), dtype=np.float64)
    for k in range(r):
        ku = max(1, int(round(density * m)))
        kv = max(1, int(round(density * n)))
        iu = rng.choice(m, size=ku, replace=False)
        iv = rng.choice(n, size=kv, replace=False, p=col_p)
        u = rng.standard_normal(ku)
        v = rng.standard_normal(kv)
        u /= np.linalg.norm(u)
        v /= np.linalg.norm(v)
        A = A + sp.csr_matrix((sigma[k] * np.outer(u, v).ravel(),
                               (np.repeat(iu, kv), np.tile(iv, ku))), shape=(m, n))
    nz = int(round(noise_nnz_per_row * m))
    if nz > 0:
        ri = rng.integers(0, m, size=nz)
        ci = rng.choice(n, size=nz, p=col_p) if col_p is not None else rng.integers(0, n, size=nz)
        A = A + sp.csr_matrix((1e-3 * rng.standard_normal(nz), (ri, ci)), shape=(m, n))
    A = sp.csr_matrix(A, dtype=dtype)
    A.sum_duplicates()
    A.sort_indices()
    return A, sigma
