"""Seeded inputs of the learned q/k head: initial network parameters and the
recipe of the training / evaluation matrices.

Matrices follow the learned-head recipe: A = U diag(sigma) V^T with U, V
orthonormal panels (QR of Gaussian panels) and sigma drawn from one of three
families (``matrices.spectrum_family``: step, polynomial, exponential).  To
keep generation cheap the planted rank is capped at ``rank_cap`` columns
(sigma_i = 0 beyond it), and every label is computed from the capped
spectrum, so features and labels describe the same matrix.  Nothing here
computes any part of the factorization or of the network.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .matrices import rng_for, spectrum_family

__all__ = ["MLP_SHAPES", "mlp_init", "QKSpec", "qk_spec", "qk_matrix"]

# (rows, cols) of W1, b1, W2, b2, W3, b3 in the flat parameter order
MLP_SHAPES = [(128, 64), (128,), (128, 128), (128,), (6, 128), (6,)]


def mlp_init(seed: int) -> np.ndarray:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases, as one flat
    float32 vector of 25606 values."""
    rng = rng_for(seed)
    parts = []
    for shp in MLP_SHAPES:
        if len(shp) == 2:
            parts.append(rng.standard_normal(shp) * np.sqrt(2.0 / shp[1]))
        else:
            parts.append(np.zeros(shp))
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


@dataclass
class QKSpec:
    index: int
    m: int
    n: int
    family: str
    sigma: np.ndarray      # planted singular values (length <= rank_cap), sigma_1 = 1
    seed_a: int            # seeds the Gaussian panels of U and V
    seed_omega: int        # the method's sketch seed


def qk_spec(index: int, base_seed: int, m_range=(512, 2048), n_range=(512, 2048),
            rank_cap: int = 256, family=None) -> QKSpec:
    """The index-th matrix of a learned-head set: sizes uniform in the ranges
    (inclusive), a random spectrum family, planted rank min(m, n, rank_cap)."""
    rng = rng_for(7_000_000 + 1009 * base_seed + index)
    m = int(rng.integers(m_range[0], m_range[1] + 1))
    n = int(rng.integers(n_range[0], n_range[1] + 1))
    r = min(m, n, rank_cap)
    fam, sigma = spectrum_family(rng, r, family)
    return QKSpec(index, m, n, fam, sigma, 5_000_000 + 1009 * base_seed + index,
                  6_000_000 + 1009 * base_seed + index)


def qk_matrix(spec: QKSpec, dtype=np.float64) -> np.ndarray:
    """Host construction of a spec's matrix (for small sizes and tests)."""
    rng = rng_for(spec.seed_a)
    r = spec.sigma.shape[0]
    u, _ = np.linalg.qr(rng.standard_normal((spec.m, r)))
    v, _ = np.linalg.qr(rng.standard_normal((spec.n, r)))
    return ((u * spec.sigma) @ v.T).astype(dtype)
