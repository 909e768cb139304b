"""FP64 CPU oracle for Projection-based Partial QLP (PbP-QLP).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run this module.  The GPU
library never calls it and shares no code with it; the only thing both sides
consume is the seeded input generator package ``synth``.

What is computed (Kaloorazi & Chen, "Projection-based QLP algorithm for
efficiently computing low-rank approximation of matrices", IEEE TSP 2021):

* Section III-A, eqs. (c), (Pbar), (D), (DQR), (R^T = Pt Rt), (Ahat): the basic
  method -- Gaussian sketch, orthonormal basis of the sketch, projection of A
  onto it, an unpivoted QR of the projection, a second unpivoted QR of R^T.
* Section III-B, Algorithm 1 (Power Iteration-coupled PbP-QLP): the same with q
  power iterations and a re-orthonormalization after every application of A
  or A^T (the paper requires this because components below
  sigma_1 * eps^(1/(2q+1)) are otherwise lost).

Orientation.  ``pbpqlp`` works on an m x n matrix A with an n x l Gaussian
Omega and returns (Q, L, P) with  A ~= Q @ L.T @ P.T : this is Algorithm 1
applied to A^T (the paper's Phi -> Omega, Pbar -> Q basis, paper-Q -> P,
paper Pt -> Qtilde, paper L -> L).  The paper's own orientation for an
n1 x n2 matrix A with an n1 x d sketch Phi is therefore pbpqlp(A.T,
Omega=Phi): its (P, L, Q) are the paper's (Q, L, P), with A ~= Q L P^T.

Readings where the paper is silent or ambiguous:
* orth() is a QR-type (upper-triangular) orthonormalization -- the paper says
  it can be "a packaged QR" -- implemented here with Householder reflections.
* Every QR is sign-normalized so that diag(R) >= 0 (a zero column keeps +1,
  i.e. the reflector is skipped and Q gets the unit vector).
* randn() is the project's Philox4x32-10 + Box-Muller generator, rounded to
  bfloat16 (round-to-nearest-even) with magnitudes below 2^-14 flushed to zero,
  so the same sketch is exactly representable in fp64/fp32/bf16/fp16.

Pins (see tests/test_oracle_*.py): numpy/LAPACK QR and SVD, an mpmath 50-digit
brute force of the plain definition on tiny inputs, the randomized-SVD
projection with the same Omega, L = chol(R R^T), the a-posteriori residual
identity, exact recovery for rank(A) <= l, the paper's deterministic theorems
(Theorems 1, 3, 4, 5, 7 and the Mathias-Stewart inequalities), Random123's
published Philox known-answer vectors and a normality test of the sketch.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional

import numpy as np

__all__ = [
    "philox4x32_10", "bf16_rne", "omega", "householder_qr", "hh_orth",
    "pbpqlp", "OracleResult", "rel_residual", "jacobi_svd",
    "validate_args",
]

# ----------------------------------------------------------------------------
# randn(): Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers:
# as easy as 1, 2, 3", SC'11) followed by the Box-Muller transform.
# ----------------------------------------------------------------------------
_MASK = np.uint64(0xFFFFFFFF)
_PHILOX_M0 = np.uint64(0xD2511F53)
_PHILOX_M1 = np.uint64(0xCD9E8D57)
_PHILOX_W0 = np.uint64(0x9E3779B9)
_PHILOX_W1 = np.uint64(0xBB67AE85)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox-4x32 rounds.  Inputs are arrays (or scalars) of 32-bit words
    held in uint64; returns the four output words.

    One round: the two multipliers take counter words 0 and 2; the new counter
    is (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0)); the
    key is bumped by the Weyl constants between rounds."""
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) & _MASK for x in (c0, c1, c2, c3))
    k0 = np.uint64(int(k0) & 0xFFFFFFFF)
    k1 = np.uint64(int(k1) & 0xFFFFFFFF)
    for _ in range(10):
        p0 = _PHILOX_M0 * c0
        p1 = _PHILOX_M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
        k0 = (k0 + _PHILOX_W0) & _MASK
        k1 = (k1 + _PHILOX_W1) & _MASK
    return c0, c1, c2, c3


def bf16_rne(x: np.ndarray) -> np.ndarray:
    """Round float64 values to the nearest bfloat16 value (8 significant bits),
    ties to even, returned as float64.  Written from the definition: with
    x = m * 2^e and 0.5 <= |m| < 1, keep rint(m * 2^8) * 2^(e-8)."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)
    return np.ldexp(np.rint(m * 256.0), e - 8)


_TWO_PI = 2.0 * math.pi
_FTZ = 2.0 ** -14


def omega(n: int, l: int, seed: int) -> np.ndarray:
    """The n x l Gaussian test matrix (spec Omega = the paper's Phi).

    Element (i, j) has flat index t = i*l + j.  Philox4x32-10 with key
    (seed mod 2^32, seed div 2^32) and counter (b mod 2^32, b div 2^32, 0, 0),
    b = t div 4, gives words x0..x3.  Words (x0, x1) feed Box-Muller for
    t mod 4 in {0, 1}, (x2, x3) for {2, 3}:  u = (x + 1/2) / 2^32,
    r = sqrt(-2 ln u_a), theta = 2 pi u_b, z = r cos(theta) (even t) or
    r sin(theta) (odd t).  z is rounded to bf16 (RNE) and |z| < 2^-14 -> 0."""
    N = n * l
    nb = (N + 3) // 4
    b = np.arange(nb, dtype=np.uint64)
    seed = int(seed)
    x0, x1, x2, x3 = philox4x32_10(b & _MASK, b >> np.uint64(32), 0, 0,
                                   seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    scale = 2.0 ** -32
    ua = (x0.astype(np.float64) + 0.5) * scale
    ub = (x1.astype(np.float64) + 0.5) * scale
    uc = (x2.astype(np.float64) + 0.5) * scale
    ud = (x3.astype(np.float64) + 0.5) * scale
    ra = np.sqrt(-2.0 * np.log(ua))
    rc = np.sqrt(-2.0 * np.log(uc))
    tb = _TWO_PI * ub
    td = _TWO_PI * ud
    z = np.stack([ra * np.cos(tb), ra * np.sin(tb), rc * np.cos(td), rc * np.sin(td)], axis=1)
    z = z.reshape(-1)[:N]
    z = bf16_rne(z)
    z = np.where(np.abs(z) < _FTZ, 0.0, z)
    return z.reshape(n, l)


# ----------------------------------------------------------------------------
# Unpivoted QR ("qr" and the packaged-QR "orth" of the paper's notation).
# ----------------------------------------------------------------------------
def householder_qr(M: np.ndarray):
    """Thin Householder QR of an r x c matrix (r >= c), LAPACK-style reflectors
    H_j = I - tau v v^T, followed by sign normalization: column j of Q and row
    j of R are negated when R_jj < 0, so diag(R) >= 0.  A column that is
    already zero below/at the diagonal gets no reflector (tau = 0), which
    leaves e_j in Q and 0 on the diagonal of R."""
    A = np.array(M, dtype=np.float64, copy=True)
    r, c = A.shape
    if r < c:
        raise ValueError("householder_qr needs rows >= cols")
    vs = []
    taus = []
    for j in range(c):
        x = A[j:, j]
        normx = np.linalg.norm(x)
        if normx == 0.0:
            vs.append(None)
            taus.append(0.0)
            continue
        alpha = -math.copysign(normx, x[0])
        v = x.copy()
        v[0] -= alpha
        tau = 2.0 / np.dot(v, v)
        w = v @ A[j:, j:]
        A[j:, j:] -= tau * np.outer(v, w)
        A[j + 1:, j] = 0.0
        vs.append(v)
        taus.append(tau)
    R = np.triu(A[:c, :c])
    Q = np.eye(r, c)
    for j in reversed(range(c)):
        v = vs[j]
        if v is None:
            continue
        Q[j:, :] -= taus[j] * np.outer(v, v @ Q[j:, :])
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d, d[:, None] * R


def hh_orth(M: np.ndarray) -> np.ndarray:
    """orth(M): the Q factor of the sign-normalized Householder QR."""
    return householder_qr(M)[0]


# ----------------------------------------------------------------------------
# PbP-QLP
# ----------------------------------------------------------------------------
def validate_args(m: int, n: int, k: int, p: int, q: int) -> int:
    """Argument rules of the problem statement (Section I-A and Algorithm 1:
    1 <= k <= d <= n2), with d = l = k + p, q >= 0 (q = 0 is the basic
    method of Section III-A) and a cap of 16 power iterations."""
    if m < 1 or n < 1:
        raise ValueError("empty matrix")
    if k < 1 or p < 0:
        raise ValueError("need k >= 1 and p >= 0")
    l = k + p
    if l > min(m, n):
        raise ValueError("l = k + p must not exceed min(m, n)")
    if q < 0 or q > 16:
        raise ValueError("q must lie in [0, 16]")
    return l


@dataclass
class OracleResult:
    Q: np.ndarray          # m x l, = Qbasis @ Qtilde (spec Q Q~)
    L: np.ndarray          # l x l lower triangular
    P: np.ndarray          # n x l
    R: np.ndarray          # l x l upper triangular, from B^T = P R (R-values on its diagonal)
    Qbasis: np.ndarray     # m x l orthonormal basis of the final sketch
    Qtilde: np.ndarray     # l x l orthogonal, from R^T = Qtilde L^T
    Omega: np.ndarray      # n x l sketch matrix actually used

    def reconstruct(self) -> np.ndarray:
        return self.Q @ self.L.T @ self.P.T


def pbpqlp(A: np.ndarray, k: int, p: int, q: int, seed: Optional[int] = None,
           Omega: Optional[np.ndarray] = None) -> OracleResult:
    """PbP-QLP of an m x n matrix A in the spec orientation (the
    method of Section III for A^T).

    Qb is an orthonormal basis of the sketch (A A^T)^q A Omega (eq. (c) with
    the power scheme of Section III-B, orthonormalized after every product
    with A or A^T, as that section requires for rounding reasons); P and R
    come from the unpivoted QR of the projection A^T Qb (eqs. (D), (DQR));
    Qtilde and U from the unpivoted QR of R^T (eq. (R^T = Pt Rt)), L = U^T;
    and the returned basis is Q = Qb Qtilde, so that A ~= Q L^T P^T, the
    paper's eq. (Ahat) written for A^T."""
    A = np.asarray(A)
    m, n = A.shape
    l = validate_args(m, n, k, p, q)
    A64 = A.astype(np.float64, copy=False)
    if Omega is None:
        if seed is None:
            raise ValueError("need seed or Omega")
        Omega = omega(n, l, seed)
    Omega = np.asarray(Omega, dtype=np.float64)
    if Omega.shape != (n, l):
        raise ValueError("Omega must be n x l")
    Y = A64 @ Omega
    Qb = hh_orth(Y)
    for _ in range(q):
        Z = A64.T @ Qb
        Ph = hh_orth(Z)
        Y = A64 @ Ph
        Qb = hh_orth(Y)
    W = A64.T @ Qb
    P, R = householder_qr(W)
    Qt, U = householder_qr(R.T)
    L = U.T
    return OracleResult(Q=Qb @ Qt, L=L, P=P, R=R, Qbasis=Qb, Qtilde=Qt, Omega=Omega)


def rel_residual(A: np.ndarray, Q: np.ndarray, L: np.ndarray, P: np.ndarray,
                 block_rows: int = 4096) -> float:
    """||A - Q L^T P^T||_F / ||A||_F in float64, streamed over row blocks so
    that no m x n temporary is formed."""
    M = np.asarray(L, dtype=np.float64).T @ np.asarray(P, dtype=np.float64).T
    Q = np.asarray(Q, dtype=np.float64)
    num = 0.0
    den = 0.0
    m = A.shape[0]
    for r0 in range(0, m, block_rows):
        r1 = min(m, r0 + block_rows)
        blk = np.asarray(A[r0:r1], dtype=np.float64)
        E = blk - Q[r0:r1] @ M
        num += float(np.einsum("ij,ij->", E, E))
        den += float(np.einsum("ij,ij->", blk, blk))
    if den == 0.0:
        return math.sqrt(num)
    return math.sqrt(num / den)


# ----------------------------------------------------------------------------
# One-sided (Hestenes) Jacobi SVD, for tiny test inputs only.
# ----------------------------------------------------------------------------
def jacobi_svd(M: np.ndarray, tol: float = 1e-15, max_sweeps: int = 80):
    """Singular values (descending) and right singular vectors of a small
    matrix by one-sided Jacobi rotations on column pairs until every pair is
    orthogonal to within tol.  Pure Python loops: tiny inputs only."""
    A = np.array(M, dtype=np.float64, copy=True)
    transposed = False
    if A.shape[0] < A.shape[1]:
        A = A.T.copy()
        transposed = True
    n = A.shape[1]
    V = np.eye(n)
    for _ in range(max_sweeps):
        rotated = False
        for i in range(n - 1):
            for j in range(i + 1, n):
                a = float(A[:, i] @ A[:, i])
                b = float(A[:, j] @ A[:, j])
                c = float(A[:, i] @ A[:, j])
                if c == 0.0 or abs(c) <= tol * math.sqrt(a * b):
                    continue
                rotated = True
                zeta = (b - a) / (2.0 * c)
                t = math.copysign(1.0, zeta) / (abs(zeta) + math.sqrt(1.0 + zeta * zeta))
                cs = 1.0 / math.sqrt(1.0 + t * t)
                sn = cs * t
                ai = A[:, i].copy()
                A[:, i] = cs * ai - sn * A[:, j]
                A[:, j] = sn * ai + cs * A[:, j]
                vi = V[:, i].copy()
                V[:, i] = cs * vi - sn * V[:, j]
                V[:, j] = sn * vi + cs * V[:, j]
        if not rotated:
            break
    s = np.sqrt(np.einsum("ij,ij->j", A, A))
    order = np.argsort(-s)
    s = s[order]
    V = V[:, order]
    if transposed:
        return s, None
    return s, V
