"""Seeded synthetic inputs shaped like the paper's test matrices.

This module only constructs input matrices (and the factors they are built
from); it holds none of the iteration's arithmetic. Both the CPU oracle's tests
and the GPU path's tests and benchmark draw their inputs here, so the two sides
see identical bytes.

Recipes (all FP64, row-major, numpy ``default_rng(seed)``):

* ``uniform``      -- entries iid U[-1, 1] (the 200x100 full-rank workload).
* ``lowrank_svd``  -- A = U diag(s) V^T, U (m x r) and V (n x r) with
  Haar-distributed orthonormal columns (QR of a Gaussian, signs fixed by
  diag(R) > 0), nonzero s log-spaced in [smin, 1] (rectangular rank-deficient
  Moore-Penrose workload; sigma_max = 1 exactly by construction).
* ``square_svd``   -- square nonsingular A = U diag(s) V^T, s log-uniform in
  [smin, 1] with the end points pinned so that sigma_max = 1 and
  sigma_min = smin exactly (mixed-precision workload).
* ``drazin_jordan`` -- A = P blockdiag(B, N) P^{-1}: B = Q diag(lam) Q^T
  nonsingular with lam ~ U[0.5, 2], N nilpotent made of Jordan blocks of size
  <= 3 (index 3), P = U_P diag(s_P) V_P^T with s_P log-spaced in [1, cond_P]
  (well conditioned), P^{-1} = V_P diag(1/s_P) U_P^T.
* ``request_stream`` -- Poisson arrivals of Moore-Penrose requests with
  m log-uniform in [64, 2048] (rounded to a multiple of 4), n = m / r with
  r uniform in {1, 2, 4}, entries iid N(0, 1), a fraction rank-deficient at
  half rank (A = G1 G2 / sqrt(k)).
* ``hilbert``      -- H_{m x n} = [1 / (i + j - 1)] (Example 8.2).
* ``grid_stencil`` -- stand-in for Example 8.3's sparse 841 x 841 matrix
  (MatrixMarket YOUNG1C, which is not available here): the 5-point stencil
  of a 29 x 29 grid, diagonal 4 + shift, each neighbour weight
  -1 + spread U(-1, 1) (nonsymmetric, not tridiagonal, strictly diagonally
  dominant for shift > 4 spread).
* ``spd``          -- symmetric positive definite Q diag(w) Q^T, Q Haar, w
  log-spaced in [1, cond] (weights of a weighted Moore-Penrose inverse).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def haar_columns(rng: np.random.Generator, m: int, r: int) -> np.ndarray:
    """m x r matrix with orthonormal columns, Haar distributed (first r columns
    of the Q factor of an m x m Gaussian; QR of the m x r Gaussian gives the same
    distribution once the signs of diag(R) are fixed)."""
    g = rng.standard_normal((m, r))
    q, rr = np.linalg.qr(g)
    sgn = np.sign(np.diag(rr))
    sgn[sgn == 0] = 1.0
    return q * sgn


def uniform(m: int = 200, n: int = 100, seed: int = 1001) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(m, n))


@dataclass
class SVDInput:
    A: np.ndarray
    U: np.ndarray
    s: np.ndarray
    V: np.ndarray


def lowrank_svd(m: int = 4096, n: int = 2048, r: int = 1536, smin: float = 1e-4,
                seed: int = 1002) -> SVDInput:
    rng = np.random.default_rng(seed)
    U = haar_columns(rng, m, r)
    V = haar_columns(rng, n, r)
    s = np.logspace(0.0, np.log10(smin), r)
    A = (U * s) @ V.T
    return SVDInput(np.ascontiguousarray(A), U, s, V)


def square_svd_device(n: int = 8192, smin: float = 1e-3, seed: int = 1003, device="cuda"):
    """The square_svd recipe built on the GPU with torch (FP64): Haar factors
    from torch.linalg.qr of seeded Gaussians (sign-fixed), s log-uniform in
    [smin, 1] with the end points pinned. Returns torch tensors (A, U, s, V).
    Used where the host QR of two n x n matrices would dominate (n = 8192)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)

    def haar(k):
        q, r = torch.linalg.qr(torch.randn(k, k, dtype=torch.float64, device=device, generator=g))
        d = torch.sign(torch.diagonal(r))
        d[d == 0] = 1.0
        return q * d

    U = haar(n)
    V = haar(n)
    s = torch.exp(torch.empty(n, dtype=torch.float64, device=device).uniform_(
        float(np.log(smin)), 0.0, generator=g))
    s[0], s[-1] = 1.0, smin
    s = torch.sort(s, descending=True).values
    A = (U * s) @ V.T.contiguous()
    return A.contiguous(), U, s, V


def square_svd(n: int = 8192, smin: float = 1e-3, seed: int = 1003) -> SVDInput:
    rng = np.random.default_rng(seed)
    U = haar_columns(rng, n, n)
    V = haar_columns(rng, n, n)
    s = np.exp(rng.uniform(np.log(smin), 0.0, size=n))
    s[0], s[-1] = 1.0, smin
    s = np.sort(s)[::-1].copy()
    A = (U * s) @ V.T
    return SVDInput(np.ascontiguousarray(A), U, s, V)


@dataclass
class DrazinInput:
    A: np.ndarray
    P: np.ndarray
    Pinv: np.ndarray
    Q: np.ndarray       # eigenvectors of the nonsingular block B
    lam: np.ndarray     # eigenvalues of B
    nil: np.ndarray     # the nilpotent block N
    index: int


def nilpotent_jordan(size: int, block: int = 3) -> tuple[np.ndarray, int]:
    """Nilpotent matrix made of Jordan blocks (ones on the superdiagonal
    inside each block) of size `block`, the last one shorter if needed.
    Returns (N, index of N)."""
    N = np.zeros((size, size))
    start = 0
    largest = 0
    while start < size:
        b = min(block, size - start)
        for i in range(b - 1):
            N[start + i, start + i + 1] = 1.0
        largest = max(largest, b)
        start += b
    return N, largest


def drazin_jordan(n: int = 2048, nb: int = 1792, cond_p: float = 10.0,
                  block: int = 3, seed: int = 1004) -> DrazinInput:
    rng = np.random.default_rng(seed)
    Q = haar_columns(rng, nb, nb)
    lam = rng.uniform(0.5, 2.0, size=nb)
    B = (Q * lam) @ Q.T
    Nn, index = nilpotent_jordan(n - nb, block)
    UP = haar_columns(rng, n, n)
    VP = haar_columns(rng, n, n)
    sP = np.logspace(0.0, np.log10(cond_p), n)
    P = (UP * sP) @ VP.T
    Pinv = (VP / sP) @ UP.T
    J = np.zeros((n, n))
    J[:nb, :nb] = B
    J[nb:, nb:] = Nn
    A = P @ J @ Pinv
    return DrazinInput(np.ascontiguousarray(A), P, Pinv, Q, lam, Nn, index)


def hilbert(m: int, n: int) -> np.ndarray:
    i = np.arange(1, m + 1)[:, None]
    j = np.arange(1, n + 1)[None, :]
    return 1.0 / (i + j - 1)


def grid_stencil(side: int = 29, shift: float = 0.5, spread: float = 0.1,
                 seed: int = 1006) -> np.ndarray:
    rng = np.random.default_rng(seed)
    n = side * side
    A = np.zeros((n, n))
    for r in range(side):
        for c in range(side):
            i = r * side + c
            A[i, i] = 4.0 + shift
            for dr, dc in ((-1, 0), (1, 0), (0, -1), (0, 1)):
                rr, cc = r + dr, c + dc
                if 0 <= rr < side and 0 <= cc < side:
                    A[i, rr * side + cc] = -1.0 + spread * rng.uniform(-1.0, 1.0)
    return A


def spd(n: int, cond: float = 10.0, seed: int = 1007) -> np.ndarray:
    rng = np.random.default_rng(seed)
    Q = haar_columns(rng, n, n)
    w = np.logspace(0.0, np.log10(cond), n)
    S = (Q * w) @ Q.T
    return (S + S.T) / 2


@dataclass
class Request:
    arrival_s: float
    A: np.ndarray
    rank_deficient: bool


def request_shape(rng: np.random.Generator, m_lo: int = 64, m_hi: int = 2048):
    m = int(round(np.exp(rng.uniform(np.log(m_lo), np.log(m_hi))) / 4.0)) * 4
    m = max(m_lo, min(m_hi, m))
    r = int(rng.choice([1, 2, 4]))
    n = max(1, m // r)
    return m, n


def request_matrix(rng: np.random.Generator, m: int, n: int, deficient: bool) -> np.ndarray:
    if not deficient:
        return rng.standard_normal((m, n))
    k = max(1, min(m, n) // 2)
    G1 = rng.standard_normal((m, k))
    G2 = rng.standard_normal((k, n))
    return (G1 @ G2) / np.sqrt(k)


def request_stream(count: int, qps: float, seed: int = 1005, m_lo: int = 64,
                   m_hi: int = 2048, deficient_frac: float = 0.1) -> list[Request]:
    """Poisson arrival trace: exponential inter-arrival gaps of mean 1/qps."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for _ in range(count):
        t += rng.exponential(1.0 / qps) if qps > 0 else 0.0
        m, n = request_shape(rng, m_lo, m_hi)
        deficient = bool(rng.uniform() < deficient_frac)
        out.append(Request(t, request_matrix(rng, m, n, deficient), deficient))
    return out
