"""Seeded synthetic inputs for the linear-response eigenproblem H = [[0, K], [M, 0]].

This module is shared by the CPU oracle (``oracle/``), the tests and the
benchmark.  It holds only input construction -- random draws, orthogonal
factors, the structured test matrices of the paper's numerical section --
and none of the eigensolver's arithmetic.

Every generator takes an explicit seed and draws from
``numpy.random.default_rng(seed)`` (PCG64) in a fixed, documented order, so
the same seed gives the same bytes on every machine up to the rounding of
the LAPACK QR used for the Haar factors.

Workloads (sizes and distributions follow the benchmark configurations):

* dense:   K = Q1 diag(k) Q1^T, M = Q2 diag(m) Q2^T, Q1/Q2 Haar-orthogonal,
           k, m ~ U[0.5, 10]; optional exact zeros in m (generalized nullspace
           on M, which the solver handles by exchanging the roles of K and M).
           Draw order: Q1 (Gaussian n*n), Q2 (Gaussian n*n), k (n), m (n).
* casida:  K = diag(delta), M = diag(delta) + 2 L L^T with delta ~ U[0.1, 20]
           sorted ascending and L ~ N(0,1)/sqrt(n) of shape n x rank
           (a diagonal-plus-low-rank stand-in for the TDDFT/Casida matrices
           of the paper's efficiency section, which are not available here).
           Draw order: delta (n), L (n*rank, column-major order of draws).
* T(s):    the tridiagonal (2, -1) matrix with corner entries s used by the
           paper's accuracy examples (Section 4.1).
* Hilbert / Lauchli: the ill-conditioned pair of the biorthogonalisation
           experiment (Section 3.1, table of biorthogonality loss).
* init:    the random starting block (U, V) of Step 1 of the BOSP algorithm,
           standard normal, U drawn before V.
* metric:  the diagonal b of an SPD metric B = diag(b) for the generalized
           LREP K x = lambda B y, M y = lambda B x: log-uniform on [lo, hi]
           (default [0.25, 4]), a stand-in for a lumped finite-element mass
           matrix (the paper's Example 4.5 uses a P3 mass matrix, not
           available here).  One draw of n uniforms.  A dense SPD metric:
           B = Q diag(beta) Q^T, Q Haar, beta log-uniform on [lo, hi]
           (default [0.25, 4]); draws: Q (Gaussian n*n), beta (n).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "haar",
    "dense_factors",
    "dense_operator",
    "casida_factors",
    "tridiag_T",
    "hilbert",
    "lauchli",
    "init_block",
    "DenseFactors",
    "CasidaFactors",
    "dense_operator_device",
    "metric_diag",
    "metric_dense",
    "dense_factors_torch",
]


def haar(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed orthogonal n x n matrix.

    QR of a standard Gaussian matrix with the signs of R's diagonal moved
    into Q (Mezzadri, "How to generate random matrices from the classical
    compact groups", Notices AMS 2007), which makes the distribution exactly
    Haar.
    """
    g = rng.standard_normal((n, n))
    q, r = np.linalg.qr(g)
    d = np.sign(np.diagonal(r)).copy()
    d[d == 0] = 1.0
    q *= d[None, :]
    return q


class DenseFactors:
    """Spectral factors of the dense workload: K = Q1 diag(k) Q1^T, M = Q2 diag(m) Q2^T."""

    def __init__(self, q1, k, q2, m):
        self.q1, self.k, self.q2, self.m = q1, k, q2, m

    @property
    def n(self) -> int:
        return self.k.shape[0]

    def K(self) -> np.ndarray:
        a = (self.q1 * self.k[None, :]) @ self.q1.T
        return 0.5 * (a + a.T)

    def M(self) -> np.ndarray:
        a = (self.q2 * self.m[None, :]) @ self.q2.T
        return 0.5 * (a + a.T)

    def null_basis_M(self) -> np.ndarray:
        """Columns of Q2 whose m is exactly zero (a basis of N(M))."""
        return self.q2[:, self.m == 0.0].copy()

    def norm_H(self) -> float:
        """||H||_2 = max(||K||_2, ||M||_2), known exactly from the factors."""
        return float(max(self.k.max(), self.m.max()))


def dense_factors(n: int, seed: int, n_zero_m: int = 0,
                  lo: float = 0.5, hi: float = 10.0) -> DenseFactors:
    """Draw the dense workload's factors.  ``n_zero_m`` sets m[0:n_zero_m] = 0
    after drawing (the zero-eigenvalue variant)."""
    rng = np.random.default_rng(seed)
    q1 = haar(n, rng)
    q2 = haar(n, rng)
    k = rng.uniform(lo, hi, n)
    m = rng.uniform(lo, hi, n)
    if n_zero_m:
        m[:n_zero_m] = 0.0
    return DenseFactors(q1, k, q2, m)


def dense_operator(n: int, seed: int, n_zero_m: int = 0):
    """(K, M, factors) for the dense workload, K and M symmetrised."""
    f = dense_factors(n, seed, n_zero_m)
    return f.K(), f.M(), f


class CasidaFactors:
    """K = diag(delta), M = diag(delta) + 2 L L^T."""

    def __init__(self, delta, L):
        self.delta, self.L = delta, L

    @property
    def n(self) -> int:
        return self.delta.shape[0]

    @property
    def rank(self) -> int:
        return self.L.shape[1]

    def K(self) -> np.ndarray:
        return np.diag(self.delta)

    def M(self) -> np.ndarray:
        return np.diag(self.delta) + 2.0 * (self.L @ self.L.T)


def casida_factors(n: int, rank: int, seed: int,
                   lo: float = 0.1, hi: float = 20.0) -> CasidaFactors:
    rng = np.random.default_rng(seed)
    delta = np.sort(rng.uniform(lo, hi, n))
    # draws fill L column by column (Fortran order), matching a column-major buffer
    L = rng.standard_normal(n * rank).reshape((n, rank), order="F") / np.sqrt(n)
    return CasidaFactors(delta, np.asfortranarray(L))


def tridiag_T(n: int, s: float) -> np.ndarray:
    """T(s): 2 on the diagonal, -1 on the first off-diagonals, s in the two corners."""
    t = 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    t[0, n - 1] += s
    t[n - 1, 0] += s
    return t


def hilbert(n: int) -> np.ndarray:
    i = np.arange(1, n + 1, dtype=np.float64)
    return 1.0 / (i[:, None] + i[None, :] - 1.0)


def lauchli(n: int, mu: float) -> np.ndarray:
    """The n x (n-1) Lauchli matrix: a row of ones over mu * I_{n-1} (Higham's test matrix)."""
    a = np.zeros((n, n - 1))
    a[0, :] = 1.0
    a[1:, :] = mu * np.eye(n - 1)
    return a


def init_block(n: int, d: int, seed: int):
    """Random starting block (U, V) of Step 1: independent standard normal, U first."""
    rng = np.random.default_rng(seed)
    U = np.asfortranarray(rng.standard_normal((d, n)).T)
    V = np.asfortranarray(rng.standard_normal((d, n)).T)
    return U, V


def dense_factors_torch(n: int, seed: int, device, n_zero_m: int = 0, lo: float = 0.5, hi: float = 10.0):
    """The dense workload's factors (Q1, k, Q2, m) with the QR factorisations
    done by torch on ``device`` (a GPU, or "cpu"): the same NumPy draws in the
    same order as ``dense_factors``, so Q1, Q2 agree with it up to rounding."""
    import torch
    rng = np.random.default_rng(seed)
    qs = []
    for _ in range(2):
        g = torch.from_numpy(rng.standard_normal((n, n))).to(device)
        q, r = torch.linalg.qr(g)
        d = torch.sign(torch.diagonal(r))
        d[d == 0] = 1.0
        qs.append(q * d[None, :])
        del g, r
    k = rng.uniform(lo, hi, n)
    m = rng.uniform(lo, hi, n)
    if n_zero_m:
        m[:n_zero_m] = 0.0
    return qs[0], k, qs[1], m


def dense_operator_device(n: int, seed: int, device, n_zero_m: int = 0,
                          lo: float = 0.5, hi: float = 10.0, return_factors: bool = False):
    """The dense workload built on a torch device: the same NumPy draws in the
    same order as ``dense_factors`` (Gaussian for Q1, Gaussian for Q2, k, m),
    with the QR factorisations and the products K = Q1 diag(k) Q1^T,
    M = Q2 diag(m) Q2^T done by torch on ``device`` (for large n, where the
    host QR takes tens of seconds).  Returns (K, M, k, m) with K, M symmetric
    FP64 device tensors and k, m NumPy vectors; with ``return_factors`` also
    the device tensors Q1, Q2."""
    import torch
    qs = [None, None]
    qs[0], k, qs[1], m = dense_factors_torch(n, seed, device, n_zero_m, lo, hi)
    out = []
    for q, v in ((qs[0], k), (qs[1], m)):
        a = (q * torch.from_numpy(v).to(device)[None, :]) @ q.T
        out.append(0.5 * (a + a.T))
    if return_factors:
        return out[0], out[1], k, m, qs[0], qs[1]
    return out[0], out[1], k, m


def metric_diag(n: int, seed: int, lo: float = 0.25, hi: float = 4.0) -> np.ndarray:
    """Diagonal of the SPD metric B: exp(U[log lo, log hi]) per entry."""
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(np.log(lo), np.log(hi), n))


def metric_dense(n: int, seed: int, lo: float = 0.25, hi: float = 4.0) -> np.ndarray:
    """Dense SPD metric B = Q diag(beta) Q^T (symmetrised), Q Haar."""
    rng = np.random.default_rng(seed)
    Q = haar(n, rng)
    beta = np.exp(rng.uniform(np.log(lo), np.log(hi), n))
    B = (Q * beta[None, :]) @ Q.T
    return np.asfortranarray(0.5 * (B + B.T))
