"""Generalized LREP with an SPD metric B (the remark on the generalized LREP
in Section 3.2; the finite-element problem of Example 4.5), plain FP64.

TEST INFRASTRUCTURE ONLY -- part of the CPU oracle.

The problem is

    [[0, K], [M, 0]] [y; x] = lambda [[B, 0], [0, B]] [y; x],

i.e. K x = lambda B y and M y = lambda B x, with K, M symmetric positive
semidefinite and B symmetric positive definite.  The eigenpairs are unique
(up to sign, for simple eigenvalues), so the oracle is their definition:

  * with B = C C^T (Cholesky), the substitution x^ = C^T x, y^ = C^T y turns
    the pencil into the standard LREP of K^ = C^-1 K C^-T, M^ = C^-1 M C^-T;
  * the positive eigenvalues of a standard LREP are the singular values of
    F1^T F2 for any factors K^ = F1 F1^T, M^ = F2 F2^T (Lemma 2.1 gives
    det(lambda I - H) = det(lambda^2 I - K^ M^)); symmetric square-root
    factors from an eigendecomposition also cover singular K or M.

A pair returned by a solver is measured by its own residuals K x - lambda B y,
M y - lambda B x and by the B-biorthogonality Y^T B X = I (the B inner
product <u, v>_B = u^T B v that MGS-Biorth uses in the remark).
"""
from __future__ import annotations

import numpy as np


def _psd_factor(A: np.ndarray) -> np.ndarray:
    """F with F F^T = A for symmetric positive semidefinite A (eigenvalues
    below zero from rounding are clipped)."""
    w, V = np.linalg.eigh(0.5 * (A + A.T))
    return V * np.sqrt(np.maximum(w, 0.0))[None, :]


def reduce_to_standard(K: np.ndarray, M: np.ndarray, B: np.ndarray):
    """(K^, M^, C) with K^ = C^-1 K C^-T, M^ = C^-1 M C^-T, C C^T = B."""
    C = np.linalg.cholesky(B)
    Ci = np.linalg.inv(C)
    Kh = Ci @ K @ Ci.T
    Mh = Ci @ M @ Ci.T
    return 0.5 * (Kh + Kh.T), 0.5 * (Mh + Mh.T), C


def generalized_spectrum(K: np.ndarray, M: np.ndarray, B: np.ndarray, count=None, zeros: int = 0):
    """Positive eigenvalues of the generalized LREP, ascending.  ``zeros`` is
    the number of exact zero eigenvalues of K^ M^ (the dimension of the
    null space the solver is told about); they are left out."""
    Kh, Mh, _ = reduce_to_standard(K, M, B)
    F1, F2 = _psd_factor(Kh), _psd_factor(Mh)
    s = np.sort(np.linalg.svd(F1.T @ F2, compute_uv=False))
    s = s[zeros:]
    return s if count is None else s[:count]


def generalized_residual(K, M, B, X, Y, lam, normH=None, normB=None):
    """Per pair: sqrt(||K x - lambda B y||^2 + ||M y - lambda B x||^2) over
    ((||H||_2 + lambda ||B||_2) sqrt(||x||^2 + ||y||^2)), a normwise backward
    error of the pencil.  ||H||_2 = max(||K||_2, ||M||_2)."""
    if normH is None:
        normH = max(np.linalg.norm(K, 2), np.linalg.norm(M, 2))
    if normB is None:
        normB = np.linalg.norm(B, 2)
    R1 = K @ X - (B @ Y) * lam[None, :]
    R2 = M @ Y - (B @ X) * lam[None, :]
    num = np.sqrt(np.sum(R1 * R1, axis=0) + np.sum(R2 * R2, axis=0))
    den = (normH + lam * normB) * np.sqrt(np.sum(X * X, axis=0) + np.sum(Y * Y, axis=0))
    return num / den


def b_biorth_error(B, X, Y) -> float:
    """max |Y^T B X - I|."""
    return float(np.abs(Y.T @ (B @ X) - np.eye(X.shape[1])).max())


def dense_metric_spectrum_smallest(q1, k, q2, m, b, count, zeros: int = 0):
    """The ``count`` smallest positive eigenvalues for the dense workload
    K = Q1 diag(k) Q1^T, M = Q2 diag(m) Q2^T with the diagonal metric
    B = diag(b), for large n.  With S = B^-1/2 the scaled pencil has factors
    F1 = S Q1 diag(sqrt k), F2 = S Q2 diag(sqrt m), so the eigenvalues are the
    singular values of F = diag(sqrt k) Q1^T B^-1 Q2 diag(sqrt m); their
    squares are taken from F^T F with a symmetric eigensolver restricted to
    the index range (``zeros`` exact zeros of m are skipped)."""
    import scipy.linalg as sla
    F = (np.sqrt(k)[:, None] * (q1.T @ (q2 / b[:, None]))) * np.sqrt(m)[None, :]
    w = sla.eigh(F.T @ F, eigvals_only=True, subset_by_index=[zeros, zeros + count - 1], driver="evr")
    return np.sqrt(np.maximum(w, 0.0))
