"""Null space of the semidefinite operator (the remark on computing the
generalized null space, Section 2.2, and Lemma 2.3), plain FP64.

TEST INFRASTRUCTURE ONLY -- part of the CPU oracle.

The basis X0~ of N(K) that the generalized null space V0 is built from is
defined as the eigenvectors of the symmetric K for the eigenvalue zero.  The
oracle takes them from a full symmetric eigendecomposition: eigenvalues at
most ``rtol * max |eigenvalue|`` count as zero.  Solvers are compared with it
through the principal angles between the two subspaces.
"""
from __future__ import annotations

import numpy as np


def null_basis(K: np.ndarray, rtol: float = 1e-10) -> np.ndarray:
    """Orthonormal basis (n x r) of N(K) for symmetric K."""
    w, V = np.linalg.eigh(0.5 * (K + K.T))
    scale = max(float(np.abs(w).max()), np.finfo(float).tiny)
    return V[:, np.abs(w) <= rtol * scale]


def subspace_distance(A: np.ndarray, B: np.ndarray) -> float:
    """sin of the largest principal angle between span(A) and span(B)
    (1.0 when the dimensions differ)."""
    if A.shape[1] != B.shape[1]:
        return 1.0
    if A.shape[1] == 0:
        return 0.0
    Qa, _ = np.linalg.qr(A)
    Qb, _ = np.linalg.qr(B)
    # ||(I - Qa Qa^T) Qb||_2 = sin(theta_max)
    return float(np.linalg.norm(Qb - Qa @ (Qa.T @ Qb), 2))
