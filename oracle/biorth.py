"""Biorthogonalisation, plain FP64 (Section 3.1 of the paper).

TEST INFRASTRUCTURE ONLY -- this module is part of the CPU oracle.  Only the
tests, the smoke check and the benchmark's CPU-baseline leg may import it.

``mgs_biorth`` is the modified Gram-Schmidt biorthogonalisation (the paper's
Algorithm "Modified Gram-Schmidt biorthogonalization"): column by column,
the new pair (x_l, y_l) is stripped of its components along every previous
pair -- the coefficient for the x side is taken against the previous q_j
*after* the earlier subtractions have been applied (Gauss-Seidel form), the
y side likewise against p_j -- and the pair is then scaled by
r_ll = sign(eta) sqrt|eta| and s_ll = sqrt|eta|, eta = p_l^T q_l, so that
p_l^T q_l = 1.

``cgs_biorth`` is the classical variant (Gauss-Jacobi form: every coefficient
is taken against the *original* x, y), kept only to reproduce the paper's
comparison of biorthogonality loss.

Breakdown handling (remark on ill-conditioned inputs in Section 3.1): a pair
whose pivot is numerically zero is discarded and the procedure continues, so
fewer than m columns may come out.  The paper does not fix the threshold;
the reading used here is scale invariant:

  drop l  if  |eta| <= cos_tol * ||p~_l|| * ||q~_l||          (near-orthogonal pair)
        or  ||p~_l|| <= dep_tol * ||x_l||  or  ||q~_l|| <= dep_tol * ||y_l||
                                                              (numerically dependent)
With cos_tol = dep_tol = 0 only an exactly zero pivot is dropped.
"""
from __future__ import annotations

import numpy as np


def mgs_biorth(X: np.ndarray, Y: np.ndarray, cos_tol: float = 0.0,
               dep_tol: float = 0.0):
    """MGS-Biorth of (X, Y), both n x m.

    Returns (P, Q, kept) with P^T Q = I (up to rounding) and ``kept`` the
    indices of the input columns that survived the breakdown test.
    """
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    n, m = X.shape
    P_cols, Q_cols, kept = [], [], []
    for l in range(m):
        p = X[:, l].copy()
        q = Y[:, l].copy()
        for j in range(len(P_cols)):
            r_jl = Q_cols[j] @ p          # against the updated p (Gauss-Seidel)
            p -= r_jl * P_cols[j]
            s_jl = P_cols[j] @ q
            q -= s_jl * Q_cols[j]
        eta = p @ q
        np_, nq = np.linalg.norm(p), np.linalg.norm(q)
        if (eta == 0.0
                or abs(eta) <= cos_tol * np_ * nq
                or np_ <= dep_tol * np.linalg.norm(X[:, l])
                or nq <= dep_tol * np.linalg.norm(Y[:, l])):
            continue
        r_ll = np.sign(eta) * np.sqrt(abs(eta))
        s_ll = np.sqrt(abs(eta))
        P_cols.append(p / r_ll)
        Q_cols.append(q / s_ll)
        kept.append(l)
    if P_cols:
        P = np.stack(P_cols, axis=1)
        Q = np.stack(Q_cols, axis=1)
    else:
        P = np.zeros((n, 0))
        Q = np.zeros((n, 0))
    return P, Q, kept


def cgs_biorth(X: np.ndarray, Y: np.ndarray):
    """Classical Gram-Schmidt biorthogonalisation: coefficients against the
    original columns x_l, y_l (Gauss-Jacobi form).  No breakdown handling."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    n, m = X.shape
    P = np.zeros((n, m))
    Q = np.zeros((n, m))
    for l in range(m):
        x, y = X[:, l], Y[:, l]
        p, q = x.copy(), y.copy()
        for j in range(l):
            p -= P[:, j] * (Q[:, j] @ x)
            q -= Q[:, j] * (P[:, j] @ y)
        eta = p @ q
        P[:, l] = p / (np.sign(eta) * np.sqrt(abs(eta)))
        Q[:, l] = q / np.sqrt(abs(eta))
    return P, Q
