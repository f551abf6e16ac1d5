"""Exact spectra of the synthetic workloads, plain FP64 (pins for the oracle).

TEST INFRASTRUCTURE ONLY -- part of the CPU oracle.

* Factored form.  If K = F1 F1^T and M = F2 F2^T then the nonzero
  eigenvalues of K M are the squared singular values of F1^T F2, so the
  positive eigenvalues of H = [[0, K], [M, 0]] are sigma(F1^T F2)
  (Lemma 2.1: det(lambda I - H) = det(lambda^2 I - K M)).  For the dense
  workload F1 = Q1 diag(sqrt k), F2 = Q2 diag(sqrt m); for Example 4.2
  F1 = D^T (D the periodic first-difference matrix, D^T D = T(-1)) and
  F2 = chol(T(0)).
* Example 4.1 (K = M = T(0)): lambda_l = 4 sin^2(pi l / (2 (n + 1))).
* Casida workload: lambda^2 are the eigenvalues of S = D^2 + W W^T with
  D = diag(delta), W = sqrt(2) D^(1/2) L.  The number of eigenvalues of H
  below sqrt(mu) follows from Haynsworth inertia additivity applied to the
  bordered matrix [[D^2 - mu I, W], [W^T, -I]]:
      #{lambda^2 < mu} = #{delta^2 < mu} - #neg eig(I + W^T (D^2 - mu I)^-1 W).
"""
from __future__ import annotations

import numpy as np


def dense_spectrum(q1, k, q2, m, count=None):
    """Positive eigenvalues of H for K = Q1 diag(k) Q1^T, M = Q2 diag(m) Q2^T,
    ascending; exact zeros (from zero k or m) are excluded."""
    F = (np.sqrt(k)[:, None] * (q1.T @ q2)) * np.sqrt(m)[None, :]
    s = np.linalg.svd(F, compute_uv=False)
    nz = int(min(np.count_nonzero(k), np.count_nonzero(m)))
    s = np.sort(s)[::-1][:nz][::-1]
    return s if count is None else s[:count]


def dense_spectrum_smallest(q1, k, q2, m, count):
    """The ``count`` smallest positive eigenvalues of H for the dense workload
    (same definition as ``dense_spectrum``), for large n: they are the square
    roots of the smallest eigenvalues of F^T F, F = diag(sqrt k) Q1^T Q2
    diag(sqrt m), taken with a symmetric eigensolver restricted to that index
    range.  Forming F^T F squares the condition number: the absolute error of
    sigma^2 is about eps ||F||^2, i.e. a relative error in sigma of about
    eps max(k) max(m) / (2 sigma^2), below 1e-13 for k, m in [0.5, 10] and
    sigma >= 0.5.  Exact zeros of k or m are excluded as in dense_spectrum."""
    import scipy.linalg as sla
    F = (np.sqrt(k)[:, None] * (q1.T @ q2)) * np.sqrt(m)[None, :]
    nzero = int(q1.shape[0] - min(np.count_nonzero(k), np.count_nonzero(m)))
    w = sla.eigh(F.T @ F, eigvals_only=True, subset_by_index=[nzero, nzero + count - 1], driver="evr")
    return np.sqrt(np.maximum(w, 0.0))


def periodic_difference(n):
    """D with (D x)_i = x_i - x_{i-1} (indices mod n); D^T D = T(-1)."""
    D = np.eye(n)
    D[np.arange(n), np.arange(n) - 1] -= 1.0
    return D


def example_4_2_spectrum(n, count):
    """Smallest positive eigenvalues for K = T(-1), M = T(0)."""
    T0 = 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    L2 = np.linalg.cholesky(T0)
    s = np.linalg.svd(periodic_difference(n) @ L2, compute_uv=False)
    s = np.sort(s)
    s = s[s > 1e-8 * s[-1]]                 # the one zero singular value (N(K) = span 1)
    return s[:count]


def example_4_1_spectrum(n, count):
    l = np.arange(1, count + 1, dtype=np.float64)
    return 4.0 * np.sin(np.pi * l / (2.0 * (n + 1))) ** 2


def casida_count_below(delta, L, lam):
    """Number of positive eigenvalues of H strictly below ``lam`` for
    K = diag(delta), M = diag(delta) + 2 L L^T (Haynsworth inertia count)."""
    mu = lam * lam
    d2 = delta * delta - mu
    W = np.sqrt(2.0 * delta)[:, None] * L
    S = np.eye(L.shape[1]) + W.T @ (W / d2[:, None])
    ev = np.linalg.eigvalsh(0.5 * (S + S.T))
    return int(np.count_nonzero(d2 < 0) - np.count_nonzero(ev < 0))


def casida_count_below_many(delta, L, lams, chunk=16384):
    """casida_count_below for every value in ``lams`` (the same Haynsworth
    count, with W formed once and the sum W^T (D^2 - mu I)^-1 W taken over
    row chunks); returns a list of counts in the order of ``lams``."""
    W = np.sqrt(2.0 * delta)[:, None] * L
    d2all = delta * delta
    r = L.shape[1]
    out = []
    for lam in lams:
        mu = float(lam) * float(lam)
        S = np.eye(r)
        for s in range(0, W.shape[0], chunk):
            Wc = W[s:s + chunk]
            S += Wc.T @ (Wc / (d2all[s:s + chunk] - mu)[:, None])
        ev = np.linalg.eigvalsh(0.5 * (S + S.T))
        out.append(int(np.count_nonzero(d2all - mu < 0) - np.count_nonzero(ev < 0)))
    return out


def dense_spectrum_smallest_torch(q1, k, q2, m, count):
    """dense_spectrum_smallest with plain PyTorch CPU FP64 operations (for
    n in the tens of thousands, where the host LAPACK eigensolver of NumPy /
    SciPy is slow): the square roots of the smallest eigenvalues of F^T F,
    F = diag(sqrt k) Q1^T Q2 diag(sqrt m), exact zeros of k or m excluded.
    q1, q2 are CPU tensors or arrays; the products are formed in place to
    keep three n x n arrays alive at most."""
    import torch
    q1 = torch.as_tensor(q1, dtype=torch.float64)
    q2 = torch.as_tensor(q2, dtype=torch.float64)
    n = q1.shape[0]
    F = q1.T @ q2
    F *= torch.sqrt(torch.as_tensor(k, dtype=torch.float64))[:, None]
    F *= torch.sqrt(torch.as_tensor(m, dtype=torch.float64))[None, :]
    G = F.T @ F
    del F
    G = 0.5 * (G + G.T)
    w = torch.linalg.eigvalsh(G)
    nzero = int(n - min(int(np.count_nonzero(k)), int(np.count_nonzero(m))))
    w = w[nzero:nzero + count].numpy()
    return np.sqrt(np.maximum(w, 0.0))
