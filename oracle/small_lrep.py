"""Small structured LREP of the Rayleigh-Ritz step, plain FP64.

TEST INFRASTRUCTURE ONLY -- part of the CPU oracle.

The projected matrix (Section 3.2, equation for H-hat) is
    H^ = [[0, K^], [M^, 0]],  K^ = U^T K U,  M^ = V^T M V,  both SPD,
and its smallest positive eigenpairs  K^ X^ = Y^ Lambda,  M^ Y^ = X^ Lambda,
X^^T Y^ = I are computed by the structure-preserving route the paper adopts
(two Cholesky factorisations and one SVD, Section 3.2 and the cost
discussion of Section 3.3):

    K^ = L1 L1^T,  M^ = L2 L2^T,  L1^T L2 = Phi Sigma Psi^T
    Lambda = Sigma (ascending),  Y^ = L1 Phi Sigma^{-1/2},  X^ = L2 Psi Sigma^{-1/2}.

Check:  K^ X^ = L1 (L1^T L2 Psi) Sigma^{-1/2} = L1 Phi Sigma^{1/2} = Y^ Sigma,
        M^ Y^ = L2 (L2^T L1 Phi) Sigma^{-1/2} = L2 Psi Sigma^{1/2} = X^ Sigma,
        X^^T Y^ = Sigma^{-1/2} Psi^T (L2^T L1) Phi Sigma^{-1/2} = I.
"""
from __future__ import annotations

import numpy as np


class NotSPDError(ArithmeticError):
    """A projected matrix failed its Cholesky factorisation."""


def small_lrep(Khat: np.ndarray, Mhat: np.ndarray, nwant: int):
    """Smallest ``nwant`` positive eigenpairs of [[0, Khat], [Mhat, 0]].

    Returns (lam (nwant,), Xh (d x nwant), Yh (d x nwant)).
    """
    Khat = 0.5 * (Khat + Khat.T)
    Mhat = 0.5 * (Mhat + Mhat.T)
    try:
        L1 = np.linalg.cholesky(Khat)
        L2 = np.linalg.cholesky(Mhat)
    except np.linalg.LinAlgError as e:
        raise NotSPDError(str(e)) from e
    Phi, sig, PsiT = np.linalg.svd(L1.T @ L2)
    order = np.argsort(sig)[:nwant]          # ascending
    sig = sig[order]
    Phi = Phi[:, order]
    Psi = PsiT.T[:, order]
    isq = 1.0 / np.sqrt(sig)
    Yh = (L1 @ Phi) * isq[None, :]
    Xh = (L2 @ Psi) * isq[None, :]
    return sig, Xh, Yh


def small_lrep_bruteforce(Khat: np.ndarray, Mhat: np.ndarray, nwant: int):
    """Eigenvalues of the full 2d x 2d H^ by a general eigensolver: the
    smallest ``nwant`` positive ones, ascending (used only to check
    ``small_lrep``)."""
    d = Khat.shape[0]
    H = np.zeros((2 * d, 2 * d))
    H[:d, d:] = Khat
    H[d:, :d] = Mhat
    ev = np.linalg.eigvals(H).real
    ev = np.sort(ev[ev > 0])
    return ev[:nwant]
