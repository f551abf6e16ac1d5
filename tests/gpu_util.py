"""Helpers shared by the GPU tests (device tensors in column-major layout)."""
import numpy as np


def dev_colmajor(a, torch, device="cuda:0"):
    """Column-major FP64 device copy of a 2-D numpy array (or 1-D vector)."""
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        return torch.from_numpy(a.copy()).to(device)
    return torch.from_numpy(np.ascontiguousarray(a.T)).to(device).T


def dev_empty(n, k, torch, device="cuda:0"):
    return torch.zeros(k, n, dtype=torch.float64, device=device).T


def host(t):
    return t.detach().cpu().numpy()


def h_residual(K_apply, M_apply, X, Y, lam, normH):
    R1 = K_apply(X) - Y * lam
    R2 = M_apply(Y) - X * lam
    return np.sqrt((R1 ** 2).sum(0) + (R2 ** 2).sum(0)) / (normH * np.sqrt((X ** 2).sum(0) + (Y ** 2).sum(0)))
