"""BOSP subspace eigensolver for the LREP, plain FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY -- the oracle the GPU library is checked against.
Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import it; it never imports the library and the library never imports it.

Problem (Section 1, change of variables u = y + x, v = y - x):
    H [y; x] = lambda [y; x],  H = [[0, K], [M, 0]],  K = A - B, M = A + B,
i.e. K x = lambda y and M y = lambda x, with K symmetric positive
semi-definite and M symmetric positive definite.  The nev smallest positive
eigenvalues are returned with X^T Y = I (Algorithm "BOSP algorithm").

Steps, in the paper's order and notation (Section 3.2 / 3.3):

  V0      If dim N(K) = r > 0 the caller supplies a basis X0~ of N(K); the
          oracle solves M Y0~ = X0~ exactly, factors X0~^T Y0~ = C^T C and
          takes X0 = X0~ C^-1, Y0 = Y0~ C^-1 (proof of the direct-sum
          theorem, equation for the V0 basis), so X0^T Y0 = I.
  Step 1  U = [X, P, W], V = [Y, Q, Z] random with d = b + 2w columns.
  Step 2  U <- (I - X0 Y0^T) U, V <- (I - Y0 X0^T) V, then MGS-Biorth.
  Step 3  K^ = U^T K U, M^ = V^T M V, small structured LREP (two Cholesky
          factorisations and one SVD), pull back X~ = U X^, Y~ = V Y^.
  Step 4  eps_i = ||H xi_i - lambda_i xi_i|| / ((1 + lambda_i) ||xi_i||),
          xi_i = [y~_i; x~_i] (stopping rule of Section 4).
  Step 5  P^ = (I - X^ Y^^T)(X^_a - E_a), Q^ = (I - Y^ X^^T)(Y^_a - E_a),
          small MGS-Biorth, P~ = U P^, Q~ = V Q^.
  Step 6  ngs block Gauss-Seidel sweeps, W(0) = 0:
              M Z(j) = W(j-1) Lambda + (X~ Lambda - M Y~)
              K W(j) = Z(j) Lambda + (Y~ Lambda - K X~)
          each by CG (zero start, relative tolerance 1e-2, at most 20
          iterations); then W~ = (I - [X0, X~, P~][Y0, Y~, Q~]^T) W,
          Z~ = (I - [Y0, Y~, Q~][X0, X~, P~]^T) Z and MGS-Biorth of (W~, Z~).
  Step 7  U = [X~, P~, W~], V = [Y~, Q~, Z~].

Batching and moving (Section 3.3): only the first w ("n_b") unconverged
Ritz pairs -- the window a -- feed Steps 5-6.  The X block keeps b columns
(b = s * n_b under moving).  Readings of the parts the paper leaves open
(its illustration of the moving mechanism is not available):

  * converged pairs are locked from the front: when the leading 2w (or b,
    if b < 2w) Ritz pairs of the active block have converged they are moved
    to the locked set [X_c, Y_c], and the next b Ritz pairs of the *same*
    projected problem -- which come from the span of P and W -- become the
    active X block ("P, W are integrated into X").  The subspace dimension
    therefore stays d = b + 2w, independent of nev.
  * locked pairs join the converged block of the projection in Step 6:
    W is made biorthogonal to [X0, X_c, X~, P~] (Section 3.3: later pairs
    are computed in the biorthogonal complement of the converged ones).
  * E in Step 5 is [I_b; 0] restricted to the window's Ritz indices; the
    projector uses every Ritz pair kept this iteration (locked or active).
  * ngs = 1 by default (the paper does not fix it).
  * CG stops a column when ||r|| <= cg_tol ||rhs||, after cg_maxit
    iterations, or when p^T A p <= 0 (singular K: the projection that
    follows removes any N(K) component).
  * MGS-Biorth drops a pair by the scale-invariant rule documented in
    ``oracle.biorth``.
  * if the null space sits on M instead of K, K and M exchange roles and X,
    Y are exchanged back at the end: K x = lambda y, M y = lambda x is the
    same problem as M x' = lambda y', K y' = lambda x' with x' = y, y' = x.
  * each returned pair is sign-normalised: the entry of x of largest
    magnitude is made positive (y flips with it).
  * Step 1 draws one standard-normal block and uses it for both U and V
    (the algorithm draws the columns at random and needs U^T V invertible;
    V = U makes U^T V = U^T U SPD, so no restore of U^T V = I is needed at
    the start; independent U and V, passed through ``init``, reach the same
    pairs after a few restores by the biorthogonality monitor).
  * the projectors of Steps 5 and 6 are applied twice.  Both act on vectors
    that largely cancel near convergence (X^_a ~ E_a; W mostly along X~), so
    one application leaves them biorthogonal only to eps / (relative size
    of what survives); the second application, idempotent in exact
    arithmetic, restores biorthogonality to rounding level.
  * a window column whose Step-5 difference the projector annihilates
    (relative size below MGS_DEP_TOL) gives no P direction -- this happens
    when the kept Ritz vectors span the whole subspace, right after a lock.
  * when fewer than w pairs of the X block are unconverged, the window is
    continued into the next Ritz pairs of the projected problem, so every
    iteration keeps w correction directions (otherwise the last pairs of a
    batch converge only at the rate set by the gap to the first pair
    outside the block).
  * biorthogonality monitor: at the top of every iteration, if
    max |U^T V - I| > REBIORTH_TOL the whole basis is re-biorthogonalised
    with MGS-Biorth.  The small problem's X^^T Y^ = I holds only to about
    eps ||H^|| / lambda_min, which for tiny eigenvalues (Example 4.1: 1e-5
    against ||H|| = 4) compounds from one iteration to the next.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Optional

import numpy as np
import scipy.linalg as sla

from .biorth import mgs_biorth
from .small_lrep import small_lrep

Apply = Callable[[np.ndarray], np.ndarray]

# breakdown-test thresholds of MGS-Biorth inside the solver (see oracle.biorth)
MGS_COS_TOL = 1e-10
MGS_DEP_TOL = 1e-13
# re-biorthogonalise U, V when max |U^T V - I| exceeds this
REBIORTH_TOL = 1e-12


# --------------------------------------------------------------------------
# operators
# --------------------------------------------------------------------------
class DenseOperator:
    """Explicit symmetric K, M (n x n)."""

    def __init__(self, K: np.ndarray, M: np.ndarray):
        self.K = np.asarray(K, dtype=np.float64)
        self.M = np.asarray(M, dtype=np.float64)
        self.n = self.K.shape[0]
        self._cho = {}

    def apply_K(self, X):
        return self.K @ X

    def apply_M(self, X):
        return self.M @ X

    def _solve(self, which, B):
        if which not in self._cho:
            A = self.K if which == "K" else self.M
            self._cho[which] = sla.cho_factor(A, lower=True)
        return sla.cho_solve(self._cho[which], B)

    def solve_K(self, B):
        return self._solve("K", B)

    def solve_M(self, B):
        return self._solve("M", B)


class CasidaOperator:
    """K = diag(delta), M = diag(delta) + 2 L L^T (matrix-free)."""

    def __init__(self, delta: np.ndarray, L: np.ndarray):
        self.delta = np.asarray(delta, dtype=np.float64)
        self.L = np.asarray(L, dtype=np.float64)
        self.n = self.delta.shape[0]

    def apply_K(self, X):
        return self.delta[:, None] * X

    def apply_M(self, X):
        return self.delta[:, None] * X + 2.0 * (self.L @ (self.L.T @ X))

    def solve_K(self, B):
        return B / self.delta[:, None]

    def solve_M(self, B):
        # Sherman-Morrison-Woodbury: (D + 2 L L^T)^-1 = D^-1 - D^-1 L (I/2 + L^T D^-1 L)^-1 L^T D^-1
        Dinv_B = B / self.delta[:, None]
        Dinv_L = self.L / self.delta[:, None]
        S = 0.5 * np.eye(self.L.shape[1]) + self.L.T @ Dinv_L
        return Dinv_B - Dinv_L @ np.linalg.solve(S, self.L.T @ Dinv_B)


# --------------------------------------------------------------------------
# pieces of the iteration
# --------------------------------------------------------------------------
def cg_columns(apply: Apply, B: np.ndarray, tol: float, maxit: int):
    """Conjugate gradients, one independent system per column of B, zero
    initial guess; a column stops when ||r|| <= tol ||b||, after ``maxit``
    iterations, or on p^T A p <= 0.  Returns (X, applies) where ``applies``
    counts column mat-vecs."""
    X = np.zeros_like(B)
    R = B.copy()
    P = R.copy()
    rr = np.einsum("ij,ij->j", R, R)
    bb = rr.copy()
    active = rr > (tol * tol) * bb
    applies = 0
    for _ in range(maxit):
        if not active.any():
            break
        cols = np.nonzero(active)[0]
        Q = apply(P[:, cols])
        applies += cols.size
        pq = np.einsum("ij,ij->j", P[:, cols], Q)
        ok = pq > 0.0
        stop = cols[~ok]
        active[stop] = False
        cols, Q, pq = cols[ok], Q[:, ok], pq[ok]
        alpha = rr[cols] / pq
        X[:, cols] += P[:, cols] * alpha
        R[:, cols] -= Q * alpha
        rr_new = np.einsum("ij,ij->j", R[:, cols], R[:, cols])
        beta = rr_new / rr[cols]
        P[:, cols] = R[:, cols] + P[:, cols] * beta
        rr[cols] = rr_new
        active[cols] = rr_new > (tol * tol) * bb[cols]
    return X, applies


def residual_eps(KX, Y, MY, X, lam):
    """Step 4's normalised residual per column (stopping rule, Section 4)."""
    R1 = KX - Y * lam[None, :]
    R2 = MY - X * lam[None, :]
    num = np.sqrt(np.einsum("ij,ij->j", R1, R1) + np.einsum("ij,ij->j", R2, R2))
    den = (1.0 + lam) * np.sqrt(np.einsum("ij,ij->j", X, X) + np.einsum("ij,ij->j", Y, Y))
    return num / den


def sign_normalise(X, Y):
    X = X.copy()
    Y = Y.copy()
    for j in range(X.shape[1]):
        i = np.argmax(np.abs(X[:, j]))
        if X[i, j] < 0:
            X[:, j] = -X[:, j]
            Y[:, j] = -Y[:, j]
    return X, Y


def nullspace_basis(X0t: np.ndarray, solve_M: Apply):
    """Biorthonormal basis of the generalized null space from a basis X0~ of
    N(K): Y0~ = M^-1 X0~, X0~^T Y0~ = C^T C, X0 = X0~ C^-1, Y0 = Y0~ C^-1."""
    Y0t = solve_M(X0t)
    G = X0t.T @ Y0t
    G = 0.5 * (G + G.T)
    C = np.linalg.cholesky(G).T                  # upper, C^T C = G
    X0 = sla.solve_triangular(C, X0t.T, trans="T", lower=False).T
    Y0 = sla.solve_triangular(C, Y0t.T, trans="T", lower=False).T
    return X0, Y0


@dataclasses.dataclass
class BospResult:
    lam: np.ndarray
    X: np.ndarray
    Y: np.ndarray
    converged: bool
    iterations: int
    eps: np.ndarray                  # Step-4 residual of each returned pair
    stats: dict


class NotConvergedError(RuntimeError):
    pass


def bosp_solve(op, nev: int, block: int, tol: float, window: Optional[int] = None,
               X0: Optional[np.ndarray] = None, init=None, seed: int = 0,
               maxit: int = 1000, ngs: int = 1, cg_tol: float = 1e-2,
               cg_maxit: int = 20, null_on_M: bool = False,
               raise_on_maxit: bool = False, history: Optional[list] = None):
    """Run the BOSP iteration.  ``op`` provides apply_K/apply_M/solve_K/solve_M
    and n.  ``X0`` is a basis of the null space of K (or of M when
    ``null_on_M``).  ``init`` = (U, V), n x (block + 2 window), else standard
    normal from ``seed``.  Returns a BospResult."""
    if null_on_M:
        K_apply, M_apply, M_solve = op.apply_M, op.apply_K, op.solve_K
    else:
        K_apply, M_apply, M_solve = op.apply_K, op.apply_M, op.solve_M
    n = op.n
    b = int(block)
    w = int(window) if window else b
    d0 = b + 2 * w
    r0 = 0 if X0 is None else X0.shape[1]
    if not (1 <= nev <= n - r0) or b < 1 or w < 1 or d0 > n - r0:
        raise ValueError("invalid sizes")
    stats = dict(applies_K=0, applies_M=0, mgs_drops=0, locks=0, rebiorth=0)

    # generalized null space V0
    if r0:
        X0, Y0 = nullspace_basis(np.asarray(X0, dtype=np.float64), M_solve)
    else:
        X0 = np.zeros((n, 0))
        Y0 = np.zeros((n, 0))

    # Step 1
    if init is not None:
        U, V = (np.array(a, dtype=np.float64) for a in init)
    else:
        rng = np.random.default_rng(seed)
        U = rng.standard_normal((d0, n)).T.copy()
        V = U.copy()
    # Step 2
    U = U - X0 @ (Y0.T @ U)
    V = V - Y0 @ (X0.T @ V)
    U, V, kept = mgs_biorth(U, V, MGS_COS_TOL, MGS_DEP_TOL)
    stats["mgs_drops"] += d0 - len(kept)

    Xc = np.zeros((n, 0))
    Yc = np.zeros((n, 0))
    lamc = np.zeros(0)
    epsc = np.zeros(0)
    lock_unit = min(2 * w, b)

    for it in range(1, maxit + 1):
        d = U.shape[1]
        c = lamc.size
        need = nev - c
        # biorthogonality monitor: restore U^T V = I when rounding has eroded it
        S = U.T @ V - np.eye(d)
        if np.abs(S).max() > REBIORTH_TOL:
            U, V, kept = mgs_biorth(U, V, MGS_COS_TOL, MGS_DEP_TOL)
            stats["mgs_drops"] += d - len(kept)
            stats["rebiorth"] += 1
            d = U.shape[1]
        # Step 3: projection and small LREP (all d Ritz pairs, ascending)
        KU = K_apply(U)
        MV = M_apply(V)
        stats["applies_K"] += d
        stats["applies_M"] += d
        lam_all, Xh_all, Yh_all = small_lrep(U.T @ KU, V.T @ MV, d)

        cache = {}

        def pull(g):
            """Pulled-back Ritz pair g: (x~, y~, K x~, M y~)."""
            if g not in cache:
                cache[g] = (U @ Xh_all[:, g], V @ Yh_all[:, g],
                            KU @ Xh_all[:, g], MV @ Yh_all[:, g])
            return cache[g]

        def block(idx):
            cols = [pull(g) for g in idx]
            return tuple(np.stack([cl[k] for cl in cols], axis=1) if cols
                         else np.zeros((n, 0)) for k in range(4))

        nr = min(b, d)
        Xt, Yt, KXt, MYt = block(range(nr))
        # Step 4
        eps = residual_eps(KXt, Yt, MYt, Xt, lam_all[:nr])
        conv = eps <= tol
        p = nr if conv.all() else int(np.argmin(conv))
        if history is not None:
            history.append(dict(it=it, locked=c, d=d, eps=eps.copy(),
                                lam=lam_all[:nr].copy()))
        if p >= need:
            lam = np.concatenate([lamc, lam_all[:need]])
            X = np.hstack([Xc, Xt[:, :need]])
            Y = np.hstack([Yc, Yt[:, :need]])
            epsout = np.concatenate([epsc, eps[:need]])
            if null_on_M:
                X, Y = Y, X
            X, Y = sign_normalise(X, Y)
            return BospResult(lam, X, Y, True, it, epsout, stats)

        # locking with the moving mechanism
        L = lock_unit if (p >= lock_unit and d > lock_unit) else 0
        if L:
            Xc = np.hstack([Xc, Xt[:, :L]])
            Yc = np.hstack([Yc, Yt[:, :L]])
            lamc = np.concatenate([lamc, lam_all[:L]])
            epsc = np.concatenate([epsc, eps[:L]])
            stats["locks"] += 1
        hi = min(L + b, d)                        # active X block: Ritz [L, hi)
        known = {g: eps[g] for g in range(nr)}
        win = [g for g in range(L, hi) if known.get(g, np.inf) > tol][:w]
        # fewer than w unconverged in the block: continue the window into the
        # next Ritz pairs of the projected problem
        win += list(range(hi, min(d, hi + w - len(win))))
        Xa, Ya, KXa, MYa = block(range(L, hi))

        if not win:
            U, V = Xa, Ya
            continue

        # Step 5
        ga = np.array(win)
        XhK = Xh_all[:, :hi]
        YhK = Yh_all[:, :hi]
        E = np.zeros((d, ga.size))
        E[ga, np.arange(ga.size)] = 1.0
        Ph0 = Xh_all[:, ga] - E
        Qh0 = Yh_all[:, ga] - E
        Ph, Qh = Ph0, Qh0
        for _ in range(2):               # projector applied twice (see module notes)
            Ph = Ph - XhK @ (YhK.T @ Ph)
            Qh = Qh - YhK @ (XhK.T @ Qh)
        # a difference the projector annihilates carries no new direction
        # (e.g. when the kept Ritz vectors already span the whole subspace)
        live = ((np.linalg.norm(Ph, axis=0) > MGS_DEP_TOL * np.linalg.norm(Ph0, axis=0))
                & (np.linalg.norm(Qh, axis=0) > MGS_DEP_TOL * np.linalg.norm(Qh0, axis=0)))
        Ph, Qh, kept = mgs_biorth(Ph[:, live], Qh[:, live], MGS_COS_TOL, MGS_DEP_TOL)
        stats["mgs_drops"] += ga.size - len(kept)
        Pt = U @ Ph
        Qt = V @ Qh

        # Step 6
        lw = lam_all[ga][None, :]
        Xw, Yw, KXw, MYw = block(ga)
        W = np.zeros_like(Xw)
        for _ in range(ngs):
            Z, na = cg_columns(M_apply, W * lw + Xw * lw - MYw, cg_tol, cg_maxit)
            stats["applies_M"] += na
            W, na = cg_columns(K_apply, Z * lw + Yw * lw - KXw, cg_tol, cg_maxit)
            stats["applies_K"] += na
        Xall = np.hstack([X0, Xc, Xa, Pt])
        Yall = np.hstack([Y0, Yc, Ya, Qt])
        for _ in range(2):               # projector applied twice (see module notes)
            W = W - Xall @ (Yall.T @ W)
            Z = Z - Yall @ (Xall.T @ Z)
        W, Z, kept = mgs_biorth(W, Z, MGS_COS_TOL, MGS_DEP_TOL)
        stats["mgs_drops"] += ga.size - len(kept)

        # Step 7
        U = np.hstack([Xa, Pt, W])
        V = np.hstack([Ya, Qt, Z])

    if raise_on_maxit:
        raise NotConvergedError(f"not converged in {maxit} iterations")
    # not converged: return the converged prefix (locked pairs) only
    X, Y = (Yc, Xc) if null_on_M else (Xc, Yc)
    X, Y = sign_normalise(X, Y)
    return BospResult(lamc, X, Y, False, maxit, epsc, stats)
