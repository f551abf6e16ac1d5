"""Pins for the oracle's MGS-Biorth / CGS-Biorth (Section 3.1)."""
import numpy as np
import pytest

import gen
from oracle import mgs_biorth, cgs_biorth
from conftest import load_golden


def _e1(n):
    m = n // 2
    return gen.hilbert(n)[:, :m], gen.lauchli(n, 1e-3)[:, :m], m


@pytest.mark.parametrize("row", list(range(5)))
def test_biorth_loss_table(row):
    """Reproduce the paper's table of biorthogonality loss.  The Lauchli
    parameter is not printed; mu = 1e-3 reproduces kappa(Y) exactly."""
    tab = load_golden("biorth_loss_table.txt")
    n, kx, ky, skxy, cgs_p, mgs_p = tab[row]
    X, Y, m = _e1(int(n))
    # condition numbers: the printed digits are truncated to 3 significant figures
    assert np.floor(np.linalg.cond(X) / 10 ** np.floor(np.log10(kx)) * 100) / 100 == pytest.approx(kx / 10 ** np.floor(np.log10(kx)), abs=1e-9)
    assert np.floor(np.linalg.cond(Y) / 10 ** np.floor(np.log10(ky)) * 100) / 100 == pytest.approx(ky / 10 ** np.floor(np.log10(ky)), abs=1e-9)
    if n <= 12:       # beyond that kappa(X^T Y) exceeds what FP64 can resolve
        assert np.sqrt(np.linalg.cond(X.T @ Y)) == pytest.approx(skxy, rel=1e-2)
    P, Q, kept = mgs_biorth(X, Y)
    Pc, Qc = cgs_biorth(X, Y)
    assert len(kept) == m
    mgs_loss = np.linalg.norm(P.T @ Q - np.eye(m), 2)
    cgs_loss = np.linalg.norm(Pc.T @ Qc - np.eye(m), 2)
    # rounding-order dependent: agree with the printed value in order of magnitude
    assert abs(np.log10(mgs_loss) - np.log10(mgs_p)) < 1.0
    assert abs(np.log10(cgs_loss) - np.log10(cgs_p)) < 1.0
    if n >= 8:
        assert cgs_loss > 5 * mgs_loss
    # conjectured bound ||P^T Q - I|| = O(eps) sqrt(kappa(X^T Y)), constant <= 1e4
    if n <= 12:
        assert mgs_loss <= 1e4 * np.finfo(float).eps * np.sqrt(np.linalg.cond(X.T @ Y))


def test_mgs_biorth_with_equal_inputs_is_mgs_qr():
    """With Y = X, X^T Y = X^T X is SPD, every pivot is positive and
    MGS-Biorth is MGS orthogonalisation: P = Q = the QR factor with a
    positive diagonal."""
    rng = np.random.default_rng(3)
    X = rng.standard_normal((40, 7))
    P, Q, kept = mgs_biorth(X, X)
    q, r = np.linalg.qr(X)
    q *= np.sign(np.diag(r))[None, :]
    assert kept == list(range(7))
    np.testing.assert_allclose(P, q, atol=1e-13)
    np.testing.assert_allclose(Q, q, atol=1e-13)


def test_mgs_biorth_pivots_are_ratios_of_leading_minors():
    """Exact-arithmetic identity: X = P R, Y = Q S with R, S upper triangular,
    so X^T Y = R^T S is an unpivoted LU of X^T Y and the l-th pivot eta_l =
    r_ll s_ll = det(G_l) / det(G_{l-1}) (G_l the leading l x l block)."""
    rng = np.random.default_rng(4)
    n, m = 30, 6
    X = rng.standard_normal((n, m))
    Y = X + 0.3 * rng.standard_normal((n, m))
    P, Q, kept = mgs_biorth(X, Y)
    R = Q.T @ X
    S = P.T @ Y
    np.testing.assert_allclose(np.tril(R, -1), 0, atol=1e-12)
    np.testing.assert_allclose(np.tril(S, -1), 0, atol=1e-12)
    G = X.T @ Y
    np.testing.assert_allclose(R.T @ S, G, rtol=1e-12, atol=1e-12)
    dets = [1.0] + [np.linalg.det(G[:l, :l]) for l in range(1, m + 1)]
    eta = np.array([dets[l] / dets[l - 1] for l in range(1, m + 1)])
    np.testing.assert_allclose(np.diag(R) * np.diag(S), eta, rtol=1e-10)
    # normalisation of Algorithm MGS-Biorth: r_ll = sign(eta) sqrt|eta|, s_ll = sqrt|eta|
    np.testing.assert_allclose(np.diag(S), np.sqrt(np.abs(eta)), rtol=1e-10)
    np.testing.assert_allclose(np.sign(np.diag(R)), np.sign(eta))
    np.testing.assert_allclose(P.T @ Q, np.eye(m), atol=1e-13)


def test_mgs_biorth_negative_pivot():
    """A pair with x^T y < 0 is kept and normalised with r = -sqrt|eta|."""
    x = np.array([[1.0], [2.0], [0.0]])
    y = np.array([[-1.0], [0.0], [1.0]])
    P, Q, kept = mgs_biorth(x, y)
    assert kept == [0]
    assert P[0, 0] == pytest.approx(-1.0) and Q[0, 0] == pytest.approx(-1.0)
    assert (P.T @ Q)[0, 0] == pytest.approx(1.0)


def test_mgs_biorth_drops_dependent_and_orthogonal_pairs():
    """Remark on ill-conditioned inputs: pairs whose pivot vanishes are
    discarded and the procedure continues."""
    rng = np.random.default_rng(5)
    X = rng.standard_normal((20, 4))
    Y = X.copy()
    X[:, 2] = X[:, 0] + X[:, 1]           # dependent on earlier columns
    Y[:, 2] = Y[:, 0] - Y[:, 1]
    P, Q, kept = mgs_biorth(X, Y, cos_tol=1e-10, dep_tol=1e-12)
    assert kept == [0, 1, 3]
    np.testing.assert_allclose(P.T @ Q, np.eye(3), atol=1e-12)
    # exactly orthogonal pair: eta = 0 is always dropped
    x = np.array([[1.0], [0.0]])
    y = np.array([[0.0], [1.0]])
    P, Q, kept = mgs_biorth(x, y)
    assert kept == [] and P.shape == (2, 0)
