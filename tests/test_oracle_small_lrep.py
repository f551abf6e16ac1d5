"""Pins for the oracle's small structured LREP (Cholesky + SVD)."""
import numpy as np
import pytest

from oracle import small_lrep, small_lrep_bruteforce, NotSPDError


def _spd(rng, d, cond):
    q, _ = np.linalg.qr(rng.standard_normal((d, d)))
    ev = np.geomspace(1.0, cond, d)
    return (q * ev) @ q.T


@pytest.mark.parametrize("d,cond", [(5, 10.0), (24, 1e3), (48, 1e5)])
def test_small_lrep_matches_bruteforce_eig(d, cond):
    """Positive eigenvalues of the 2d x 2d H^ by a general eigensolver."""
    rng = np.random.default_rng(d)
    Kh = _spd(rng, d, cond)
    Mh = _spd(rng, d, cond)
    nwant = d // 2
    lam, Xh, Yh = small_lrep(Kh, Mh, nwant)
    ref = small_lrep_bruteforce(Kh, Mh, nwant)
    np.testing.assert_allclose(lam, ref, rtol=1e-9 * cond ** 0.5)
    assert np.all(np.diff(lam) >= 0)
    # K^ X^ = Y^ Lambda, M^ Y^ = X^ Lambda, X^T Y^ = I
    scale = np.linalg.norm(Kh, 2) + np.linalg.norm(Mh, 2)
    assert np.abs(Kh @ Xh - Yh * lam).max() <= 1e-12 * scale * np.abs(Xh).max()
    assert np.abs(Mh @ Yh - Xh * lam).max() <= 1e-12 * scale * np.abs(Yh).max()
    np.testing.assert_allclose(Xh.T @ Yh, np.eye(nwant), atol=1e-12 * cond)


def test_small_lrep_commuting_case_closed_form():
    """K^ = Q diag(k) Q^T, M^ = Q diag(m) Q^T share eigenvectors: lambda =
    sqrt(k m), x = (m/k)^(1/4) q, y = (k/m)^(1/4) q."""
    rng = np.random.default_rng(9)
    d = 12
    q, _ = np.linalg.qr(rng.standard_normal((d, d)))
    k = rng.uniform(0.5, 10, d)
    m = rng.uniform(0.5, 10, d)
    lam, Xh, Yh = small_lrep((q * k) @ q.T, (q * m) @ q.T, d)
    order = np.argsort(np.sqrt(k * m))
    np.testing.assert_allclose(lam, np.sqrt(k * m)[order], rtol=1e-13)
    for j, i in enumerate(order):
        s = np.sign(Xh[:, j] @ q[:, i])
        np.testing.assert_allclose(s * Xh[:, j], (m[i] / k[i]) ** 0.25 * q[:, i], atol=1e-12)
        np.testing.assert_allclose(s * Yh[:, j], (k[i] / m[i]) ** 0.25 * q[:, i], atol=1e-12)


def test_small_lrep_rejects_indefinite():
    Kh = np.diag([1.0, -1.0, 2.0])
    with pytest.raises(NotSPDError):
        small_lrep(Kh, np.eye(3), 2)
