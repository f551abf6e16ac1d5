"""Pins of the generalized-LREP oracle (K x = lambda B y, M y = lambda B x).

Each check is fixed by something other than the oracle's own formula: a
closed form, the library eigensolver on the full 2n x 2n pencil, an
exact invariance, or the standard-LREP spectrum computed another way.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import exact, generalized as G


def _spd(n, rng, lo=0.5, hi=10.0):
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (Q * rng.uniform(lo, hi, n)[None, :]) @ Q.T


def test_diagonal_closed_form():
    # diagonal K, M, B: the pencil splits into 2 x 2 blocks with
    # lambda_i = sqrt(k_i m_i) / b_i
    rng = np.random.default_rng(1)
    n = 40
    k, m, b = rng.uniform(0.5, 10, n), rng.uniform(0.5, 10, n), rng.uniform(0.2, 5, n)
    got = G.generalized_spectrum(np.diag(k), np.diag(m), np.diag(b))
    np.testing.assert_allclose(got, np.sort(np.sqrt(k * m) / b), rtol=1e-13)


def test_against_full_pencil_eig():
    # the library's generalized eigensolver on the 2n x 2n pencil itself
    rng = np.random.default_rng(2)
    n = 7
    K, M, B = _spd(n, rng), _spd(n, rng), _spd(n, rng, 0.3, 3.0)
    Z = np.zeros((n, n))
    ev = sla.eigvals(np.block([[Z, K], [M, Z]]), np.block([[B, Z], [Z, B]]))
    assert np.abs(ev.imag).max() < 1e-9
    pos = np.sort(ev.real[ev.real > 0])
    np.testing.assert_allclose(G.generalized_spectrum(K, M, B), pos, rtol=1e-10)


def test_identity_metric_is_the_standard_spectrum():
    # B = I: the factored-form spectrum of the dense workload
    rng = np.random.default_rng(3)
    n = 30
    q1, _ = np.linalg.qr(rng.standard_normal((n, n)))
    q2, _ = np.linalg.qr(rng.standard_normal((n, n)))
    k, m = rng.uniform(0.5, 10, n), rng.uniform(0.5, 10, n)
    K, M = (q1 * k) @ q1.T, (q2 * m) @ q2.T
    np.testing.assert_allclose(G.generalized_spectrum(K, M, np.eye(n)), exact.dense_spectrum(q1, k, q2, m),
                               rtol=1e-12)


def test_metric_scaling_and_congruence():
    rng = np.random.default_rng(4)
    n = 12
    K, M, B = _spd(n, rng), _spd(n, rng), _spd(n, rng, 0.3, 3.0)
    ref = G.generalized_spectrum(K, M, B)
    # B -> beta B scales every eigenvalue by 1 / beta
    np.testing.assert_allclose(G.generalized_spectrum(K, M, 2.5 * B), ref / 2.5, rtol=1e-12)
    # congruence with any invertible P leaves the pencil's spectrum unchanged
    P = rng.standard_normal((n, n)) + 3 * np.eye(n)
    np.testing.assert_allclose(G.generalized_spectrum(P.T @ K @ P, P.T @ M @ P, P.T @ B @ P), ref, rtol=1e-9)


def test_singular_K_leaves_out_the_null_space():
    # K with a 2-dimensional null space: two zero eigenvalues of K^ M^, the
    # rest from the diagonal closed form
    rng = np.random.default_rng(5)
    n = 20
    k, m, b = rng.uniform(0.5, 10, n), rng.uniform(0.5, 10, n), rng.uniform(0.2, 5, n)
    k[[3, 11]] = 0.0
    got = G.generalized_spectrum(np.diag(k), np.diag(m), np.diag(b), zeros=2)
    ref = np.sort(np.sqrt(k * m) / b)[2:]
    np.testing.assert_allclose(got, ref, rtol=1e-12)


def test_residual_and_biorth_of_exact_pairs():
    # exact pairs from the reduction have zero residual and Y^T B X = I;
    # a wrong eigenvalue or a dropped B shows up in the residual
    rng = np.random.default_rng(6)
    n = 10
    K, M, B = _spd(n, rng), _spd(n, rng), _spd(n, rng, 0.3, 3.0)
    Kh, Mh, C = G.reduce_to_standard(K, M, B)
    w, V = np.linalg.eig(Kh @ Mh)       # K^ M^ y^ = lambda^2 y^
    order = np.argsort(w.real)
    lam = np.sqrt(w.real[order])
    Yh = V.real[:, order]
    Xh = (Mh @ Yh) / lam[None, :]       # M^ y^ = lambda x^
    s = np.einsum("ij,ij->j", Xh, Yh)
    Xh, Yh = Xh / np.sqrt(s), Yh / np.sqrt(s)
    Ci = np.linalg.inv(C)
    X, Y = Ci.T @ Xh, Ci.T @ Yh
    np.testing.assert_allclose(lam, G.generalized_spectrum(K, M, B), rtol=1e-10)
    assert G.generalized_residual(K, M, B, X, Y, lam).max() < 1e-13
    assert G.b_biorth_error(B, X, Y) < 1e-12
    assert G.generalized_residual(K, M, np.eye(n), X, Y, lam).max() > 1e-3
    assert G.generalized_residual(K, M, B, X, Y, lam * (1 + 1e-6)).max() > 1e-8


@pytest.mark.parametrize("n_zero_m", [0, 3])
def test_dense_metric_factored_form_against_reduction(n_zero_m):
    # the large-n factored form of the dense workload with a diagonal metric
    # against the Cholesky reduction of the assembled matrices
    import gen
    n, count = 60, 12
    f = gen.dense_factors(n, 21, n_zero_m=n_zero_m)
    b = gen.metric_diag(n, 22)
    K, M = (f.q1 * f.k) @ f.q1.T, (f.q2 * f.m) @ f.q2.T
    ref = G.generalized_spectrum(K, M, np.diag(b), count, zeros=n_zero_m)
    got = G.dense_metric_spectrum_smallest(f.q1, f.k, f.q2, f.m, b, count, zeros=n_zero_m)
    np.testing.assert_allclose(got, ref, rtol=1e-11)
