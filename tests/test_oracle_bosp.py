"""Pins for the oracle's BOSP iteration and exact spectra (Sections 2-4)."""
import numpy as np
import pytest

import gen
import oracle
from oracle import exact
from conftest import load_golden


def _solve(op, nev, block, tol, window=None, X0=None, null_on_M=False, seed=7, **kw):
    d = block + 2 * (window or block)
    U, _ = gen.init_block(op.n, d, seed)
    return oracle.bosp_solve(op, nev, block, tol, window=window, X0=X0,
                             init=(U, U), null_on_M=null_on_M, **kw)


def _invariants(op, res, normH, tol_res=1e-8, tol_bi=1e-12):
    X, Y, lam = res.X, res.Y, res.lam
    k = lam.size
    # biorthogonality X^T Y = I (definition of biorthogonal matrices, Section 2)
    assert np.abs(X.T @ Y - np.eye(k)).max() <= tol_bi
    # H-normalised residual ||H z - lambda z|| / (||H|| ||z||), z = [y; x]
    R1 = op.apply_K(X) - Y * lam
    R2 = op.apply_M(Y) - X * lam
    rel = np.sqrt((R1 ** 2).sum(0) + (R2 ** 2).sum(0)) / (
        normH * np.sqrt((X ** 2).sum(0) + (Y ** 2).sum(0)))
    assert rel.max() <= tol_res
    # +-lambda pairing (Lemma 2.1 (iii)): H [-y; x] = -lambda [-y; x]
    np.testing.assert_allclose(op.apply_K(X), Y * lam, atol=10 * tol_res * normH * np.abs(Y).max())
    np.testing.assert_allclose(op.apply_M(-Y), -(X * lam), atol=10 * tol_res * normH * np.abs(X).max())
    # trace identity at convergence (Theorem 2.5): 1/2 tr(X^T K X + Y^T M Y) = sum lambda
    tr = 0.5 * (np.einsum("ij,ij->", X, op.apply_K(X)) + np.einsum("ij,ij->", Y, op.apply_M(Y)))
    assert tr == pytest.approx(lam.sum(), rel=1e-9)
    assert np.all(np.diff(lam) >= -1e-12 * lam.max())
    return rel


def test_example_4_1_against_printed_values():
    """Example 4.1: K = M = T(0), n = 1000, n_e = n_b = 10, tol 1e-10."""
    n = 1000
    T0 = gen.tridiag_T(n, 0.0)
    op = oracle.DenseOperator(T0, T0)
    res = _solve(op, 10, 10, 1e-10)
    assert res.converged
    printed = load_golden("example_4_1_eigenvalues.txt")[:, 1]
    np.testing.assert_allclose(exact.example_4_1_spectrum(n, 10), printed, rtol=1e-15)
    np.testing.assert_allclose(res.lam, printed, rtol=1e-10)
    _invariants(op, res, 4.0, tol_res=1e-10)
    # eigenvectors: x = y = [sin(j l pi/(n+1))]_j (error measure eta_l of Section 4.1)
    j = np.arange(1, n + 1)
    for l in range(10):
        xe = np.sin(j * (l + 1) * np.pi / (n + 1))
        ze = np.concatenate([xe, xe]) / np.linalg.norm(np.concatenate([xe, xe]))
        z = np.concatenate([res.Y[:, l], res.X[:, l]])
        z /= np.linalg.norm(z)
        assert min(np.linalg.norm(z - ze), np.linalg.norm(z + ze)) < 1e-6


def test_example_4_2_against_printed_values():
    """Example 4.2: K = T(-1) (null space span{1}), M = T(0), n = 1000."""
    n = 1000
    K = gen.tridiag_T(n, -1.0)
    M = gen.tridiag_T(n, 0.0)
    op = oracle.DenseOperator(K, M)
    x0 = np.ones((n, 1))
    # closed form of the generalized null space (Example 4.2): M y0 = x0
    l = np.arange(1, n + 1, dtype=float)
    y0 = l * (n - l + 1) / 2.0
    np.testing.assert_allclose(M @ y0, x0[:, 0], atol=1e-9)
    np.testing.assert_allclose(K @ x0[:, 0], 0.0, atol=0)
    res = _solve(op, 10, 10, 1e-10, X0=x0)
    assert res.converged
    printed = load_golden("example_4_2_eigenvalues.txt")[:, 1]
    np.testing.assert_allclose(exact.example_4_2_spectrum(n, 10), printed, rtol=5e-12)
    np.testing.assert_allclose(res.lam, printed, rtol=1e-10)
    _invariants(op, res, 4.0, tol_res=1e-10)
    # Lemma 2.3 (iii): nonzero eigenvectors are biorthogonal to the null space pair
    X0, Y0 = oracle.nullspace_basis(x0, op.solve_M)
    assert np.abs(Y0.T @ res.X).max() <= 1e-12 * np.linalg.norm(Y0) * np.abs(res.X).max() * n
    assert np.abs(X0.T @ res.Y).max() <= 1e-12


def test_nullspace_basis_normalisation():
    """Equation for the V0 basis: X0^T Y0 = I, K X0 = 0, M Y0 = X0."""
    n = 50
    K = gen.tridiag_T(n, -1.0)
    op = oracle.DenseOperator(K, gen.tridiag_T(n, 0.0))
    X0, Y0 = oracle.nullspace_basis(3.0 * np.ones((n, 1)), op.solve_M)
    np.testing.assert_allclose(X0.T @ Y0, np.eye(1), atol=1e-14)
    np.testing.assert_allclose(K @ X0, 0, atol=1e-14)
    np.testing.assert_allclose(op.M @ Y0, X0, atol=1e-12)


def test_dense_spectrum_against_bruteforce_eig():
    """Factored singular-value form vs eig of the 2n x 2n H (Lemma 2.1)."""
    K, M, f = gen.dense_operator(40, 11)
    H = np.block([[np.zeros((40, 40)), K], [M, np.zeros((40, 40))]])
    ev = np.sort(np.linalg.eigvals(H).real)
    np.testing.assert_allclose(exact.dense_spectrum(f.q1, f.k, f.q2, f.m), ev[ev > 0], rtol=1e-11)
    np.testing.assert_allclose(-exact.dense_spectrum(f.q1, f.k, f.q2, f.m)[::-1], ev[ev < 0], rtol=1e-11)
    # lambda^2 in spec(K M)
    km = np.sort(np.linalg.eigvals(K @ M).real)
    np.testing.assert_allclose(exact.dense_spectrum(f.q1, f.k, f.q2, f.m) ** 2, km, rtol=1e-10)


def test_dense_spectrum_smallest_against_bruteforce():
    """The F^T F route for large n against eig of H, with and without exact
    zeros in m (the zero-eigenvalue variant)."""
    for zeros in (0, 5):
        K, M, f = gen.dense_operator(60, 12 + zeros, n_zero_m=zeros)
        H = np.block([[np.zeros((60, 60)), K], [M, np.zeros((60, 60))]])
        ev = np.sort(np.linalg.eigvals(H).real)
        pos = ev[ev > 1e-6]
        got = exact.dense_spectrum_smallest(f.q1, f.k, f.q2, f.m, 12)
        np.testing.assert_allclose(got, pos[:12], rtol=1e-11)
        np.testing.assert_allclose(got, exact.dense_spectrum(f.q1, f.k, f.q2, f.m, 12), rtol=1e-12)


def test_config1_dense_n256():
    """Dense n = 256, 8 smallest, block 16, tol 1e-10."""
    K, M, f = gen.dense_operator(256, 1001)
    op = oracle.DenseOperator(K, M)
    res = _solve(op, 8, 16, 1e-10)
    assert res.converged and res.lam.size == 8
    np.testing.assert_allclose(res.lam, exact.dense_spectrum(f.q1, f.k, f.q2, f.m, 8), rtol=1e-10)
    _invariants(op, res, f.norm_H())
    assert np.all(res.eps <= 1e-10)


@pytest.mark.parametrize("n,seed,nev,block,window", [(256, 1001, 8, 16, 8), (600, 1005, 16, 16, 8)])
def test_independent_start_blocks_reach_the_same_pairs(n, seed, nev, block, window):
    """Step 1 of the algorithm draws U and V at random; the oracle (and the
    library) take V = U (reading Z6).  Independent U and V must lead to the
    same pairs: the biorthogonality monitor restores U^T V = I where the
    independent start erodes it, and the iteration count stays within a few
    iterations of the V = U start (measured: 22 vs 21 and 60 vs 66)."""
    K, M, f = gen.dense_operator(n, seed)
    op = oracle.DenseOperator(K, M)
    U, V = gen.init_block(n, block + 2 * window, 7)
    ref = exact.dense_spectrum(f.q1, f.k, f.q2, f.m, nev)
    same = oracle.bosp_solve(op, nev, block, 1e-10, window=window, init=(U, U.copy()), maxit=400)
    indep = oracle.bosp_solve(op, nev, block, 1e-10, window=window, init=(U, V), maxit=400)
    for res in (same, indep):
        assert res.converged and res.lam.size == nev
        np.testing.assert_allclose(res.lam, ref, rtol=1e-10)
        _invariants(op, res, f.norm_H())
    assert indep.stats["rebiorth"] >= 1 and same.stats["rebiorth"] == 0
    assert abs(indep.iterations - same.iterations) <= 0.15 * same.iterations + 2


def test_commuting_case_closed_form():
    """Q1 = Q2: lambda_i = sqrt(k_i m_i) exactly."""
    n = 120
    f = gen.dense_factors(n, 21)
    f.q2 = f.q1
    op = oracle.DenseOperator(f.K(), f.M())
    res = _solve(op, 6, 8, 1e-11)
    np.testing.assert_allclose(res.lam, np.sort(np.sqrt(f.k * f.m))[:6], rtol=1e-11)


@pytest.mark.slow
def test_zero_variant_role_swap_and_moving():
    """Dense with 8 exact zeros in m (null space on M, roles exchanged),
    nev > block so the moving mechanism locks pairs."""
    n = 400
    K, M, f = gen.dense_operator(n, 1012, n_zero_m=8)
    op = oracle.DenseOperator(K, M)
    res = _solve(op, 24, 16, 1e-10, window=8, X0=f.null_basis_M(), null_on_M=True)
    assert res.converged and res.stats["locks"] >= 1
    np.testing.assert_allclose(res.lam, exact.dense_spectrum(f.q1, f.k, f.q2, f.m, 24), rtol=1e-10)
    _invariants(op, res, f.norm_H())
    # returned pairs are biorthogonal to the generalized null space (Lemma 2.3 (iii))
    Xn = f.null_basis_M()                    # N(M); after the exchange it plays N(K)
    assert np.abs(Xn.T @ res.X).max() <= 1e-10


def test_casida_count_against_bruteforce():
    f = gen.casida_factors(300, 12, 5)
    H = np.block([[np.zeros((300, 300)), f.K()], [f.M(), np.zeros((300, 300))]])
    ev = np.sort(np.linalg.eigvals(H).real)
    pos = ev[ev > 0]
    lams = [0.2, 0.5, 1.3, 7.0] + list(np.sort(pos)[[0, 5, 40, 120]] * (1 + 1e-9))
    for lam in lams:
        assert exact.casida_count_below(f.delta, f.L, lam) == int(np.count_nonzero(pos < lam))
    # the batched form (W formed once, row chunks smaller than n) gives the same counts
    assert exact.casida_count_below_many(f.delta, f.L, lams, chunk=64) == [
        int(np.count_nonzero(pos < lam)) for lam in lams]


@pytest.mark.slow
def test_casida_lowrank_moving():
    """K = diag(delta), M = diag(delta) + 2 L L^T; nev = 32 in batches."""
    n, r = 1500, 16
    f = gen.casida_factors(n, r, 1003)
    op = oracle.CasidaOperator(f.delta, f.L)
    res = _solve(op, 32, 16, 1e-9, window=8)
    assert res.converged and res.stats["locks"] >= 1
    # exact: K = F1 F1^T with F1 = diag(sqrt delta), M = L2 L2^T
    L2 = np.linalg.cholesky(f.M())
    ref = np.sort(np.linalg.svd(np.sqrt(f.delta)[:, None] * L2, compute_uv=False))[:32]
    np.testing.assert_allclose(res.lam, ref, rtol=1e-10)
    _invariants(op, res, np.linalg.norm(f.M(), 2))
    # no eigenvalue skipped (Haynsworth inertia count)
    assert exact.casida_count_below(f.delta, f.L, res.lam[-1] * (1 + 1e-9)) == 32


def test_casida_operator_and_woodbury():
    f = gen.casida_factors(200, 7, 2)
    op = oracle.CasidaOperator(f.delta, f.L)
    X = np.random.default_rng(0).standard_normal((200, 3))
    np.testing.assert_allclose(op.apply_M(X), f.M() @ X, rtol=1e-13)
    np.testing.assert_allclose(op.apply_K(X), f.K() @ X, rtol=1e-15)
    np.testing.assert_allclose(f.M() @ op.solve_M(X), X, atol=1e-11)


def test_cg_columns_exact_with_many_iterations():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((30, 30))
    A = A @ A.T + 30 * np.eye(30)
    B = rng.standard_normal((30, 4))
    B[:, 2] = 0.0                       # zero right-hand side stays zero
    X, _ = oracle.cg_columns(lambda v: A @ v, B, 1e-14, 200)
    np.testing.assert_allclose(X, np.linalg.solve(A, B), atol=1e-10)
    # relative stopping rule: ||r|| <= tol ||b|| per column
    X, _ = oracle.cg_columns(lambda v: A @ v, B, 1e-2, 20)
    for j in [0, 1, 3]:
        assert np.linalg.norm(B[:, j] - A @ X[:, j]) <= 1e-2 * np.linalg.norm(B[:, j]) * (1 + 1e-12)


def test_not_converged_returns_prefix():
    K, M, f = gen.dense_operator(128, 3)
    res = _solve(oracle.DenseOperator(K, M), 8, 8, 1e-12, maxit=2)
    assert not res.converged and res.iterations == 2
    with pytest.raises(oracle.NotConvergedError):
        _solve(oracle.DenseOperator(K, M), 8, 8, 1e-12, maxit=2, raise_on_maxit=True)


def test_dense_spectrum_torch_form_matches_the_numpy_form():
    """The PyTorch CPU form of the dense closed form (used for n = 32768)
    gives the NumPy form's eigenvalues, also with exact zeros in m, and the
    torch QR of the generator gives the same spectrum as the host QR."""
    f = gen.dense_factors(300, 17, n_zero_m=3)
    a = exact.dense_spectrum_smallest(f.q1, f.k, f.q2, f.m, 20)
    b = exact.dense_spectrum_smallest_torch(f.q1, f.k, f.q2, f.m, 20)
    np.testing.assert_allclose(b, a, rtol=1e-13)
    np.testing.assert_allclose(a, exact.dense_spectrum(f.q1, f.k, f.q2, f.m, 20), rtol=1e-12)
    q1, k, q2, m = gen.dense_factors_torch(300, 17, "cpu", n_zero_m=3)
    np.testing.assert_allclose(exact.dense_spectrum_smallest_torch(q1, k, q2, m, 20), a, rtol=1e-12)
