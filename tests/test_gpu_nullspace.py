"""lrep_find_nullspace: the null space of the semidefinite operator computed
on the device (the remark on computing the generalized null space), against
the oracle's eigendecomposition basis, and whole solves on top of it.

Bars: subspace distance (sin of the largest principal angle) to the oracle's
N(A) <= 1e-10; the solve on the found null space meets the same eigenvalue,
residual and biorthogonality bars as with a declared basis.
"""
import numpy as np
import pytest

import gen
import paper_2506_08355_amd as L
from oracle import exact, generalized as G, nullspace as N
from conftest import load_golden
from gpu_util import dev_colmajor, h_residual

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    c = L.lrep_init(0)
    yield c
    L.lrep_finalize(c)


def gpu_solve(ctx, op, n, nev, block, tol, window=0, init=None):
    lam = np.zeros(nev)
    X = np.zeros((n, nev), order="F")
    Y = np.zeros((n, nev), order="F")
    opts = L.make_opts(window=window, init=None if init is None else np.asfortranarray(init))
    rc, st = L.lrep_solve(op, n, nev, block, tol, opts, lam, X, Y, ctx=ctx, check=False)
    return rc, st, lam, X, Y


def test_example_4_2_constant_null_vector(ctx):
    n = 1000
    print(f"[nullspace] Example 4.2 n={n}", flush=True)
    K, M = gen.tridiag_T(n, -1.0), gen.tridiag_T(n, 0.0)
    op = L.lrep_create_dense(ctx, dev_colmajor(K, torch), dev_colmajor(M, torch))
    r, res = L.lrep_find_nullspace(op, 4, 1e-10, 11, ctx)
    assert r == 1 and res <= 1e-10
    # the basis the library kept is biorthonormal (X0, Y0); the oracle's N(K) is span(1)
    U, _ = gen.init_block(n, 30, 7)
    rc, st, lam, X, Y = gpu_solve(ctx, op, n, 10, 10, 1e-10, init=U)
    L.lrep_destroy_op(op)
    assert rc == L.LREP_OK, L.lrep_last_error(ctx)
    printed = load_golden("example_4_2_eigenvalues.txt")[:, 1]
    np.testing.assert_allclose(lam, printed, rtol=1e-10)
    assert h_residual(lambda v: K @ v, lambda v: M @ v, X, Y, lam, 4.0).max() <= 1e-8
    assert np.abs(X.T @ Y - np.eye(10)).max() <= 1e-12


@pytest.mark.parametrize("metric", [False, True], ids=["plain", "with_metric"])
def test_zero_variant_found_null_space(ctx, metric):
    n, nev, block, window, tol = 400, 24, 16, 8, 1e-10
    print(f"[nullspace] zero variant n={n} metric={metric}", flush=True)
    K, M, f = gen.dense_operator(n, 1012, n_zero_m=8)
    op = L.lrep_create_dense(ctx, dev_colmajor(K, torch), dev_colmajor(M, torch), L.LREP_NULL_ON_M)
    b = gen.metric_diag(n, 1106)
    if metric:
        L.lrep_set_metric(op, b, ctx)
    r, res = L.lrep_find_nullspace(op, 16, 1e-10, 12, ctx)
    assert r == 8 and res <= 1e-10
    U, _ = gen.init_block(n, block + 2 * window, 7)
    rc, st, lam, X, Y = gpu_solve(ctx, op, n, nev, block, tol, window=window, init=U)
    L.lrep_destroy_op(op)
    assert rc == L.LREP_OK, L.lrep_last_error(ctx)
    if metric:
        ref = G.generalized_spectrum(K, M, np.diag(b), nev, zeros=8)
        np.testing.assert_allclose(lam, ref, rtol=1e-10)
        assert G.generalized_residual(K, M, np.diag(b), X, Y, lam, normH=f.norm_H(),
                                      normB=float(b.max())).max() <= 1e-8
        assert G.b_biorth_error(np.diag(b), X, Y) <= 1e-12
    else:
        np.testing.assert_allclose(lam, exact.dense_spectrum(f.q1, f.k, f.q2, f.m, nev), rtol=1e-10)
        assert h_residual(lambda v: K @ v, lambda v: M @ v, X, Y, lam, f.norm_H()).max() <= 1e-8
        assert np.abs(X.T @ Y - np.eye(nev)).max() <= 1e-12
        # the null space the solve worked against is the oracle's N(M): X is orthogonal to it
        Z = N.null_basis(M)
        assert Z.shape[1] == 8 and np.abs(Z.T @ X).max() <= 1e-10


def test_lowrank_found_basis_matches_declared_one(ctx):
    """A low-rank operator with two zeros in delta: N(K) is spanned by two
    coordinate vectors (the oracle's null basis of a diagonal with zeros).
    Solving on the found null space and on the declared coordinate vectors
    gives the same eigenvalues, and the pairs meet the residual bar."""
    n, r, nev, block, window, tol = 1500, 16, 16, 16, 8, 1e-9
    print(f"[nullspace] low rank n={n} with two zeros in delta", flush=True)
    fc = gen.casida_factors(n, r, 1003)
    delta = fc.delta.copy()
    delta[[5, 700]] = 0.0
    U, _ = gen.init_block(n, block + 2 * window, 7)
    out = []
    for found in (True, False):
        op = L.lrep_create_lowrank(ctx, dev_colmajor(delta, torch), dev_colmajor(fc.L, torch))
        if found:
            k, res = L.lrep_find_nullspace(op, 8, 1e-10, 13, ctx)
            assert k == 2 and res <= 1e-10
        else:
            E = np.zeros((n, 2), order="F")
            E[5, 0] = E[700, 1] = 1.0
            L.lrep_set_nullspace(op, E, ctx)
        rc, st, lam, X, Y = gpu_solve(ctx, op, n, nev, block, tol, window=window, init=U)
        L.lrep_destroy_op(op)
        assert rc == L.LREP_OK, L.lrep_last_error(ctx)
        out.append((lam, X, Y))
    np.testing.assert_allclose(out[0][0], out[1][0], rtol=1e-10)
    Kd = np.diag(delta)
    Md = Kd + 2.0 * fc.L @ fc.L.T
    assert h_residual(lambda v: Kd @ v, lambda v: Md @ v, out[0][1], out[0][2], out[0][0],
                      np.linalg.norm(Md, 2)).max() <= 1e-8


def test_definite_operator_and_small_rmax(ctx):
    n = 256
    K, M, f = gen.dense_operator(n, 1001)
    op = L.lrep_create_dense(ctx, dev_colmajor(K, torch), dev_colmajor(M, torch))
    r, res = L.lrep_find_nullspace(op, 8, 1e-10, 14, ctx)
    assert r == 0                                   # K is definite: nothing found
    with pytest.raises(L.LrepError) as e:
        L.lrep_find_nullspace(op, 65, 1e-10, 14, ctx)
    assert e.value.code == L.LREP_EINVAL
    L.lrep_destroy_op(op)
    # rmax below dim N(M): r == rmax signals that the null space may be larger
    K, M, f = gen.dense_operator(400, 1012, n_zero_m=8)
    op = L.lrep_create_dense(ctx, dev_colmajor(K, torch), dev_colmajor(M, torch), L.LREP_NULL_ON_M)
    r, res = L.lrep_find_nullspace(op, 4, 1e-10, 15, ctx)
    assert r == 4 and res <= 1e-10
    L.lrep_destroy_op(op)
