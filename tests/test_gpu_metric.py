"""Generalized LREP with a diagonal SPD metric (K x = lambda B y,
M y = lambda B x, B = diag(b)) through lrep_set_metric, against the oracle's
generalized spectrum on the same seeded inputs.

Bars: eigenvalues within 1e-10 relative of the oracle's; the pencil's
normwise backward error sqrt(||K x - lambda B y||^2 + ||M y - lambda B x||^2)
/ ((||H|| + lambda ||B||) ||(x, y)||) <= 1e-8; max |Y^T B X - I| <= 1e-12.
The metric b is log-uniform on [0.25, 4] (a lumped mass-matrix stand-in).
"""
import numpy as np
import pytest

import gen
import paper_2506_08355_amd as L
from oracle import generalized as G
from gpu_util import dev_colmajor

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    c = L.lrep_init(0)
    yield c
    L.lrep_finalize(c)


def gpu_solve(ctx, op, n, nev, block, tol, window=0, init=None, **kw):
    lam = np.zeros(nev)
    X = np.zeros((n, nev), order="F")
    Y = np.zeros((n, nev), order="F")
    opts = L.make_opts(window=window, init=None if init is None else np.asfortranarray(init), **kw)
    rc, st = L.lrep_solve(op, n, nev, block, tol, opts, lam, X, Y, ctx=ctx, check=False)
    return rc, st, lam, X, Y


def check_generalized(lam, X, Y, ref, K, M, b):
    np.testing.assert_allclose(lam, ref, rtol=1e-10, atol=0)
    B = np.diag(b)
    normH = max(np.linalg.norm(K, 2), np.linalg.norm(M, 2))
    res = G.generalized_residual(K, M, B, X, Y, lam, normH=normH, normB=float(b.max()))
    assert res.max() <= 1e-8, res.max()
    assert G.b_biorth_error(B, X, Y) <= 1e-12


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "bf16_cg_applies"])
def test_dense_metric(ctx, precision):
    n, nev, block, tol = 256, 8, 16, 1e-10
    print(f"[metric] dense n={n} precision={precision}", flush=True)
    K, M, f = gen.dense_operator(n, 1001)
    b = gen.metric_diag(n, 1101)
    U, _ = gen.init_block(n, 3 * block, 7)
    op = L.lrep_create_dense(ctx, dev_colmajor(K, torch), dev_colmajor(M, torch))
    if precision:
        # a first solve makes the 16-bit copies of the unscaled operator; the
        # metric must replace them
        rc, *_ = gpu_solve(ctx, op, n, nev, block, tol, init=U, precision=precision)
        assert rc == L.LREP_OK, L.lrep_last_error(ctx)
    L.lrep_set_metric(op, b, ctx)
    rc, st, lam, X, Y = gpu_solve(ctx, op, n, nev, block, tol, init=U, precision=precision)
    L.lrep_destroy_op(op)
    assert rc == L.LREP_OK, L.lrep_last_error(ctx)
    ref = G.generalized_spectrum(K, M, np.diag(b), nev)
    check_generalized(lam, X, Y, ref, K, M, b)
    assert st.n_converged == nev


def test_dense_metric_nullspace_role_swap(ctx):
    """Zero variant (8 exact zeros in m, roles exchanged): the null-space basis
    is given in the original coordinates."""
    n, nev, block, window, tol = 400, 24, 16, 8, 1e-10
    print(f"[metric] zero variant n={n}", flush=True)
    K, M, f = gen.dense_operator(n, 1012, n_zero_m=8)
    b = gen.metric_diag(n, 1102)
    U, _ = gen.init_block(n, block + 2 * window, 7)
    op = L.lrep_create_dense(ctx, dev_colmajor(K, torch), dev_colmajor(M, torch), L.LREP_NULL_ON_M)
    L.lrep_set_metric(op, dev_colmajor(b, torch), ctx)           # device copy of b
    L.lrep_set_nullspace(op, np.asfortranarray(f.null_basis_M()), ctx)
    rc, st, lam, X, Y = gpu_solve(ctx, op, n, nev, block, tol, window=window, init=U)
    L.lrep_destroy_op(op)
    assert rc == L.LREP_OK, L.lrep_last_error(ctx)
    assert st.locks >= 1
    ref = G.generalized_spectrum(K, M, np.diag(b), nev, zeros=8)
    check_generalized(lam, X, Y, ref, K, M, b)
    # n0 in N(M): 0 = n0^T M y = lambda n0^T B x, so X is B-orthogonal to N(M)
    assert np.abs(f.null_basis_M().T @ (b[:, None] * X)).max() <= 1e-10


def test_lowrank_metric(ctx):
    n, r, nev, block, window, tol = 1500, 16, 32, 16, 8, 1e-9
    print(f"[metric] low rank n={n} rank={r}", flush=True)
    fc = gen.casida_factors(n, r, 1003)
    b = gen.metric_diag(n, 1103)
    U, _ = gen.init_block(n, block + 2 * window, 7)
    op = L.lrep_create_lowrank(ctx, dev_colmajor(fc.delta, torch), dev_colmajor(fc.L, torch))
    L.lrep_set_metric(op, b, ctx)
    rc, st, lam, X, Y = gpu_solve(ctx, op, n, nev, block, tol, window=window, init=U)
    L.lrep_destroy_op(op)
    assert rc == L.LREP_OK, L.lrep_last_error(ctx)
    K, M = fc.K(), fc.M()
    ref = G.generalized_spectrum(K, M, np.diag(b), nev)
    np.testing.assert_allclose(lam, ref, rtol=1e-10, atol=0)
    normH = np.linalg.norm(M, 2)
    res = G.generalized_residual(K, M, np.diag(b), X, Y, lam, normH=normH, normB=float(b.max()))
    # tol 1e-9 on the scaled pencil's relative residual
    assert res.max() <= 1e-8, res.max()
    assert G.b_biorth_error(np.diag(b), X, Y) <= 1e-12


def test_metric_rejections_leave_the_operator_unchanged(ctx):
    n, nev, block, tol = 128, 4, 8, 1e-10
    K, M, f = gen.dense_operator(n, 1001)
    U, _ = gen.init_block(n, 3 * block, 7)
    Kd, Md = dev_colmajor(K, torch), dev_colmajor(M, torch)
    op = L.lrep_create_dense(ctx, Kd, Md)
    good = gen.metric_diag(n, 1104)
    for bad_value in (0.0, -1.0, np.nan, np.inf):
        b = good.copy()
        b[17] = bad_value
        with pytest.raises(L.LrepError) as e:
            L.lrep_set_metric(op, b, ctx)
        assert e.value.code == L.LREP_EINVAL
    with pytest.raises(L.LrepError):
        L.lrep_set_metric(op, good[:-1], ctx)                    # wrong length
    # nothing was scaled: the standard spectrum
    rc, st, lam, X, Y = gpu_solve(ctx, op, n, nev, block, tol, init=U)
    assert rc == L.LREP_OK
    from oracle import exact
    np.testing.assert_allclose(lam, exact.dense_spectrum(f.q1, f.k, f.q2, f.m, nev), rtol=1e-10)
    L.lrep_set_metric(op, good, ctx)
    with pytest.raises(L.LrepError):
        L.lrep_set_metric(op, good, ctx)                         # only once
    L.lrep_destroy_op(op)
    # after the null space: refused (any X0 with X0^T M^-1 X0 SPD is accepted
    # by lrep_set_nullspace, which is all this needs)
    op = L.lrep_create_dense(ctx, Kd, Md)
    L.lrep_set_nullspace(op, np.ones((n, 1)), ctx)
    with pytest.raises(L.LrepError):
        L.lrep_set_metric(op, good, ctx)
    L.lrep_destroy_op(op)
    # a callback operator: refused (it applies the scaled pencil itself)
    op = L.lrep_create_callback(ctx, n, lambda *a: 0)
    with pytest.raises(L.LrepError):
        L.lrep_set_metric(op, good, ctx)
    L.lrep_destroy_op(op)
    # borrowed arrays: refused
    op = L.lrep_create_dense(ctx, Kd, Md, L.LREP_BORROW)
    with pytest.raises(L.LrepError):
        L.lrep_set_metric(op, good, ctx)
    L.lrep_destroy_op(op)


@pytest.mark.parametrize("n", [256, 300, 2048])
def test_dense_metric_matrix(ctx, n):
    """A dense SPD metric B (Haar eigenvectors, eigenvalues log-uniform on
    [0.25, 4]); n = 300 leaves a ragged last Cholesky block, n = 2048 runs the
    panel and trailing updates on the tall-skinny products."""
    nev, block, tol = 8, 16, 1e-10
    print(f"[metric] dense B n={n}", flush=True)
    K, M, f = gen.dense_operator(n, 1001 if n == 256 else 1020 + n)
    B = gen.metric_dense(n, 1107)
    U, _ = gen.init_block(n, 3 * block, 7)
    op = L.lrep_create_dense(ctx, dev_colmajor(K, torch), dev_colmajor(M, torch))
    L.lrep_set_metric_dense(op, B, ctx)
    rc, st, lam, X, Y = gpu_solve(ctx, op, n, nev, block, tol, init=U)
    L.lrep_destroy_op(op)
    assert rc == L.LREP_OK, L.lrep_last_error(ctx)
    ref = G.generalized_spectrum(K, M, B, nev)
    np.testing.assert_allclose(lam, ref, rtol=1e-10, atol=0)
    normH = max(np.linalg.norm(K, 2), np.linalg.norm(M, 2))
    res = G.generalized_residual(K, M, B, X, Y, lam, normH=normH, normB=np.linalg.norm(B, 2))
    assert res.max() <= 1e-8, res.max()
    assert G.b_biorth_error(B, X, Y) <= 1e-12


def test_dense_metric_matrix_zero_variant_found_null_space(ctx):
    n, nev, block, window, tol = 400, 24, 16, 8, 1e-10
    print(f"[metric] dense B zero variant n={n}", flush=True)
    K, M, f = gen.dense_operator(n, 1012, n_zero_m=8)
    B = gen.metric_dense(n, 1108)
    U, _ = gen.init_block(n, block + 2 * window, 7)
    op = L.lrep_create_dense(ctx, dev_colmajor(K, torch), dev_colmajor(M, torch), L.LREP_NULL_ON_M)
    L.lrep_set_metric_dense(op, dev_colmajor(B, torch), ctx)
    r, res = L.lrep_find_nullspace(op, 16, 1e-10, 12, ctx)
    assert r == 8 and res <= 1e-10
    rc, st, lam, X, Y = gpu_solve(ctx, op, n, nev, block, tol, window=window, init=U)
    L.lrep_destroy_op(op)
    assert rc == L.LREP_OK, L.lrep_last_error(ctx)
    ref = G.generalized_spectrum(K, M, B, nev, zeros=8)
    np.testing.assert_allclose(lam, ref, rtol=1e-10, atol=0)
    res = G.generalized_residual(K, M, B, X, Y, lam, normH=f.norm_H(), normB=np.linalg.norm(B, 2))
    assert res.max() <= 1e-8, res.max()
    assert G.b_biorth_error(B, X, Y) <= 1e-12
    # n0 in N(M): 0 = n0^T M y = lambda n0^T B x
    assert np.abs(f.null_basis_M().T @ (B @ X)).max() <= 1e-10


def test_dense_metric_matrix_declared_null_space(ctx):
    """The declared basis of N(M) in the original coordinates, with a dense B."""
    n, nev, block, window, tol = 400, 24, 16, 8, 1e-10
    K, M, f = gen.dense_operator(n, 1012, n_zero_m=8)
    B = gen.metric_dense(n, 1109)
    U, _ = gen.init_block(n, block + 2 * window, 7)
    op = L.lrep_create_dense(ctx, dev_colmajor(K, torch), dev_colmajor(M, torch), L.LREP_NULL_ON_M)
    L.lrep_set_metric_dense(op, B, ctx)
    L.lrep_set_nullspace(op, np.asfortranarray(f.null_basis_M()), ctx)
    rc, st, lam, X, Y = gpu_solve(ctx, op, n, nev, block, tol, window=window, init=U)
    L.lrep_destroy_op(op)
    assert rc == L.LREP_OK, L.lrep_last_error(ctx)
    np.testing.assert_allclose(lam, G.generalized_spectrum(K, M, B, nev, zeros=8), rtol=1e-10, atol=0)
    assert G.b_biorth_error(B, X, Y) <= 1e-12


def test_dense_metric_matrix_rejections(ctx):
    n = 128
    K, M, f = gen.dense_operator(n, 1001)
    op = L.lrep_create_dense(ctx, dev_colmajor(K, torch), dev_colmajor(M, torch))
    B = gen.metric_dense(n, 1110)
    Bbad = B.copy()
    Bbad[70, 70] = -5.0                        # indefinite
    with pytest.raises(L.LrepError) as e:
        L.lrep_set_metric_dense(op, np.asfortranarray(Bbad), ctx)
    assert e.value.code == L.LREP_EINVAL
    lam = np.zeros(4)
    X = np.zeros((n, 4), order="F")
    Y = np.zeros((n, 4), order="F")
    U, _ = gen.init_block(n, 24, 7)
    rc, st = L.lrep_solve(op, n, 4, 8, 1e-10, L.make_opts(init=np.asfortranarray(U)), lam, X, Y, ctx=ctx,
                          check=False)
    assert rc == L.LREP_OK
    from oracle import exact
    np.testing.assert_allclose(lam, exact.dense_spectrum(f.q1, f.k, f.q2, f.m, 4), rtol=1e-10)
    L.lrep_set_metric_dense(op, B, ctx)
    with pytest.raises(L.LrepError):
        L.lrep_set_metric(op, gen.metric_diag(n, 1), ctx)      # one metric per operator
    L.lrep_destroy_op(op)
    fc = gen.casida_factors(n, 4, 3)
    op = L.lrep_create_lowrank(ctx, dev_colmajor(fc.delta, torch), dev_colmajor(fc.L, torch))
    with pytest.raises(L.LrepError):
        L.lrep_set_metric_dense(op, B, ctx)                    # low rank: refused
    L.lrep_destroy_op(op)
