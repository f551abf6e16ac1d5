"""Parity of the GPU solver (through the C ABI) with the FP64 CPU oracle on
the same seeded inputs and the same starting block.

Bars (from the build's accuracy contract):
  eigenvalues       |lambda_gpu - lambda_oracle| / lambda_oracle <= 1e-10
  residual          ||H z - lambda z|| / (||H|| ||z||) <= 1e-8, z = [y; x]
  biorthogonality   max |Y^T X - I| <= 1e-12 (looser where the paper's own
                    problem bounds it: eps ||H|| / lambda_min for tiny lambda)
"""
import numpy as np
import pytest

import gen
import oracle
import paper_2506_08355_amd as L
from oracle import exact
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


def gpu_solve(ctx, op, n, nev, block, tol, window=0, init=None, **kw):
    lam = np.zeros(nev)
    X = np.zeros((n, nev), order="F")
    Y = np.zeros((n, nev), order="F")
    opts = L.make_opts(window=window, init=None if init is None else np.asfortranarray(init), **kw)
    rc, st = L.lrep_solve(op, n, nev, block, tol, opts, lam, X, Y, ctx=ctx, check=False)
    return rc, st, lam, X, Y


def check_pair(lam, X, Y, ref_lam, K_apply, M_apply, normH, bi_tol=1e-12, lam_tol=1e-10):
    np.testing.assert_allclose(lam, ref_lam, rtol=lam_tol, atol=0)
    res = h_residual(K_apply, M_apply, X, Y, lam, normH)
    assert res.max() <= 1e-8, res.max()
    k = lam.size
    assert np.abs(X.T @ Y - np.eye(k)).max() <= bi_tol
    return res


def null_cosines(X0, Y0, X, Y):
    """Largest |cos| between the columns of Y0 and of X, and of X0 and of Y."""
    cy = np.abs(Y0.T @ X) / (np.linalg.norm(Y0, axis=0)[:, None] * np.linalg.norm(X, axis=0)[None, :])
    cx = np.abs(X0.T @ Y) / (np.linalg.norm(X0, axis=0)[:, None] * np.linalg.norm(Y, axis=0)[None, :])
    return float(cy.max()), float(cx.max())


# refresh=1 applies K and M to the whole subspace every iteration (the paper's
# cost model); the default carries the images between refreshes
REFRESH = [pytest.param(1, id="refresh1"), pytest.param(0, id="refresh_default")]


@pytest.mark.parametrize("refresh,precision", [pytest.param(1, 0, id="refresh1"),
                                               pytest.param(0, 0, id="refresh_default"),
                                               pytest.param(0, 1, id="bf16_cg_applies"),
                                               pytest.param(0, 2, id="fp16_cg_applies")])
def test_config1_dense_n256(ctx, refresh, precision):
    """Also with the CG applies in BF16 / FP16 (FP32 accumulate): the other
    steps stay FP64, so the eigenpairs must meet the same FP64 bars."""
    n, nev, block, tol = 256, 8, 16, 1e-10
    K, M, f = gen.dense_operator(n, 1001)
    U, _ = gen.init_block(n, 3 * block, 7)
    op = L.lrep_create_dense(ctx, dev_colmajor(K, torch), dev_colmajor(M, torch))
    rc, st, lam, X, Y = gpu_solve(ctx, op, n, nev, block, tol, init=U, refresh=refresh, precision=precision)
    L.lrep_destroy_op(op)
    assert rc == L.LREP_OK, L.lrep_last_error(ctx)
    ref = oracle.bosp_solve(oracle.DenseOperator(K, M), nev, block, tol, init=(U, U))
    check_pair(lam, X, Y, ref.lam, lambda v: K @ v, lambda v: M @ v, f.norm_H())
    np.testing.assert_allclose(lam, exact.dense_spectrum(f.q1, f.k, f.q2, f.m, nev), rtol=1e-10)
    # same eigenvectors as the oracle (both sign-normalised; spectrum is simple here)
    np.testing.assert_allclose(X, ref.X, atol=1e-7 * np.abs(ref.X).max())
    np.testing.assert_allclose(Y, ref.Y, atol=1e-7 * np.abs(ref.Y).max())
    assert st.n_converged == nev and st.max_eps <= tol


def test_config1_default_start_block(ctx):
    """The library's own Philox starting block reaches the same eigenpairs."""
    n, nev, block, tol = 256, 8, 16, 1e-10
    K, M, f = gen.dense_operator(n, 1001)
    op = L.lrep_create_dense(ctx, dev_colmajor(K, torch), dev_colmajor(M, torch))
    rc, st, lam, X, Y = gpu_solve(ctx, op, n, nev, block, tol, seed=12345)
    L.lrep_destroy_op(op)
    assert rc == L.LREP_OK, L.lrep_last_error(ctx)
    check_pair(lam, X, Y, exact.dense_spectrum(f.q1, f.k, f.q2, f.m, nev), lambda v: K @ v, lambda v: M @ v,
               f.norm_H())


def test_example_4_1(ctx):
    n = 1000
    T0 = gen.tridiag_T(n, 0.0)
    U, _ = gen.init_block(n, 30, 7)
    op = L.lrep_create_dense(ctx, dev_colmajor(T0, torch), dev_colmajor(T0, torch))
    rc, st, lam, X, Y = gpu_solve(ctx, op, n, 10, 10, 1e-10, init=U)
    L.lrep_destroy_op(op)
    assert rc == L.LREP_OK, L.lrep_last_error(ctx)
    printed = load_golden("example_4_1_eigenvalues.txt")[:, 1]
    check_pair(lam, X, Y, printed, lambda v: T0 @ v, lambda v: T0 @ v, 4.0)


def test_example_4_2_nullspace(ctx):
    n = 1000
    K = gen.tridiag_T(n, -1.0)
    M = gen.tridiag_T(n, 0.0)
    U, _ = gen.init_block(n, 30, 7)
    op = L.lrep_create_dense(ctx, dev_colmajor(K, torch), dev_colmajor(M, torch))
    L.lrep_set_nullspace(op, np.ones((n, 1)), ctx)
    rc, st, lam, X, Y = gpu_solve(ctx, op, n, 10, 10, 1e-10, init=U)
    L.lrep_destroy_op(op)
    assert rc == L.LREP_OK, L.lrep_last_error(ctx)
    printed = load_golden("example_4_2_eigenvalues.txt")[:, 1]
    check_pair(lam, X, Y, printed, lambda v: K @ v, lambda v: M @ v, 4.0)
    # Lemma 2.3 (iii): the pairs of nonzero eigenvalues are biorthogonal to the
    # generalized null space, Y0^T x = 0 and X0^T y = 0 (X0^T Y0 = I basis),
    # measured as cosines
    X0, Y0 = oracle.nullspace_basis(np.ones((n, 1)), oracle.DenseOperator(K, M).solve_M)
    cy, cx = null_cosines(X0, Y0, X, Y)
    print(f"Lemma 2.3 (iii): max cos(Y0, x) = {cy:.2e}, max cos(X0, y) = {cx:.2e}")
    assert cy <= 1e-12 and cx <= 1e-12, (cy, cx)


@pytest.mark.parametrize("refresh", REFRESH)
def test_zero_variant_role_swap_moving(ctx, refresh):
    n, nev, block, window, tol = 400, 24, 16, 8, 1e-10
    K, M, f = gen.dense_operator(n, 1012, n_zero_m=8)
    U, _ = gen.init_block(n, block + 2 * window, 7)
    op = L.lrep_create_dense(ctx, dev_colmajor(K, torch), dev_colmajor(M, torch), L.LREP_NULL_ON_M)
    L.lrep_set_nullspace(op, np.asfortranarray(f.null_basis_M()), ctx)
    rc, st, lam, X, Y = gpu_solve(ctx, op, n, nev, block, tol, window=window, init=U, refresh=refresh)
    L.lrep_destroy_op(op)
    assert rc == L.LREP_OK, L.lrep_last_error(ctx)
    assert st.locks >= 1
    ref = oracle.bosp_solve(oracle.DenseOperator(K, M), nev, block, tol, window=window, init=(U, U),
                            X0=f.null_basis_M(), null_on_M=True)
    check_pair(lam, X, Y, ref.lam, lambda v: K @ v, lambda v: M @ v, f.norm_H())
    np.testing.assert_allclose(lam, exact.dense_spectrum(f.q1, f.k, f.q2, f.m, nev), rtol=1e-10)
    assert np.abs(f.null_basis_M().T @ X).max() <= 1e-10


@pytest.mark.parametrize("refresh", REFRESH)
def test_casida_lowrank_moving(ctx, refresh):
    n, r, nev, block, window, tol = 1500, 16, 32, 16, 8, 1e-9
    f = gen.casida_factors(n, r, 1003)
    U, _ = gen.init_block(n, block + 2 * window, 7)
    op = L.lrep_create_lowrank(ctx, dev_colmajor(f.delta, torch), dev_colmajor(f.L, torch))
    rc, st, lam, X, Y = gpu_solve(ctx, op, n, nev, block, tol, window=window, init=U, refresh=refresh)
    L.lrep_destroy_op(op)
    assert rc == L.LREP_OK, L.lrep_last_error(ctx)
    cop = oracle.CasidaOperator(f.delta, f.L)
    ref = oracle.bosp_solve(cop, nev, block, tol, window=window, init=(U, U))
    normH = np.linalg.norm(f.M(), 2)
    check_pair(lam, X, Y, ref.lam, cop.apply_K, cop.apply_M, normH)
    assert exact.casida_count_below(f.delta, f.L, lam[-1] * (1 + 1e-9)) == nev


@pytest.mark.parametrize("n,r,fused", [(1500, 16, 1), (1500, 16, -1), (1502, 100, 1), (3002, 256, 1),
                                       (1501, 100, 1), (2048, 64, 1)])
def test_casida_fused_cg(ctx, n, r, fused):
    """The Step-6 CG on the low-rank operator as one pass per step (fused=1,
    the default: L read once per step, L^T p carried by the direction
    recurrence) and as the plain two-pass CG (fused=-1): both meet the oracle's
    eigenvalues, residual and biorthogonality bars.  Ragged row tiles (n = 1502,
    3002), ranks whose row copy has 1, 2 or 4 wavefronts of columns (16, 100,
    256) and an odd n (1501, which takes the plain CG) are covered."""
    nev, block, window, tol = 16, 16, 8, 1e-9
    print(f"[fused cg] n={n} rank={r} fused={fused}", flush=True)
    f = gen.casida_factors(n, r, 1000 + r)
    U, _ = gen.init_block(n, block + 2 * window, 7)
    op = L.lrep_create_lowrank(ctx, dev_colmajor(f.delta, torch), dev_colmajor(f.L, torch))
    rc, st, lam, X, Y = gpu_solve(ctx, op, n, nev, block, tol, window=window, init=U, fused_cg=fused)
    L.lrep_destroy_op(op)
    assert rc == L.LREP_OK, L.lrep_last_error(ctx)
    cop = oracle.CasidaOperator(f.delta, f.L)
    ref = oracle.bosp_solve(cop, nev, block, tol, window=window, init=(U, U))
    normH = np.linalg.norm(f.M(), 2)
    check_pair(lam, X, Y, ref.lam, cop.apply_K, cop.apply_M, normH)
    assert exact.casida_count_below(f.delta, f.L, lam[-1] * (1 + 1e-9)) == nev
    assert st.applies_M > 0 and st.applies_K > 0


@pytest.mark.parametrize("n,r", [(1502, 100), (3002, 256), (2048, 64)])
def test_casida_fused_cg_fp32_rows(ctx, n, r):
    """precision 4: the fused CG passes read an FP32 copy of L's rows (only
    the Step-6 CG changes, by ~1e-7 relative against its 1e-2 tolerance); the
    returned pairs meet the same oracle bars as the FP64 solve.  Ragged row
    tiles (1502, 3002) and 1, 2 or 4 wavefronts of columns (64, 100, 256)."""
    nev, block, window, tol = 16, 16, 8, 1e-9
    print(f"[fused cg fp32 rows] n={n} rank={r}", flush=True)
    f = gen.casida_factors(n, r, 1000 + r)
    U, _ = gen.init_block(n, block + 2 * window, 7)
    op = L.lrep_create_lowrank(ctx, dev_colmajor(f.delta, torch), dev_colmajor(f.L, torch))
    rc, st, lam, X, Y = gpu_solve(ctx, op, n, nev, block, tol, window=window, init=U, precision=4)
    L.lrep_destroy_op(op)
    assert rc == L.LREP_OK, L.lrep_last_error(ctx)
    cop = oracle.CasidaOperator(f.delta, f.L)
    ref = oracle.bosp_solve(cop, nev, block, tol, window=window, init=(U, U))
    normH = np.linalg.norm(f.M(), 2)
    check_pair(lam, X, Y, ref.lam, cop.apply_K, cop.apply_M, normH)
    assert exact.casida_count_below(f.delta, f.L, lam[-1] * (1 + 1e-9)) == nev


def test_fp32_rows_only_for_low_rank(ctx):
    """precision 4 on a dense operator is rejected before any work, and
    precision 5 on any operator."""
    n = 256
    K, M, _ = gen.dense_operator(n, 3)
    op = L.lrep_create_dense(ctx, dev_colmajor(K, torch), dev_colmajor(M, torch))
    rc, *_ = gpu_solve(ctx, op, n, 4, 8, 1e-8, precision=4)
    assert rc == L.LREP_EINVAL
    rc, *_ = gpu_solve(ctx, op, n, 4, 8, 1e-8, precision=5)
    assert rc == L.LREP_EINVAL
    L.lrep_destroy_op(op)


def test_error_paths(ctx):
    n = 64
    K, M, f = gen.dense_operator(n, 3)
    op = L.lrep_create_dense(ctx, dev_colmajor(K, torch), dev_colmajor(M, torch))
    # block too large for the device's small solver
    rc, *_ = gpu_solve(ctx, op, n, 4, 60, 1e-8)
    assert rc == L.LREP_EINVAL
    # n mismatch
    lam = np.zeros(4); X = np.zeros((n, 4), order="F"); Y = np.zeros((n, 4), order="F")
    rc, _ = L.lrep_solve(op, n + 1, 4, 4, 1e-8, L.make_opts(), lam, X, Y, check=False)
    assert rc == L.LREP_EINVAL
    # maxit reached: converged prefix only
    rc, st, lam, X, Y = gpu_solve(ctx, op, n, 4, 4, 1e-14, maxit=2)
    assert rc == L.LREP_ENOTCONV and st.iterations == 2
    L.lrep_destroy_op(op)
    # NaN in the operator
    Kn = K.copy(); Kn[3, 5] = np.nan
    op = L.lrep_create_dense(ctx, dev_colmajor(Kn, torch), dev_colmajor(M, torch))
    rc, *_ = gpu_solve(ctx, op, n, 4, 4, 1e-8)
    assert rc in (L.LREP_ENUMERIC, L.LREP_ENOTSPD)
    L.lrep_destroy_op(op)


@pytest.mark.parametrize("null_on_m", [False, True], ids=["km", "role_swap"])
def test_callback_operator(ctx, null_on_m):
    """Matrix-free operator (lrep_create_callback): the products come from a
    caller function, here one that forwards to a dense operator's apply on
    the same context (so on the solve's stream).  The solve takes the
    generic CG path and must reach the oracle's eigenpairs of config 1; with
    the role flag the function is asked for the exchanged operators."""
    n, nev, block, tol = 256, 8, 16, 1e-10
    K, M, f = gen.dense_operator(n, 1001)
    U, _ = gen.init_block(n, 3 * block, 7)
    inner = L.lrep_create_dense(ctx, dev_colmajor(K, torch), dev_colmajor(M, torch))
    calls = {"K": 0, "M": 0}

    def apply(which, cols, X, ldx, Y, ldy, stream):
        if ldx != n or ldy != n:
            return 1
        calls["K" if which == 0 else "M"] += 1
        return L.lib().lrep_test_apply(inner, which, cols, X, Y)

    # with the role flag the library exchanges the roles inside and back on
    # return: the function still sees which = 0 as K, and X, Y come back in
    # the caller's roles
    flags = L.LREP_NULL_ON_M if null_on_m else 0
    op = L.lrep_create_callback(ctx, n, apply, flags)
    rc, st, lam, X, Y = gpu_solve(ctx, op, n, nev, block, tol, init=U)
    L.lrep_destroy_op(op)
    L.lrep_destroy_op(inner)
    assert rc == L.LREP_OK, L.lrep_last_error(ctx)
    assert calls["K"] > 0 and calls["M"] > 0
    ref_lam = exact.dense_spectrum(f.q1, f.k, f.q2, f.m, nev)
    check_pair(lam, X, Y, ref_lam, lambda v: K @ v, lambda v: M @ v, f.norm_H())
    assert st.n_converged == nev


def test_callback_error_ends_solve(ctx):
    """A product function that reports failure ends the solve with
    LREP_EDEVICE and a message naming the callback (no device fault)."""
    n = 256

    def apply(which, cols, X, ldx, Y, ldy, stream):
        return 7

    op = L.lrep_create_callback(ctx, n, apply)
    U, _ = gen.init_block(n, 48, 7)
    rc, st, lam, X, Y = gpu_solve(ctx, op, n, 8, 16, 1e-10, init=U)
    L.lrep_destroy_op(op)
    assert rc == L.LREP_EDEVICE
    assert "callback" in L.lrep_last_error(ctx)


@pytest.mark.parametrize("case", ["dense", "zero_variant", "lowrank", "bf16"])
def test_step6_graph_replay_is_bitwise_the_stream_path(ctx, case):
    """Step 6 captured as a HIP graph and replayed gives bitwise the results
    of issuing the same launches on the stream (each replay reruns every CG
    step; steps after convergence return at once on the device flag)."""
    print(f"[graphs] {case}", flush=True)
    if case == "lowrank":
        n, nev, block, window, tol = 1500, 16, 16, 8, 1e-9
        f = gen.casida_factors(n, 16, 1003)
        make = lambda: L.lrep_create_lowrank(ctx, dev_colmajor(f.delta, torch), dev_colmajor(f.L, torch))
    elif case == "zero_variant":
        n, nev, block, window, tol = 400, 24, 16, 8, 1e-10
        K, M, f = gen.dense_operator(n, 1012, n_zero_m=8)

        def make():
            op = L.lrep_create_dense(ctx, dev_colmajor(K, torch), dev_colmajor(M, torch), L.LREP_NULL_ON_M)
            L.lrep_set_nullspace(op, np.asfortranarray(f.null_basis_M()), ctx)
            return op
    else:
        n, nev, block, window, tol = 256, 8, 16, 16, 1e-10
        K, M, f = gen.dense_operator(n, 1001)
        make = lambda: L.lrep_create_dense(ctx, dev_colmajor(K, torch), dev_colmajor(M, torch))
    U, _ = gen.init_block(n, block + 2 * window, 7)
    out = []
    for graphs in (-1, 1):
        op = make()
        rc, st, lam, X, Y = gpu_solve(ctx, op, n, nev, block, tol, window=window, init=U, graphs=graphs,
                                      precision=1 if case == "bf16" else 0)
        L.lrep_destroy_op(op)
        assert rc == L.LREP_OK, L.lrep_last_error(ctx)
        out.append((lam, X, Y, st.iterations))
    assert out[0][3] == out[1][3]
    for a, b in zip(out[0][:3], out[1][:3]):
        assert np.array_equal(a, b)


def test_xy_to_uv_solves_the_original_problem(ctx):
    """u = y + x, v = y - x (Section 1) solve [[A, B], [-B, -A]] [u; v] =
    lambda [u; v] with A = (K + M) / 2, B = (M - K) / 2."""
    n, nev, block, tol = 256, 8, 16, 1e-10
    K, M, f = gen.dense_operator(n, 1001)
    U0, _ = gen.init_block(n, 3 * block, 7)
    op = L.lrep_create_dense(ctx, dev_colmajor(K, torch), dev_colmajor(M, torch))
    lam = torch.zeros(nev, dtype=torch.float64, device="cuda:0")
    X = torch.zeros(nev, n, dtype=torch.float64, device="cuda:0").T
    Y = torch.zeros(nev, n, dtype=torch.float64, device="cuda:0").T
    opts = L.make_opts(init=np.asfortranarray(U0), result_on_device=True)
    L.lrep_solve(op, n, nev, block, tol, opts, lam, X, Y, ctx=ctx)
    L.lrep_destroy_op(op)
    Ud = torch.zeros(nev, n, dtype=torch.float64, device="cuda:0").T
    Vd = torch.zeros(nev, n, dtype=torch.float64, device="cuda:0").T
    L.lrep_xy_to_uv(ctx, X, Y, Ud, Vd)
    u, v, x, y, lm = (t.cpu().numpy() for t in (Ud, Vd, X, Y, lam))
    np.testing.assert_array_equal(u, y + x)
    np.testing.assert_array_equal(v, y - x)
    A, B = 0.5 * (K + M), 0.5 * (M - K)
    R1 = A @ u + B @ v - u * lm
    R2 = -B @ u - A @ v - v * lm
    res = np.sqrt((R1 ** 2).sum(0) + (R2 ** 2).sum(0)) / (f.norm_H() * np.sqrt((u ** 2).sum(0) + (v ** 2).sum(0)))
    assert res.max() <= 1e-8, res.max()
