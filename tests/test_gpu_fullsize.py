"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times (same operators, start block, nev, block, window and tol).

The oracle cannot run BOSP itself at these sizes in test time, so the GPU
result is checked against what the oracle computes exactly for these
workloads:
  dense n = 8192       all 64 eigenvalues against the oracle's exact
                       spectrum (smallest eigenvalues of F^T F,
                       F = diag(sqrt k) Q1^T Q2 diag(sqrt m));
  zero variant         the same with 8 exact zeros in m, plus the
                       biorthogonality to the generalized null space;
  Casida n = 262144    every eigenvalue bracketed by the oracle's
                       Haynsworth inertia count (no eigenvalue skipped, each
                       within 1e-10 relative of the k-th);
  dense n = 32768      (mixed precision) all 64 eigenvalues against the
                       oracle's exact spectrum, stored by
                       tests/golden/make_dense32768_spectrum.py, for the
                       FP64, BF16 and FP16 CG applies, per-pair errors printed;
and, for all, the FP64 residual ||H z - lambda z|| / (||H|| ||z||) <= 1e-8
and max |Y^T X - I| <= 1e-12, evaluated on the host.
"""
import numpy as np
import pytest

import gen
from oracle import exact
import paper_2506_08355_amd as L
from gpu_util import h_residual

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    c = L.lrep_init(0)
    yield c
    L.lrep_finalize(c)


def solve(ctx, op, n, nev, block, window, tol, init, precision=0):
    lam = np.zeros(nev)
    X = np.zeros((n, nev), order="F")
    Y = np.zeros((n, nev), order="F")
    opts = L.make_opts(window=window, init=np.asfortranarray(init), precision=precision)
    rc, st = L.lrep_solve(op, n, nev, block, tol, opts, lam, X, Y, ctx=ctx, check=False)
    return rc, st, lam, X, Y


@pytest.mark.parametrize("zeros,seed,precision", [(0, 1002, 0), (8, 1012, 0), (0, 1002, 1), (0, 1002, 2),
                                                  (0, 1002, 3)],
                         ids=["dense8192", "dense8192_zero_variant", "dense8192_bf16_cg", "dense8192_fp16_cg",
                              "dense8192_bf16x3_cg"])
def test_config2_full_size(ctx, zeros, seed, precision):
    """The mixed-precision cases (CG applies in BF16 / FP16 / BF16x3) are held to the
    same bars: per pair, eigenvalue error against the exact spectrum <= 1e-10
    relative and FP64 residual <= 1e-8."""
    n, nev, block, window, tol = 8192, 64, 64, 32, 1e-10
    print(f"[fullsize] dense n={n} zeros={zeros} seed={seed}", flush=True)
    Kd, Md, k, m, Q1, Q2 = gen.dense_operator_device(n, seed, "cuda:0", n_zero_m=zeros, return_factors=True)
    U, _ = gen.init_block(n, block + 2 * window, 7)
    flags = L.LREP_NULL_ON_M if zeros else 0
    op = L.lrep_create_dense(ctx, Kd.T, Md.T, flags)      # symmetric: the transpose view is column-major
    q2 = Q2.cpu().numpy()
    null = np.asfortranarray(q2[:, m == 0.0])
    if zeros:
        L.lrep_set_nullspace(op, null, ctx)
    rc, st, lam, X, Y = solve(ctx, op, n, nev, block, window, tol, U, precision)
    L.lrep_destroy_op(op)
    assert rc == L.LREP_OK, L.lrep_last_error(ctx)
    print(f"[fullsize] iterations {st.iterations}", flush=True)
    K, M = Kd.cpu().numpy(), Md.cpu().numpy()
    del Kd, Md
    ref = exact.dense_spectrum_smallest(Q1.cpu().numpy(), k, q2, m, nev)
    np.testing.assert_allclose(lam, ref, rtol=1e-10, atol=0)
    res = h_residual(lambda v: K @ v, lambda v: M @ v, X, Y, lam, float(max(k.max(), m.max())))
    assert res.max() <= 1e-8, res.max()
    assert np.abs(X.T @ Y - np.eye(nev)).max() <= 1e-12
    if zeros:
        # Lemma 2.3 (iii): the returned X is biorthogonal to the null space of M
        assert np.abs(null.T @ X).max() <= 1e-10


@pytest.mark.parametrize("precision", [0, 4], ids=["fp64", "fp32_rows_cg"])
def test_config3_casida_full_size(ctx, precision):
    """The Casida workload at full size; precision 4 runs the Step-6 CG
    passes on the FP32 copy of L's rows and must meet the same bars."""
    n, r, nev, block, window, tol = 262144, 256, 128, 64, 32, 1e-8
    print(f"[fullsize] casida n={n} rank={r} precision={precision}", flush=True)
    f = gen.casida_factors(n, r, 1003)
    delta_d = torch.from_numpy(f.delta).to("cuda:0")
    L_d = torch.from_numpy(np.ascontiguousarray(f.L.T)).to("cuda:0").T
    U, _ = gen.init_block(n, block + 2 * window, 7)
    op = L.lrep_create_lowrank(ctx, delta_d, L_d)
    rc, st, lam, X, Y = solve(ctx, op, n, nev, block, window, tol, U, precision=precision)
    L.lrep_destroy_op(op)
    assert rc == L.LREP_OK, L.lrep_last_error(ctx)
    Lh, dl = f.L, f.delta

    def apply_M(v):
        return dl[:, None] * v + 2.0 * (Lh @ (Lh.T @ v))

    v = np.random.default_rng(5).standard_normal(n)
    for _ in range(40):                      # ||M||_2 (>= ||K||_2 = max delta) by power iteration
        v = apply_M(v[:, None])[:, 0]
        v /= np.linalg.norm(v)
    normH = float(v @ apply_M(v[:, None])[:, 0])
    res = h_residual(lambda x: dl[:, None] * x, apply_M, X, Y, lam, normH)
    assert res.max() <= 1e-8, res.max()
    assert np.abs(X.T @ Y - np.eye(nev)).max() <= 1e-12
    assert np.all(np.diff(lam) >= 0)
    # every eigenvalue bracketed by the inertia count: at most k - 1 eigenvalues
    # of H lie below lam_k (1 - 1e-10) and at least k below lam_k (1 + 1e-10),
    # so each lam_k is within 1e-10 relative of the k-th smallest eigenvalue
    lo = exact.casida_count_below_many(dl, Lh, lam * (1 - 1e-10))
    hi = exact.casida_count_below_many(dl, Lh, lam * (1 + 1e-10))
    bad = [kk for kk in range(1, nev + 1) if not (lo[kk - 1] <= kk - 1 and hi[kk - 1] >= kk)]
    print(f"[fullsize] casida: {nev - len(bad)} of {nev} eigenvalues bracketed at 1e-10", flush=True)
    assert not bad, [(kk, lo[kk - 1], hi[kk - 1]) for kk in bad[:10]]


def test_config2_full_size_metric(ctx):
    """The dense n = 8192 workload as a generalized LREP with a diagonal
    metric B (K x = lambda B y, M y = lambda B x): eigenvalues against the
    oracle's factored form, the pencil's backward error <= 1e-8 and
    max |Y^T B X - I| <= 1e-12."""
    from oracle import generalized as G
    n, nev, block, window, tol = 8192, 64, 64, 32, 1e-10
    print(f"[fullsize] dense n={n} metric", flush=True)
    Kd, Md, k, m, Q1, Q2 = gen.dense_operator_device(n, 1002, "cuda:0", return_factors=True)
    b = gen.metric_diag(n, 1105)
    U, _ = gen.init_block(n, block + 2 * window, 7)
    op = L.lrep_create_dense(ctx, Kd.T, Md.T)
    L.lrep_set_metric(op, b, ctx)
    rc, st, lam, X, Y = solve(ctx, op, n, nev, block, window, tol, U)
    L.lrep_destroy_op(op)
    assert rc == L.LREP_OK, L.lrep_last_error(ctx)
    print(f"[fullsize] iterations {st.iterations}", flush=True)
    K, M = Kd.cpu().numpy(), Md.cpu().numpy()
    del Kd, Md
    ref = G.dense_metric_spectrum_smallest(Q1.cpu().numpy(), k, Q2.cpu().numpy(), m, b, nev)
    np.testing.assert_allclose(lam, ref, rtol=1e-10, atol=0)
    B = np.diag(b)
    res = G.generalized_residual(K, M, B, X, Y, lam, normH=float(max(k.max(), m.max())), normB=float(b.max()))
    assert res.max() <= 1e-8, res.max()
    assert G.b_biorth_error(B, X, Y) <= 1e-12


def test_config2_zero_variant_found_null_space(ctx):
    """The zero variant at n = 8192 with N(M) computed on the device
    (lrep_find_nullspace) instead of declared: the same bars as with the
    declared basis, and X orthogonal to the true N(M)."""
    n, nev, block, window, tol = 8192, 64, 64, 32, 1e-10
    print(f"[fullsize] dense n={n} zero variant, found null space", flush=True)
    Kd, Md, k, m, Q1, Q2 = gen.dense_operator_device(n, 1012, "cuda:0", n_zero_m=8, return_factors=True)
    U, _ = gen.init_block(n, block + 2 * window, 7)
    op = L.lrep_create_dense(ctx, Kd.T, Md.T, L.LREP_NULL_ON_M)
    r, res = L.lrep_find_nullspace(op, 16, 1e-10, 21, ctx)
    assert r == 8 and res <= 1e-10, (r, res)
    rc, st, lam, X, Y = solve(ctx, op, n, nev, block, window, tol, U)
    L.lrep_destroy_op(op)
    assert rc == L.LREP_OK, L.lrep_last_error(ctx)
    K, M = Kd.cpu().numpy(), Md.cpu().numpy()
    del Kd, Md
    q2 = Q2.cpu().numpy()
    ref = exact.dense_spectrum_smallest(Q1.cpu().numpy(), k, q2, m, nev)
    np.testing.assert_allclose(lam, ref, rtol=1e-10, atol=0)
    res = h_residual(lambda v: K @ v, lambda v: M @ v, X, Y, lam, float(max(k.max(), m.max())))
    assert res.max() <= 1e-8, res.max()
    assert np.abs(X.T @ Y - np.eye(nev)).max() <= 1e-12
    assert np.abs(q2[:, m == 0.0].T @ X).max() <= 1e-10


GOLDEN32768 = "dense32768_seed1004_spectrum.txt"


@pytest.fixture(scope="module")
def dense32768(ctx):
    """The n = 32768 dense workload (seed 1004) on the device, borrowed by
    the operator (16 GiB of FP64 operators), and the oracle's spectrum."""
    import os
    from conftest import GOLDEN, load_golden
    if not os.path.exists(os.path.join(GOLDEN, GOLDEN32768)):
        pytest.skip("the n = 32768 spectrum has not been generated (tests/golden/make_dense32768_spectrum.py)")
    ref = load_golden(GOLDEN32768)[:, 1]
    n = 32768
    print(f"[fullsize] dense n={n} generating", flush=True)
    Kd, Md, k, m = gen.dense_operator_device(n, 1004, "cuda:0")
    op = L.lrep_create_dense(ctx, Kd.T, Md.T, L.LREP_BORROW)
    yield op, Kd, Md, float(max(k.max(), m.max())), ref
    L.lrep_destroy_op(op)
    del Kd, Md
    torch.cuda.empty_cache()


@pytest.mark.parametrize("precision", [0, 1, 2, 3], ids=["fp64", "bf16_cg", "fp16_cg", "bf16x3_cg"])
def test_config4_dense32768_full_size(ctx, dense32768, precision):
    """The mixed-precision configuration at its own size: n = 32768, nev 64,
    block 64, window 32, tol 1e-10, the CG applies of Step 6 in FP64, BF16,
    FP16 or BF16x3 (FP32 accumulation), everything else FP64.  Every eigenvalue
    within 1e-10 relative of the oracle's exact spectrum (the error of each
    pair is printed), residual <= 1e-8 and max |X^T Y - I| <= 1e-12 (device
    FP64 products, independent of the library)."""
    op, Kd, Md, normH, ref = dense32768
    n, nev, block, window, tol = 32768, 64, 64, 32, 1e-10
    U, _ = gen.init_block(n, block + 2 * window, 7)
    print(f"[fullsize] dense n={n} precision={precision}", flush=True)
    rc, st, lam, X, Y = solve(ctx, op, n, nev, block, window, tol, U, precision=precision)
    assert rc == L.LREP_OK, L.lrep_last_error(ctx)
    err = np.abs(lam - ref[:nev]) / ref[:nev]
    print(f"[fullsize] precision={precision} iterations {st.iterations}; relative eigenvalue error per pair: "
          + " ".join(f"{e:.1e}" for e in err), flush=True)
    assert err.max() <= 1e-10, err.max()
    Xd, Yd = torch.from_numpy(X).to("cuda:0"), torch.from_numpy(Y).to("cuda:0")
    ld = torch.from_numpy(lam).to("cuda:0")
    with torch.no_grad():
        R1 = Kd @ Xd - Yd * ld
        R2 = Md @ Yd - Xd * ld
        res = torch.sqrt((R1 ** 2).sum(0) + (R2 ** 2).sum(0)) / (normH * torch.sqrt((Xd ** 2).sum(0) + (Yd ** 2).sum(0)))
        bi = float((Xd.T @ Yd - torch.eye(nev, dtype=torch.float64, device="cuda:0")).abs().max())
    print(f"[fullsize] precision={precision} max residual {float(res.max()):.2e}, max |X^T Y - I| {bi:.2e}",
          flush=True)
    assert float(res.max()) <= 1e-8
    assert bi <= 1e-12
