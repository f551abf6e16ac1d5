"""Kernel-level GPU tests through the testing entry points of the C ABI,
against plain FP64 NumPy (and the oracle's small LREP / MGS-Biorth)."""
import numpy as np
import pytest

import gen
import oracle
import paper_2506_08355_amd as L
from gpu_util import dev_colmajor, dev_empty, host

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    c = L.lrep_init(0)
    yield c
    L.lrep_finalize(c)


@pytest.mark.parametrize("m,p,q,ksplit,beta", [
    (16, 4, 16, 0, 0.0), (300, 257, 33, 0, 0.0), (1000, 1000, 32, 4, 0.0), (129, 48, 16, 0, 0.5),
    (517, 130, 100, 0, 0.0), (4096, 4096, 32, 0, 0.0), (2048, 2048, 128, 0, 0.0),
    (8192, 192, 64, 0, 0.5), (1000, 37, 19, 0, 0.0), (600, 1024, 8, 0, -1.0), (513, 3, 1, 0, 0.0)])
def test_gemm_nn(ctx, m, p, q, ksplit, beta):
    """Tall-skinny shapes (m >= 512, k <= 1024) take the register-direct
    kernel: k in whole 16-deep units split over four waves plus a partial
    unit (37, 130, 3), ragged row and column blocks (1000 x 19, 517 x 100);
    large k and explicit splits take the LDS-tiled kernel."""
    rng = np.random.default_rng(m + p + q)
    A = rng.standard_normal((m, p))
    B = rng.standard_normal((p, q))
    C0 = rng.standard_normal((m, q))
    Ad, Bd, Cd = dev_colmajor(A, torch), dev_colmajor(B, torch), dev_colmajor(C0, torch)
    torch.cuda.synchronize()
    L.lrep_test_gemm_nn(ctx, Ad, Bd, Cd, alpha=1.5, beta=beta, ksplit=ksplit)
    ref = 1.5 * A @ B + beta * C0
    scale = np.sqrt(max(p, 1)) * 4
    np.testing.assert_allclose(host(Cd), ref, atol=1e-14 * scale * 8, rtol=0)


@pytest.mark.parametrize("n,p,q,sym", [(64, 16, 16, False), (5000, 70, 33, False), (8192, 128, 128, True),
                                       (100003, 32, 64, False), (3, 5, 7, False), (8192, 192, 32, False),
                                       (1000, 257, 17, False), (513, 5, 3, False), (262144, 256, 64, False)])
def test_gemm_tn(ctx, n, p, q, sym):
    """n >= 512 takes the register-direct Gram kernel: row splits with a
    ragged last unit (100003, 1000, 513), narrow (q <= 32) and wide column
    blocks, ragged output blocks (257, 33, 17), symmetrisation."""
    rng = np.random.default_rng(n + p)
    A = rng.standard_normal((n, p))
    B = A[:, :q] + 0.1 * rng.standard_normal((n, q)) if sym else rng.standard_normal((n, q))
    Cd = dev_empty(p, q, torch)
    L.lrep_test_gemm_tn(ctx, dev_colmajor(A, torch), dev_colmajor(B, torch), Cd, symmetrize=sym)
    ref = A.T @ B
    if sym:
        ref = 0.5 * (ref + ref.T)
    np.testing.assert_allclose(host(Cd), ref, atol=1e-13 * np.sqrt(n) * 4, rtol=0)


def _spd(rng, d, cond):
    q, _ = np.linalg.qr(rng.standard_normal((d, d)))
    return (q * np.geomspace(1.0, cond, d)) @ q.T


@pytest.mark.parametrize("d,cond", [(1, 1.0), (10, 10.0), (30, 1e3), (32, 10.0), (33, 1e2), (48, 1e4), (64, 1e2),
                                    (65, 1e3), (100, 1e3), (127, 10.0), (128, 1e5)])
def test_small_lrep_against_oracle(ctx, d, cond):
    rng = np.random.default_rng(d)
    Kh, Mh = _spd(rng, d, cond), _spd(rng, d, cond)
    lam = torch.zeros(d, dtype=torch.float64, device="cuda:0")
    Xh = dev_empty(128, 128, torch)
    Yh = dev_empty(128, 128, torch)
    rc = L.lrep_test_small_lrep(ctx, dev_colmajor(Kh, torch), dev_colmajor(Mh, torch), lam, Xh, Yh)
    assert rc == L.LREP_OK
    lam_h, X, Y = host(lam), host(Xh)[:d, :d], host(Yh)[:d, :d]
    ref, _, _ = oracle.small_lrep(Kh, Mh, d)
    np.testing.assert_allclose(lam_h, ref, rtol=1e-12 * cond)
    np.testing.assert_allclose(X.T @ Y, np.eye(d), atol=1e-12 * cond)
    scale = np.abs(Kh).max() + np.abs(Mh).max()
    assert np.abs(Kh @ X - Y * lam_h).max() <= 1e-11 * scale * max(np.abs(X).max(), 1)
    assert np.abs(Mh @ Y - X * lam_h).max() <= 1e-11 * scale * max(np.abs(Y).max(), 1)


@pytest.mark.parametrize("d", [37, 100, 128])
def test_small_lrep_uses_the_symmetric_part(ctx, d):
    """The projected matrices are symmetric only up to rounding (K^ = U^T (K U)
    with carried images); the small solver factors their symmetric parts
    (K^ + K^T)/2.  A non-symmetric perturbation of relative size 1e-3 makes
    a factorisation of one triangle alone (or of one element twice) move the
    eigenvalues by ~8e-4, far above the 1e-10 tolerance."""
    rng = np.random.default_rng(500 + d)
    Kh = _spd(rng, d, 1e2) + 1e-3 * rng.standard_normal((d, d))
    Mh = _spd(rng, d, 1e2) + 1e-3 * rng.standard_normal((d, d))
    lam = torch.zeros(d, dtype=torch.float64, device="cuda:0")
    Xh, Yh = dev_empty(128, 128, torch), dev_empty(128, 128, torch)
    rc = L.lrep_test_small_lrep(ctx, dev_colmajor(Kh, torch), dev_colmajor(Mh, torch), lam, Xh, Yh)
    assert rc == L.LREP_OK
    lam_h, X, Y = host(lam), host(Xh)[:d, :d], host(Yh)[:d, :d]
    ref, _, _ = oracle.small_lrep(Kh, Mh, d)
    np.testing.assert_allclose(lam_h, ref, rtol=1e-10)
    Ks, Ms = 0.5 * (Kh + Kh.T), 0.5 * (Mh + Mh.T)
    scale = np.abs(Ks).max() + np.abs(Ms).max()
    assert np.abs(Ks @ X - Y * lam_h).max() <= 1e-11 * scale * max(np.abs(X).max(), 1)
    assert np.abs(Ms @ Y - X * lam_h).max() <= 1e-11 * scale * max(np.abs(Y).max(), 1)


def test_small_lrep_reports_not_spd(ctx):
    d = 6
    Kh = np.diag([1.0, 2.0, -1.0, 3.0, 1.0, 1.0])
    lam = torch.zeros(d, dtype=torch.float64, device="cuda:0")
    Xh, Yh = dev_empty(128, 128, torch), dev_empty(128, 128, torch)
    rc = L.lrep_test_small_lrep(ctx, dev_colmajor(Kh, torch), dev_colmajor(np.eye(d), torch), lam, Xh, Yh)
    assert rc == L.LREP_ENOTSPD


@pytest.mark.parametrize("n,m,same", [(200, 7, True), (5000, 32, False), (3000, 128, True), (1000, 48, False)])
def test_block_mgs_biorth(ctx, n, m, same):
    rng = np.random.default_rng(n + m)
    X = rng.standard_normal((n, m))
    Y = X.copy() if same else X + 0.5 * rng.standard_normal((n, m))
    Xd, Yd = dev_colmajor(X, torch).T.contiguous().T, dev_colmajor(Y, torch).T.contiguous().T
    k = L.lrep_test_block_mgs(ctx, Xd, Yd)
    assert k == m
    P, Q = host(Xd)[:, :k], host(Yd)[:, :k]
    np.testing.assert_allclose(P.T @ Q, np.eye(m), atol=1e-12)
    # same spans as the inputs (X = P R with R upper triangular)
    R = Q.T @ X
    np.testing.assert_allclose(np.tril(R, -1), 0, atol=1e-10 * np.abs(R).max())
    if same:                      # MGS-Biorth with Y = X is MGS orthogonalisation
        q, r = np.linalg.qr(X)
        q *= np.sign(np.diag(r))
        np.testing.assert_allclose(P, q, atol=1e-12)
    Po, Qo, kept = oracle.mgs_biorth(X, Y)
    np.testing.assert_allclose(P, Po, atol=1e-9 * np.abs(Po).max())
    np.testing.assert_allclose(Q, Qo, atol=1e-9 * np.abs(Qo).max())


@pytest.mark.parametrize("row", list(range(5)))
def test_block_mgs_biorth_ill_conditioned_table(ctx, row):
    """The inputs of the paper's table of biorthogonality loss (Section 3.1):
    X = the first m columns of the n x n Hilbert matrix, Y = the first m
    columns of the Lauchli matrix (mu = 1e-3), m = n / 2, n = 4 ... 20, with
    zero rows appended up to 64 (inner products unchanged).  The block form
    (two coefficient passes) must lose no more biorthogonality than the
    paper's column-by-column MGS-Biorth (its printed ||P^T Q - I||_2) and keep
    every pair the oracle keeps; at n = 20 the second pass may drop the last
    pair, whose pivot after the first pass is below the near-orthogonality
    bar (|eta| <= 1e-10 ||p|| ||q||)."""
    from conftest import load_golden
    tab = load_golden("biorth_loss_table.txt")
    n, mgs_printed = int(tab[row][0]), tab[row][5]
    m = n // 2
    X = np.zeros((64, m))
    Y = np.zeros((64, m))
    X[:n] = gen.hilbert(n)[:, :m]
    Y[:n] = gen.lauchli(n, 1e-3)[:, :m]
    Xd, Yd = dev_colmajor(X, torch).T.contiguous().T, dev_colmajor(Y, torch).T.contiguous().T
    print(f"[mgs table] n={n} m={m}", flush=True)
    k = L.lrep_test_block_mgs(ctx, Xd, Yd)
    P, Q = host(Xd)[:, :k], host(Yd)[:, :k]
    loss = np.linalg.norm(P.T @ Q - np.eye(k), 2) if k else 0.0
    Po, Qo, kept = oracle.mgs_biorth(X, Y)
    oloss = np.linalg.norm(Po.T @ Qo - np.eye(len(kept)), 2)
    print(f"[mgs table] n={n}: block kept {k}/{m}, loss {loss:.2e}; oracle MGS kept {len(kept)}, loss {oloss:.2e}; "
          f"printed MGS {mgs_printed:.2e}", flush=True)
    assert np.all(P[n:] == 0.0) and np.all(Q[n:] == 0.0)
    assert k == len(kept) or (n == 20 and k == len(kept) - 1), (k, len(kept))
    assert loss <= mgs_printed, (loss, mgs_printed)
    # the kept columns still span the inputs (least-squares residual of X in span(P))
    c = np.linalg.lstsq(P, X, rcond=None)[0]
    assert np.abs(X - P @ c).max() <= 1e-9 * np.abs(X).max()


def test_block_mgs_drops_dependent_columns(ctx):
    rng = np.random.default_rng(11)
    X = rng.standard_normal((500, 6))
    X[:, 3] = X[:, 0] - 2 * X[:, 1]
    Xd = dev_colmajor(X, torch).T.contiguous().T
    Yd = Xd.clone().T.contiguous().T
    k = L.lrep_test_block_mgs(ctx, Xd, Yd)
    assert k == 5
    P, Q = host(Xd)[:, :k], host(Yd)[:, :k]
    np.testing.assert_allclose(P.T @ Q, np.eye(5), atol=1e-12)


@pytest.mark.parametrize("kind,n,cols", [("dense", 1500, 19), ("dense", 1501, 32), ("dense", 4096, 32),
                                         ("dense", 700, 48), ("lowrank24", 1500, 19), ("lowrank24", 1501, 19),
                                         ("lowrank256", 5002, 32),
                                         ("lowrank100", 4098, 70), ("lowrank256", 262144, 32),
                                         ("dense_swap", 1500, 19)])
def test_operator_apply(ctx, kind, n, cols):
    """Dense applies with <= 32 columns and an even leading dimension take the
    streaming kernel (ragged row tiles at 1500), odd n and wide blocks the
    tiled product.  Low-rank M applies take the two streaming passes (L^T Y,
    then L T + delta o Y) 32 columns at a time: rank below one wavefront's 64
    columns, not a multiple of 16, the full 256; rows not a multiple of the
    8-row step (5002: leftover rows and a ragged last row tile); odd n falls
    back to the tiled product (1501); the full-size n = 262144."""
    rng = np.random.default_rng(5)
    Xh = rng.standard_normal((n, cols))
    if kind.startswith("lowrank"):
        f = gen.casida_factors(n, int(kind[7:]), 3)
        op = L.lrep_create_lowrank(ctx, dev_colmajor(f.delta, torch), dev_colmajor(f.L, torch))
        dl, Lf = f.delta, f.L

        class _Op:   # K = diag(delta), M = diag(delta) + 2 L L^T without forming n x n
            def __init__(self, m):
                self.m = m

            def __matmul__(self, x):
                return dl[:, None] * x + (2.0 * (Lf @ (Lf.T @ x)) if self.m else 0.0)

        K, M = _Op(False), _Op(True)
    else:
        K, M, _ = gen.dense_operator(n, 4)
        flags = L.LREP_NULL_ON_M if kind == "dense_swap" else 0
        op = L.lrep_create_dense(ctx, dev_colmajor(K, torch), dev_colmajor(M, torch), flags)
        if kind == "dense_swap":
            K, M = M, K
    Xd = dev_colmajor(Xh, torch).T.contiguous().T
    Yd = dev_empty(n, cols, torch).T.contiguous().T
    for which, A in ((0, K), (1, M)):
        L.lrep_test_apply(op, which, Xd, Yd)
        np.testing.assert_allclose(host(Yd), A @ Xh, atol=1e-12 * np.abs(A @ Xh).max())
    L.lrep_destroy_op(op)


def test_input_ab_forms_k_and_m(ctx):
    rng = np.random.default_rng(8)
    n = 200
    A = rng.standard_normal((n, n)); A = A + A.T
    B = rng.standard_normal((n, n)); B = B + B.T
    op = L.lrep_create_dense(ctx, dev_colmajor(A, torch), dev_colmajor(B, torch), L.LREP_INPUT_AB)
    X = rng.standard_normal((n, 3))
    Xd = dev_colmajor(X, torch).T.contiguous().T
    Yd = dev_empty(n, 3, torch).T.contiguous().T
    L.lrep_test_apply(op, 0, Xd, Yd)
    np.testing.assert_allclose(host(Yd), (A - B) @ X, atol=1e-11)
    L.lrep_test_apply(op, 1, Xd, Yd)
    np.testing.assert_allclose(host(Yd), (A + B) @ X, atol=1e-11)
    L.lrep_destroy_op(op)


@pytest.mark.parametrize("d", [24, 96, 128])
def test_small_lrep_clustered_spectrum(ctx, d):
    """Clustered Ritz values (K^ = M^ = I + small symmetric noise): many
    near-equal singular values of B, where Jacobi takes 45-degree rotations."""
    rng = np.random.default_rng(7 * d)
    e = rng.standard_normal((d, d)) * 1e-6
    Kh = np.eye(d) + 0.5 * (e + e.T)
    Mh = np.eye(d) + 1e-3 * np.diag(np.repeat([0.0, 1.0], (d + 1) // 2)[:d])
    lam = torch.zeros(d, dtype=torch.float64, device="cuda:0")
    Xh, Yh = dev_empty(128, 128, torch), dev_empty(128, 128, torch)
    rc = L.lrep_test_small_lrep(ctx, dev_colmajor(Kh, torch), dev_colmajor(Mh, torch), lam, Xh, Yh)
    assert rc == L.LREP_OK
    lam_h, X, Y = host(lam), host(Xh)[:d, :d], host(Yh)[:d, :d]
    ref, _, _ = oracle.small_lrep(Kh, Mh, d)
    np.testing.assert_allclose(lam_h, ref, rtol=1e-13)
    np.testing.assert_allclose(X.T @ Y, np.eye(d), atol=1e-12)
    assert np.abs(Kh @ X - Y * lam_h).max() <= 1e-12
    assert np.abs(Mh @ Y - X * lam_h).max() <= 1e-12



def _round16(x, precision):
    """Host rounding of FP64 values the way the 16-bit copies are made: one
    rounding to nearest even straight to BF16 (8 significant bits, normal
    exponents from -126) or FP16 (11 bits, from -14, subnormals below),
    done in FP64 arithmetic (exact scaling by the quantum, then rint)."""
    p, emin = (8, -126) if precision == 1 else (11, -14)
    x = np.asarray(x, dtype=np.float64)
    _, e = np.frexp(x)                        # |x| = f 2^e, f in [0.5, 1)
    q = np.exp2(np.maximum(e - 1, emin) - (p - 1))
    r = np.rint(x / q) * q                    # representable: the casts below are exact
    return torch.from_numpy(r).to(torch.float32).to(_dtype16(precision))


def _dtype16(precision):
    return torch.bfloat16 if precision == 1 else torch.float16


@pytest.mark.parametrize("precision", [1, 2], ids=["bf16", "fp16"])
@pytest.mark.parametrize("n", [64, 1000, 1001, 4104])
def test_convert16_bitwise(ctx, precision, n):
    """The 16-bit operator copy is bitwise the host's round-to-nearest-even of
    the symmetric part: a non-symmetric input pins the transpose in the tiled
    conversion, odd n and n = 1000 the ragged 32 x 32 tiles, a leading
    dimension above n the strided reads; two conversions back to back into
    two buffers must both be right."""
    rng = np.random.default_rng(n)
    lda = n + 3
    outs = []
    for rep in range(2):
        A = rng.standard_normal((lda, n)) * (10.0 ** rng.uniform(-3, 3, (lda, n)))
        Ad = torch.from_numpy(np.ascontiguousarray(A.T)).to("cuda:0").T[:n]    # column-major, ld = lda
        out = torch.empty(n * n, dtype=torch.int16, device="cuda:0")
        L.lrep_test_convert16(ctx, precision, Ad, out)
        outs.append((A[:n], out))
    for A, out in outs:
        S = 0.5 * (A + A.T)
        want = _round16(S, precision).view(torch.int16).numpy()
        got = out.cpu().numpy().reshape(n, n).T      # column-major n x n
        assert np.array_equal(got, want), int((got != want).sum())


@pytest.mark.parametrize("precision", [1, 2], ids=["bf16", "fp16"])
@pytest.mark.parametrize("n,cols", [(64, 5), (1000, 32), (4104, 19), (8192, 32)])
def test_apply16_against_rounded_operands(ctx, precision, n, cols):
    """The 16-bit CG apply equals the exact product of the rounded operands up
    to FP32 accumulation (|err_i| <= n 2^-24 (|A16| |X16|)_i, X16 rounded on
    the host the way the kernel rounds it), so a wrong fragment layout, split
    or row tile shows as an O(1) error.  n = 1000 ends in a partial k-step, 4104
    splits k four ways with a ragged last chunk and a ragged last row tile,
    8192 is the dense workload's size.  FP16 scales each column by
    2^round(log2 sqrt(n / |x_j|^2)) before rounding; columns of norm 1e-6 and
    1e6 check that the scaling is applied and undone.  K and M go through
    the same buffers one after the other."""
    Kd, Md, _, _ = gen.dense_operator_device(n, 40 + n, "cuda:0")
    rng = np.random.default_rng(n)
    Xh = rng.standard_normal((n, cols))
    Xh[:, 0] *= 1e-6
    Xh[:, cols - 1] *= 1e6
    rr = (Xh * Xh).sum(axis=0)
    Xd = dev_colmajor(Xh, torch).T.contiguous().T
    rrd = torch.from_numpy(rr).to("cuda:0")
    Yd = dev_empty(n, cols, torch).T.contiguous().T
    A16 = torch.empty(n * n, dtype=torch.int16, device="cuda:0")
    sc = np.exp2(np.rint(0.5 * np.log2(n / rr))) if precision == 2 else np.ones(cols)
    X16 = _round16(Xh * sc, precision).to(torch.float64).numpy()
    for Ad in (Kd, Md):
        L.lrep_test_convert16(ctx, precision, Ad.T, A16)
        L.lrep_test_apply16(ctx, precision, A16, Xd, rrd, Yd)
        A16h = A16.cpu().view(_dtype16(precision)).to(torch.float64).numpy().reshape(n, n).T
        ref = (A16h @ X16) / sc
        absprod = np.abs(A16h) @ np.abs(X16)
        bound = n * 2.0 ** -24 * absprod / sc
        err = np.abs(host(Yd) - ref)
        assert np.all(err <= bound), float((err / bound).max())
        # and the product is the operator's to 16-bit accuracy
        exact = Ad.cpu().numpy() @ Xh
        assert np.abs(host(Yd) - exact).max() <= 2e-2 * np.abs(exact).max()


def _split3_host(v):
    """The three BF16 parts of FP64 values, each the rounding (to nearest
    even) of what the earlier parts leave, as FP64 arrays."""
    parts = []
    r = np.array(v, dtype=np.float64)
    for _ in range(3):
        h = _round16(r, 1).to(torch.float64).numpy()
        parts.append(h)
        r = r - h
    return parts


@pytest.mark.parametrize("n", [64, 1001, 4104])
def test_convert16_bf16x3_parts(ctx, n):
    """BF16x3 operator copy: three BF16 matrices whose parts are bitwise the
    host's successive roundings of the symmetric part, and whose sum carries
    at least FP32's 24 bits (|S - (hi + mid + lo)| <= 2^-24 |S|)."""
    rng = np.random.default_rng(n + 7)
    lda = n + 3
    A = rng.standard_normal((lda, n)) * (10.0 ** rng.uniform(-3, 3, (lda, n)))
    Ad = torch.from_numpy(np.ascontiguousarray(A.T)).to("cuda:0").T[:n]
    out = torch.empty(3 * n * n, dtype=torch.int16, device="cuda:0")
    L.lrep_test_convert16(ctx, 3, Ad, out)
    S = 0.5 * (A[:n] + A[:n].T)
    want = _split3_host(S)
    got = out.cpu().view(torch.bfloat16).to(torch.float64).numpy().reshape(3, n, n).transpose(0, 2, 1)
    for q in range(3):
        assert np.array_equal(got[q], want[q]), (q, int((got[q] != want[q]).sum()))
    assert np.all(np.abs(S - (got[0] + got[1] + got[2])) <= 2.0 ** -24 * np.abs(S))


@pytest.mark.parametrize("n,cols", [(64, 5), (1000, 32), (4104, 19), (8192, 32)])
def test_apply16_bf16x3_is_fp32_accurate(ctx, n, cols):
    """The BF16x3 CG apply: the six part products of order <= 2 summed in
    FP32 give the FP64 product to FP32 accuracy, |err_i| <= (n + 8) 2^-23
    (|A| |X|)_i (16-bit products: 2e-2 of the largest entry), so a missing or
    doubled part, a wrong part offset or the 16-bit layout shows at once.
    Ragged k (1000), split k with a ragged last chunk (4104), the workload's
    size (8192); columns of norm 1e-6 and 1e6."""
    Kd, Md, _, _ = gen.dense_operator_device(n, 40 + n, "cuda:0")
    rng = np.random.default_rng(n)
    Xh = rng.standard_normal((n, cols))
    Xh[:, 0] *= 1e-6
    Xh[:, cols - 1] *= 1e6
    rr = (Xh * Xh).sum(axis=0)
    Xd = dev_colmajor(Xh, torch).T.contiguous().T
    rrd = torch.from_numpy(rr).to("cuda:0")
    Yd = dev_empty(n, cols, torch).T.contiguous().T
    A16 = torch.empty(3 * n * n, dtype=torch.int16, device="cuda:0")
    for Ad in (Kd, Md):
        L.lrep_test_convert16(ctx, 3, Ad.T, A16)
        L.lrep_test_apply16(ctx, 3, A16, Xd, rrd, Yd)
        A = Ad.cpu().numpy()
        exact = A @ Xh
        bound = (n + 8) * 2.0 ** -23 * (np.abs(A) @ np.abs(Xh))
        err = np.abs(host(Yd) - exact)
        assert np.all(err <= bound), float((err / bound).max())
        # far tighter than the BF16 product (~4e-3 relative)
        assert (err / (np.abs(A) @ np.abs(Xh))).max() <= 1e-4


@pytest.mark.parametrize("n,r", [(1502, 16), (20002, 100), (262144, 256)])
@pytest.mark.parametrize("which", [0, 1])
def test_fused_cg_matches_plain_cg_and_the_oracle(ctx, n, r, which):
    """The Step-6 CG on a low-rank operator (K = diag(delta), M = diag(delta) +
    2 L L^T) in its fused form -- one pass over the rows per step, L^T p
    carried by the direction recurrence, alpha from carried sums -- against
    the plain CG (two passes over L per product, separate updates) and the
    oracle's CG: 32 columns, tolerance 1e-2, 20 steps.  Several row tiles per
    workgroup at n = 20002 and 262144."""
    f = gen.casida_factors(n, r, 900 + r)
    B = np.random.default_rng(n + which).standard_normal((n, 32))
    op = L.lrep_create_lowrank(ctx, dev_colmajor(f.delta, torch), dev_colmajor(f.L, torch))
    Bd = dev_colmajor(B, torch).T.contiguous().T
    Xf, Xp = dev_empty(n, 32, torch), dev_empty(n, 32, torch)
    torch.cuda.synchronize()
    print(f"[cg] n={n} rank={r} which={which}", flush=True)
    af = L.lrep_test_cg(op, which, Bd, Xf, 1e-2, 20, 1)
    ap = L.lrep_test_cg(op, which, Bd, Xp, 1e-2, 20, -1)
    L.lrep_destroy_op(op)
    Xf, Xp = host(Xf), host(Xp)
    scale = np.abs(Xp).max()
    print(f"[cg] applies fused {af} plain {ap}; max |X_fused - X_plain| / max |X| = "
          f"{np.abs(Xf - Xp).max() / scale:.2e}", flush=True)
    assert af == ap
    assert np.abs(Xf - Xp).max() <= 1e-10 * scale
    if n <= 20002:
        cop = oracle.CasidaOperator(f.delta, f.L)
        Xo, ao = oracle.bosp.cg_columns(cop.apply_K if which == 0 else cop.apply_M, B, 1e-2, 20)
        assert ao == af
        assert np.abs(Xf - Xo).max() <= 1e-10 * np.abs(Xo).max()
