"""Serving interface (lrep_submit / lrep_poll / lrep_cancel): requests of
different operators, sizes and nev run concurrently on the context's worker
streams, admitted against the HBM budget.  Every kernel reduces in a fixed
order and nothing in a solve depends on timing, so each result must be
bitwise the one the same request gives alone."""
import time

import numpy as np
import pytest

import gen
import paper_2506_08355_amd as L
from gpu_util import dev_colmajor

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# (operator, nev, block, window, tol)
REQUESTS = [(0, 8, 16, 16, 1e-8), (1, 24, 32, 16, 1e-8), (2, 16, 16, 16, 1e-8), (0, 32, 32, 16, 1e-8),
            (1, 4, 16, 16, 1e-8), (2, 40, 48, 24, 1e-8), (3, 12, 16, 8, 1e-8)]


def make_ops(ctx, factors=None):
    ops, sizes = [], []
    for n, seed in ((512, 1201), (1024, 1202)):
        K, M, f = gen.dense_operator(n, seed)
        ops.append(L.lrep_create_dense(ctx, dev_colmajor(K, torch), dev_colmajor(M, torch)))
        sizes.append(n)
        if factors is not None:
            factors.append(f)
    for n, r, seed in ((16384, 64, 1203), (20000, 100, 1204)):
        f = gen.casida_factors(n, r, seed)
        ops.append(L.lrep_create_lowrank(ctx, dev_colmajor(f.delta, torch), dev_colmajor(f.L, torch)))
        sizes.append(n)
        if factors is not None:
            factors.append(f)
    return ops, sizes


def request_inputs(sizes):
    out = []
    for i, (o, nev, block, window, tol) in enumerate(REQUESTS):
        U, _ = gen.init_block(sizes[o], block + 2 * window, 100 + i)
        out.append(np.asfortranarray(U))
    return out


def run_alone(ctx, ops, sizes, inits):
    res = []
    for (o, nev, block, window, tol), U in zip(REQUESTS, inits):
        n = sizes[o]
        lam, X, Y = np.zeros(nev), np.zeros((n, nev), order="F"), np.zeros((n, nev), order="F")
        rc, st = L.lrep_solve(ops[o], n, nev, block, tol, L.make_opts(window=window, init=U), lam, X, Y, ctx=ctx)
        assert rc == L.LREP_OK
        res.append((lam, X, Y))
    return res


def run_mix(ctx, ops, sizes, inits, copies):
    jobs = []
    for c in range(copies):
        for k, ((o, nev, block, window, tol), U) in enumerate(zip(REQUESTS, inits)):
            n = sizes[o]
            lam, X, Y = np.zeros(nev), np.zeros((n, nev), order="F"), np.zeros((n, nev), order="F")
            opts = L.make_opts(window=window, init=U)
            t = L.lrep_submit(ctx, ops[o], nev, block, tol, opts, lam, X, Y)
            jobs.append((k, t, lam, X, Y, opts))
    pending = {j[1] for j in jobs}
    deadline = time.time() + 240
    saw_pending = False
    while pending and time.time() < deadline:
        for t in list(pending):
            rc, st = L.lrep_poll(ctx, t)
            if rc == L.LREP_EAGAIN:
                saw_pending = True
                continue
            assert rc == L.LREP_OK, (rc, L.lrep_strerror(rc))
            pending.discard(t)
        time.sleep(0.005)
    assert not pending, "served requests did not finish"
    return jobs, saw_pending


@pytest.fixture(scope="module")
def served():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    ctx = L.lrep_init(0)
    factors = []
    ops, sizes = make_ops(ctx, factors)
    inits = request_inputs(sizes)
    alone = run_alone(ctx, ops, sizes, inits)
    yield ctx, ops, sizes, inits, alone, factors
    for op in ops:
        L.lrep_destroy_op(op)
    L.lrep_finalize(ctx)


def test_mix_is_bitwise_alone(served):
    ctx, ops, sizes, inits, alone, _ = served
    jobs, saw_pending = run_mix(ctx, ops, sizes, inits, copies=2)
    assert saw_pending   # the requests were in flight together
    for k, t, lam, X, Y, _ in jobs:
        a_lam, a_X, a_Y = alone[k]
        assert np.array_equal(lam, a_lam), k
        assert np.array_equal(X, a_X), k
        assert np.array_equal(Y, a_Y), k


def test_served_results_match_the_oracle(served):
    """Every served result, checked against the exact spectrum rather than
    against the library: dense operators against the factored closed form
    (eigenvalues within 1e-10 relative), low-rank ones by the inertia count
    (each eigenvalue bracketed at 1e-10 relative); all against the residual
    bar ||H z - lambda z|| / (||H|| ||z||) <= 1e-8 and max |X^T Y - I| <= 1e-12."""
    from oracle import exact
    from gpu_util import h_residual
    ctx, ops, sizes, inits, alone, factors = served
    jobs, _ = run_mix(ctx, ops, sizes, inits, copies=1)
    for k, t, lam, X, Y, _ in jobs:
        o = REQUESTS[k][0]
        f = factors[o]
        nev = lam.size
        if o < 2:
            np.testing.assert_allclose(lam, exact.dense_spectrum(f.q1, f.k, f.q2, f.m, nev), rtol=1e-10, atol=0)
            K, M = f.K(), f.M()
            res = h_residual(lambda v: K @ v, lambda v: M @ v, X, Y, lam, f.norm_H())
        else:
            lo = exact.casida_count_below_many(f.delta, f.L, lam * (1 - 1e-10))
            hi = exact.casida_count_below_many(f.delta, f.L, lam * (1 + 1e-10))
            assert all(lo[i] <= i and hi[i] >= i + 1 for i in range(nev)), (k, lo, hi)
            apply_M = lambda v: f.delta[:, None] * v + 2.0 * (f.L @ (f.L.T @ v))
            normH = float(f.delta.max() + 2.0 * np.linalg.norm(f.L, 2) ** 2)   # >= ||M||_2 >= ||K||_2
            res = h_residual(lambda v: f.delta[:, None] * v, apply_M, X, Y, lam, normH)
        assert res.max() <= 1e-8, (k, res.max())
        assert np.abs(X.T @ Y - np.eye(nev)).max() <= 1e-12, k


def test_request_larger_than_the_budget_fails_without_blocking():
    """Two concurrent requests whose footprint alone exceeds what the budget
    leaves beside the operator: both report LREP_ENOMEM (no request waits for
    memory that can never come), and lrep_finalize returns."""
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    n = 1024
    K, M, _ = gen.dense_operator(n, 1202)
    ctx = L.lrep_init(0, 2 * n * n * 8 + (1 << 20))   # the operator and 1 MiB
    op = L.lrep_create_dense(ctx, dev_colmajor(K, torch), dev_colmajor(M, torch))
    outs, tickets = [], []
    for i in range(2):
        lam, X, Y = np.zeros(8), np.zeros((n, 8), order="F"), np.zeros((n, 8), order="F")
        opts = L.make_opts(window=16)
        outs.append((lam, X, Y, opts))
        tickets.append(L.lrep_submit(ctx, op, 8, 16, 1e-8, opts, lam, X, Y))
    deadline = time.time() + 60
    rcs = {}
    while len(rcs) < 2 and time.time() < deadline:
        for t in tickets:
            if t not in rcs:
                rc, _ = L.lrep_poll(ctx, t)
                if rc != L.LREP_EAGAIN:
                    rcs[t] = rc
        time.sleep(0.005)
    assert sorted(rcs.values()) == [L.LREP_ENOMEM, L.LREP_ENOMEM], rcs
    L.lrep_destroy_op(op)
    t0 = time.time()
    L.lrep_finalize(ctx)
    assert time.time() - t0 < 30


def test_budget_admission_queues_and_matches():
    """A context whose HBM budget holds the operators and about one solve's
    workspace at a time: requests wait for memory instead of failing, and
    still return the alone results."""
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    # size the budget from an unbudgeted context's per-solve footprint
    probe = L.lrep_init(0)
    ops, sizes = make_ops(probe)
    inits = request_inputs(sizes)
    alone = run_alone(probe, ops, sizes, inits)
    for op in ops:
        L.lrep_destroy_op(op)
    L.lrep_finalize(probe)
    # dense K, M; low-rank delta and L plus the row-major copy of L (rank rounded up to 64)
    op_bytes = (sum(2 * n * n * 8 for n in sizes[:2]) + 16384 * 65 * 8 + 20000 * 101 * 8
                + 16384 * 64 * 8 + 20000 * 128 * 8)
    budget = op_bytes + 400 * (1 << 20)   # the largest solve needs about 300 MiB
    ctx = L.lrep_init(0, budget)
    ops, sizes = make_ops(ctx)
    try:
        jobs, _ = run_mix(ctx, ops, sizes, inits, copies=1)
        for k, t, lam, X, Y, _ in jobs:
            a_lam, a_X, a_Y = alone[k]
            assert np.array_equal(lam, a_lam), k
            assert np.array_equal(X, a_X), k
    finally:
        for op in ops:
            L.lrep_destroy_op(op)
        L.lrep_finalize(ctx)


def test_cancel_queued_request(served):
    ctx, ops, sizes, inits, alone, _ = served
    # fill the workers, then cancel the last request while it is still queued
    jobs = []
    for i in range(6):
        o, nev, block, window, tol = REQUESTS[5]
        n = sizes[o]
        lam, X, Y = np.zeros(nev), np.zeros((n, nev), order="F"), np.zeros((n, nev), order="F")
        opts = L.make_opts(window=window, init=inits[5])
        jobs.append((L.lrep_submit(ctx, ops[o], nev, block, tol, opts, lam, X, Y), lam, X, Y, opts))
    last = jobs[-1][0]
    rc_cancel = L.lrep_cancel(ctx, last)
    assert rc_cancel in (L.LREP_OK, L.LREP_EAGAIN)
    deadline = time.time() + 240
    for t, *_ in jobs:
        while time.time() < deadline:
            rc, _ = L.lrep_poll(ctx, t)
            if rc != L.LREP_EAGAIN:
                break
            time.sleep(0.005)
        if t == last and rc_cancel == L.LREP_OK:
            assert rc == L.LREP_ECANCELED
        else:
            assert rc == L.LREP_OK


def test_concurrent_cg_solves_run_batched_and_bitwise_alone(served):
    """Continuous batching of Step 6: eight requests on one operator at once
    (window 8, so up to four jobs fill a 32-column block CG) -- their CG
    solves run as shared block CGs (stats: cg_batched, cg_batch_columns),
    every result bitwise the request's result alone, and the same with
    batching switched off (serve_batch = -1)."""
    ctx, ops, sizes, _, _, _ = served
    for o, nev, block, window in ((0, 8, 16, 8), (2, 8, 16, 8)):
        n = sizes[o]
        U = np.asfortranarray(gen.init_block(n, block + 2 * window, 300 + o)[0])
        lam0, X0, Y0 = np.zeros(nev), np.zeros((n, nev), order="F"), np.zeros((n, nev), order="F")
        rc, _ = L.lrep_solve(ops[o], n, nev, block, 1e-8, L.make_opts(window=window, init=U), lam0, X0, Y0, ctx=ctx)
        assert rc == L.LREP_OK
        for batch in (0, -1):
            jobs = []
            for c in range(8):
                lam, X, Y = np.zeros(nev), np.zeros((n, nev), order="F"), np.zeros((n, nev), order="F")
                opts = L.make_opts(window=window, init=U, serve_batch=batch)
                jobs.append((L.lrep_submit(ctx, ops[o], nev, block, 1e-8, opts, lam, X, Y), lam, X, Y, opts))
            stats, deadline = {}, time.time() + 120
            while len(stats) < len(jobs) and time.time() < deadline:
                for t, *_ in jobs:
                    if t not in stats:
                        rc, st = L.lrep_poll(ctx, t)
                        if rc != L.LREP_EAGAIN:
                            assert rc == L.LREP_OK, (o, batch, rc)
                            stats[t] = st
                time.sleep(0.002)
            assert len(stats) == len(jobs), "served requests did not finish"
            for t, lam, X, Y, _ in jobs:
                assert np.array_equal(lam, lam0), (o, batch)
                assert np.array_equal(X, X0), (o, batch)
                assert np.array_equal(Y, Y0), (o, batch)
            batched = sum(st.cg_batched for st in stats.values())
            shared_cols = sum(st.cg_batch_columns for st in stats.values())
            if batch == 0:
                assert batched > 0 and shared_cols > 0, (o, batched, shared_cols)
            else:
                assert batched == 0 and shared_cols == 0, (o, batched, shared_cols)


def test_concurrent_fp32_row_requests_share_one_copy(served):
    """precision 4 (the CG passes on the FP32 rows of L) under serving: six
    requests submitted at once on a fresh low-rank operator race to make its
    FP32 copy (made once, under the operator's lock) and batch their CG
    solves; every result is bitwise the same request solved alone afterwards,
    and its eigenvalues match the FP64 solve to 1e-10."""
    ctx = served[0]
    n, r, nev, block, window = 16384, 64, 8, 16, 8
    f = gen.casida_factors(n, r, 1205)
    op = L.lrep_create_lowrank(ctx, dev_colmajor(f.delta, torch), dev_colmajor(f.L, torch))
    U = np.asfortranarray(gen.init_block(n, block + 2 * window, 310)[0])
    jobs = []
    for c in range(6):
        lam, X, Y = np.zeros(nev), np.zeros((n, nev), order="F"), np.zeros((n, nev), order="F")
        opts = L.make_opts(window=window, init=U, precision=4)
        jobs.append((L.lrep_submit(ctx, op, nev, block, 1e-8, opts, lam, X, Y), lam, X, Y, opts))
    done, deadline = set(), time.time() + 120
    while len(done) < len(jobs) and time.time() < deadline:
        for t, *_ in jobs:
            if t not in done:
                rc, _ = L.lrep_poll(ctx, t)
                if rc != L.LREP_EAGAIN:
                    assert rc == L.LREP_OK, rc
                    done.add(t)
        time.sleep(0.002)
    assert len(done) == len(jobs), "served requests did not finish"
    lam1, X1, Y1 = np.zeros(nev), np.zeros((n, nev), order="F"), np.zeros((n, nev), order="F")
    rc, _ = L.lrep_solve(op, n, nev, block, 1e-8, L.make_opts(window=window, init=U, precision=4), lam1, X1, Y1,
                         ctx=ctx)
    assert rc == L.LREP_OK
    lam0, X0, Y0 = np.zeros(nev), np.zeros((n, nev), order="F"), np.zeros((n, nev), order="F")
    rc, _ = L.lrep_solve(op, n, nev, block, 1e-8, L.make_opts(window=window, init=U), lam0, X0, Y0, ctx=ctx)
    assert rc == L.LREP_OK
    L.lrep_destroy_op(op)
    for t, lam, X, Y, _ in jobs:
        assert np.array_equal(lam, lam1) and np.array_equal(X, X1) and np.array_equal(Y, Y1)
    np.testing.assert_allclose(lam1, lam0, rtol=1e-10, atol=0)
