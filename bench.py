#!/usr/bin/env python3
"""Throughput benchmark of the MI355X BOSP eigensolver.

One step = one complete lrep_solve (every row of the hot path: block operator
applies, Rayleigh-Ritz projection and small LREP, residuals, P/Q update, CG
search directions, MGS-Biorth against the converged and active blocks) on a
device-resident operator, from the same seeded starting block each step.

Default workload: the matrix-free Casida-style operator, FP64, n = 262144:
K = diag(delta), M = diag(delta) + 2 L L^T, delta ~ U[0.1, 20] sorted, L an
n x 256 Gaussian matrix scaled by 1/sqrt(n) (seed 1003); the 128 smallest
positive eigenpairs at residual tolerance 1e-8, block 64, window 32 (moving
mechanism).  value = eigenpairs per second over the timed steps, which run
with every profiling hook off.  `--workload dense8192` selects the dense
n = 8192 workload (tolerance 1e-10) and the others listed in WORKLOADS.

Also reported on the same JSON line, from one extra profiled solve after the
timed region:
  roofline      the dominant kernel (the low-rank M apply of the CG inner
                solves for the Casida workload, the FP64 MFMA streaming block
                apply for the dense ones) timed live with HIP events on the
                solve's stream; its algorithmic bytes per launch against the
                8 TB/s HBM peak.  `traffic` is the HBM bytes per launch
                measured with hardware counters (rocprofv3 --pmc FETCH_SIZE /
                WRITE_SIZE, scaled by the same counters on a plain copy of
                known size), read from the committed profile summary, and
                null when the kernel source has changed since the counters
                were taken;
  phases        per-phase GPU time of that solve in the paper's five buckets;
  cpu_baseline  the FP64 CPU oracle on the same operator and start block,
                to convergence where that takes a minute or less on the host,
                else for a bounded number of outer iterations scaled to the
                iteration count of the GPU solve (the line says which).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6

WORKLOADS = {
    "dense8192": dict(kind="dense", n=8192, seed=1002, nev=64, block=64, window=32, tol=1e-10, zeros=0),
    "dense8192z": dict(kind="dense", n=8192, seed=1012, nev=64, block=64, window=32, tol=1e-10, zeros=8),
    "dense256": dict(kind="dense", n=256, seed=1001, nev=8, block=16, window=16, tol=1e-10, zeros=0),
    "dense32768": dict(kind="dense", n=32768, seed=1004, nev=64, block=64, window=32, tol=1e-10, zeros=0,
                       cpu_iters=4),
    # mixed precision (growth direction 1): BF16 / FP16 operator copies for the CG applies
    "dense32768bf16": dict(kind="dense", n=32768, seed=1004, nev=64, block=64, window=32, tol=1e-10, zeros=0,
                           precision=1, cpu_iters=4),
    "dense32768fp16": dict(kind="dense", n=32768, seed=1004, nev=64, block=64, window=32, tol=1e-10, zeros=0,
                           precision=2, cpu_iters=4),
    "dense8192bf16": dict(kind="dense", n=8192, seed=1002, nev=64, block=64, window=32, tol=1e-10, zeros=0,
                          precision=1),
    "dense8192fp16": dict(kind="dense", n=8192, seed=1002, nev=64, block=64, window=32, tol=1e-10, zeros=0,
                          precision=2),
    # BF16x3: operator and CG block split into hi/mid/lo BF16 parts, FP32-accurate CG products
    "dense32768bf16x3": dict(kind="dense", n=32768, seed=1004, nev=64, block=64, window=32, tol=1e-10, zeros=0,
                             precision=3, cpu_iters=4),
    "dense8192bf16x3": dict(kind="dense", n=8192, seed=1002, nev=64, block=64, window=32, tol=1e-10, zeros=0,
                            precision=3),
    # one oracle iteration takes about a minute on the host: the baseline is a bounded sample
    "casida262144": dict(kind="casida", n=262144, rank=256, seed=1003, nev=128, block=64, window=32, tol=1e-8,
                         cpu_iters=1),
    # the same with the Step-6 CG passes reading an FP32 copy of L's rows (growth direction 1)
    "casida262144f32": dict(kind="casida", n=262144, rank=256, seed=1003, nev=128, block=64, window=32, tol=1e-8,
                            cpu_iters=1, precision=4),
    # generalized LREP K x = lambda B y, M y = lambda B x with a diagonal metric B (growth direction f4)
    "dense8192metric": dict(kind="dense", n=8192, seed=1002, nev=64, block=64, window=32, tol=1e-10, zeros=0,
                            metric_seed=1105),
    "dense8192metricB": dict(kind="dense", n=8192, seed=1002, nev=64, block=64, window=32, tol=1e-10, zeros=0,
                             metric_seed=1111, metric_dense=True),
}


# every step solves from the same start block, drawn with this seed (the
# outer iteration count, and so the rate, depends on the draw)
START_BLOCK_SEED = 7

# counter summaries of the dominant kernel, per workload: file, kernel source
# the counters were taken on, and the key under which its SHA-256 is stored
TRAFFIC = {
    "dense8192": ("apply_stream_kernel.dense8192.traffic.md", "apply.hip", "apply_hip_sha256"),
    "casida262144": ("lowrank_cg.casida262144.traffic.md", "lowrank.hip", "lowrank_hip_sha256"),
    "casida262144f32": ("lowrank_cg_f32rows.casida262144.traffic.md", "lowrank.hip", "lowrank_hip_sha256"),
}
CSRC = os.path.join(ROOT, "paper_2506_08355_amd", "csrc")


def measured_traffic(workload):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, if one was taken on this workload and on the current source."""
    if workload not in TRAFFIC:
        return None
    fname, src, key = TRAFFIC[workload]
    path = os.path.join(ROOT, "profiles", fname)
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    with open(os.path.join(CSRC, src), "rb") as fh:
        sha = hashlib.sha256(fh.read()).hexdigest()
    if fields.get(key) != sha:
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_calibration(mib):
    """One plain device copy of `mib` MiB through the library's copy kernel
    (reference for the byte counters); prints the bytes it moves."""
    import torch
    import paper_2506_08355_amd as L
    count = mib * (1 << 20) // 8
    src = torch.ones(count, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    ctx = L.lrep_init(0)
    L.lrep_test_copy(ctx, src, dst)
    torch.cuda.synchronize()
    ok = bool(torch.equal(src, dst))
    L.lrep_finalize(ctx)
    print(json.dumps({"copy_kernel": "copy_kernel", "read_bytes": count * 8, "write_bytes": count * 8,
                      "correct": ok}), flush=True)


def hbm_probe(mib):
    """The HBM read rate the hardware reaches with the library's plain
    streaming read kernel over `mib` MiB (20 launches back to back, timed
    with HIP events on the library's stream); prints one JSON line."""
    import torch
    import paper_2506_08355_amd as L
    count = mib * (1 << 20) // 8
    src = torch.ones(count, dtype=torch.float64, device="cuda:0")
    ctx = L.lrep_init(0)
    res = {"probe": "hbm_read", "bytes": count * 8, "launches": 20}
    for blocks in (1024, 2048, 4096):
        out = torch.empty(blocks, dtype=torch.float64, device="cuda:0")
        L.lrep_test_read(ctx, src, out)
        ok = abs(float(out.sum()) - count) <= 1e-9 * count
        ms = L.lrep_test_read(ctx, src, out, iters=20)
        res[f"read_GBps_{blocks}_blocks"] = round(count * 8 * 20 / (ms * 1e-3) / 1e9, 1)
        res[f"read_ok_{blocks}"] = ok
    L.lrep_finalize(ctx)
    print(json.dumps(res), flush=True)


def serve(args, np, torch, gen, L):
    """Serving workload (continuous admission through lrep_submit/lrep_poll):
    a pool of dense and low-rank operators, requests of random nev drawn 50/50
    over them, first all at once (closed-loop solve rate), then with Poisson
    arrivals at rho times that rate; latency = submit to completed poll.
    `--serve-sizes full` draws the serving configuration's ranges (dense n
    in [512, 16384], low-rank n in [16384, 262144]); the default caps them
    (dense n <= 8192, low-rank n <= 32768) so that a run stays within a few
    minutes.  `--budget-gib` caps the context's HBM (requests then queue for
    memory).  With `--sequential 1` the same requests also run one after
    the other through the blocking lrep_solve on the same context (the
    sequential rate the served rate is compared with); every served and
    sequential result is checked (verify)."""
    rng = np.random.default_rng(1005)
    dev = torch.device("cuda:0")
    full = args.serve_sizes == "full"
    dmax, lmax = (16384, 262144) if full else (8192, 32768)
    ctx = L.lrep_init(0, int(args.budget_gib * (1 << 30)))
    pool, t0 = [], time.time()
    checks = []              # per operator: what the served results are checked against
    shared = args.serve_pool == "shared"
    for i in range(1 if shared else 6):       # dense, n log-uniform [512, dmax], multiple of 64
        n = int(64 * round(np.exp(rng.uniform(np.log(512), np.log(dmax))) / 64))
        if shared:
            n = 8192
        Kd, Md, kk, mm, Q1, Q2 = gen.dense_operator_device(n, 2000 + i, dev, return_factors=True)
        pool.append((L.lrep_create_dense(ctx, Kd.T, Md.T), n))
        checks.append(dict(kind="dense", K=Kd, M=Md, q1=Q1, q2=Q2, k=kk, m=mm, normH=float(max(kk.max(), mm.max()))))
    for i in range(1 if shared else 6):       # low rank, n log-uniform [16384, lmax], rank uniform {64..256}
        n = int(64 * round(np.exp(rng.uniform(np.log(16384), np.log(lmax))) / 64))
        r = int(rng.integers(64, 257))
        if shared:
            n, r = 65536, 128
        f = gen.casida_factors(n, r, 3000 + i)
        dd = torch.from_numpy(f.delta).to(dev)
        Ld = torch.from_numpy(np.ascontiguousarray(f.L.T)).to(dev).T
        pool.append((L.lrep_create_lowrank(ctx, dd, Ld), n))
        checks.append(dict(kind="lowrank", f=f, delta=dd, L=Ld,
                           normH=float(f.delta.max() + 2.0 * np.linalg.norm(f.L, 2) ** 2)))
    torch.cuda.synchronize()
    print(f"[serve] operator pool ready in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    reqs = []
    nd = 1 if shared else 6
    for i in range(args.requests):
        k = int(rng.integers(0, nd)) + (nd if rng.uniform() < 0.5 else 0)
        nev = int(rng.integers(4, 65))
        block = 16 * ((nev + 15) // 16)
        window = block // 2 if block >= 32 else block
        if shared:
            # small windows, so that up to four concurrent CG solves share one 32-column block
            nev = int(rng.integers(4, 17))
            block, window = 16, 8
        reqs.append((k, nev, block, window))

    def check_vectors(j, lam, X, Y):
        """One result against bars independent of the library: the residual
        ||H z - lambda z|| / (||H|| ||z||) <= 1e-8 and max |X^T Y - I| <= 1e-12
        (torch FP64 products).  Returns a failure record or None."""
        k = reqs[j][0]
        c = checks[k]
        Xd, Yd = torch.from_numpy(X).to(dev), torch.from_numpy(Y).to(dev)
        ld = torch.from_numpy(lam).to(dev)
        if c["kind"] == "dense":
            KX, MY = c["K"] @ Xd, c["M"] @ Yd
        else:
            KX = c["delta"][:, None] * Xd
            MY = c["delta"][:, None] * Yd + 2.0 * (c["L"] @ (c["L"].T @ Yd))
        res = torch.sqrt(((KX - Yd * ld) ** 2).sum(0) + ((MY - Xd * ld) ** 2).sum(0)) / (
            c["normH"] * torch.sqrt((Xd ** 2).sum(0) + (Yd ** 2).sum(0)))
        bi = float((Xd.T @ Yd - torch.eye(lam.size, dtype=torch.float64, device=dev)).abs().max())
        if float(res.max()) > 1e-8 or bi > 1e-12:
            return [j, "residual/biorth", float(res.max()), bi]
        return None

    def reference_values(lams):
        """The reference eigenvalues of every operator some result in lams
        (list of (request, lambda)) belongs to: dense, the oracle's factored
        closed form for the longest prefix asked; low rank, the longest
        returned prefix with each value bracketed at 1e-10 relative by the
        oracle's inertia count.  Returns (ref, failures)."""
        from oracle import exact
        bad, ref = [], {}
        for k in sorted({reqs[j][0] for j, _ in lams}):
            c = checks[k]
            longest = max((lam for j, lam in lams if reqs[j][0] == k), key=lambda a: a.size)
            if c["kind"] == "dense":
                ref[k] = exact.dense_spectrum_smallest(c["q1"].cpu().numpy(), c["k"], c["q2"].cpu().numpy(), c["m"],
                                                       longest.size)
            else:
                lo = exact.casida_count_below_many(c["f"].delta, c["f"].L, longest * (1 - 1e-10))
                hi = exact.casida_count_below_many(c["f"].delta, c["f"].L, longest * (1 + 1e-10))
                if not all(lo[i] <= i and hi[i] >= i + 1 for i in range(longest.size)):
                    bad.append([int(k), "bracket"])
                ref[k] = longest
        return ref, bad

    def check_values(lams, ref):
        bad = []
        for j, lam in lams:
            r = ref[reqs[j][0]][:lam.size]
            if np.abs(lam - r).max() > 1e-10 * r.max():
                bad.append([j, "eigenvalues", float(np.abs(lam - r).max())])
        return bad

    def run(arrivals, keep):
        jobs, done = [], {}
        start = time.perf_counter()
        i = 0
        pending = {}
        while i < len(reqs) or pending:
            now = time.perf_counter() - start
            while i < len(reqs) and arrivals[i] <= now:
                k, nev, block, window = reqs[i]
                op, n = pool[k]
                lam, X, Y = np.zeros(nev), np.zeros((n, nev), order="F"), np.zeros((n, nev), order="F")
                opts = L.make_opts(window=window, seed=17 + i, graphs=args.graphs, serve_batch=args.serve_batch)
                t = L.lrep_submit(ctx, op, nev, block, 1e-8, opts, lam, X, Y)
                pending[t] = (i, time.perf_counter(), (lam, X, Y, opts))
                i += 1
            for t in list(pending):
                rc, st = L.lrep_poll(ctx, t)
                if rc == L.LREP_EAGAIN:
                    continue
                j, ts, outs = pending.pop(t)
                done[j] = (rc, (time.perf_counter() - ts) * 1e3, outs[:3] if keep else None,
                           (st.cg_batched, st.cg_batch_columns))
                print(f"[serve] request {j} rc={rc} {done[j][1]:.0f} ms ({len(done)}/{len(reqs)})",
                      file=sys.stderr, flush=True)
            time.sleep(0.0005)
        return time.perf_counter() - start, done

    seq_time, seq_bad, seq_lams = None, [], []
    if args.sequential:
        # the same requests one at a time through the blocking call
        # (each result is checked right after its solve, outside the timed sum)
        seq_time = 0.0
        for j, (k, nev, block, window) in enumerate(reqs):
            op, n = pool[k]
            lam, X, Y = np.zeros(nev), np.zeros((n, nev), order="F"), np.zeros((n, nev), order="F")
            t1 = time.perf_counter()
            rc, _ = L.lrep_solve(op, n, nev, block, 1e-8, L.make_opts(window=window, seed=17 + j, graphs=args.graphs),
                                 lam, X, Y, ctx=ctx, check=False)
            seq_time += time.perf_counter() - t1
            if rc == L.LREP_OK:
                f = check_vectors(j, lam, X, Y)
                if f:
                    seq_bad.append(f)
                seq_lams.append((j, lam))
            else:
                seq_bad.append([j, "rc", rc])
            if j % 16 == 15:
                print(f"[serve] sequential {j + 1}/{len(reqs)}: {seq_time:.1f}s of solves, {len(seq_bad)} failures",
                      file=sys.stderr, flush=True)
    closed_time, closed = run([0.0] * len(reqs), False)
    rate = len(reqs) / closed_time
    gaps = rng.exponential(1.0 / (args.rho * rate), len(reqs))
    arrivals = np.cumsum(gaps) - gaps[0]
    open_time, done = run(list(arrivals), True)
    lat = np.array([done[j][1] for j in range(len(reqs))])
    ok = all(done[j][0] == L.LREP_OK for j in range(len(reqs))) and all(
        closed[j][0] == L.LREP_OK for j in range(len(reqs)))
    tv = time.time()
    bad = []
    for j in range(len(reqs)):
        if done[j][0] == L.LREP_OK:
            f = check_vectors(j, *done[j][2])
            if f:
                bad.append(f)
    served_lams = [(j, done[j][2][0]) for j in range(len(reqs)) if done[j][0] == L.LREP_OK]
    ref, rbad = reference_values(served_lams + seq_lams)
    bad += rbad + check_values(served_lams, ref)
    seq_bad += check_values(seq_lams, ref)
    print(f"[serve] results checked in {time.time() - tv:.1f}s: {len(bad)} failures", file=sys.stderr, flush=True)
    failed = [[j, done[j][0], pool[reqs[j][0]][1], reqs[j][1], "dense" if reqs[j][0] < nd else "lowrank"]
              for j in range(len(reqs)) if done[j][0] != L.LREP_OK][:10]
    slowest = sorted(range(len(reqs)), key=lambda j: -done[j][1])[:5]
    slow = [[j, round(done[j][1], 1), pool[reqs[j][0]][1], reqs[j][1], "dense" if reqs[j][0] < nd else "lowrank"]
            for j in slowest]
    for op, _ in pool:
        L.lrep_destroy_op(op)
    L.lrep_finalize(ctx)
    out = {
        "metric": "serving: solves/s under Poisson arrivals; p50/p99 solve latency",
        "value": round(len(reqs) / open_time, 3), "unit": "solves/s", "n_gpus": 1, "steps": len(reqs),
        "warmup": 0, "ms_per_step": round(open_time * 1e3 / len(reqs), 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": (f"serving: 6 dense (n log-uniform 512-{dmax}) + 6 low-rank (n log-uniform "
                                f"16384-{lmax}, rank 64-256) operators, requests 50/50, nev uniform 4-64, tol 1e-8, "
                                f"Poisson arrivals at rho={args.rho} of the closed-loop rate") if not shared else
                               (f"serving, shared operators: one dense (n=8192) and one low-rank (n=65536, rank 128) "
                                f"operator, requests 50/50, nev uniform 4-16, block 16, window 8, tol 1e-8, Poisson "
                                f"arrivals at rho={args.rho} of the closed-loop rate"),
                   "cg_batching": args.serve_batch == 0,
                   "requests": len(reqs), "workers": 4,
                   "hbm_budget_gib": args.budget_gib if args.budget_gib else None,
                   "operator_n": [n for _, n in pool]},
        "closed_loop_solves_per_s": round(rate, 3),
        "cg_solves_batched": int(sum(done[j][3][0] for j in range(len(reqs)))),
        "cg_columns_shared": int(sum(done[j][3][1] for j in range(len(reqs)))),
        "sequential_solves_per_s": round(len(reqs) / seq_time, 3) if seq_time else None,
        "sequential_failures": seq_bad[:10],
        "p50_ms": round(float(np.percentile(lat, 50)), 2), "p99_ms": round(float(np.percentile(lat, 99)), 2),
        "all_ok": ok and not bad, "oracle_failures": bad[:10], "failed": failed, "slowest": slow,
    }
    print(json.dumps(out), flush=True)


def describe(w):
    if w["kind"] == "dense":
        z = f", {w['zeros']} exact zeros in m" if w["zeros"] else ""
        z += {0: "", 1: "; CG applies in BF16 (f32 accumulate)", 2: "; CG applies in FP16 (f32 accumulate)",
              3: "; CG applies in BF16x3 (hi/mid/lo BF16 parts, six part products, f32 accumulate)"}[
            w.get("precision", 0)]
        if w.get("metric_dense"):
            z += ("; generalized LREP K x = lambda B y, M y = lambda B x, dense B = Q diag(beta) Q^T, Q Haar, "
                  "beta log-uniform on [0.25, 4] (Cholesky reduction set up before the timed solves)")
        elif w.get("metric_seed"):
            z += "; generalized LREP K x = lambda B y, M y = lambda B x, B = diag(b), b log-uniform on [0.25, 4]"
        return (f"dense FP64 n={w['n']}: K=Q1 diag(k) Q1^T, M=Q2 diag(m) Q2^T, Haar Q1/Q2, k,m~U[0.5,10]{z}; "
                f"nev={w['nev']}, block={w['block']}, window={w['window']}, tol={w['tol']:g}")
    z = "; Step-6 CG passes read an FP32 copy of L's rows (FP64 products)" if w.get("precision", 0) == 4 else ""
    return (f"Casida low-rank FP64 n={w['n']}: K=diag(delta), M=diag(delta)+2LL^T, delta~U[0.1,20] sorted, "
            f"L n x {w['rank']} Gaussian/sqrt(n){z}; nev={w['nev']}, block={w['block']}, window={w['window']}, "
            f"tol={w['tol']:g}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="casida262144", choices=sorted(WORKLOADS) + ["serve"])
    ap.add_argument("--requests", type=int, default=512, help="serve: number of requests (the configuration's 512)")
    ap.add_argument("--serve-pool", choices=["mixed", "shared"], default="mixed",
                    help="serve: the configuration's pool of 6 dense + 6 low-rank operators, or 'shared': every "
                         "request on one dense (n = 8192) or one low-rank (n = 65536, rank 128) operator")
    ap.add_argument("--serve-batch", type=int, default=0, choices=[-1, 0],
                    help="serve: Step-6 CG solves of concurrent requests on one operator batched (0) or not (-1)")
    ap.add_argument("--sequential", type=int, default=1, choices=[0, 1],
                    help="serve: also run the same requests one at a time through lrep_solve (the comparison)")
    ap.add_argument("--serve-sizes", choices=["reduced", "full"], default="reduced",
                    help="serve: operator size ranges (full: dense n <= 16384, low-rank n <= 262144)")
    ap.add_argument("--budget-gib", type=float, default=0.0, help="serve: HBM budget of the context (0: none)")
    ap.add_argument("--rho", type=float, default=0.7,
                    help="serve: Poisson arrival rate as a fraction of the closed-loop solve rate")
    ap.add_argument("--graphs", type=int, default=0, choices=[-1, 0, 1],
                    help="Step 6 as a replayed HIP graph: 1 on, -1 off, 0 the library's default")
    ap.add_argument("--fused-cg", type=int, default=0, choices=[-1, 0, 1],
                    help="low-rank operators: Step-6 CG as one pass per step (0 or 1, the default) or the plain "
                         "two-pass CG (-1)")
    ap.add_argument("--cpu-iters", type=int, default=-1,
                    help="outer iterations of the CPU oracle baseline (0: skip; -1: the workload's default, "
                         "to convergence where that takes about a minute on the host, else a bounded sample)")
    ap.add_argument("--operator-cache", default="", metavar="NPZ",
                    help="dense workloads: load K, M from this .npz if it exists, else generate and save them "
                         "(lets profiler passes skip the device QR of the generator)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run one plain device copy of MIB MiB (counter calibration) and exit")
    ap.add_argument("--hbm-probe", type=int, default=0, metavar="MIB",
                    help="only time the library's plain streaming read kernel over MIB MiB and exit")
    args = ap.parse_args()
    if args.hbm_probe:
        hbm_probe(args.hbm_probe)
        return
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the solver runs on a single MI355X; "
              "--gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import gen
    import paper_2506_08355_amd as L

    if args.workload == "serve":
        serve(args, np, torch, gen, L)
        return
    w = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    n, nev, block, window, tol = w["n"], w["nev"], w["block"], w["window"], w["tol"]
    t0 = time.time()
    print(f"[bench] generating {args.workload} ...", file=sys.stderr, flush=True)
    if w["kind"] == "dense":
        cache = args.operator_cache
        if w["zeros"] and cache:
            raise SystemExit("the operator cache does not hold the null basis of the zero variant")
        if cache and os.path.exists(cache):
            with np.load(cache, allow_pickle=False) as z:
                if int(z["n"]) != n or int(z["seed"]) != w["seed"]:
                    raise SystemExit(f"{cache} holds another workload")
                Kd, Md = torch.from_numpy(z["K"]).to(dev), torch.from_numpy(z["M"]).to(dev)
                kk, mm = z["k"], z["m"]
        else:
            Kd, Md, kk, mm, _, Q2 = gen.dense_operator_device(n, w["seed"], dev, n_zero_m=w["zeros"],
                                                               return_factors=True)
            if w["zeros"]:
                null = np.asfortranarray(Q2.cpu().numpy()[:, mm == 0.0])
            del Q2
            if cache:
                np.savez(cache, K=Kd.cpu().numpy(), M=Md.cpu().numpy(), k=kk, m=mm, n=n, seed=w["seed"])
        normH = float(max(kk.max(), mm.max()))
    else:
        f = gen.casida_factors(n, w["rank"], w["seed"])
        delta_d = torch.from_numpy(f.delta).to(dev)
        L_d = torch.from_numpy(np.ascontiguousarray(f.L.T)).to(dev).T
        normH = None
    U0, _ = gen.init_block(n, block + 2 * window, START_BLOCK_SEED)
    U0d = torch.from_numpy(np.ascontiguousarray(U0.T)).to(dev).T
    torch.cuda.synchronize()
    print(f"[bench] inputs ready in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)

    ctx = L.lrep_init(0)
    metric_setup_ms = None
    if w["kind"] == "dense":
        op = L.lrep_create_dense(ctx, Kd.T, Md.T, L.LREP_NULL_ON_M if w["zeros"] else 0)
        if w.get("metric_dense"):
            Bmat = torch.from_numpy(np.ascontiguousarray(gen.metric_dense(n, w["metric_seed"]).T)).to(dev).T
            torch.cuda.synchronize()
            tm = time.perf_counter()
            L.lrep_set_metric_dense(op, Bmat, ctx)
            metric_setup_ms = (time.perf_counter() - tm) * 1e3
            print(f"[bench] dense metric set up in {metric_setup_ms:.1f} ms", file=sys.stderr, flush=True)
        elif w.get("metric_seed"):
            bmetric = gen.metric_diag(n, w["metric_seed"])
            L.lrep_set_metric(op, bmetric, ctx)
        if w["zeros"]:
            L.lrep_set_nullspace(op, null, ctx)     # the 8 columns of Q2 with m = 0
    else:
        op = L.lrep_create_lowrank(ctx, delta_d, L_d)
    lam = torch.zeros(nev, dtype=torch.float64, device=dev)
    X = torch.zeros(nev, n, dtype=torch.float64, device=dev).T
    Y = torch.zeros(nev, n, dtype=torch.float64, device=dev).T

    def step(profile):
        opts = L.make_opts(window=window, init=U0d, profile=profile, precision=w.get("precision", 0),
                           graphs=args.graphs, fused_cg=args.fused_cg)
        rc, st = L.lrep_solve(op, n, nev, block, tol, opts, lam, X, Y, ctx=ctx)
        return st

    for i in range(args.warmup):
        st = step(False)
        print(f"[bench] warmup {i}: {st.time_ms:.1f} ms, {st.iterations} iterations", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    lat = []
    iters = 0
    restores = 0
    t_start = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        st = step(False)
        lat.append((time.perf_counter() - ts) * 1e3)
        iters = st.iterations
        restores = st.rebiorth
        print(f"[bench] step {i}: {lat[-1]:.1f} ms, {st.iterations} iterations, {st.rebiorth} restores, "
              f"applies K/M {st.applies_K}/{st.applies_M}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    value = nev * args.steps / total

    # one profiled solve outside the timed region: HIP events around every CG
    # apply and at the phase boundaries (the roofline and the phase split)
    tp = time.perf_counter()
    st = step(True)
    torch.cuda.synchronize()
    profiled_ms = (time.perf_counter() - tp) * 1e3
    prof_ms, prof_bytes, prof_flops, prof_launches = st.prof_ms, st.prof_bytes, st.prof_flops, st.prof_launches
    phase_ms = list(st.phase_ms)
    print(f"[bench] profiled solve: {profiled_ms:.1f} ms, {st.iterations} iterations, {prof_launches} timed "
          f"applies", file=sys.stderr, flush=True)

    # accuracy of the last result, independently of the library (torch FP64 products)
    with torch.no_grad():
        if w["kind"] == "dense":
            KX, MY = Kd @ X, Md @ Y
        else:
            KX = delta_d[:, None] * X
            MY = delta_d[:, None] * Y + 2.0 * (L_d @ (L_d.T @ Y))
            if normH is None:
                v = torch.randn(n, dtype=torch.float64, device=dev)
                for _ in range(30):
                    v = delta_d * v + 2.0 * (L_d @ (L_d.T @ v))
                    v = v / torch.linalg.norm(v)
                normH = float(torch.dot(v, delta_d * v + 2.0 * (L_d @ (L_d.T @ v))))
        if w.get("metric_seed"):
            # generalized pencil: residuals K x - lambda B y, M y - lambda B x over
            # (||H|| + lambda ||B||) ||(x, y)||, and Y^T B X = I
            if w.get("metric_dense"):
                applyB = lambda V: Bmat @ V
                normB = float(torch.linalg.matrix_norm(Bmat, 2))
            else:
                bd = torch.from_numpy(bmetric).to(dev)[:, None]
                applyB = lambda V: bd * V
                normB = float(bmetric.max())
            BX, BY = applyB(X), applyB(Y)
            R1 = KX - BY * lam[None, :]
            R2 = MY - BX * lam[None, :]
            res = torch.sqrt((R1 ** 2).sum(0) + (R2 ** 2).sum(0)) / (
                (normH + lam * normB) * torch.sqrt((X ** 2).sum(0) + (Y ** 2).sum(0)))
            biorth = float((Y.T @ BX - torch.eye(nev, dtype=torch.float64, device=dev)).abs().max())
        else:
            R1 = KX - Y * lam[None, :]
            R2 = MY - X * lam[None, :]
            res = torch.sqrt((R1 ** 2).sum(0) + (R2 ** 2).sum(0)) / (
                normH * torch.sqrt((X ** 2).sum(0) + (Y ** 2).sum(0)))
            biorth = float((X.T @ Y - torch.eye(nev, dtype=torch.float64, device=dev)).abs().max())
        max_res = float(res.max())

    achieved = prof_bytes / (prof_ms * 1e-3) / 1e9 if prof_ms > 0 else None
    roofline = None
    if achieved is not None:
        traffic = measured_traffic(args.workload)
        if w["kind"] == "dense" and w.get("precision", 0) == 3:
            kname = "apply16x3_stream_kernel (BF16x3 CG block apply: three BF16 operator parts, w=%d)" % window
            abytes = 6.0 * n * n + 14.0 * n * window
        elif w["kind"] == "dense" and w.get("precision", 0):
            kname = "apply16_stream_kernel (16-bit CG block apply, w=%d)" % window
            abytes = 2.0 * n * n + 10.0 * n * window
        elif w["kind"] == "dense":
            kname = "apply_stream_kernel (CG block apply, w=%d)" % window
            abytes = 8.0 * n * n + 16.0 * n * window
        elif w.get("precision", 0) == 4:
            kname = ("fcg_pass_M_kernel<float> (fused CG step on M = diag(delta) + 2 L L^T, w=%d: FP32 rows of L "
                     "read once, x, r, p read and written, delta read)" % window)
            abytes = 4.0 * n * w["rank"] + 48.0 * n * window + 8.0 * n
        else:
            kname = ("fcg_pass_M_kernel (fused CG step on M = diag(delta) + 2 L L^T, w=%d: L read once, "
                     "x, r, p read and written, delta read)" % window)
            abytes = 8.0 * n * w["rank"] + 48.0 * n * window + 8.0 * n
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "algorithmic_bytes_per_launch": abytes,
                    "kernel": kname,
                    "launches": prof_launches, "avg_us": round(prof_ms * 1e3 / max(prof_launches, 1), 2),
                    "tflops": round(prof_flops / (prof_ms * 1e-3) / 1e12, 2),
                    "tflops_frac_fp64": round(prof_flops / (prof_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4)}

    cpu = None
    cpu_iters = w.get("cpu_iters", 0) if args.cpu_iters < 0 else args.cpu_iters
    if args.cpu_iters != 0:
        import oracle
        try:
            import threadpoolctl
            info = threadpoolctl.threadpool_info()
            cores = max([i.get("num_threads", 1) for i in info] or [os.cpu_count()])
        except Exception:
            cores = os.cpu_count()
        what = f"{cpu_iters} iterations" if cpu_iters else "to convergence"
        print(f"[bench] CPU oracle baseline: {what} ...", file=sys.stderr, flush=True)
        if w["kind"] == "dense" and w.get("metric_dense"):
            # the transformed pencil L^-1 K L^-T, L^-1 M L^-T (B = L L^T) that the library solves
            import scipy.linalg as sla
            Lc = np.linalg.cholesky(Bmat.cpu().numpy())
            def _tr(A):
                T = sla.solve_triangular(Lc, A, lower=True)
                T = sla.solve_triangular(Lc, T.T, lower=True)
                return 0.5 * (T + T.T)
            cop = oracle.DenseOperator(_tr(Kd.cpu().numpy()), _tr(Md.cpu().numpy()))
        elif w["kind"] == "dense" and w.get("metric_seed"):
            # the scaled pencil S K S, S M S (S = B^-1/2) that the library solves
            sv = 1.0 / np.sqrt(bmetric)
            cop = oracle.DenseOperator(sv[:, None] * Kd.cpu().numpy() * sv[None, :],
                                       sv[:, None] * Md.cpu().numpy() * sv[None, :])
        elif w["kind"] == "dense":
            cop = oracle.DenseOperator(Kd.cpu().numpy(), Md.cpu().numpy())
        else:
            cop = oracle.CasidaOperator(f.delta, f.L)
        tc = time.perf_counter()
        extra = dict(X0=null, null_on_M=True) if w.get("zeros") else {}
        if cpu_iters:
            extra["maxit"] = cpu_iters
        r = oracle.bosp_solve(cop, nev, block, tol, window=window, init=(U0, U0), **extra)
        tcpu = time.perf_counter() - tc
        if not r.converged:
            per_it = tcpu / max(r.iterations, 1)
            cpu = {"value": round(nev / (per_it * iters), 4), "unit": "eigenpairs/s", "cores": cores,
                   "kind": "oracle",
                   "sample": f"oracle BOSP on the same operator and start block: start-up and {r.iterations} "
                             f"outer iteration(s) in {tcpu:.1f}s, scaled to the {iters} iterations the GPU solve "
                             f"needed (a solve to convergence would take hours on the host)"}
        else:
            cpu = {"value": round(nev / tcpu, 4), "unit": "eigenpairs/s", "cores": cores, "kind": "oracle",
                   "sample": f"oracle BOSP on the same operator and start block, solved to convergence: "
                             f"{r.iterations} outer iterations (the GPU solve: {iters}) in {tcpu:.1f}s",
                   "iterations": r.iterations}

    lat_s = sorted(lat)
    out = {
        "metric": "eigenpairs/s at 1e-8 residual; MFMA/HBM roofline fraction; p50/p99 solve latency",
        "value": round(value, 3), "unit": "eigenpairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(total * 1e3 / args.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {0: "f64", 1: "bf16 CG applies (f32 accumulate), f64 elsewhere",
                  2: "f16 CG applies (f32 accumulate), f64 elsewhere",
                  3: "bf16x3 CG applies (f32 accumulate), f64 elsewhere",
                  4: "f64 (CG passes read an f32 copy of L)"}[w.get("precision", 0)],
        "data": "synthetic",
        "config": {"workload": describe(w), "n": n, "nev": nev, "block": block, "window": window, "tol": tol,
                   "seed": w["seed"], "start_block_seed": START_BLOCK_SEED, "parallelism": "single GPU"},
        "p50_ms": round(lat_s[len(lat_s) // 2], 3), "p99_ms": round(lat_s[min(len(lat_s) - 1, int(0.99 * len(lat_s)))], 3),
        "iterations": iters, "biorth_restores": restores, "max_residual_Hnorm": max_res, "biorth": biorth,
        "phase_ms_per_solve": dict(zip(["init", "small_problem", "convergence_check", "pq", "wz"],
                                       [round(v, 2) for v in phase_ms])),
        "profiled_solve_ms": round(profiled_ms, 1),
        "roofline": roofline, "cpu_baseline": cpu,
    }
    if metric_setup_ms is not None:
        out["metric_setup_ms"] = round(metric_setup_ms, 1)   # one-time, outside the timed solves
    L.lrep_destroy_op(op)
    L.lrep_finalize(ctx)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
