/* A whole solve through the C ABI from plain C99, with host arrays: reads
 * n, nev, block, tol and column-major K, M, U0 (float64) from a file, solves,
 * and writes lambda, X, Y to another file (tests/test_gpu_cabi.py checks
 * them against the oracle).  Usage: abi_solve IN OUT */
#include <stdio.h>
#include <stdlib.h>

#include "lrep.h"

static int rd(FILE* f, void* p, size_t sz, size_t cnt) { return fread(p, sz, cnt, f) == cnt ? 0 : 1; }

int main(int argc, char** argv) {
    if (argc != 3) return 10;
    FILE* fi = fopen(argv[1], "rb");
    if (!fi) return 11;
    int64_t hdr[4];
    double tol;
    if (rd(fi, hdr, sizeof(int64_t), 4) || rd(fi, &tol, sizeof(double), 1)) return 12;
    const int64_t n = hdr[0], nev = hdr[1], block = hdr[2], d0 = hdr[3];
    double* K = malloc(sizeof(double) * n * n);
    double* M = malloc(sizeof(double) * n * n);
    double* U = malloc(sizeof(double) * n * d0);
    double* lam = malloc(sizeof(double) * nev);
    double* X = malloc(sizeof(double) * n * nev);
    double* Y = malloc(sizeof(double) * n * nev);
    if (!K || !M || !U || !lam || !X || !Y) return 13;
    if (rd(fi, K, sizeof(double), n * n) || rd(fi, M, sizeof(double), n * n) || rd(fi, U, sizeof(double), n * d0))
        return 14;
    fclose(fi);

    lrep_ctx_t ctx = NULL;
    lrep_op_t op = NULL;
    int rc = lrep_init(&ctx, 0, 0, NULL);
    if (rc != LREP_OK) return 20;
    rc = lrep_create_dense(ctx, n, K, M, n, 0, &op);
    if (rc != LREP_OK) return 21;
    lrep_solve_opts_t opts = {0};
    opts.init_U = U;
    opts.ld_init = n;
    lrep_stats_t st;
    rc = lrep_solve(op, n, nev, block, tol, &opts, lam, X, Y, n, &st);
    if (rc != LREP_OK) {
        fprintf(stderr, "lrep_solve: %s (%s)\n", lrep_strerror(rc), lrep_last_error(ctx));
        return 22;
    }
    printf("iterations %lld converged %lld max_eps %.3e\n", (long long)st.iterations, (long long)st.n_converged,
           st.max_eps);
    lrep_destroy_op(op);
    lrep_finalize(ctx);

    FILE* fo = fopen(argv[2], "wb");
    if (!fo) return 30;
    if (fwrite(lam, sizeof(double), nev, fo) != (size_t)nev || fwrite(X, sizeof(double), n * nev, fo) != (size_t)(n * nev) ||
        fwrite(Y, sizeof(double), n * nev, fo) != (size_t)(n * nev))
        return 31;
    fclose(fo);
    free(K);
    free(M);
    free(U);
    free(lam);
    free(X);
    free(Y);
    return 0;
}
