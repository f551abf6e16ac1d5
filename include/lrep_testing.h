/*
 * lrep_testing.h -- kernel-level entry points of the BOSP library, exported
 * for the library's own unit tests.  Each runs one internal kernel family on
 * caller-owned device buffers, synchronously on the context's stream.  All
 * matrices are column-major FP64 device arrays; return 0 or an LREP_E* code.
 */
#ifndef LREP_TESTING_H
#define LREP_TESTING_H
#include "lrep.h"

#ifdef __cplusplus
extern "C" {
#endif

/* C (m x q, ldc) = alpha * A (m x p, lda) * B (p x q, ldb) + beta * C,
 * the FP64 MFMA product used by the dense apply and the pull-back.
 * ksplit > 0 forces the split of the p dimension (deterministic second
 * stage), 0 lets the library choose. */
int lrep_test_gemm_nn(lrep_ctx_t ctx, int m, int q, int p, const double* A, int64_t lda, const double* B,
                      int64_t ldb, double* C, int64_t ldc, double alpha, double beta, int ksplit);

/* C (p x q, ldc) = A^T B, A n x p (lda), B n x q (ldb): the tall-skinny Gram
 * product; symmetrize != 0 returns (C + C^T)/2 (p == q). */
int lrep_test_gemm_tn(lrep_ctx_t ctx, int n, int p, int q, const double* A, int64_t lda, const double* B,
                      int64_t ldb, double* C, int64_t ldc, int symmetrize);

/* Small structured LREP (Step 3): Kh, Mh d x d (ld ldh), d <= 128.
 * Outputs lam (d, ascending), Xh, Yh (d x d, ld 128).  Returns
 * LREP_ENOTSPD when a Cholesky factorisation fails. */
int lrep_test_small_lrep(lrep_ctx_t ctx, int d, const double* Kh, const double* Mh, int64_t ldh, double* lam,
                         double* Xh, double* Yh);

/* Block MGS-Biorth (two coefficient passes) of (X, Y), n x m, ld n, m <= 128,
 * in place; *kept receives the number of columns kept (compacted to the
 * front). */
int lrep_test_block_mgs(lrep_ctx_t ctx, int n, int m, double* X, double* Y, int* kept);

/* Y = A X for an operator (which = 0: K, 1: M, after the role exchange of
 * LREP_NULL_ON_M), X n x cols (ld n), Y n x cols (ld n). */
int lrep_test_apply(lrep_op_t op, int which, int cols, const double* X, double* Y);

/* One CG solve of Step 6 (the block Gauss-Seidel solves, Section 3.2): A X = B
 * for A = K (which = 0) or M (which = 1), nw <= 32 columns (B, X device, ld
 * n), zero start, per-column relative tolerance tol, at most maxit steps, as
 * the solver runs it: fused = 1 the fused low-rank CG, -1 the plain CG, 0 the
 * solver's choice.  *applies (nullable) receives the column applies made. */
int lrep_test_cg(lrep_op_t op, int which, int nw, const double* B, double* X, double tol, int maxit, int fused,
                 int64_t* applies);

/* out (n x n, ld n, 16-bit) = the BF16 (precision 1) or FP16 (precision 2)
 * copy of 0.5 (A + A^T) that the mixed-precision CG applies use: each value
 * rounded once, to nearest even, from FP64 to 16 bits.  Precision 3 (BF16x3):
 * three such matrices, the hi, mid and lo BF16 parts (each the rounding of
 * what the earlier parts leave), at out, out + n^2, out + 2 n^2.  A is a
 * device FP64 matrix (ld lda), out a device array of n * n 16-bit values
 * (3 n * n for precision 3). */
int lrep_test_convert16(lrep_ctx_t ctx, int precision, int n, const double* A, int64_t lda, uint16_t* out);

/* Y = A16 X through the mixed-precision CG apply: A16 a 16-bit copy made as
 * above, X scaled column by column by a power of two from rr[j] = |x_j|^2
 * before its conversion when precision is 2 (FP16), X split in three BF16
 * parts when precision is 3, FP32 accumulation, FP64 result.  X, rr and Y are device arrays, X and Y n x cols (ld n),
 * cols <= 32; n a multiple of 8, n >= 64. */
int lrep_test_apply16(lrep_ctx_t ctx, int precision, int n, int cols, const uint16_t* A16, const double* X,
                      const double* rr, double* Y);

/* out[b] = sum of block b's grid-stride share of src[0:count] (device FP64,
 * 16-byte aligned, count even; out holds `blocks` doubles), `iters` launches
 * back to back on the context's stream, *ms = their total time from HIP
 * events on that stream: a plain streaming read, the reference for the HBM
 * read rate the hardware reaches. */
int lrep_test_read(lrep_ctx_t ctx, const double* src, int64_t count, int blocks, int iters, double* out,
                   double* ms);

/* dst[0:count] = src[0:count] (device FP64 arrays, 16-byte aligned): a
 * plain streaming copy of known size, the reference against which hardware
 * byte counters (FETCH_SIZE, WRITE_SIZE) are scaled. */
int lrep_test_copy(lrep_ctx_t ctx, const double* src, double* dst, int64_t count);

#ifdef __cplusplus
}
#endif
#endif
