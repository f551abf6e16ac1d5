/*
 * lrep.h -- C ABI of the MI355X (gfx950) BOSP eigensolver for the linear
 * response eigenvalue problem (LREP).
 *
 * Problem (paper Section 1, change of variables u = y + x, v = y - x):
 *
 *     [[A, B], [-B, -A]] [u; v] = lambda [u; v]   <=>   H [y; x] = lambda [y; x],
 *     H = [[0, K], [M, 0]],  K = A - B,  M = A + B,
 *
 * i.e. K x = lambda y and M y = lambda x, with K symmetric positive
 * semi-definite and M symmetric positive definite (or the reverse, see
 * LREP_NULL_ON_M).  lrep_solve returns the nev smallest positive eigenvalues
 * in ascending order with X^T Y = I (Algorithm "BOSP algorithm", Sections
 * 3.2-3.3 of the paper).
 *
 * Conventions for every entry point
 *   - matrices are column-major IEEE FP64 with an explicit leading dimension
 *     (ld >= number of rows);
 *   - pointers are host pointers unless a flag or option says "device"
 *     (a device pointer is a HIP device allocation on the context's device);
 *   - the library runs on its own non-blocking streams (or the stream given
 *     to lrep_init) and does not order itself after any other stream: the
 *     data behind a device pointer must be complete when the call is made
 *     (synchronize the stream that produced it first), and a blocking call
 *     returns only after its device results are written;
 *   - every function returns 0 (LREP_OK) or a negative LREP_E* code and never
 *     aborts; lrep_strerror(code) gives a static message and
 *     lrep_last_error(ctx) the detail of the last failure on a context;
 *   - the library owns every workspace it allocates; the caller owns every
 *     buffer it passes.
 */
#ifndef LREP_H
#define LREP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- codes */
#define LREP_OK           0
#define LREP_EINVAL      -1   /* bad argument: sizes, null pointer, nev > n - r, ...   */
#define LREP_ENOMEM      -2   /* HBM budget of the context or hipMalloc exhausted       */
#define LREP_ENOTCONV    -3   /* maxit reached; converged prefix written, count in stats */
#define LREP_EBREAKDOWN  -4   /* MGS-Biorth dropped so many columns that the subspace
                                 cannot hold the requested Ritz block                   */
#define LREP_ENOTSPD     -5   /* Cholesky of a projected matrix failed (operator not
                                 SPD on the subspace)                                   */
#define LREP_ENUMERIC    -6   /* NaN or Inf met (operator or iteration)                 */
#define LREP_EDEVICE     -7   /* HIP runtime error, detail in lrep_last_error           */
#define LREP_EAGAIN      -8   /* lrep_poll: request still pending                        */
#define LREP_ECANCELED   -9   /* lrep_poll: request was cancelled                        */

/* ---------------------------------------------------------------- flags */
#define LREP_DEVICE_PTR  0x1u /* operator arrays are device pointers                   */
#define LREP_BORROW      0x2u /* with LREP_DEVICE_PTR: use the caller's device arrays in
                                 place (caller keeps them alive and unchanged until
                                 lrep_destroy_op); otherwise they are copied            */
#define LREP_INPUT_AB    0x4u /* dense: the two matrices are A and B; the library forms
                                 K = A - B and M = A + B (paper Section 1)              */
#define LREP_NULL_ON_M   0x8u /* the semi-definite operator is M, not K: the solver
                                 exchanges the roles of K and M (exact:
                                 K x = l y, M y = l x <=> M y = l x, K x = l y with
                                 x, y exchanged) and exchanges X, Y back on output    */

typedef struct lrep_ctx_s* lrep_ctx_t;
typedef struct lrep_op_s*  lrep_op_t;
typedef uint64_t           lrep_ticket_t;

/* Solver options.  Zero-initialise and set what you need; every zero field
 * takes the documented default. */
typedef struct lrep_solve_opts {
    int64_t window;        /* w = n_b, width of the P/Q and W/Z blocks (default: block) */
    int64_t maxit;         /* outer iterations (default 1000)                          */
    int32_t ngs;           /* block Gauss-Seidel sweeps in Step 6 (default 1)           */
    int32_t cg_maxit;      /* CG iterations per solve (default 20)                      */
    double  cg_tol;        /* CG relative residual tolerance (default 1e-2)             */
    uint64_t seed;         /* seed of the library's own starting block (Philox4x32-10,
                              Box-Muller) when init_U is NULL                           */
    const double* init_U;  /* optional starting block, n x (block + 2 window), ld_init;
                              used for both U and V (the paper's Step 1)                */
    int64_t ld_init;
    int32_t init_on_device;   /* init_U is a device pointer                             */
    int32_t result_on_device; /* lambda, X, Y are device pointers                       */
    int32_t precision;        /* 0: FP64 everywhere (default).  Dense operators only:
                                 1: the CG applies of Step 6 use a BF16 copy of K and
                                 M and a BF16 copy of the CG block, FP32 accumulation
                                 (MFMA), FP64 result; 2: the same in FP16 with each CG
                                 column scaled by a power of two; 3: BF16x3, the
                                 operator and the CG block each split into three
                                 BF16 parts (hi, mid, lo) and the six part products
                                 of order <= 2 summed in FP32 (an FP32-accurate
                                 product).  Everything else (Rayleigh-Ritz images,
                                 residuals, MGS-Biorth, small problem) stays FP64.
                                 The 16-bit copies (2 n^2 bytes each, 6 n^2 for
                                 BF16x3, charged to the context budget) are made at
                                 the first such solve and kept with the operator; n
                                 must be a multiple of 8.  Low-rank operators ignore
                                 1-3.  4 (low-rank operators with rank >= 1 only,
                                 else LREP_EINVAL): the fused CG steps of Step 6 read
                                 an FP32 copy of L's rows (each value rounded to
                                 nearest even once, widened exactly to FP64 in the
                                 kernel; FP64 products and sums), half the bytes of L
                                 per step; the CG solves the system of diag(delta) +
                                 2 L~ L~^T with L~ the rounded L, a relative change of
                                 ~1e-7, far below the CG's 1e-2 tolerance.  The copy
                                 (4 n ceil64(rank) bytes, charged to the budget) is
                                 made at the first such solve.                        */
    int32_t profile;          /* 1: time every Step-6 operator apply with HIP events on
                                 the solve's stream (results in lrep_stats_t.prof_*)  */
    double  rebiorth_tol;  /* re-biorthogonalise U,V when max|U^T V - I| exceeds this
                              (default 1e-12)                                          */
    int32_t refresh;       /* longest interval, in iterations, between applications of
                              K and M to the whole subspace (default 8; 1 = every
                              iteration).  In between, K U and M V follow the basis
                              through the same coefficient products (Ritz pull-back,
                              P~ = U P^) and only the new W~, Z~ block is applied.
                              The interval starts at 2 and adapts to the measured
                              relative drift of the carried images (halved at
                              1e-2 tol, doubled below 1e-3 tol); images are always
                              fresh after a biorthogonality restoration and before
                              pairs are locked or returned.                           */
    int32_t graphs;        /* 1: Step 6 (right-hand sides, both CG solves, copies)
                              as a HIP graph, captured once per block width and
                              basis buffer and replayed; 0 (default) or -1: issued
                              on the stream.  The replay issues all cg_maxit CG
                              steps; steps after convergence return at once on the
                              device flag.  Results are bitwise those of the
                              stream path.  Ignored for callback operators and
                              with profile.                                           */
    int32_t fused_cg;      /* low-rank operators: 0 (default) or 1: each CG step of
                              Step 6 is one pass over the rows (direction update,
                              product, x and r updates; L read once per step, with
                              L^T p carried by the direction recurrence); -1: the
                              plain CG (L^T p and L (L^T p) as two passes, then
                              separate vector updates).  Same iteration, different
                              rounding order.                                         */
    int32_t serve_batch;   /* served requests (lrep_submit) on dense or low-rank
                              operators: 0 (default) -- a Step-6 CG solve that
                              starts while a CG of another request on the same
                              operator (same CG settings) runs on the device
                              waits for it; the solves then waiting run as one
                              block CG over their concatenated columns (at most
                              32), the operator streamed once per step for all
                              (one such block CG per operator at a time); every column's
                              arithmetic is the one it has alone, so results are
                              bitwise those of the request alone.  -1: never.
                              Ignored by lrep_solve.                                 */
} lrep_solve_opts_t;

/* Per-solve statistics (all optional to read). */
typedef struct lrep_stats {
    int64_t iterations;        /* outer iterations run                                 */
    int64_t n_converged;       /* eigenpairs written (== nev on LREP_OK)               */
    int64_t applies_K;         /* column mat-vecs with K (served with batching: those
                                  of the block CGs this request led, other requests'
                                  columns included)                                  */
    int64_t applies_M;         /* column mat-vecs with M (likewise)                    */
    int64_t mgs_drops;         /* columns dropped by MGS-Biorth breakdown handling      */
    int64_t locks;             /* moving-mechanism lock events                          */
    int64_t rebiorth;          /* biorthogonality restorations                          */
    double  max_eps;           /* max Step-4 residual of the returned pairs            */
    double  time_ms;           /* wall time of the solve                               */
    /* per-phase GPU time (ms) in the paper's five buckets: initialise U,V /
       small-scale problem (incl. projection and pull-back) / convergence check /
       P,Q / W,Z (incl. CG and MGS-Biorth)                                         */
    double  phase_ms[5];
    /* with opts.profile: the block operator applies of the CG inner solves
       (w columns each), timed kernel by kernel with HIP events               */
    int64_t prof_launches;     /* timed apply-kernel launches                          */
    double  prof_ms;           /* their summed GPU time                                */
    double  prof_bytes;        /* algorithmic bytes they move (operator read once,
                                  block read once, result written once)               */
    double  prof_flops;        /* algorithmic flops (2 n^2 w dense)                     */
    int64_t cg_batched;        /* served: Step-6 CG solves of this request that ran
                                  in one block CG with other requests' columns       */
    int64_t cg_batch_columns;  /* served: CG columns of other requests that ran in
                                  the block CGs this request's worker thread led    */
} lrep_stats_t;

/* Request for the serving interface (lrep_submit). */
typedef struct lrep_request {
    int64_t nev;
    int64_t block;
    double  tol;
    lrep_solve_opts_t opts;    /* as for lrep_solve; result_on_device applies        */
    double* lambda;            /* nev                                                 */
    double* X;                 /* n x nev, ld = ldxy                                  */
    double* Y;
    int64_t ldxy;
} lrep_request_t;

/* ------------------------------------------------------------ context */

/* Create a context on HIP device `device`.  `hbm_budget_bytes` caps the
 * device memory the context may hold for operators and workspaces (0 = no
 * cap beyond the device).  `hip_stream` is a hipStream_t to run on, or NULL
 * for a stream the context creates (default priority).
 * Errors: LREP_EINVAL (bad device), LREP_EDEVICE. */
int lrep_init(lrep_ctx_t* ctx, int device, size_t hbm_budget_bytes, void* hip_stream);

/* Destroy the context: cancels pending requests, waits for the running one,
 * frees every workspace.  Operators must be destroyed first (else they are
 * destroyed here). */
int lrep_finalize(lrep_ctx_t ctx);

/* ----------------------------------------------------------- operators */

/* Dense operator (paper equation for H).  K and M are n x n symmetric,
 * column-major with leading dimension ld (with LREP_INPUT_AB they are A and
 * B).  Only the lower triangle is read when symmetrising is not needed; both
 * triangles are used by the apply.  Host arrays are copied to HBM; device
 * arrays are copied, or borrowed with LREP_BORROW.
 * Errors: LREP_EINVAL (n < 1, ld < n, null pointer), LREP_ENOMEM, LREP_EDEVICE. */
int lrep_create_dense(lrep_ctx_t ctx, int64_t n, const double* K, const double* M,
                      int64_t ld, uint32_t flags, lrep_op_t* op);

/* Diagonal-plus-low-rank (Casida-type) operator, matrix-free:
 *     K = diag(delta),  M = diag(delta) + 2 L L^T,
 * delta: n values (> 0), L: n x rank column-major with leading dimension ldl.
 * Storage on the device is n + n*rank doubles.
 * Errors: LREP_EINVAL, LREP_ENOMEM, LREP_EDEVICE. */
int lrep_create_lowrank(lrep_ctx_t ctx, int64_t n, int64_t rank, const double* delta,
                        const double* L, int64_t ldl, uint32_t flags, lrep_op_t* op);

/* Matrix-free operator: the method touches K and M only through block
 * products (Section 3.2), so an operator may be supplied as a function
 *   apply(user, which, cols, X, ldx, Y, ldy, stream)
 * that makes Y = K X (which = 0) or Y = M X (which = 1) for the device
 * blocks X (n x cols, leading dimension ldx) and Y (n x cols, ld ldy), with
 * K and M as in lrep_create_dense (symmetric, M positive definite, or the
 * roles exchanged with LREP_NULL_ON_M).  The library's work that produces X
 * is already enqueued on `stream` (a hipStream_t); the function enqueues its
 * product on that stream, or finishes it before returning, and returns 0
 * (any other value ends the solve with LREP_EDEVICE).  It is called from
 * the thread that runs the solve (the caller of lrep_solve, or a serving
 * worker), from several threads at once when requests of the operator are
 * served concurrently.  `user` is passed through; the library holds no
 * device memory for the operator.  Mixed precision (opts.precision) does
 * not apply to it.
 * Errors: LREP_EINVAL. */
typedef int (*lrep_apply_fn)(void* user, int32_t which, int64_t cols, const double* X, int64_t ldx, double* Y,
                             int64_t ldy, void* stream);
int lrep_create_callback(lrep_ctx_t ctx, int64_t n, lrep_apply_fn apply, void* user, uint32_t flags,
                         lrep_op_t* op);

/* Declare the generalized null space (Lemma 2.3, Remark on computing V0):
 * X0 (n x r, ld) spans N(K) (or N(M) with LREP_NULL_ON_M).  The library
 * solves M Y0~ = X0~ by CG on the device, factors X0~^T Y0~ = C^T C and keeps
 * X0 = X0~ C^-1, Y0 = Y0~ C^-1 (equation for the V0 basis) so that every
 * later iterate is biorthogonal to V0.  r = 0 clears it.
 * Errors: LREP_EINVAL, LREP_ENOTSPD (X0~^T Y0~ not SPD), LREP_ENOMEM. */
int lrep_set_nullspace(lrep_op_t op, int64_t r, const double* X0, int64_t ld, int32_t on_device);

/* Eigenvectors of the original problem [[A, B], [-B, -A]] [u; v] = lambda
 * [u; v] from the returned pairs, by the change of variables of Section 1:
 * U = Y + X, V = Y - X (each n x nev, column-major).  X, Y (ld ldxy) and
 * U, V (ld lduv) are device arrays of the context's device; U and V must not
 * overlap X or Y.  Blocking.
 * Errors: LREP_EINVAL, LREP_EDEVICE. */
int lrep_xy_to_uv(lrep_ctx_t ctx, int64_t n, int64_t nev, const double* X, const double* Y, int64_t ldxy, double* U,
                  double* V, int64_t lduv);

/* Allocation-free block apply, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): Y = K X (which = 0) or Y = M X (which = 1, after the
 * role exchange of LREP_NULL_ON_M), the products of lrep_test_apply, with X
 * and Y device arrays of n x cols (ld n, n = the operator's size) on the
 * operator's device.  Every intermediate lives in one fixed 40 MiB device
 * array of the library (one per device, held until the process ends); the
 * call allocates nothing and returns when Y is complete (the context's
 * stream is synchronised).  Calls on one device share that array: calls that
 * overlap on one device (other streams or contexts) race.  Limits: dense
 * operators n <= 73728 for cols <= 32; low-rank M applies rank * cols <=
 * 524288; beyond them LREP_EINVAL with the reason in lrep_last_error.
 * Errors: LREP_EINVAL, LREP_EDEVICE (also when the operator's callback
 * fails). */
int lrep_apply_noalloc(lrep_op_t op, int which, int cols, const double* X, double* Y);

/* Compute the null space instead of declaring it (the remark on computing the
 * generalized null space, Section 2.2: the zero eigenvectors of the
 * semidefinite operator A = K, or M with LREP_NULL_ON_M).  rmax (1..64,
 * below n) random vectors from `seed` are projected onto N(A) by CG on
 * A x = A x0 from a zero start (x0 - x is x0's component in N(A)); the
 * projections are orthonormalised by block MGS, which drops dependent ones,
 * and projections at rounding level are discarded.  The basis found is then
 * declared as with lrep_set_nullspace (r = 0 clears any earlier one).
 * *r_out (required) receives its dimension r; r == rmax means N(A) may be
 * larger: call again with a larger rmax.  *res_out (may be NULL) receives
 * max ||A z|| / ||A||_est over the orthonormal basis vectors, with ||A||_est =
 * max ||A x0|| / ||x0|| over the random vectors.
 * Errors: LREP_EINVAL, LREP_ENOTCONV (that residual above tol: the operator
 * is too ill-conditioned for the CG to separate N(A); the operator is then
 * left without a null space), LREP_ENUMERIC (A zero or not finite),
 * LREP_ENOTSPD, LREP_ENOMEM, LREP_EDEVICE. */
int lrep_find_nullspace(lrep_op_t op, int64_t rmax, double tol, uint64_t seed, int64_t* r_out, double* res_out);

/* Generalized LREP with a diagonal SPD metric (the remark on the generalized
 * LREP in Section 3.2; Example 4.5 has this form):
 *     K x = lambda B y,   M y = lambda B x,   B = diag(b), b_i > 0,
 * solved in the B inner product <u, v>_B = u^T B v.  b (n values, host, or
 * device with LREP_DEVICE_PTR in flags; n must equal the operator's) is read
 * once.  With S = B^-1/2 the
 * pencil is the standard LREP of S K S and S M S in x^ = B^1/2 x, y^ =
 * B^1/2 y, and Euclidean MGS-Biorth on (x^, y^) is MGS-Biorth in the B inner
 * product on (x, y); the library scales its copy of the operator once
 * (dense: K and M; low rank: delta and L) and keeps S.  Afterwards:
 *   - lrep_set_nullspace takes X0 spanning N(K) (or N(M)) in the original
 *     coordinates;
 *   - a start block in opts.init is taken in the original coordinates;
 *   - lrep_solve returns X, Y in the original coordinates with
 *     Y^T B X = I, and stats.max_eps / the convergence test use the
 *     residual of the scaled pencil, ||S (K x - lambda B y)|| and
 *     ||S (M y - lambda B x)||, over (1 + lambda) ||(x^, y^)||.
 * Call it at most once per operator, before lrep_set_nullspace, and not
 * while a solve of the operator runs.  Operators from lrep_create_callback
 * and operators that borrow the caller's arrays (LREP_BORROW) are refused:
 * their data is not the library's to scale (a callback can apply S K S
 * itself).  Nothing is changed when an error is returned.
 * Errors: LREP_EINVAL (also for an entry of b that is not positive and
 * finite), LREP_ENOMEM, LREP_EDEVICE. */
int lrep_set_metric(lrep_op_t op, int64_t n, const double* b, uint32_t flags);

/* The same generalized LREP with a dense SPD metric B (n x n, column-major,
 * ld ldb >= n, host, or device with LREP_DEVICE_PTR; only its lower triangle
 * is read), for dense operators.  With the Cholesky factor B = L L^T the
 * pencil is the standard LREP of L^-1 K L^-T and L^-1 M L^-T in x^ = L^T x,
 * y^ = L^T y, and Euclidean MGS-Biorth on (x^, y^) is MGS-Biorth in the B
 * inner product on (x, y).  The library factors B on the device (blocked,
 * 64-wide diagonal blocks), replaces its copies of K and M by the transformed
 * (symmetrised) operators and keeps L^T and L^-T (2 n^2 doubles) for the
 * coordinate changes; the one-time cost is about 6 n^3 flops on the MFMA
 * products.  Null-space bases, start blocks and results are in the original
 * coordinates as with lrep_set_metric, and the stopping rule measures
 * ||L^-1 (K x - lambda B y)|| and ||L^-1 (M y - lambda B x)||.  The same
 * preconditions as lrep_set_metric hold; low-rank and callback operators are
 * refused.
 * Errors: LREP_EINVAL (also when B is not positive definite: a Cholesky pivot
 * is not positive; K and M are then unchanged), LREP_ENOMEM, LREP_EDEVICE (the
 * operator may then be partly transformed and must be destroyed). */
int lrep_set_metric_dense(lrep_op_t op, int64_t n, const double* B, int64_t ldb, uint32_t flags);

/* Free an operator's device memory (borrowed arrays are not freed). */
int lrep_destroy_op(lrep_op_t op);

/* --------------------------------------------------------------- solve */

/* Blocking solve on the context's stream (Algorithm "BOSP algorithm").
 *   n      must equal the operator's dimension;
 *   nev    number of eigenpairs, 1 <= nev <= n - r;
 *   block  width b of the Ritz block X (b = s * n_b under the moving
 *          mechanism); the subspace has d = b + 2w columns, w = opts->window;
 *          requires d <= n - r and d <= 128 (the small problem runs in one
 *          workgroup on the device);
 *   tol    stopping tolerance on ||H z - l z|| / ((1 + l) ||z||) (Section 4);
 *   lambda (nev), X, Y (n x nev, ld = ldxy) outputs, host or device per
 *          opts->result_on_device; X^T Y = I, K X = Y diag(lambda),
 *          M Y = X diag(lambda); each x is sign-normalised so that its
 *          entry of largest magnitude is positive.
 * Errors: LREP_EINVAL, LREP_ENOMEM, LREP_ENOTCONV (maxit reached: the
 * converged prefix is written, stats->n_converged says how many),
 * LREP_EBREAKDOWN, LREP_ENOTSPD, LREP_ENUMERIC, LREP_EDEVICE. */
int lrep_solve(lrep_op_t op, int64_t n, int64_t nev, int64_t block, double tol,
               const lrep_solve_opts_t* opts, double* lambda, double* X, double* Y,
               int64_t ldxy, lrep_stats_t* stats);

/* ------------------------------------------------------------- serving */

/* Queue a solve on `op` (thread-safe).  The request struct is copied; its
 * output buffers must stay valid until lrep_poll reports completion.
 * At submission the library computes the request's device footprint (every
 * workspace the solve allocates, and 16-bit operator copies it would make).
 * Four worker streams take queued requests in arrival order, passing over
 * any whose footprint does not fit the context's free HBM budget at that
 * moment; an admitted request reserves its whole footprint until it
 * completes, so it never waits for memory once started.  A request whose
 * footprint exceeds what the budget leaves beside the operators fails with
 * LREP_ENOMEM at poll time.  Admitted requests run concurrently; results are
 * identical to lrep_solve with the same arguments.
 * Errors: LREP_EINVAL (bad request: the checks of lrep_solve), LREP_EDEVICE
 * (the context's workers could not start). */
int lrep_submit(lrep_ctx_t ctx, lrep_op_t op, const lrep_request_t* req, lrep_ticket_t* ticket);

/* Completion status of a ticket (thread-safe, non-blocking): LREP_EAGAIN
 * while pending or running, otherwise the solve's own return code (once
 * reported, the ticket is released).  stats_out may be NULL. */
int lrep_poll(lrep_ctx_t ctx, lrep_ticket_t ticket, lrep_stats_t* stats_out);

/* Cancel a ticket that is still queued: LREP_OK, and lrep_poll then reports
 * LREP_ECANCELED.  A request already running (or finished) is not
 * interrupted: LREP_EAGAIN, and lrep_poll reports its own outcome.
 * LREP_EINVAL for an unknown ticket. */
int lrep_cancel(lrep_ctx_t ctx, lrep_ticket_t ticket);

/* ---------------------------------------------------------------- misc */
const char* lrep_strerror(int code);
const char* lrep_last_error(lrep_ctx_t ctx);
int lrep_version(void);   /* 100 * major + minor */

#ifdef __cplusplus
}
#endif
#endif /* LREP_H */
