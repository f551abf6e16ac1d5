// Host-side launchers of the gfx950 kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <algorithm>

namespace lrep {

constexpr int kMaxSeg = 4;
constexpr int kMaxD = 128;     // largest subspace the one-workgroup small solver takes

// A column segment of a larger logical matrix.
struct Seg {
    const double* p;
    int64_t ld;
    int cols;
};

// Status words written by kernels and read back by the driver.
enum StatusSlot : int {
    ST_NOTSPD = 0,       // Cholesky failure in the small problem
    ST_NONFINITE = 1,    // NaN/Inf seen
    ST_NKEPT = 2,        // columns kept by the last coefficient MGS
    ST_NP = 3,           // columns of P^ kept by Step 5
    ST_SWEEPS = 4,       // Jacobi sweeps of the last small LREP
    ST_COUNT = 8
};

// Launchers taking `active_flag` skip all work when *active_flag == 0 (used
// by the CG loop, which runs a fixed number of launches without host syncs).
// ---- gemm.hip ------------------------------------------------------------
hipError_t gemm_nn(hipStream_t st, int m, int q, int p, const Seg* A, int nsegA,
                   const double* B, int64_t ldb, double* C, int64_t ldc, double alpha,
                   double beta, double* work, size_t work_elems,
                   const double* delta = nullptr, const double* Yd = nullptr,
                   int64_t ldyd = 0, int ksplit_hint = 0, const int* active_flag = nullptr,
                   hipEvent_t* ev = nullptr);   // ev[0], ev[1] recorded around the product kernel

// nb (<= 4) independent products C_i = alpha A_i B_i + beta C_i of one shape
// (A_i single segments) in a single launch.
hipError_t gemm_nn_batch(hipStream_t st, int m, int q, int p, int nb, const Seg* A,
                         const double* const* B, int64_t ldb, double* const* C, int64_t ldc,
                         double alpha, double beta);

hipError_t gemm_tn(hipStream_t st, int n, int p, int q, const Seg* A, int nsegA,
                   const Seg* B, int nsegB, double* C, int64_t ldc, double alpha,
                   int symmetrize, double* work, size_t work_elems,
                   const int* active_flag = nullptr);

// ---- apply.hip -----------------------------------------------------------
// C = alpha * A X + beta * C for a dense A (m x p, lda even, 16-byte aligned)
// and a narrow X (p x q, q <= 32): the streaming block apply.  `ev`
// (optional) brackets the main product kernel.
hipError_t dense_apply_narrow(hipStream_t st, int m, int q, int p, const double* A, int64_t lda,
                              const double* X, int64_t ldx, double* C, int64_t ldc, double alpha,
                              double beta, double* work, size_t work_elems,
                              const int* active_flag = nullptr, hipEvent_t* ev = nullptr);

// M Y for the low-rank operator M = diag(delta) + 2 L L^T (n x r, r <= 256,
// w <= 32 columns; ld even, 16-byte aligned): T = 2 L^T Y by a streaming
// MFMA reduction over n, then C = L T + delta o Y by the streaming apply with
// a direct epilogue.  `ev` (optional) brackets both passes.
hipError_t lowrank_apply_M(hipStream_t st, int n, int r, int w, const double* delta, const double* L,
                           int64_t ldl, const double* Y, int64_t ldy, double* C, int64_t ldc, double* work,
                           size_t work_elems, const int* active_flag = nullptr, hipEvent_t* ev = nullptr);

// ---- apply16.hip ---------------------------------------------------------
// out (16-bit, n x n, ld n) = round(0.5 (A + A^T)); precision 1 = BF16, 2 = FP16
hipError_t convert_operator16(hipStream_t st, int precision, int n, const double* A, int64_t lda,
                              uint16_t* out);
// The mixed-precision counterpart of cg_dense_apply: same contract, with the
// product taken on the 16-bit operator copy A16 (n x n, n a multiple of 8)
// and a 16-bit copy of P (FP16: columns scaled by powers of two from rr).
hipError_t cg_dense_apply16(hipStream_t st, int precision, int n, int w, const uint16_t* A16, double* P,
                            const double* R, const double* beta, const int* active, const double* rr,
                            int first, double* Q, double* pq, double* work, size_t work_elems,
                            const int* any_active, hipEvent_t* ev = nullptr, int* flag_log = nullptr);

// 64-row tiles of the streaming apply for m rows
size_t stream_tiles(int m);

// One CG step's operator work on the dense path (n x n, w <= 32 columns, all
// ld n): p = r + beta p for the active columns (skipped when `first`), then
// Q = A P, and pq[t * 32 + j] = the sum over tile t's rows of P[:, j] Q[:, j].
// `flag_log` (optional) receives *any_active as the step starts.
hipError_t cg_dense_apply(hipStream_t st, int n, int w, const double* A, int64_t lda, double* P,
                          const double* R, const double* beta, const int* active, int first,
                          double* Q, double* pq, double* work, size_t work_elems,
                          const int* any_active, hipEvent_t* ev = nullptr, int* flag_log = nullptr);

// ---- lowrank.hip ---------------------------------------------------------
// leading dimension of the row-major copy of L (rank rounded up to 64)
int64_t lowrank_row_ld(int64_t r);
// Lr (n x lowrank_row_ld(r), row-major, zero-padded) = L (n x r, ld ldl), r <= 256
hipError_t lowrank_make_rows(hipStream_t st, int n, int r, const double* L, int64_t ldl, double* Lr);
// Lr32 = the FP32 copy of the row-major Lr (n x lowrank_row_ld(r)), each value
// rounded to nearest even
hipError_t lowrank_rows_f32(hipStream_t st, int n, int r, const double* Lr, float* Lr32);
// C = delta o Y + 2 L (L^T Y) from the row-major copy, w <= 32 columns of Y
// (ld even, 16-byte aligned); `work` holds 256 * 32 + nchunk * 8192 doubles.
// With pq, also pq[t * 32 + j] = the sum over the 64-row tile t of Y[:, j] C[:, j].
hipError_t lowrank_apply_M_rows(hipStream_t st, int n, int r, int w, const double* delta, const double* Lr,
                                const double* Y, int64_t ldy, double* C, int64_t ldc, double* work,
                                size_t work_elems, const int* active_flag = nullptr, hipEvent_t* ev = nullptr,
                                double* pq = nullptr);

// ---- vec.hip -------------------------------------------------------------
// ---- diagonal metric (metric.hip)
// s = b^-1/2 where every b_i is positive and finite; else *bad = 1
hipError_t metric_prepare(hipStream_t st, int64_t n, const double* b, double* s, int* bad);
// A (n x n, ld) <- diag(s) A diag(s)
hipError_t metric_scale_sym(hipStream_t st, int64_t n, double* A, int64_t ld, const double* s);
// d <- s o s o d
hipError_t metric_scale_diag(hipStream_t st, int64_t n, double* d, const double* s);
// dense metric B (n x n, ld n, in Lb) = L L^T: L^T into LT, L^-T into LinvT,
// L^-1 into Xb; Tb (n x 64), Vall (64 x n), Wb (64 x 64), Pt (64 x n) are
// workspace; *bad = 1 when a pivot is not positive
hipError_t metric_dense_setup(hipStream_t st, int64_t n, double* Lb, double* Xb, double* Tb, double* LT,
                              double* LinvT, double* Vall, double* Wb, double* Pt, double* work, size_t work_elems,
                              int* bad);
// A (n x n, ld lda) <- Linv A Linv^T, symmetrised; Tb n x n workspace
hipError_t metric_dense_apply(hipStream_t st, int64_t n, double* A, int64_t lda, const double* Linv,
                              const double* LinvT, double* Tb, double* work, size_t work_elems);
// X (n x cols, ld) <- diag(s) X, or diag(s)^-1 X with inverse
hipError_t metric_scale_rows(hipStream_t st, int64_t n, int cols, double* X, int64_t ldx, const double* s,
                             bool inverse);

// Y[:, j] = delta o X[:, j]
hipError_t diag_scale(hipStream_t st, int n, int cols, const double* delta,
                      const double* X, int64_t ldx, double* Y, int64_t ldy,
                      const int* active_flag = nullptr);
// the same for cols <= 32 with pq[t * 32 + j] = the sum over the 64-row tile
// t of X[:, j] Y[:, j] (the CG's p . A p per tile)
hipError_t diag_scale_pq(hipStream_t st, int n, int cols, const double* delta, const double* X, int64_t ldx,
                         double* Y, int64_t ldy, double* pq, const int* active_flag = nullptr);
// the same on CG vectors (ld n) with the pending direction update folded in:
// P = R + beta P for the active columns first (as cg_direction), then Q, pq
hipError_t diag_dir_scale_pq(hipStream_t st, int n, int cols, const double* delta, double* P, const double* R,
                             const double* beta, const int* active, double* Q, double* pq,
                             const int* active_flag = nullptr);

// Step-4 residuals.  For Ritz columns j in [0, cols):
//   eps[j] = sqrt(|KX_j - l_j Y_j|^2 + |MY_j - l_j X_j|^2) / ((1 + l_j) sqrt(|X_j|^2 + |Y_j|^2))
// `part` holds (n/chunk) * cols * 4 doubles; `ticket` one unsigned (zeroed).
hipError_t residual_eps(hipStream_t st, int n, int cols, const double* X, const double* Y,
                        const double* KX, const double* MY, int64_t ld, const double* lam,
                        double* eps, double* part, size_t part_elems, unsigned* ticket);

// Block CG state for `w` independent systems A x_j = b_j (Step 6).
struct CgState {
    double *X, *R, *P, *Q;     // n x w, ld = n
    double *rr, *bb, *alpha, *beta;   // w
    int *active;               // w
    int *any_active;           // 1
    double* part;              // partial sums
    size_t part_elems;
    unsigned* ticket;          // 1
    unsigned long long* napplies;   // running count of column applies (active columns)
    // optional host-visible note (mapped pinned memory): 2 seq + any_active,
    // written whenever any_active is (re)computed, so that the host can stop
    // issuing steps of solve `seq` once every column has converged
    unsigned long long* note;
    unsigned long long seq;
    // fused CG on a low-rank operator (lowrank.hip): c = p^T diag(delta) p of
    // the current direction (w), T = L^T p (k-major, rows of L x 32)
    double* c;
    double* T;
};
// x = 0, r = p = b (B may alias R), rr = bb = |b|^2, active = rr > tol^2 bb
hipError_t cg_init(hipStream_t st, int n, int w, const CgState& s, const double* B, int64_t ldb,
                   double tol);
// alpha_j = rr_j / (p_j . q_j) for active columns (p.q <= 0 stops the column)
hipError_t cg_alpha(hipStream_t st, int n, int w, const CgState& s);
// alpha from the per-tile sums and cg_update in one launch: every block forms alpha of its
// column from the tile sums in the same fixed order
// pq holds cg_pq_elems(ntiles) doubles: the per-tile sums (ntiles x 32) and
// room behind them where long tile lists are first folded 128 tiles at a time
hipError_t cg_update_tiles(hipStream_t st, int n, int w, int ntiles, double* pq, const CgState& s, double tol);
size_t cg_pq_elems(int ntiles);
// x += alpha p, r -= alpha q, rr_new, beta, active update
hipError_t cg_update(hipStream_t st, int n, int w, const CgState& s, double tol);
// p = r + beta p for active columns
hipError_t cg_direction(hipStream_t st, int n, int w, const CgState& s);

// ---- fused CG on a low-rank operator (lowrank.hip) ------------------------
// CG for A = diag(delta) + 2 L L^T (Lr: the row-major copy of L, rank r) or,
// with Lr == nullptr, A = diag(delta), on w <= 32 columns of the CgState
// vectors (ld n, n even).  Each step is one pass over the rows: the direction
// update p = r + beta p, A p = delta o p + 2 L T with T = L^T p carried by its
// own recurrence (L^T p_new = L^T r_new + beta L^T p), x += alpha p,
// r -= alpha A p, and the sums that give the next alpha and beta (L is read
// once per step), then a fixed-order reduction and finishing launch.
// `work` holds fused_cg_work_elems(n, r, w) doubles.  With Lr32 (the FP32 copy
// of Lr) the steps read L from it, widened exactly to FP64 (half the bytes of
// L; the products are those of the FP32-rounded L); the first T = L^T b still
// comes from Lr.
size_t fused_cg_work_elems(int n, int r, int w);
hipError_t fused_cg_init(hipStream_t st, int n, int r, int w, const double* delta, const double* Lr,
                         const CgState& s, const double* B, int64_t ldb, double tol, double* work,
                         size_t work_elems);
hipError_t fused_cg_step(hipStream_t st, int n, int r, int w, const double* delta, const double* Lr,
                         const CgState& s, double tol, double* work, size_t work_elems, hipEvent_t* ev = nullptr,
                         int* flag_log = nullptr, const float* Lr32 = nullptr);
// Bx = I - (G - I)^T / 2, By = I - (G - I) / 2 for G = X^T Y (c x c): the
// first-order correction (X Bx)^T (Y By) = I + O(|G - I|^2)
hipError_t biorth_fix_coef(hipStream_t st, int c, const double* G, int64_t ldg, double* Bx, double* By, int64_t ldb);

// Right-hand sides of the block Gauss-Seidel sweep (equation for the sweep):
//   out[:, j] = lam[j] * (S[:, j] + T[:, g_j]) - U[:, g_j]
// with g_j = win[j] indexing columns of T and U (S may be null = 0).
hipError_t gs_rhs(hipStream_t st, int n, int w, const double* S, int64_t lds, const double* T,
                  const double* U, int64_t ldt, const int* win, const double* lam_w,
                  double* out, int64_t ldo);

// max over the columns j of both pairs of |A_j - B_j| / |B_j| (n x cols, ld):
// the relative drift of carried images A against fresh ones B
hipError_t image_drift(hipStream_t st, int n, int cols, const double* A1, const double* B1, const double* A2,
                       const double* B2, int64_t ld, double* part, size_t part_elems, double* out);

// out = in, column block copy with leading dimensions
// U = Y + X, V = Y - X (n x cols)
hipError_t xy_to_uv(hipStream_t st, int n, int cols, const double* X, const double* Y, int64_t ldxy, double* U,
                    double* V, int64_t lduv);
// C = A - B (n x cols)
hipError_t sub_cols(hipStream_t st, int n, int cols, const double* A, int64_t lda, const double* B, int64_t ldb,
                    double* C, int64_t ldc);
hipError_t copy_cols(hipStream_t st, int n, int cols, const double* in, int64_t ldi, double* out,
                     int64_t ldo);

// max |S - I| over a d x d matrix (one workgroup); result into *out
hipError_t max_offidentity(hipStream_t st, int d, const double* S, int64_t lds, double* out);

// standard normal fill from the counter-based Philox4x32-10 generator
// (Salmon, Moraes, Dror, Shaw, SC'11) with Box-Muller; element (i, j) uses
// counter i + j * n so the block is independent of the launch shape.
hipError_t philox_normal(hipStream_t st, int n, int cols, uint64_t seed, double* out, int64_t ld);

// sign normalisation of returned pairs: x_j's entry of largest magnitude is
// made positive, y_j flips with it.
hipError_t sign_normalise(hipStream_t st, int n, int cols, double* X, double* Y, int64_t ld);

// K <- A - B, M <- A + B element-wise (K holds A and M holds B on entry), n x n, ld n
hipError_t combine_ab(hipStream_t st, int64_t n, double* K, double* M);


// ---- small.hip (small d x d data, d <= 128) ------------------------------
// Small structured LREP:  K^ = L1 L1^T, M^ = L2 L2^T, SVD of L2^T L1 by
// one-sided Jacobi, all d Ritz pairs ascending: lam[d], Xh (d x d, ld kMaxD),
// Yh.  `scratch` >= 4 * kMaxD^2 doubles; `work` is the block-product
// workspace.  status[ST_NOTSPD] set on Cholesky failure.
hipError_t small_lrep(hipStream_t st, int d, const double* Kh, const double* Mh, int64_t ldh,
                      double* lam, double* Xh, double* Yh, double* scratch, int* status,
                      double* work, size_t work_elems);

// Step 5 in coefficient space: for window Ritz indices win[0..nw):
//   P^ = (I - Xk Yk^T)^2 (Xh[:, g] - e_g), Q^ likewise, Xk = Xh[:, 0:hi];
// columns the projector annihilates are dropped, then MGS-Biorth (drop rule
// of the oracle).  Writes P^, Q^ (d x np, ld kMaxD) and status[ST_NP] = np.
// `scratch` >= 3 * kMaxD * 64 + 128 doubles.
hipError_t step5_pq(hipStream_t st, int d, int hi, const double* Xh, const double* Yh,
                    const int* win, int nw, double* Ph, double* Qh, double* scratch,
                    int* status, double cos_tol, double dep_tol, double* work, size_t work_elems);

// Coefficient pass of block MGS-Biorth.  G is the Gram of [X Y] (2m x 2m,
// ld ldg).  Runs the MGS-Biorth recurrence (Algorithm MGS-Biorth) on the
// coefficient vectors: P = X A, Q = Y B with A, B upper triangular (m x np,
// ld kMaxD; dropped columns compacted away).  status[ST_NKEPT] = np.
// `scratch` >= 2 * kMaxD^2 doubles.
hipError_t coef_mgs(hipStream_t st, int m, const double* G, int64_t ldg, double* A, double* B,
                    int* status, double cos_tol, double dep_tol, double* scratch);

}  // namespace lrep
