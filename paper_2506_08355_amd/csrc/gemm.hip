// FP64 MFMA (v_mfma_f64_16x16x4_f64) block products for gfx950.
//
//   gemm_nn : C = alpha * A B + beta * C  (+ diag(delta) Yd), A m x p, B p x q.
//             Covers the dense operator apply (m = p = n, q = block width,
//             split over p with a deterministic second-stage sum), the
//             pull-back X~ = U X^ (p = d), and the block updates W -= X C.
//   gemm_tn : C = alpha * A^T B, A n x p, B n x q: the tall-skinny Gram
//             products of the Rayleigh-Ritz step (K^ = U^T K U), of the
//             projections against converged/active blocks and of block
//             MGS-Biorth.  The n dimension is split over workgroups; the
//             partial p x q tiles are summed in a fixed order.
// A and B of gemm_tn and A of gemm_nn may be given as up to four column
// segments (pointer, leading dimension, columns) that act as one matrix.
//
// Every matrix is column-major FP64.  Lane layout of the 16x16x4 FP64 MFMA:
//   A (16x4):  lane l holds A[l % 16][l / 16]
//   B (4x16):  lane l holds B[l / 16][l % 16]
//   D (16x16): lane l holds D[4 * r + l / 16][l % 16] in item r = 0..3
#include "device.hpp"
#include "kernels.hpp"

namespace lrep {

namespace {

constexpr int NT = 256;     // 4 waves
constexpr int BK = 16;      // k-depth of one LDS stage
// tall-skinny products (k up to this, rows from this) take the register-direct kernels
constexpr int kSkinnyMaxK = 1024;
constexpr int kSkinnyMinRows = 512;

struct SegView {
    const double* p[kMaxSeg];
    int64_t ld[kMaxSeg];
    int start[kMaxSeg + 1];  // prefix of column counts
    int nseg;
};

// column c of a segment list; the segment fields are read with constant
// indices (uniform loads) and chosen per lane by selects, never by indexing
// the table with a per-lane value
__device__ __forceinline__ const double* seg_col(const SegView& s, int c, int64_t& ld) {
    const double* p = s.p[0];
    int64_t l = s.ld[0];
    int st = s.start[0];
#pragma unroll
    for (int t = 1; t < kMaxSeg; ++t) {
        const bool in = t < s.nseg && c >= s.start[t];
        p = in ? s.p[t] : p;
        l = in ? s.ld[t] : l;
        st = in ? s.start[t] : st;
    }
    ld = l;
    return p + (int64_t)(c - st) * l;
}

// up to four independent products of the same shape in one launch
constexpr int kMaxBatch = 4;
struct NNBatch {
    SegView A[kMaxBatch];
    const double* B[kMaxBatch];
    double* C[kMaxBatch];
};

SegView make_view(const Seg* segs, int nseg) {
    SegView v{};
    v.nseg = nseg;
    v.start[0] = 0;
    for (int i = 0; i < nseg; ++i) {
        v.p[i] = segs[i].p;
        v.ld[i] = segs[i].ld;
        v.start[i + 1] = v.start[i] + segs[i].cols;
    }
    for (int i = nseg; i < kMaxSeg; ++i) {
        v.p[i] = nullptr;
        v.ld[i] = 1;
        v.start[i + 1] = v.start[nseg];
    }
    return v;
}

// --------------------------------------------------------------------------
// C tile (BM x BN) of A B over k in [k_begin, k_end).
// Waves are arranged WM x WN; each wave owns (BM/WM) x (BN/WN) = FM x FN
// MFMA tiles of 16x16.
// --------------------------------------------------------------------------
template <int BM, int BN, int WM>
__global__ __launch_bounds__(NT) void gemm_nn_kernel(
    int m, int q, int p, NNBatch bt, int ksplit, int64_t ldb, int64_t ldc, double alpha, double beta,
    int kchunk, double* __restrict__ part, const double* __restrict__ delta,
    const double* __restrict__ Yd, int64_t ldyd, const int* __restrict__ active_flag) {
    if (active_flag && *active_flag == 0) return;
    const int bz = blockIdx.z / ksplit;
    const SegView& A = bt.A[bz];
    const double* __restrict__ B = bt.B[bz];
    double* __restrict__ C = bt.C[bz];
    constexpr int WN = 4 / WM;
    constexpr int TM = BM / WM, TN = BN / WN;
    constexpr int FM = TM / 16, FN = TN / 16;
    constexpr int APAD = 4, BPAD = 4;
    __shared__ double As[BK][BM + APAD];
    __shared__ double Bs[BK][BN + BPAD];

    const int tid = threadIdx.x, lane = tid % WAVE, wid = tid / WAVE;
    const int wm = wid % WM, wn = wid / WM;
    const int row0 = blockIdx.x * BM, col0 = blockIdx.y * BN;
    const int ks = blockIdx.z % ksplit;
    const int k_begin = ks * kchunk;
    const int k_end = min(p, k_begin + kchunk);

    d4 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

    constexpr int AE = BM * BK / NT;   // elements of A per thread per stage
    constexpr int BE = BK * BN / NT;
    double ra[AE], rb[BE];

    auto load = [&](int k0) {
#pragma unroll
        for (int e = 0; e < AE; ++e) {
            const int idx = e * NT + tid;
            const int i = idx % BM, kk = idx / BM;
            const int r = row0 + i, k = k0 + kk;
            double v = 0.0;
            if (r < m && k < k_end) {
                int64_t ld;
                const double* col = seg_col(A, k, ld);
                v = col[r];
            }
            ra[e] = v;
        }
#pragma unroll
        for (int e = 0; e < BE; ++e) {
            const int idx = e * NT + tid;
            const int kk = idx % BK, j = idx / BK;
            const int k = k0 + kk, c = col0 + j;
            rb[e] = (k < k_end && c < q) ? B[(int64_t)c * ldb + k] : 0.0;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int e = 0; e < AE; ++e) {
            const int idx = e * NT + tid;
            As[idx / BM][idx % BM] = ra[e];
        }
#pragma unroll
        for (int e = 0; e < BE; ++e) {
            const int idx = e * NT + tid;
            Bs[idx % BK][idx / BK] = rb[e];
        }
    };

    const int ntiles = (k_end - k_begin + BK - 1) / BK;
    if (ntiles > 0) {
        load(k_begin);
        store();
        __syncthreads();
        for (int t = 0; t < ntiles; ++t) {
            if (t + 1 < ntiles) load(k_begin + (t + 1) * BK);
#pragma unroll
            for (int s = 0; s < BK / 4; ++s) {
                const int kr = s * 4 + lane / 16;
                double af[FM], bf[FN];
#pragma unroll
                for (int i = 0; i < FM; ++i) af[i] = As[kr][wm * TM + i * 16 + lane % 16];
#pragma unroll
                for (int j = 0; j < FN; ++j) bf[j] = Bs[kr][wn * TN + j * 16 + lane % 16];
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
            }
            __syncthreads();
            if (t + 1 < ntiles) {
                store();
                __syncthreads();
            }
        }
    }

    // epilogue
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int c = col0 + wn * TN + j * 16 + lane % 16;
            if (c >= q) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = row0 + wm * TM + i * 16 + 4 * r + lane / 16;
                if (row >= m) continue;
                const double v = acc[i][j][r];
                if (part) {
                    part[((int64_t)ks * q + c) * m + row] = v;
                } else {
                    double o = alpha * v;
                    if (beta != 0.0) o += beta * C[(int64_t)c * ldc + row];
                    if (delta) o += delta[row] * Yd[(int64_t)c * ldyd + row];
                    C[(int64_t)c * ldc + row] = o;
                }
            }
        }
}

// C = alpha * sum_s part[s] + beta * C (+ diag(delta) Yd), fixed order over s.
__global__ __launch_bounds__(NT) void splitk_reduce_kernel(
    int m, int q, int nsplit, const double* __restrict__ part, double* __restrict__ C,
    int64_t ldc, double alpha, double beta, const double* __restrict__ delta,
    const double* __restrict__ Yd, int64_t ldyd, const int* __restrict__ active_flag) {
    if (active_flag && *active_flag == 0) return;
    const int64_t total = (int64_t)m * q;
    for (int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * NT) {
        const int row = (int)(idx % m);
        const int c = (int)(idx / m);
        double s = 0.0;
        for (int k = 0; k < nsplit; ++k) s += part[((int64_t)k * q + c) * m + row];
        double o = alpha * s;
        if (beta != 0.0) o += beta * C[(int64_t)c * ldc + row];
        if (delta) o += delta[row] * Yd[(int64_t)c * ldyd + row];
        C[(int64_t)c * ldc + row] = o;
    }
}

// --------------------------------------------------------------------------
// Gram tile: part[split][BP x BQ block] = A(rows)^T B(rows).
// --------------------------------------------------------------------------
template <int BP, int BQ>
__global__ __launch_bounds__(NT) void gemm_tn_kernel(
    int n, int p, int q, SegView A, SegView B, int rows_per_split,
    double* __restrict__ part, const int* __restrict__ active_flag) {
    if (active_flag && *active_flag == 0) return;
    constexpr int WM = 2, WN = 2;
    constexpr int TM = BP / WM, TN = BQ / WN;
    constexpr int FM = TM / 16, FN = TN / 16;
    constexpr int PAD = 4;
    __shared__ double As[BK][BP + PAD];
    __shared__ double Bs[BK][BQ + PAD];
    const int tid = threadIdx.x, lane = tid % WAVE, wid = tid / WAVE;
    const int wm = wid % WM, wn = wid / WM;
    const int c0 = blockIdx.x * BP, d0 = blockIdx.y * BQ;
    const int s = blockIdx.z;
    const int r_begin = s * rows_per_split;
    const int r_end = min(n, r_begin + rows_per_split);

    d4 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

    constexpr int AE = BP * BK / NT, BE = BQ * BK / NT;
    double ra[AE], rb[BE];
    auto load = [&](int r0) {
#pragma unroll
        for (int e = 0; e < AE; ++e) {
            const int idx = e * NT + tid;
            const int kk = idx % BK, i = idx / BK;
            const int r = r0 + kk, c = c0 + i;
            double v = 0.0;
            if (r < r_end && c < p) {
                int64_t ld;
                v = seg_col(A, c, ld)[r];
            }
            ra[e] = v;
        }
#pragma unroll
        for (int e = 0; e < BE; ++e) {
            const int idx = e * NT + tid;
            const int kk = idx % BK, j = idx / BK;
            const int r = r0 + kk, c = d0 + j;
            double v = 0.0;
            if (r < r_end && c < q) {
                int64_t ld;
                v = seg_col(B, c, ld)[r];
            }
            rb[e] = v;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int e = 0; e < AE; ++e) {
            const int idx = e * NT + tid;
            As[idx % BK][idx / BK] = ra[e];
        }
#pragma unroll
        for (int e = 0; e < BE; ++e) {
            const int idx = e * NT + tid;
            Bs[idx % BK][idx / BK] = rb[e];
        }
    };
    const int ntiles = (r_end - r_begin + BK - 1) / BK;
    if (ntiles > 0) {
        load(r_begin);
        store();
        __syncthreads();
        for (int t = 0; t < ntiles; ++t) {
            if (t + 1 < ntiles) load(r_begin + (t + 1) * BK);
#pragma unroll
            for (int ss = 0; ss < BK / 4; ++ss) {
                const int kr = ss * 4 + lane / 16;
                double af[FM], bf[FN];
#pragma unroll
                for (int i = 0; i < FM; ++i) af[i] = As[kr][wm * TM + i * 16 + lane % 16];
#pragma unroll
                for (int j = 0; j < FN; ++j) bf[j] = Bs[kr][wn * TN + j * 16 + lane % 16];
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
            }
            __syncthreads();
            if (t + 1 < ntiles) {
                store();
                __syncthreads();
            }
        }
    }
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int c = d0 + wn * TN + j * 16 + lane % 16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = c0 + wm * TM + i * 16 + 4 * r + lane / 16;
                if (row < p && c < q) part[((int64_t)s * q + c) * p + row] = acc[i][j][r];
            }
        }
}

// C (p x q, ldc) = alpha * sum_s part[s]; optional symmetrisation (p == q)
// C = (T + T^T) / 2 done in the same pass.
__global__ __launch_bounds__(NT) void gram_reduce_kernel(
    int p, int q, int nsplit, const double* __restrict__ part, double* __restrict__ C,
    int64_t ldc, double alpha, int symmetrize, const int* __restrict__ active_flag) {
    if (active_flag && *active_flag == 0) return;
    const int64_t total = (int64_t)p * q;
    for (int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * NT) {
        const int row = (int)(idx % p), c = (int)(idx / p);
        double s = 0.0;
        for (int k = 0; k < nsplit; ++k) s += part[((int64_t)k * q + c) * p + row];
        if (symmetrize) {
            double t = 0.0;
            for (int k = 0; k < nsplit; ++k) t += part[((int64_t)k * q + row) * p + c];
            s = 0.5 * (s + t);
        }
        C[(int64_t)c * ldc + row] = alpha * s;
    }
}

// --------------------------------------------------------------------------
// Register-direct tall-skinny products: the operands go from memory straight
// into MFMA fragments, no LDS staging.  The long dimension is consumed in
// units of 16: lane group g = l / 16 holds four consecutive entries 4g .. 4g+3
// of its column and feeds them to four successive MFMA steps (step e pairs
// entry 4g + e of both operands, so each product term is formed once).  The
// four waves of a workgroup take interleaved units; their accumulators are
// summed through LDS in the fixed order (w0 + w2) + (w1 + w3).  The MFMA is
// called with the operands swapped (a = the column-side operand), so that
// accumulator item r of lane l is element (c, 4 r + g) of the output tile,
// c = l % 16: 16 consecutive output rows per store.
// --------------------------------------------------------------------------
constexpr int RU = 16;   // entries of the long dimension per unit

template <int NA>
__device__ __forceinline__ void lds_reduce4(double (&acc)[NA], double* red, int w, int lane) {
    // red: 2 * NA * WAVE doubles
    if (w >= 2)
#pragma unroll
        for (int x = 0; x < NA; ++x) red[((w - 2) * NA + x) * WAVE + lane] = acc[x];
    __syncthreads();
    if (w < 2)
#pragma unroll
        for (int x = 0; x < NA; ++x) acc[x] += red[(w * NA + x) * WAVE + lane];
    __syncthreads();
    if (w == 1)
#pragma unroll
        for (int x = 0; x < NA; ++x) red[x * WAVE + lane] = acc[x];
    __syncthreads();
    if (w == 0)
#pragma unroll
        for (int x = 0; x < NA; ++x) acc[x] += red[x * WAVE + lane];
}

// part[s] (q x p slices, column-major p x q) block = A(rows of split s)^T B(rows)
// for output rows i0 .. i0 + 16 TI (columns of A) and columns j0 .. j0 + 16 TJ.
template <int TI, int TJ>
__global__ __launch_bounds__(NT) void gram_rd_kernel(int n, int p, int q, SegView A, SegView B, int rows_per_split,
                                                     double* __restrict__ part, const int* __restrict__ active_flag) {
    if (active_flag && *active_flag == 0) return;
    constexpr int NA = TI * TJ * 4;
    __shared__ double red[2 * NA * WAVE];
    const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
    const int c = lane % 16, g = lane / 16;
    const int i0 = blockIdx.x * 16 * TI, j0 = blockIdx.y * 16 * TJ, s = blockIdx.z;
    const int r_begin = s * rows_per_split;
    const int nrows = min(n, r_begin + rows_per_split) - r_begin;
    // columns beyond p / q read a valid column; those outputs are not written
    const double* ap[TI];
    const double* bp[TJ];
#pragma unroll
    for (int t = 0; t < TI; ++t) {
        int64_t ld;
        ap[t] = seg_col(A, min(i0 + 16 * t + c, p - 1), ld) + r_begin + 4 * g;
    }
#pragma unroll
    for (int t = 0; t < TJ; ++t) {
        int64_t ld;
        bp[t] = seg_col(B, min(j0 + 16 * t + c, q - 1), ld) + r_begin + 4 * g;
    }
    d4 acc[TI][TJ];
#pragma unroll
    for (int a = 0; a < TI; ++a)
#pragma unroll
        for (int b = 0; b < TJ; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
    auto compute = [&](const double (&xa)[TI][4], const double (&xb)[TJ][4]) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int a = 0; a < TI; ++a)
#pragma unroll
                for (int b = 0; b < TJ; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xb[b][e], xa[a][e], acc[a][b], 0, 0, 0);
    };
    const int nfull = nrows / RU;
    const int mine = nfull > w ? (nfull - w + 3) / 4 : 0;   // whole units w, w + 4, ...
    if (mine > 0) {
        double xa0[TI][4], xb0[TJ][4], xa1[TI][4], xb1[TJ][4];
        // surplus loads re-read this wave's last unit (in range) and are not used
        auto load = [&](double (&xa)[TI][4], double (&xb)[TJ][4], int k) {
            const int64_t off = (int64_t)(w + 4 * min(k, mine - 1)) * RU;
#pragma unroll
            for (int a = 0; a < TI; ++a)
#pragma unroll
                for (int e = 0; e < 4; ++e) xa[a][e] = ap[a][off + e];
#pragma unroll
            for (int b = 0; b < TJ; ++b)
#pragma unroll
                for (int e = 0; e < 4; ++e) xb[b][e] = bp[b][off + e];
        };
        // the scheduling barriers keep each unit's loads issued ahead of the
        // previous unit's MFMAs
        load(xa0, xb0, 0);
        for (int k = 0; k < mine; k += 2) {
            load(xa1, xb1, k + 1);
            __builtin_amdgcn_sched_barrier(0);
            compute(xa0, xb0);
            __builtin_amdgcn_sched_barrier(0);
            load(xa0, xb0, k + 2);
            __builtin_amdgcn_sched_barrier(0);
            if (k + 1 < mine) compute(xa1, xb1);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    const int tail = nrows - nfull * RU;
    if (tail > 0 && w == (nfull & 3)) {
        // last partial unit: rows at or beyond the end read the last row and count zero
        const int64_t off = (int64_t)nfull * RU;
        double xa[TI][4], xb[TJ][4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const bool in = 4 * g + e < tail;
            const int64_t o = off + min(4 * g + e, tail - 1) - 4 * g;
#pragma unroll
            for (int a = 0; a < TI; ++a) {
                const double v = ap[a][o];
                xa[a][e] = in ? v : 0.0;
            }
#pragma unroll
            for (int b = 0; b < TJ; ++b) {
                const double v = bp[b][o];
                xb[b][e] = in ? v : 0.0;
            }
        }
        compute(xa, xb);
    }
    double flat[NA];
#pragma unroll
    for (int a = 0; a < TI; ++a)
#pragma unroll
        for (int b = 0; b < TJ; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) flat[(a * TJ + b) * 4 + r] = acc[a][b][r];
    lds_reduce4<NA>(flat, red, w, lane);
    if (w != 0) return;
#pragma unroll
    for (int a = 0; a < TI; ++a)
#pragma unroll
        for (int b = 0; b < TJ; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + 16 * a + c, j = j0 + 16 * b + 4 * r + g;
                if (i < p && j < q) part[((int64_t)s * q + j) * p + i] = flat[(a * TJ + b) * 4 + r];
            }
}

// C = alpha * sum_s part[s] (+ symmetrisation), four split groups per output
// summed in a fixed order.
__global__ __launch_bounds__(NT) void gram_reduce4_kernel(int p, int q, int nsplit, const double* __restrict__ part,
                                                          double* __restrict__ C, int64_t ldc, double alpha,
                                                          int symmetrize, const int* __restrict__ active_flag) {
    if (active_flag && *active_flag == 0) return;
    __shared__ double red[2][4][WAVE];
    const int lane = threadIdx.x % WAVE, sg = threadIdx.x / WAVE;
    const int64_t total = (int64_t)p * q;
    const int64_t idx = (int64_t)blockIdx.x * WAVE + lane;
    double s = 0.0, t = 0.0;
    if (idx < total) {
        const int row = (int)(idx % p), c = (int)(idx / p);
        for (int k = sg; k < nsplit; k += 4) s += part[((int64_t)k * q + c) * p + row];
        if (symmetrize)
            for (int k = sg; k < nsplit; k += 4) t += part[((int64_t)k * q + row) * p + c];
    }
    red[0][sg][lane] = s;
    red[1][sg][lane] = t;
    __syncthreads();
    if (sg == 0 && idx < total) {
        const int row = (int)(idx % p), c = (int)(idx / p);
        double v = (red[0][0][lane] + red[0][2][lane]) + (red[0][1][lane] + red[0][3][lane]);
        if (symmetrize) {
            const double u = (red[1][0][lane] + red[1][2][lane]) + (red[1][1][lane] + red[1][3][lane]);
            v = 0.5 * (v + u);
        }
        C[(int64_t)c * ldc + row] = alpha * v;
    }
}

// C (m x q) = alpha A B + beta C (+ diag(delta) Yd) for a block of 16 TR rows
// and 16 TC columns, A m x p (segments), B p x q (ldb); the four waves take
// interleaved 16-deep units of k.  Batch member = blockIdx.z.
template <int TR, int TC>
__global__ __launch_bounds__(NT) void nn_rd_kernel(int m, int q, int p, NNBatch bt, int64_t ldb, int64_t ldc,
                                                   double alpha, double beta, const double* __restrict__ delta,
                                                   const double* __restrict__ Yd, int64_t ldyd,
                                                   const int* __restrict__ active_flag) {
    if (active_flag && *active_flag == 0) return;
    constexpr int NA = TR * TC * 4;
    __shared__ double red[2 * NA * WAVE];
    const SegView& A = bt.A[blockIdx.z];
    const double* __restrict__ B = bt.B[blockIdx.z];
    double* __restrict__ C = bt.C[blockIdx.z];
    const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
    const int c = lane % 16, g = lane / 16;
    const int r0 = blockIdx.x * 16 * TR, c0 = blockIdx.y * 16 * TC;
    // rows beyond m and columns beyond q read valid memory; those outputs are not written
    int rowc[TR];
#pragma unroll
    for (int t = 0; t < TR; ++t) rowc[t] = min(r0 + 16 * t + c, m - 1);
    const double* bcol[TC];
#pragma unroll
    for (int t = 0; t < TC; ++t) bcol[t] = B + (int64_t)min(c0 + 16 * t + c, q - 1) * ldb;
    d4 acc[TR][TC];
#pragma unroll
    for (int a = 0; a < TR; ++a)
#pragma unroll
        for (int b = 0; b < TC; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
    auto compute = [&](const double (&xa)[TR][4], const double (&xb)[TC][4]) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int a = 0; a < TR; ++a)
#pragma unroll
                for (int b = 0; b < TC; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xb[b][e], xa[a][e], acc[a][b], 0, 0, 0);
    };
    const int nfull = p / RU;
    const int mine = nfull > w ? (nfull - w + 3) / 4 : 0;
    if (mine > 0) {
        double xa0[TR][4], xb0[TC][4], xa1[TR][4], xb1[TC][4];
        auto load = [&](double (&xa)[TR][4], double (&xb)[TC][4], int k) {
            const int kb = (w + 4 * min(k, mine - 1)) * RU + 4 * g;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                int64_t ld;
                const double* col = seg_col(A, kb + e, ld);
#pragma unroll
                for (int a = 0; a < TR; ++a) xa[a][e] = col[rowc[a]];
            }
#pragma unroll
            for (int b = 0; b < TC; ++b)
#pragma unroll
                for (int e = 0; e < 4; ++e) xb[b][e] = bcol[b][kb + e];
        };
        // the scheduling barriers keep each unit's loads issued ahead of the
        // previous unit's MFMAs
        load(xa0, xb0, 0);
        for (int k = 0; k < mine; k += 2) {
            load(xa1, xb1, k + 1);
            __builtin_amdgcn_sched_barrier(0);
            compute(xa0, xb0);
            __builtin_amdgcn_sched_barrier(0);
            load(xa0, xb0, k + 2);
            __builtin_amdgcn_sched_barrier(0);
            if (k + 1 < mine) compute(xa1, xb1);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    const int tail = p - nfull * RU;
    if (tail > 0 && w == (nfull & 3)) {
        double xa[TR][4], xb[TC][4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int kk = nfull * RU + 4 * g + e;
            const bool in = kk < p;
            const int kc = min(kk, p - 1);
            int64_t ld;
            const double* col = seg_col(A, kc, ld);
#pragma unroll
            for (int a = 0; a < TR; ++a) {
                const double v = col[rowc[a]];
                xa[a][e] = in ? v : 0.0;
            }
#pragma unroll
            for (int b = 0; b < TC; ++b) {
                const double v = bcol[b][kc];
                xb[b][e] = in ? v : 0.0;
            }
        }
        compute(xa, xb);
    }
    double flat[NA];
#pragma unroll
    for (int a = 0; a < TR; ++a)
#pragma unroll
        for (int b = 0; b < TC; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) flat[(a * TC + b) * 4 + r] = acc[a][b][r];
    lds_reduce4<NA>(flat, red, w, lane);
    if (w != 0) return;
#pragma unroll
    for (int a = 0; a < TR; ++a)
#pragma unroll
        for (int b = 0; b < TC; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = r0 + 16 * a + c, col = c0 + 16 * b + 4 * r + g;
                if (row < m && col < q) {
                    double o = alpha * flat[(a * TC + b) * 4 + r];
                    if (beta != 0.0) o += beta * C[(int64_t)col * ldc + row];
                    if (delta) o += delta[row] * Yd[(int64_t)col * ldyd + row];
                    C[(int64_t)col * ldc + row] = o;
                }
            }
}

// Launch of the tall-skinny product: blocks of 64 rows and 32 columns, or for
// 33..64 columns blocks of 32 rows and 64 columns, so that A is streamed once
// (two 32-column blocks read it twice; 185 against 190 us for 262144 x 128
// times 128 x 64, and 64 rows x 64 columns took 244 us).
void nn_rd_launch(hipStream_t st, int m, int q, int p, int nb, const NNBatch& bt, int64_t ldb, int64_t ldc,
                  double alpha, double beta, const double* delta, const double* Yd, int64_t ldyd,
                  const int* active_flag) {
    if (q > 32 && q <= 64)
        hipLaunchKernelGGL((nn_rd_kernel<2, 4>), dim3((m + 31) / 32, 1, nb),
                           dim3(NT), 0, st, m, q, p, bt, ldb, ldc, alpha, beta, delta, Yd, ldyd, active_flag);
    else
        hipLaunchKernelGGL((nn_rd_kernel<4, 2>), dim3((m + 63) / 64, (q + 31) / 32, nb), dim3(NT), 0, st, m, q, p, bt,
                           ldb, ldc, alpha, beta, delta, Yd, ldyd, active_flag);
}

}  // namespace

// ----------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------
hipError_t gemm_nn(hipStream_t st, int m, int q, int p, const Seg* A, int nsegA,
                   const double* B, int64_t ldb, double* C, int64_t ldc, double alpha,
                   double beta, double* work, size_t work_elems, const double* delta,
                   const double* Yd, int64_t ldyd, int ksplit_hint, const int* active_flag, hipEvent_t* ev) {
    if (m <= 0 || q <= 0) return hipSuccess;
    SegView av = make_view(A, nsegA);
    if (p > 0 && p <= kSkinnyMaxK && m >= kSkinnyMinRows && ksplit_hint <= 0) {
        // tall-skinny product: whole k per workgroup, register-direct
        NNBatch bt{};
        bt.A[0] = av;
        bt.B[0] = B;
        bt.C[0] = C;
        if (ev) (void)hipEventRecord(ev[0], st);
        nn_rd_launch(st, m, q, p, 1, bt, ldb, ldc, alpha, beta, delta, Yd, ldyd, active_flag);
        if (ev) (void)hipEventRecord(ev[1], st);
        return hipGetLastError();
    }
    int ksplit = 1;
    if (p <= 0) {
        // C = beta C (+ delta Yd): nothing to multiply
        hipLaunchKernelGGL(splitk_reduce_kernel, dim3(std::min<int64_t>(4096, ((int64_t)m * q + NT - 1) / NT)),
                           dim3(NT), 0, st, m, q, 0, (const double*)nullptr, C, ldc, alpha, beta, delta, Yd, ldyd, active_flag);
        return hipGetLastError();
    }
    // tile choice
    const bool wide = q > 32;
    const int BM = wide ? 64 : 128;
    const int BN = wide ? 64 : 32;
    const int mt = (m + BM - 1) / BM, nt = (q + BN - 1) / BN;
    if (ksplit_hint > 0) {
        ksplit = ksplit_hint;
    } else {
        // aim for >= 1024 workgroups on the large-p (operator) products
        const int base = mt * nt;
        while (base * ksplit < 1024 && p / (ksplit * 2) >= 256) ksplit *= 2;
    }
    int kchunk = (p + ksplit - 1) / ksplit;
    kchunk = ((kchunk + BK - 1) / BK) * BK;
    ksplit = (p + kchunk - 1) / kchunk;
    double* part = nullptr;
    while (ksplit > 1 && (size_t)ksplit * m * q > work_elems) {
        ksplit = (ksplit + 1) / 2;
        kchunk = (p + ksplit - 1) / ksplit;
        kchunk = ((kchunk + BK - 1) / BK) * BK;
        ksplit = (p + kchunk - 1) / kchunk;
    }
    if (ksplit > 1) part = work;
    else kchunk = p;
    NNBatch bt{};
    bt.A[0] = av;
    bt.B[0] = B;
    bt.C[0] = C;
    dim3 grid(mt, nt, ksplit);
    if (ev) (void)hipEventRecord(ev[0], st);
    if (wide)
        hipLaunchKernelGGL((gemm_nn_kernel<64, 64, 2>), grid, dim3(NT), 0, st, m, q, p, bt, ksplit, ldb, ldc, alpha,
                           beta, kchunk, part, delta, Yd, ldyd, active_flag);
    else
        hipLaunchKernelGGL((gemm_nn_kernel<128, 32, 4>), grid, dim3(NT), 0, st, m, q, p, bt, ksplit, ldb, ldc, alpha,
                           beta, kchunk, part, delta, Yd, ldyd, active_flag);
    if (ev) (void)hipEventRecord(ev[1], st);
    if (part) {
        const int64_t tot = (int64_t)m * q;
        const int nb = (int)std::min<int64_t>(8192, (tot + NT - 1) / NT);
        hipLaunchKernelGGL(splitk_reduce_kernel, dim3(nb), dim3(NT), 0, st, m, q, ksplit, part, C, ldc,
                           alpha, beta, delta, Yd, ldyd, active_flag);
    }
    return hipGetLastError();
}

hipError_t gemm_nn_batch(hipStream_t st, int m, int q, int p, int nb, const Seg* A, const double* const* B,
                         int64_t ldb, double* const* C, int64_t ldc, double alpha, double beta) {
    if (m <= 0 || q <= 0 || nb <= 0) return hipSuccess;
    if (nb > kMaxBatch || p <= 0) return hipErrorInvalidValue;
    NNBatch bt{};
    for (int i = 0; i < nb; ++i) {
        bt.A[i] = make_view(&A[i], 1);
        bt.B[i] = B[i];
        bt.C[i] = C[i];
    }
    // p = subspace size: the whole k per workgroup; the batch and the row
    // blocks provide the parallelism
    if (p <= kSkinnyMaxK && m >= kSkinnyMinRows) {
        nn_rd_launch(st, m, q, p, nb, bt, ldb, ldc, alpha, beta, nullptr, nullptr, 0, nullptr);
        return hipGetLastError();
    }
    const int BM = 64, BN = 64;
    dim3 grid((m + BM - 1) / BM, (q + BN - 1) / BN, nb);
    hipLaunchKernelGGL((gemm_nn_kernel<64, 64, 2>), grid, dim3(NT), 0, st, m, q, p, bt, 1, ldb, ldc, alpha, beta, p,
                       (double*)nullptr, (const double*)nullptr, (const double*)nullptr, (int64_t)0,
                       (const int*)nullptr);
    return hipGetLastError();
}

hipError_t gemm_tn(hipStream_t st, int n, int p, int q, const Seg* A, int nsegA, const Seg* B,
                   int nsegB, double* C, int64_t ldc, double alpha, int symmetrize,
                   double* work, size_t work_elems, const int* active_flag) {
    if (p <= 0 || q <= 0) return hipSuccess;
    SegView av = make_view(A, nsegA), bv = make_view(B, nsegB);
    if (n >= kSkinnyMinRows) {
        // register-direct Gram: about one workgroup per CU, at least 64 rows each
        const bool narrow = q <= 32;
        const int pt = (p + 63) / 64, qt = narrow ? 1 : (q + 63) / 64;
        int nsplit = std::max(1, std::min((n + 63) / 64, 256 / (pt * qt)));
        while ((size_t)nsplit * p * q > work_elems && nsplit > 1) nsplit = (nsplit + 1) / 2;
        int rows = (n + nsplit - 1) / nsplit;
        rows = ((rows + 15) / 16) * 16;
        nsplit = (n + rows - 1) / rows;
        if ((size_t)nsplit * p * q > work_elems) return hipErrorInvalidValue;
        if (narrow)
            hipLaunchKernelGGL((gram_rd_kernel<4, 2>), dim3(pt, qt, nsplit), dim3(NT), 0, st, n, p, q, av, bv, rows,
                               work, active_flag);
        else
            hipLaunchKernelGGL((gram_rd_kernel<4, 4>), dim3(pt, qt, nsplit), dim3(NT), 0, st, n, p, q, av, bv, rows,
                               work, active_flag);
        const int64_t tot = (int64_t)p * q;
        hipLaunchKernelGGL(gram_reduce4_kernel, dim3((unsigned)((tot + WAVE - 1) / WAVE)), dim3(NT), 0, st, p, q,
                           nsplit, work, C, ldc, alpha, symmetrize, active_flag);
        return hipGetLastError();
    }
    constexpr int BP = 64, BQ = 64;
    const int pt = (p + BP - 1) / BP, qt = (q + BQ - 1) / BQ;
    // rows per split: >= 256 rows of work per workgroup, <= ~1024 workgroups
    int nsplit = std::max(1, std::min((n + 255) / 256, std::max(1, 1024 / (pt * qt))));
    while ((size_t)nsplit * p * q > work_elems && nsplit > 1) nsplit /= 2;
    int rows = (n + nsplit - 1) / nsplit;
    rows = ((rows + BK - 1) / BK) * BK;
    nsplit = std::max(1, (n + rows - 1) / rows);
    if ((size_t)nsplit * p * q > work_elems) return hipErrorInvalidValue;
    hipLaunchKernelGGL((gemm_tn_kernel<BP, BQ>), dim3(pt, qt, nsplit), dim3(NT), 0, st, n, p, q, av, bv,
                       rows, work, active_flag);
    const int64_t tot = (int64_t)p * q;
    hipLaunchKernelGGL(gram_reduce_kernel, dim3((int)std::min<int64_t>(4096, (tot + NT - 1) / NT)), dim3(NT),
                       0, st, p, q, nsplit, work, C, ldc, alpha, symmetrize, active_flag);
    return hipGetLastError();
}

}  // namespace lrep
