// Streaming FP64 MFMA block apply Y = A X for a dense operator A (m x p,
// column-major) and a narrow block X (p x q, q <= 32): the CG inner solves of
// Step 6 (block Gauss-Seidel), where every launch reads the whole operator
// once and the product sits at the HBM/FP64-MFMA ridge (2 m p q flops over
// 8 m p bytes: q/4 flop/byte against a ridge of 9.8 on MI355X).
//
// Design for gfx950:
//  * no LDS and no barriers in the main loop.  Each wavefront (one per
//    workgroup) owns WR = 64 rows and streams its A panel straight from HBM
//    into registers with 16-byte loads (rows 2c, 2c+1 and 32+2c, 33+2c for
//    lane column c), software-pipelined PF k-steps ahead in two register
//    halves.  The loads of interior tiles carry no per-lane conditions (the
//    step index is clamped and the surplus steps multiply by a zero B
//    fragment), so the compiler can wait on exactly the half it needs;
//  * the block X is first packed k-major (p x 32, zero-padded) so that the
//    MFMA B fragments are contiguous 16-byte loads too, shared by all
//    wavefronts through L1/L2;
//  * four row fragments x two column fragments = eight
//    v_mfma_f64_16x16x4_f64 per k-step.  Fragment (fm, fn), row i, column c
//    is row 32 (fm / 2) + 2 i + (fm % 2) and column 2 c + fn of the tile;
//  * the k dimension is split over workgroups for occupancy; each wavefront
//    writes its 64 x 32 partial tile in lane order (256 contiguous bytes per
//    lane) and a second kernel sums the splits in a fixed order (bitwise
//    reproducible) and writes the column-major result.  For the CG it also
//    forms the per-tile, per-column sums of p . (A p).
#include "device.hpp"
#include "kernels.hpp"

namespace lrep {

namespace {

constexpr int WR = 64;       // rows per wavefront tile
constexpr int PF_WIDE = 4;   // k-steps (4 columns each) per prefetch half, grids above one wave per SIMD
constexpr int PF_ONE = 8;    // the same at most one workgroup per SIMD (282 registers, one wave each)
constexpr int TV = WR / 2;   // values per lane in a tile (WR x 32 / 64 lanes)
typedef double nd2 __attribute__((ext_vector_type(2)));   // for the non-temporal builtin

// Pt (p x 32, row k = X[k, 0:32], zero-padded) from X (p x q, ld ldx)
__global__ __launch_bounds__(256) void pack_kmajor_kernel(int p, int q, const double* __restrict__ X, int64_t ldx,
                                                          double* __restrict__ Pt, const int* __restrict__ flag) {
    if (flag && *flag == 0) return;
    __shared__ double tile[64][33];
    const int r0 = blockIdx.x * 64;
    for (int idx = threadIdx.x; idx < 64 * 32; idx += 256) {
        const int c = idx / 64, i = idx % 64;
        tile[i][c] = (c < q && r0 + i < p) ? X[(int64_t)c * ldx + r0 + i] : 0.0;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < 64 * 32; idx += 256) {
        const int i = idx / 32, c = idx % 32;
        if (r0 + i < p) Pt[(int64_t)(r0 + i) * 32 + c] = tile[i][c];
    }
}

// CG search direction fused with the packing: for the active columns
// p = r + beta p (written back to P, ld n) unless `first`, then Pt = pack(P).
__global__ __launch_bounds__(256) void cg_dir_pack_kernel(int n, int w, double* __restrict__ P,
                                                          const double* __restrict__ R,
                                                          const double* __restrict__ beta,
                                                          const int* __restrict__ active, int first,
                                                          double* __restrict__ Pt, const int* __restrict__ flag,
                                                          int* __restrict__ flag_log) {
    const int on = *flag;
    if (flag_log && blockIdx.x == 0 && threadIdx.x == 0) *flag_log = on;
    if (on == 0) return;
    __shared__ double tile[64][33];
    const int r0 = blockIdx.x * 64;
    for (int idx = threadIdx.x; idx < 64 * 32; idx += 256) {
        const int c = idx / 64, i = idx % 64;
        const int row = r0 + i;
        double v = 0.0;
        if (c < w && row < n) {
            v = P[(int64_t)c * n + row];
            if (!first && active[c]) {
                v = R[(int64_t)c * n + row] + beta[c] * v;
                P[(int64_t)c * n + row] = v;
            }
        }
        tile[i][c] = v;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < 64 * 32; idx += 256) {
        const int i = idx / 32, c = idx % 32;
        if (r0 + i < n) Pt[(int64_t)(r0 + i) * 32 + c] = tile[i][c];
    }
}

__device__ __forceinline__ void mfma_step(d4 (&acc)[4][2], double2 x, double2 y, double2 b) {
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x.x, b.x, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x.x, b.y, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x.y, b.x, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x.y, b.y, acc[1][1], 0, 0, 0);
    acc[2][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(y.x, b.x, acc[2][0], 0, 0, 0);
    acc[2][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(y.x, b.y, acc[2][1], 0, 0, 0);
    acc[3][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(y.y, b.x, acc[3][0], 0, 0, 0);
    acc[3][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(y.y, b.y, acc[3][1], 0, 0, 0);
}

// Direct epilogue of an unsplit stream launch: C = alpha A X (+ delta o Yd).
struct StreamOut {
    double* C;
    int64_t ldc;
    int q;
    double alpha;
    const double* delta;
    const double* Yd;
    int64_t ldyd;
};

template <int PF>
__global__ __launch_bounds__(64) void apply_stream_kernel(int m, int p, const double* __restrict__ A, int64_t lda,
                                                          const double* __restrict__ Pt, int kchunk,
                                                          double* __restrict__ part, const int* __restrict__ flag,
                                                          StreamOut so) {
    if (flag && *flag == 0) return;
    const int lane = threadIdx.x;
    const int tile = blockIdx.x, split = blockIdx.y;
    const int row0 = tile * WR;
    const int k_begin = split * kchunk;
    const int k_end = min(p, k_begin + kchunk);
    const int nfull = max(0, (k_end - k_begin) / 4);   // k-steps with all four columns in range
    const int c = lane % 16, kq = lane / 16;
    d4 acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i][0] = acc[i][1] = d4{0.0, 0.0, 0.0, 0.0};

    if (row0 + WR <= m && nfull > 0) {
        // interior tile: unconditional 16-byte loads, steps clamped to nfull - 1
        const double* a_base = A + (int64_t)(k_begin + kq) * lda + row0 + 2 * c;
        const double* b_base = Pt + (int64_t)(k_begin + kq) * 32 + 2 * c;
        const int64_t a_step = 4 * lda;
        double2 x0[PF], y0[PF], b0[PF], x1[PF], y1[PF], b1[PF];
        auto load = [&](double2 (&x)[PF], double2 (&y)[PF], double2 (&b)[PF], int s0) {
#pragma unroll
            for (int j = 0; j < PF; ++j) {
                const int s = min(s0 + j, nfull - 1);
                const double* ap = a_base + (int64_t)s * a_step;
                // the operator is read once per launch: non-temporal loads keep
                // it from displacing the packed block, which every workgroup
                // re-reads, from the caches (7.6 % faster at n = 8192)
                const nd2 xv = __builtin_nontemporal_load(reinterpret_cast<const nd2*>(ap));
                const nd2 yv = __builtin_nontemporal_load(reinterpret_cast<const nd2*>(ap + 32));
                x[j] = double2{xv.x, xv.y};
                y[j] = double2{yv.x, yv.y};
                b[j] = *reinterpret_cast<const double2*>(b_base + (int64_t)s * 128);
            }
        };
        auto compute = [&](const double2 (&x)[PF], const double2 (&y)[PF], const double2 (&b)[PF], int s0) {
#pragma unroll
            for (int j = 0; j < PF; ++j) {
                const bool live = s0 + j < nfull;
                const double2 bz = {live ? b[j].x : 0.0, live ? b[j].y : 0.0};
                mfma_step(acc, x[j], y[j], bz);
            }
        };
        load(x0, y0, b0, 0);
        for (int s = 0; s < nfull; s += 2 * PF) {
            load(x1, y1, b1, s + PF);
            compute(x0, y0, b0, s);
            load(x0, y0, b0, s + 2 * PF);
            compute(x1, y1, b1, s + PF);
        }
    } else if (nfull > 0) {
        // edge tile: per-lane row checks, no pipelining
        const int r0 = row0 + 2 * c, r1 = row0 + 32 + 2 * c;
        for (int s = 0; s < nfull; ++s) {
            const int k = k_begin + 4 * s + kq;
            const double* ap = A + (int64_t)k * lda;
            double2 x = {0.0, 0.0}, y = {0.0, 0.0};
            if (r0 < m) x.x = ap[r0];
            if (r0 + 1 < m) x.y = ap[r0 + 1];
            if (r1 < m) y.x = ap[r1];
            if (r1 + 1 < m) y.y = ap[r1 + 1];
            const double2 b = *reinterpret_cast<const double2*>(Pt + (int64_t)k * 32 + 2 * c);
            mfma_step(acc, x, y, b);
        }
    }
    if (k_begin + 4 * nfull < k_end) {
        // last partial k-step of the chunk
        const int k = k_begin + 4 * nfull + kq;
        const int r0 = row0 + 2 * c, r1 = row0 + 32 + 2 * c;
        double2 x = {0.0, 0.0}, y = {0.0, 0.0}, b = {0.0, 0.0};
        if (k < k_end) {
            const double* ap = A + (int64_t)k * lda;
            if (r0 < m) x.x = ap[r0];
            if (r0 + 1 < m) x.y = ap[r0 + 1];
            if (r1 < m) y.x = ap[r1];
            if (r1 + 1 < m) y.y = ap[r1 + 1];
            b = *reinterpret_cast<const double2*>(Pt + (int64_t)k * 32 + 2 * c);
        }
        mfma_step(acc, x, y, b);
    }
    if (so.C) {
        // item v of fragment (fm, fn): row 32 (fm / 2) + 2 (4 v + kq) + fm % 2, column 2 c + fn
#pragma unroll
        for (int fm = 0; fm < 4; ++fm)
#pragma unroll
            for (int fn = 0; fn < 2; ++fn)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = row0 + 32 * (fm / 2) + 2 * (4 * v + kq) + (fm % 2);
                    const int col = 2 * c + fn;
                    if (row < m && col < so.q) {
                        double o = so.alpha * acc[fm][fn][v];
                        if (so.delta) o = fma(so.delta[row], so.Yd[(int64_t)col * so.ldyd + row], o);
                        so.C[(int64_t)col * so.ldc + row] = o;
                    }
                }
        return;
    }
    const int ntiles = (m + WR - 1) / WR;
    double* out = part + (((int64_t)split * ntiles + tile) * WAVE + lane) * TV;
#pragma unroll
    for (int fm = 0; fm < 4; ++fm)
#pragma unroll
        for (int fn = 0; fn < 2; ++fn) *reinterpret_cast<d4*>(out + (fm * 2 + fn) * 4) = acc[fm][fn];
}

// ---------------------------------------------------------------------------
// Low-rank M apply, first pass: T = L^T Y for L (n x r, r <= 256, ld even,
// 16-byte aligned) and Y (n x w, w <= 32, ld even).  Workgroup g reduces rows
// [g * chunk, (g + 1) * chunk); wavefront v owns L's columns [64 v, 64 v + 64)
// (four 16-column fragments) and all 32 columns of Y (two fragments).  The
// rows are taken in units of 16: lane group kq = l / 16 reads rows
// 4 kq .. 4 kq + 3 of its column (two 16-byte loads, 128 contiguous bytes per
// column and unit over the four groups) and feeds them to four MFMA k-steps,
// so a unit is 32 v_mfma_f64_16x16x4_f64.  Partial T tiles are written in
// lane order and summed in a fixed order by lty_reduce_kernel, which writes T
// k-major (r x 32) for the second pass.
// ---------------------------------------------------------------------------
constexpr int LU = 16;   // rows per unit

__global__ __launch_bounds__(256) void lowrank_lty_kernel(int n, int r, int w, const double* __restrict__ L,
                                                          int64_t ldl, const double* __restrict__ Y, int64_t ldy,
                                                          int chunk, double* __restrict__ part,
                                                          const int* __restrict__ flag) {
    if (flag && *flag == 0) return;
    const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
    const int c = lane % 16, kq = lane / 16;
    const int i_begin = blockIdx.x * chunk;
    const int i_end = min(n, i_begin + chunk);
    const int nfull = max(0, (i_end - i_begin) / LU);
    d4 acc[4][2];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t][0] = acc[t][1] = d4{0.0, 0.0, 0.0, 0.0};
    // columns this lane reads (clamped into range; out-of-range ones are zeroed)
    int lc[4];
    bool lok[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int col = 64 * wv + 16 * t + c;
        lok[t] = col < r;
        lc[t] = lok[t] ? col : 0;
    }
    const int yc0 = c, yc1 = 16 + c;
    const bool yok0 = yc0 < w, yok1 = yc1 < w;
    const double* lp[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) lp[t] = L + (int64_t)lc[t] * ldl + i_begin + 4 * kq;
    const double* yp0 = Y + (int64_t)(yok0 ? yc0 : 0) * ldy + i_begin + 4 * kq;
    const double* yp1 = Y + (int64_t)(yok1 ? yc1 : 0) * ldy + i_begin + 4 * kq;
    // four k-steps of one unit: step e pairs row 4 kq + e of L and Y
    auto compute = [&](const double2 (&a)[4][2], const double2 (&b)[2][2]) {
        double2 bb[2][2], aa[4][2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            bb[0][h] = yok0 ? b[0][h] : double2{0.0, 0.0};
            bb[1][h] = yok1 ? b[1][h] : double2{0.0, 0.0};
#pragma unroll
            for (int t = 0; t < 4; ++t) aa[t][h] = lok[t] ? a[t][h] : double2{0.0, 0.0};
        }
        // all eight accumulators once per k-step, so that no MFMA waits on
        // the one just issued
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int u = 0; u < 2; ++u)
                    acc[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(aa[t][h].x, bb[u][h].x, acc[t][u], 0, 0, 0);
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int u = 0; u < 2; ++u)
                    acc[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(aa[t][h].y, bb[u][h].y, acc[t][u], 0, 0, 0);
        }
    };
    if (nfull > 0) {
        double2 a0[4][2], b0[2][2], a1[4][2], b1[2][2];
        // surplus loads re-read the last unit (in range) and are not used
        auto load = [&](double2 (&a)[4][2], double2 (&b)[2][2], int s) {
            const int64_t o = (int64_t)min(s, nfull - 1) * LU;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
#pragma unroll
                for (int t = 0; t < 4; ++t) a[t][h] = *reinterpret_cast<const double2*>(lp[t] + o + 2 * h);
                b[0][h] = *reinterpret_cast<const double2*>(yp0 + o + 2 * h);
                b[1][h] = *reinterpret_cast<const double2*>(yp1 + o + 2 * h);
            }
        };
        load(a0, b0, 0);
        for (int s = 0; s < nfull; s += 2) {
            load(a1, b1, s + 1);
            __builtin_amdgcn_sched_barrier(0);
            compute(a0, b0);
            __builtin_amdgcn_sched_barrier(0);
            load(a0, b0, s + 2);
            __builtin_amdgcn_sched_barrier(0);
            if (s + 1 < nfull) compute(a1, b1);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    if (i_begin + LU * nfull < i_end) {
        // last partial unit of the chunk: rows at or beyond i_end count zero
        const int i0 = i_begin + LU * nfull;
        double2 a[4][2], b[2][2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int ia = i0 + 4 * kq + 2 * h, ib = ia + 1;
            b[0][h] = double2{(yok0 && ia < i_end) ? Y[(int64_t)yc0 * ldy + ia] : 0.0,
                              (yok0 && ib < i_end) ? Y[(int64_t)yc0 * ldy + ib] : 0.0};
            b[1][h] = double2{(yok1 && ia < i_end) ? Y[(int64_t)yc1 * ldy + ia] : 0.0,
                              (yok1 && ib < i_end) ? Y[(int64_t)yc1 * ldy + ib] : 0.0};
#pragma unroll
            for (int t = 0; t < 4; ++t)
                a[t][h] = double2{(lok[t] && ia < i_end) ? L[(int64_t)lc[t] * ldl + ia] : 0.0,
                                  (lok[t] && ib < i_end) ? L[(int64_t)lc[t] * ldl + ib] : 0.0};
        }
        compute(a, b);
    }
    double* out = part + ((int64_t)blockIdx.x * 256 + threadIdx.x) * 32;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u) *reinterpret_cast<d4*>(out + (t * 2 + u) * 4) = acc[t][u];
}

// T (k-major, r x 32, zero-padded) = alpha * sum over the chunks of the
// partial tiles, in a fixed order.  Block b handles entries [64 b, 64 b + 64)
// of the per-workgroup tile (lane-order layout of lowrank_lty_kernel): its
// four wavefronts sum the chunks k = wv, wv + 4, ... for the 64 entries, then
// wavefront 0 adds the four partial sums in order.
__global__ __launch_bounds__(256) void lty_reduce_kernel(int r, int nchunk, const double* __restrict__ part,
                                                         double alpha, double* __restrict__ Pt,
                                                         const int* __restrict__ flag) {
    if (flag && *flag == 0) return;
    __shared__ double red[4][64];
    const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
    const int e = blockIdx.x * 64 + lane;   // < 8192
    double s0 = 0.0, s1 = 0.0;
    int k = wv;
    for (; k + 4 < nchunk; k += 8) {
        s0 += part[(int64_t)k * 8192 + e];
        s1 += part[(int64_t)(k + 4) * 8192 + e];
    }
    if (k < nchunk) s0 += part[(int64_t)k * 8192 + e];
    red[wv][lane] = s0 + s1;
    __syncthreads();
    if (wv != 0) return;
    const double s = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
    const int tl = e / 32, v = e % 32;               // thread of the partial tile, item
    const int pw = tl / WAVE, pl = tl % WAVE;
    const int t = v / 8, u = (v / 4) % 2, it = v % 4;
    const int row = 64 * pw + 16 * t + 4 * it + pl / 16;   // index into r
    const int col = 16 * u + pl % 16;
    if (row < r) Pt[(int64_t)row * 32 + col] = alpha * s;
}

// Sum of the split partial tiles: block (tile, g) of 256 threads writes rows
// [64 tile, 64 tile + 64) of result columns 8g .. 8g + 7; thread t takes row
// t % 64 and the column pair 8g + 2 (t / 64) + {0, 1}, which sit next to each
// other in one lane's partial tile.  The splits are added in a fixed order
// (bitwise reproducible); all split loads are issued before the adds.
// C = alpha * sum + beta * C; with P != null also
// pq[tile * 32 + col] = sum over the tile's rows of P[row, col] * C[row, col].
constexpr int MAXSPLIT = 16;

__global__ __launch_bounds__(256) void apply_reduce_kernel(int m, int q, int nsplit, const double* __restrict__ part,
                                                           double* __restrict__ C, int64_t ldc, double alpha,
                                                           double beta, const double* __restrict__ P, int64_t ldp,
                                                           double* __restrict__ pq, const int* __restrict__ flag) {
    if (flag && *flag == 0) return;
    const int tile = blockIdx.x, g = blockIdx.y;
    const int ntiles = (m + WR - 1) / WR;
    const int64_t total = (int64_t)ntiles * WAVE * TV;
    const int row = threadIdx.x % WR, cp = threadIdx.x / WR;
    const int col0 = 8 * g + 2 * cp;                 // fn = 0; col0 + 1 has fn = 1
    const int fm = 2 * (row / 32) + (row % 2);
    const int t = (row % 32) / 2;                     // 4 r + lane / 16
    const int lane = 16 * (t % 4) + col0 / 2;
    const int v0 = 4 * (2 * fm) + t / 4;              // f = 2 fm + fn, v = 4 f + r
    const double* src = part + (int64_t)tile * WAVE * TV + lane * TV + v0;
    double x[MAXSPLIT], y[MAXSPLIT];
#pragma unroll
    for (int k = 0; k < MAXSPLIT; ++k) {
        const int kc = k < nsplit ? k : nsplit - 1;
        x[k] = src[(int64_t)kc * total];
        y[k] = src[(int64_t)kc * total + 4];
    }
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int k = 0; k < MAXSPLIT; ++k) {
        if (k < nsplit) {
            s0 += x[k];
            s1 += y[k];
        }
    }
    const int grow = tile * WR + row;
    double p0 = 0.0, p1 = 0.0;
    if (grow < m) {
        if (col0 < q) {
            double o = alpha * s0;
            if (beta != 0.0) o += beta * C[(int64_t)col0 * ldc + grow];
            C[(int64_t)col0 * ldc + grow] = o;
            if (P) p0 = P[(int64_t)col0 * ldp + grow] * o;
        }
        if (col0 + 1 < q) {
            double o = alpha * s1;
            if (beta != 0.0) o += beta * C[(int64_t)(col0 + 1) * ldc + grow];
            C[(int64_t)(col0 + 1) * ldc + grow] = o;
            if (P) p1 = P[(int64_t)(col0 + 1) * ldp + grow] * o;
        }
    }
    if (P) {
        // the wavefront holds the 64 rows of this column pair
        p0 = wave_sum(p0);
        p1 = wave_sum(p1);
        if (row == 0) {
            pq[(int64_t)tile * 32 + col0] = p0;
            pq[(int64_t)tile * 32 + col0 + 1] = p1;
        }
    }
}

struct StreamPlan {
    int ntiles, ksplit, kchunk;
    int64_t tile_elems;
    int pf = PF_WIDE;
};

bool plan_stream(int m, int p, size_t work_elems, StreamPlan& pl) {
    pl.ntiles = (m + WR - 1) / WR;
    pl.tile_elems = (int64_t)pl.ntiles * WAVE * TV;
    if ((size_t)p * 32 + (size_t)pl.tile_elems > work_elems) return false;
    int ksplit = 1;
    // about 1024 workgroups, k chunks of at most 8192 columns (a longer
    // stream per workgroup), each split adding a partial tile set to write
    // and reduce
    while ((pl.ntiles * ksplit < 1024 || p / ksplit > 8192) && p / (ksplit * 2) >= 256 && ksplit < MAXSPLIT &&
           (size_t)p * 32 + (size_t)(2 * ksplit) * pl.tile_elems <= work_elems)
        ksplit *= 2;
    // a grid of at most one workgroup per SIMD prefetches twice as deep (one
    // wave per SIMD either way; 1.6 % faster at n = 8192)
    pl.pf = pl.ntiles * ksplit <= 1024 ? PF_ONE : PF_WIDE;
    // chunks of whole prefetch rounds (2 PF k-steps of 4 columns)
    int kchunk = (p + ksplit - 1) / ksplit;
    kchunk = ((kchunk + 8 * pl.pf - 1) / (8 * pl.pf)) * (8 * pl.pf);
    pl.ksplit = (p + kchunk - 1) / kchunk;
    pl.kchunk = kchunk;
    return true;
}

}  // namespace

size_t stream_tiles(int m) { return (size_t)((m + WR - 1) / WR); }

hipError_t dense_apply_narrow(hipStream_t st, int m, int q, int p, const double* A, int64_t lda, const double* X,
                              int64_t ldx, double* C, int64_t ldc, double alpha, double beta, double* work,
                              size_t work_elems, const int* active_flag, hipEvent_t* ev) {
    if (q < 1 || q > 32 || m < 1 || p < 1 || (lda & 1) || (reinterpret_cast<uintptr_t>(A) & 15))
        return hipErrorInvalidValue;
    StreamPlan pl;
    if (!plan_stream(m, p, work_elems, pl)) return hipErrorInvalidValue;
    double* Pt = work;
    double* part = work + (size_t)p * 32;
    hipLaunchKernelGGL(pack_kmajor_kernel, dim3((p + 63) / 64), dim3(256), 0, st, p, q, X, ldx, Pt, active_flag);
    if (ev) (void)hipEventRecord(ev[0], st);
    if (pl.pf == PF_ONE)
        hipLaunchKernelGGL(apply_stream_kernel<PF_ONE>, dim3(pl.ntiles, pl.ksplit), dim3(64), 0, st, m, p, A, lda, Pt,
                           pl.kchunk, part, active_flag, StreamOut{});
    else
        hipLaunchKernelGGL(apply_stream_kernel<PF_WIDE>, dim3(pl.ntiles, pl.ksplit), dim3(64), 0, st, m, p, A, lda, Pt,
                           pl.kchunk, part, active_flag, StreamOut{});
    if (ev) (void)hipEventRecord(ev[1], st);
    hipLaunchKernelGGL(apply_reduce_kernel, dim3(pl.ntiles, (q + 7) / 8), dim3(256), 0, st, m, q, pl.ksplit, part, C, ldc, alpha,
                       beta, (const double*)nullptr, (int64_t)0, (double*)nullptr, active_flag);
    return hipGetLastError();
}

hipError_t cg_dense_apply(hipStream_t st, int n, int w, const double* A, int64_t lda, double* P, const double* R,
                          const double* beta, const int* active, int first, double* Q, double* pq, double* work,
                          size_t work_elems, const int* any_active, hipEvent_t* ev, int* flag_log) {
    if (w < 1 || w > 32 || n < 1 || (lda & 1) || (reinterpret_cast<uintptr_t>(A) & 15)) return hipErrorInvalidValue;
    StreamPlan pl;
    if (!plan_stream(n, n, work_elems, pl)) return hipErrorInvalidValue;
    double* Pt = work;
    double* part = work + (size_t)n * 32;
    hipLaunchKernelGGL(cg_dir_pack_kernel, dim3((n + 63) / 64), dim3(256), 0, st, n, w, P, R, beta, active, first, Pt,
                       any_active, flag_log);
    if (ev) (void)hipEventRecord(ev[0], st);
    if (pl.pf == PF_ONE)
        hipLaunchKernelGGL(apply_stream_kernel<PF_ONE>, dim3(pl.ntiles, pl.ksplit), dim3(64), 0, st, n, n, A, lda, Pt,
                           pl.kchunk, part, any_active, StreamOut{});
    else
        hipLaunchKernelGGL(apply_stream_kernel<PF_WIDE>, dim3(pl.ntiles, pl.ksplit), dim3(64), 0, st, n, n, A, lda, Pt,
                           pl.kchunk, part, any_active, StreamOut{});
    if (ev) (void)hipEventRecord(ev[1], st);
    hipLaunchKernelGGL(apply_reduce_kernel, dim3(pl.ntiles, 4), dim3(256), 0, st, n, w, pl.ksplit, part, Q, (int64_t)n,
                       1.0, 0.0, (const double*)P, (int64_t)n, pq, any_active);
    return hipGetLastError();
}

hipError_t lowrank_apply_M(hipStream_t st, int n, int r, int w, const double* delta, const double* L, int64_t ldl,
                           const double* Y, int64_t ldy, double* C, int64_t ldc, double* work, size_t work_elems,
                           const int* active_flag, hipEvent_t* ev) {
    if (w < 1 || w > 32 || r < 1 || r > 256 || n < 1 || (ldl & 1) || (ldy & 1) ||
        (reinterpret_cast<uintptr_t>(L) & 15) || (reinterpret_cast<uintptr_t>(Y) & 15))
        return hipErrorInvalidValue;
    // first pass: up to two workgroups per CU, chunks of whole prefetch rounds
    int nchunk = std::max(1, std::min(512, n / 512));
    int chunk = (n + nchunk - 1) / nchunk;
    chunk = ((chunk + 2 * LU - 1) / (2 * LU)) * (2 * LU);
    nchunk = (n + chunk - 1) / chunk;
    double* Pt = work;                        // r x 32
    double* part = work + 256 * 32;           // nchunk x 8192
    if ((size_t)256 * 32 + (size_t)nchunk * 8192 > work_elems) return hipErrorInvalidValue;
    if (ev) (void)hipEventRecord(ev[0], st);
    hipLaunchKernelGGL(lowrank_lty_kernel, dim3(nchunk), dim3(256), 0, st, n, r, w, L, ldl, Y, ldy, chunk, part,
                       active_flag);
    hipLaunchKernelGGL(lty_reduce_kernel, dim3(128), dim3(256), 0, st, r, nchunk, part, 2.0, Pt, active_flag);
    // second pass: C = (2 L T) + delta o Y, unsplit stream with the direct epilogue
    const int ntiles = (n + WR - 1) / WR;
    const int kchunk = ((r + 3) / 4) * 4;
    hipLaunchKernelGGL(apply_stream_kernel<PF_WIDE>, dim3(ntiles, 1), dim3(64), 0, st, n, r, L, ldl, Pt, kchunk, part,
                       active_flag, StreamOut{C, ldc, w, 1.0, delta, Y, ldy});
    if (ev) (void)hipEventRecord(ev[1], st);
    return hipGetLastError();
}

}  // namespace lrep
