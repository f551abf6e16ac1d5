// Low-rank M apply, M Y = delta o Y + 2 L (L^T Y), on a row-major copy of L.
//
// L (n x r, r <= 256) is kept a second time row by row (row i = L[i, 0:r],
// zero-padded to ldr = r rounded up to 64), so that both passes stream it in
// long contiguous runs: a 16-row unit of the first pass reads 16 whole rows
// (ldr * 128 bytes), and a wavefront of the second pass reads, for each of
// its 64 rows, one contiguous run per 16-deep unit.  With the column-major
// layout every column of a row chunk is a separate short run 8 n bytes away
// from the next, which held the first pass at about 2.5 TB/s.
//
//   pass 1  T = L^T Y, reduction over n: workgroup g takes rows
//           [g chunk, (g + 1) chunk); wavefront v owns L's columns
//           [64 v, 64 v + 64) and all 32 columns of Y.  Lane group q = l / 16
//           takes rows 4 q .. 4 q + 3 of a unit and feeds them to four MFMA
//           k-steps.  Partial tiles in lane order, summed over the chunks in
//           a fixed order into T (k-major, ldr x 32, times 2).
//   pass 2  C = (2 L) T + delta o Y: one wavefront per 64 rows, k over ldr in
//           16-deep units (lane group q holds k = 4 q .. 4 q + 3 of each of
//           its rows: one 32-byte run), the MFMA called with T as the first
//           operand so that each store covers 16 consecutive rows.
#include "device.hpp"
#include "kernels.hpp"

namespace lrep {

namespace {

constexpr int RU = 16;   // rows (pass 1) or k (pass 2) per unit
constexpr int RW = 64;   // rows per wavefront in pass 2

// Lr (n x ldr, row-major, zero-padded) = L (n x r, column-major, ld ldl);
// 64 x 64 tiles through LDS
__global__ __launch_bounds__(256) void lrow_kernel(int n, int r, int ldr, const double* __restrict__ L, int64_t ldl,
                                                   double* __restrict__ Lr) {
    __shared__ double t[64][65];
    const int i0 = blockIdx.x * 64, k0 = blockIdx.y * 64;
    for (int idx = threadIdx.x; idx < 64 * 64; idx += 256) {
        const int i = idx % 64, k = idx / 64;
        t[k][i] = (i0 + i < n && k0 + k < r) ? L[(int64_t)(k0 + k) * ldl + i0 + i] : 0.0;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < 64 * 64; idx += 256) {
        const int k = idx % 64, i = idx / 64;
        if (i0 + i < n && k0 + k < ldr) Lr[(int64_t)(i0 + i) * ldr + k0 + k] = t[k][i];
    }
}

__global__ __launch_bounds__(256) void lr_lty_kernel(int n, int ldr, int w, const double* __restrict__ Lr,
                                                     const double* __restrict__ Y, int64_t ldy, int chunk,
                                                     double* __restrict__ part, const int* __restrict__ flag) {
    if (flag && *flag == 0) return;
    const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
    const int c = lane % 16, g = lane / 16;
    const int i_begin = blockIdx.x * chunk;
    const int i_end = min(n, i_begin + chunk);
    const int nfull = max(0, (i_end - i_begin) / RU);
    d4 acc[4][2];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t][0] = acc[t][1] = d4{0.0, 0.0, 0.0, 0.0};
    if (64 * wv < ldr) {   // wavefront-uniform: this wavefront's columns exist (ldr is a multiple of 64)
        const double* lp = Lr + (int64_t)(i_begin + 4 * g) * ldr + 64 * wv + c;   // + 16 t + e ldr
        const int yc0 = c, yc1 = 16 + c;
        const bool yok0 = yc0 < w, yok1 = yc1 < w;
        const double* yp0 = Y + (int64_t)(yok0 ? yc0 : 0) * ldy + i_begin + 4 * g;
        const double* yp1 = Y + (int64_t)(yok1 ? yc1 : 0) * ldy + i_begin + 4 * g;
        // use = false (wavefront-uniform) multiplies the unit by zero
        auto compute = [&](const double (&a)[4][4], const double2 (&b)[2][2], bool use) {
            const bool u0 = yok0 && use, u1 = yok1 && use;
            double bb[2][4];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                bb[0][2 * h] = u0 ? b[0][h].x : 0.0;
                bb[0][2 * h + 1] = u0 ? b[0][h].y : 0.0;
                bb[1][2 * h] = u1 ? b[1][h].x : 0.0;
                bb[1][2 * h + 1] = u1 ? b[1][h].y : 0.0;
            }
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int u = 0; u < 2; ++u)
                        acc[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t][e], bb[u][e], acc[t][u], 0, 0, 0);
        };
        if (nfull > 0) {
            double a0[4][4], a1[4][4];
            double2 b0[2][2], b1[2][2];
            // surplus loads re-read the last unit (in range) and are not used
            auto load = [&](double (&a)[4][4], double2 (&b)[2][2], int s) {
                const int64_t o = (int64_t)min(s, nfull - 1) * RU;
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int t = 0; t < 4; ++t) a[t][e] = lp[(o + e) * ldr + 16 * t];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    b[0][h] = *reinterpret_cast<const double2*>(yp0 + o + 2 * h);
                    b[1][h] = *reinterpret_cast<const double2*>(yp1 + o + 2 * h);
                }
            };
            // both halves are computed unconditionally (a surplus odd unit
            // counts zero): with a conditional second half the compiler sinks
            // its loads behind the first half's products and nothing overlaps
            load(a0, b0, 0);
            for (int s = 0; s < nfull; s += 2) {
                load(a1, b1, s + 1);
                __builtin_amdgcn_sched_barrier(0);
                compute(a0, b0, true);
                __builtin_amdgcn_sched_barrier(0);
                load(a0, b0, s + 2);
                __builtin_amdgcn_sched_barrier(0);
                compute(a1, b1, s + 1 < nfull);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        if (i_begin + RU * nfull < i_end) {
            // last partial unit of the chunk: rows at or beyond i_end count zero
            const int i0 = i_begin + RU * nfull;
            double a[4][4];
            double2 b[2][2];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = i0 + 4 * g + e;
                const bool in = row < i_end;
                const int rr = in ? row : i_end - 1;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const double v = Lr[(int64_t)rr * ldr + 64 * wv + 16 * t + c];
                    a[t][e] = in ? v : 0.0;
                }
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int ia = i0 + 4 * g + 2 * h, ib = ia + 1;
                b[0][h] = double2{(yok0 && ia < i_end) ? Y[(int64_t)yc0 * ldy + ia] : 0.0,
                                  (yok0 && ib < i_end) ? Y[(int64_t)yc0 * ldy + ib] : 0.0};
                b[1][h] = double2{(yok1 && ia < i_end) ? Y[(int64_t)yc1 * ldy + ia] : 0.0,
                                  (yok1 && ib < i_end) ? Y[(int64_t)yc1 * ldy + ib] : 0.0};
            }
            compute(a, b, true);
        }
    }
    double* out = part + ((int64_t)blockIdx.x * 256 + threadIdx.x) * 32;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u) *reinterpret_cast<d4*>(out + (t * 2 + u) * 4) = acc[t][u];
}

// T (k-major, rows 0 .. ldr - 1, 32 columns) = alpha * sum over the chunks of
// the partial tiles, in a fixed order.  Block b handles entries
// [32 b, 32 b + 32) of the per-workgroup tile (lane order of lr_lty_kernel);
// thread (entry t % 32, phase q = t / 32) sums the chunks q, q + 16, ... in
// two interleaved partial sums, and the 16 phase sums are added in order.
constexpr int RED_PH = 16;
__global__ __launch_bounds__(32 * RED_PH) void lr_reduce_kernel(int ldr, int nchunk, const double* __restrict__ part,
                                                               double alpha, double* __restrict__ Pt,
                                                               const int* __restrict__ flag) {
    if (flag && *flag == 0) return;
    __shared__ double red[RED_PH][32];
    const int x = threadIdx.x % 32, q = threadIdx.x / 32;
    const int e = blockIdx.x * 32 + x;   // < 8192
    double s0 = 0.0, s1 = 0.0;
    int k = q;
    for (; k + RED_PH < nchunk; k += 2 * RED_PH) {
        s0 += part[(int64_t)k * 8192 + e];
        s1 += part[(int64_t)(k + RED_PH) * 8192 + e];
    }
    if (k < nchunk) s0 += part[(int64_t)k * 8192 + e];
    red[q][x] = s0 + s1;
    __syncthreads();
    if (q != 0) return;
    double s = red[0][x];
#pragma unroll
    for (int p = 1; p < RED_PH; ++p) s += red[p][x];
    const int tl = e / 32, v = e % 32;               // thread of the partial tile, item
    const int pw = tl / WAVE, pl = tl % WAVE;
    const int t = v / 8, u = (v / 4) % 2, it = v % 4;
    const int row = 64 * pw + 16 * t + 4 * it + pl / 16;   // index into the columns of L
    const int col = 16 * u + pl % 16;
    if (row < ldr) Pt[(int64_t)row * 32 + col] = alpha * s;
}

// C (n x w, ld ldc) = Lr T + delta o Y; T = Pt (k-major, ldr x 32)
__global__ __launch_bounds__(64) void lr_apply_kernel(int n, int ldr, int w, const double* __restrict__ Lr,
                                                      const double* __restrict__ Pt,
                                                      const double* __restrict__ delta,
                                                      const double* __restrict__ Y, int64_t ldy,
                                                      double* __restrict__ C, int64_t ldc,
                                                      double* __restrict__ pq,
                                                      const int* __restrict__ flag) {
    if (flag && *flag == 0) return;
    const int lane = threadIdx.x, c = lane % 16, g = lane / 16;
    // tiles in reverse launch order: the first pass has just streamed L from
    // the first row to the last, so the last rows are the ones still in the
    // MALL; ending at row 0 in turn hands the first rows to the next first
    // pass (3-4 % on each pass)
    const int tile = gridDim.x - 1 - blockIdx.x;
    const int row0 = tile * RW;
    // rows beyond n read row n - 1; those outputs are not written
    const double* ap[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) ap[f] = Lr + (int64_t)min(row0 + 16 * f + c, n - 1) * ldr + 4 * g;
    const double* bp = Pt + (int64_t)(4 * g) * 32 + c;   // + (k0 + e) 32 + 16 u
    d4 acc[4][2];
#pragma unroll
    for (int f = 0; f < 4; ++f) acc[f][0] = acc[f][1] = d4{0.0, 0.0, 0.0, 0.0};
    const int nunits = ldr / RU;   // ldr is a multiple of 64
    double2 a0[4][2], a1[4][2];
    double b0[2][4], b1[2][4];
    auto load = [&](double2 (&a)[4][2], double (&b)[2][4], int s) {
        const int k0 = min(s, nunits - 1) * RU;
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            a[f][0] = *reinterpret_cast<const double2*>(ap[f] + k0);
            a[f][1] = *reinterpret_cast<const double2*>(ap[f] + k0 + 2);
        }
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int e = 0; e < 4; ++e) b[u][e] = bp[(int64_t)(k0 + e) * 32 + 16 * u];
    };
    auto compute = [&](const double2 (&a)[4][2], const double (&b)[2][4]) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                const double av = (e == 0) ? a[f][0].x : (e == 1) ? a[f][0].y : (e == 2) ? a[f][1].x : a[f][1].y;
#pragma unroll
                for (int u = 0; u < 2; ++u)
                    acc[f][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[u][e], av, acc[f][u], 0, 0, 0);
            }
    };
    // nunits is a multiple of 4, so both halves always run; they carry no
    // condition, which keeps the next half's loads ahead of the products
    load(a0, b0, 0);
    for (int s = 0; s < nunits; s += 2) {
        load(a1, b1, s + 1);
        __builtin_amdgcn_sched_barrier(0);
        compute(a0, b0);
        __builtin_amdgcn_sched_barrier(0);
        load(a0, b0, s + 2);
        __builtin_amdgcn_sched_barrier(0);
        compute(a1, b1);
        __builtin_amdgcn_sched_barrier(0);
    }
    // item r of (f, u): column 16 u + 4 r + g, row row0 + 16 f + c; with pq,
    // also the tile's sums Y[:, col] . C[:, col] (the CG's p . A p), summed
    // over f in order and then over the 16 lanes of the column
    double yc[2][4];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r) yc[u][r] = 0.0;
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = row0 + 16 * f + c, col = 16 * u + 4 * r + g;
                if (row < n && col < w) {
                    const double yv = Y[(int64_t)col * ldy + row];
                    const double o = fma(delta[row], yv, acc[f][u][r]);
                    C[(int64_t)col * ldc + row] = o;
                    yc[u][r] = fma(yv, o, yc[u][r]);
                }
            }
    if (pq) {
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double v = yc[u][r];
                v += __shfl_xor(v, 1, WAVE);
                v += __shfl_xor(v, 2, WAVE);
                v += __shfl_xor(v, 4, WAVE);
                v += __shfl_xor(v, 8, WAVE);
                if (c == 0) pq[(int64_t)tile * 32 + 16 * u + 4 * r + g] = v;
            }
    }
}

}  // namespace

int64_t lowrank_row_ld(int64_t r) { return ((r + 63) / 64) * 64; }

hipError_t lowrank_make_rows(hipStream_t st, int n, int r, const double* L, int64_t ldl, double* Lr) {
    const int ldr = (int)lowrank_row_ld(r);
    if (n < 1 || r < 1 || r > 256) return hipErrorInvalidValue;
    hipLaunchKernelGGL(lrow_kernel, dim3((n + 63) / 64, ldr / 64), dim3(256), 0, st, n, r, ldr, L, ldl, Lr);
    return hipGetLastError();
}

hipError_t lowrank_apply_M_rows(hipStream_t st, int n, int r, int w, const double* delta, const double* Lr,
                                const double* Y, int64_t ldy, double* C, int64_t ldc, double* work,
                                size_t work_elems, const int* active_flag, hipEvent_t* ev, double* pq) {
    const int ldr = (int)lowrank_row_ld(r);
    if (w < 1 || w > 32 || r < 1 || r > 256 || n < 1 || (ldy & 1) || (reinterpret_cast<uintptr_t>(Y) & 15) ||
        (reinterpret_cast<uintptr_t>(Lr) & 31))
        return hipErrorInvalidValue;
    // first pass: up to two workgroups per CU, chunks of whole prefetch rounds
    int nchunk = std::max(1, std::min(512, n / 512));
    int chunk = (n + nchunk - 1) / nchunk;
    chunk = ((chunk + 2 * RU - 1) / (2 * RU)) * (2 * RU);
    nchunk = (n + chunk - 1) / chunk;
    double* Pt = work;                        // ldr (<= 256) x 32
    double* part = work + 256 * 32;           // nchunk x 8192
    if ((size_t)256 * 32 + (size_t)nchunk * 8192 > work_elems) return hipErrorInvalidValue;
    if (ev) (void)hipEventRecord(ev[0], st);
    hipLaunchKernelGGL(lr_lty_kernel, dim3(nchunk), dim3(256), 0, st, n, ldr, w, Lr, Y, ldy, chunk, part,
                       active_flag);
    hipLaunchKernelGGL(lr_reduce_kernel, dim3(8192 / 32), dim3(32 * RED_PH), 0, st, ldr, nchunk, part, 2.0, Pt,
                       active_flag);
    hipLaunchKernelGGL(lr_apply_kernel, dim3((n + RW - 1) / RW), dim3(64), 0, st, n, ldr, w, Lr, Pt, delta, Y, ldy,
                       C, ldc, pq, active_flag);
    if (ev) (void)hipEventRecord(ev[1], st);
    return hipGetLastError();
}

}  // namespace lrep
