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

// ---------------------------------------------------------------------------
// Fused CG steps (Step 6 on a low-rank operator).
//
// CG for A = diag(delta) + 2 L L^T in a single pass over L per step.  With
// T_k = L^T p_k known before step k (a 256 x 32 block), A p_k = delta o p_k +
// 2 L T_k needs L only once; the same pass forms S = L^T r_{k+1} from the new
// residual, and since p_{k+1} = r_{k+1} + beta_k p_k, T_{k+1} = S + beta_k T_k.
// The step length alpha_k = rho_k / p_k^T A p_k uses p^T A p = p^T diag(delta) p
// + 2 |T|^2, where c_{k+1} = p_{k+1}^T diag(delta) p_{k+1} = a + 2 beta b +
// beta^2 c_k with a = r_{k+1}^T diag(delta) r_{k+1}, b = r_{k+1}^T diag(delta)
// p_k, both summed in the pass.  So alpha_k is known when step k starts and
// x, r, p are each read and written once per step.  (A plain CG step reads L
// twice -- for L^T p and for L (L^T p) -- and streams x, r, p, A p in separate
// passes.)
//
// Pass (fcg_pass_M_kernel): one workgroup of 512 threads per CU (LDS
// 142 KiB), run as two pipelines of four wavefronts over interleaved tiles of
// 16 rows; wavefront v of a pipeline owns L's columns [64 v, 64 v + 64).  Per
// tile j a pipeline runs two phases, each closed by a workgroup barrier:
//  A  (MFMA) the wavefront's 16 x 64 slice of tile j (rows 4 s + g, columns
//     32 h + 2 c and 32 h + 2 c + 1 in lane (g, c) = (lane / 16, lane % 16),
//     16-byte loads) goes to LDS; the partial product L_slice T_slice (A
//     operand read back with row on c, column on g) is interleaved with
//     S += L_{j-1}^T r_{j-1} from the previous slice, still in registers
//     (row on g); the next tile's slice is requested into the registers just
//     freed, and the partial product replaces the slice in LDS;
//  B  (vector) every thread takes two rows of one column: p = r + beta p,
//     A p = delta p + 2 (sum of the four partials in a fixed order),
//     x += alpha p, r -= alpha A p; x, r, p are stored, r goes to LDS, and the
//     next tile's vectors are requested.
// The second pipeline starts one phase late, so that while one pipeline's
// wavefronts are in their MFMA phase the other's are in their vector phase:
// the matrix cores and the memory stream see work in every interval.  Only
// T (read-only) is shared between the pipelines.  At the end the second
// pipeline hands its block of S and its column sums to the first through LDS,
// and S and the column sums leave the workgroup as one record.
// ---------------------------------------------------------------------------
constexpr int PT = 16;               // rows per tile
constexpr int FLS = 65;              // LDS stride of a wavefront's slice (16 rows x 64 columns of L)
constexpr int FMS = 33;              // LDS stride of the 32-column arrays (T, r, partial products)
constexpr int PSL = 4 * PT * FLS;    // doubles of a pipeline's slices
constexpr int PSR = PT * FMS;        // doubles of a pipeline's r
constexpr int FREC = 128;            // column sums per record: (rho, a, b, 0) for 32 columns
constexpr int FSINK = 6;             // doubles of the store sink per thread

// two consecutive entries of a row of L as loaded: a 16-byte load of the FP64
// rows or an 8-byte load of the FP32 rows; FP32 values are widened exactly to
// FP64 where they are used (LDS store, MFMA operand), so that registers hold
// the narrow form while the loads are in flight
template <typename LT> struct LPair;
template <> struct LPair<double> { using type = double2; };
template <> struct LPair<float> { using type = float2; };

template <typename LT>
__global__ __launch_bounds__(512) void fcg_pass_M_kernel(int n, int ldr, int w, int tpw,
                                                         const LT* __restrict__ Lr,
                                                         const double* __restrict__ delta, double* __restrict__ X,
                                                         double* __restrict__ R, double* __restrict__ P,
                                                         const double* __restrict__ T,
                                                         const double* __restrict__ alpha,
                                                         const double* __restrict__ beta,
                                                         const int* __restrict__ active, const int* __restrict__ any,
                                                         double* __restrict__ rec, int stride,
                                                         double* __restrict__ sink,
                                                         int* __restrict__ flag_log) {
    using P2 = typename LPair<LT>::type;
    const int on = *any;
    if (flag_log && blockIdx.x == 0 && threadIdx.x == 0) *flag_log = on;
    if (on == 0) return;
    __shared__ double sl[2 * PSL];     // per pipeline: wavefront slices of L, then the partial products
    __shared__ double stt[256 * FMS];  // T, k-major (rows from ldr on are zero); at the end the hand-over
    __shared__ double sr[2 * PSR];     // per pipeline: r of the tile
    const int tid = threadIdx.x;
    const int pp = __builtin_amdgcn_readfirstlane(tid >> 8);   // pipeline (wavefront-uniform)
    const int lt = tid & 255, lane = tid % WAVE, v = lt / WAVE, c = lane % 16, g = lane / 16;
    for (int idx = tid; idx < 256 * 32; idx += 512)
        stt[(idx >> 5) * FMS + (idx & 31)] = idx < ldr * 32 ? T[idx] : 0.0;
    // r starts at zero: the first phase A multiplies it by a zero slice
    for (int idx = tid; idx < 2 * PSR; idx += 512) sr[idx] = 0.0;

    // wavefronts beyond ldr / 64 stream a copy of the first column block and
    // multiply it by the zero rows of T: every wavefront runs the same
    // branch-free code, so the compiler can count the loads in flight exactly
    const bool hasL = 64 * v < ldr;
    const LT* lbase = Lr + (hasL ? 64 * v : 0) + 2 * c;
    double* slp = sl + pp * PSL;          // the pipeline's four slices / partials
    double* slv = slp + v * PT * FLS;     // this wavefront's
    double* srp = sr + pp * PSR;
    // phase B: thread -> column ej, rows 2 eq, 2 eq + 1 of the tile
    const int ej = lt >> 3, eq = lt & 7;
    const bool ecol = ej < w;
    const int ejc = ecol ? ej : 0;
    const bool eact = ecol && active[ej] != 0;
    const double ea = eact ? alpha[ej] : 0.0, eb = eact ? beta[ej] : 0.0;
    double* const mysink = sink + ((int64_t)blockIdx.x * 512 + tid) * FSINK;
    double srho = 0.0, sa = 0.0, sb = 0.0;
    d4 acc2[4][2];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc2[t][0] = acc2[t][1] = d4{0.0, 0.0, 0.0, 0.0};

    // this pipeline's tiles: tbeg + pp + 2 j, j < nj
    const int ntile = (n + PT - 1) / PT;
    const int tbeg = blockIdx.x * tpw, tend = min(ntile, tbeg + tpw);
    const int nj = (tend - tbeg - pp + 1) / 2;
    auto tile_of = [&](int j) { return tbeg + pp + 2 * max(0, min(j, nj - 1)); };

    // A tile's slice; rows beyond n read row n - 1 and tiles beyond the
    // pipeline's last read its last tile (an L2 hit); those rows are masked
    // in phase B.  No select on loaded values: nothing waits for them early.
    auto loadL = [&](P2 (&a)[4][2], int j) {
        const int tl = tile_of(j);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int row = min(tl * PT + 4 * s + g, n - 1);
            const LT* lp = lbase + (int64_t)row * ldr;
#pragma unroll
            for (int h = 0; h < 2; ++h) a[s][h] = *reinterpret_cast<const P2*>(lp + 32 * h);
        }
    };
    // A tile's x, r, p, delta at rows (2 eq, 2 eq + 1): one 16-byte load per
    // vector, clamped to the last pair (n is even: a pair is inside or beyond n)
    auto loadV = [&](double2 (&vv)[4], int j) {
        const int r0 = min(tile_of(j) * PT + 2 * eq, n - 2);
        const int64_t o = (int64_t)ejc * n + r0;
        vv[0] = *reinterpret_cast<const double2*>(X + o);
        vv[1] = *reinterpret_cast<const double2*>(R + o);
        vv[2] = *reinterpret_cast<const double2*>(P + o);
        vv[3] = *reinterpret_cast<const double2*>(delta + r0);
    };
    // S += L_slice^T r (rows 4 s + g): block u of S takes k = 64 v + 32 (u / 2)
    // + 2 c + u % 2 in its row c, so that item i of its 16 x 16 result is
    // S row ku(u, i) = 64 v + 32 (u / 2) + 8 i + 2 g + u % 2
    auto lpart = [](const P2 (&a)[4][2], int s, int u) {
        return (double)((u & 1) ? a[s][u >> 1].y : a[s][u >> 1].x);
    };
    auto stage4 = [&](const P2 (&a)[4][2]) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const double b0 = srp[(4 * s + g) * FMS + c], b1 = srp[(4 * s + g) * FMS + 16 + c];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                acc2[u][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(lpart(a, s, u), b0, acc2[u][0], 0, 0, 0);
                acc2[u][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(lpart(a, s, u), b1, acc2[u][1], 0, 0, 0);
            }
        }
    };
    auto srow = [&](int u, int i) { return 64 * v + 32 * (u >> 1) + 8 * i + 2 * g + (u & 1); };

    double2 vv[4];
    // one tile: cur holds its slice, old the previous tile's (zero before the first)
    auto tile_step = [&](P2 (&cur)[4][2], P2 (&old)[4][2], int j) {
        // ---- phase A: the slice to LDS; then the partial product L_slice
        // T_slice (row c, k = 4 ks + g) interleaved with the previous tile's
        // S += L^T r (slice in registers), so that the LDS reads of the one
        // hide behind the MFMAs of the other; then the next tile's slice into
        // the registers just freed
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                slv[(4 * s + g) * FLS + 32 * h + 2 * c] = (double)cur[s][h].x;
                slv[(4 * s + g) * FLS + 32 * h + 2 * c + 1] = (double)cur[s][h].y;
            }
        double rb0[4], rb1[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            rb0[s] = srp[(4 * s + g) * FMS + c];
            rb1[s] = srp[(4 * s + g) * FMS + 16 + c];
        }
        d4 acc1[2];
        acc1[0] = acc1[1] = d4{0.0, 0.0, 0.0, 0.0};
        const double* tb = stt + (64 * v + g) * FMS + c;
        // operands of step ks are read one step ahead; the scheduling
        // barriers keep each step's reads ahead of the previous step's MFMAs
        double a0 = slv[c * FLS + g], b0 = tb[0], b1 = tb[16];
#pragma unroll
        for (int ks = 0; ks < 16; ++ks) {
            const double a0c = a0, b0c = b0, b1c = b1;
            if (ks < 15) {
                a0 = slv[c * FLS + 4 * (ks + 1) + g];
                b0 = tb[4 * (ks + 1) * FMS];
                b1 = tb[4 * (ks + 1) * FMS + 16];
            }
            const int s4 = ks >> 2, t4 = ks & 3;
            acc1[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0c, b0c, acc1[0], 0, 0, 0);
            acc1[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0c, b1c, acc1[1], 0, 0, 0);
            acc2[t4][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(lpart(old, s4, t4), rb0[s4], acc2[t4][0], 0, 0, 0);
            acc2[t4][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(lpart(old, s4, t4), rb1[s4], acc2[t4][1], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
        }
        loadL(old, j + 1);
        // the partial product replaces the slice (same wavefront, after its
        // reads); item i of a 16 x 16 result holds row 4 i + g, column c
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
            for (int i = 0; i < 4; ++i) slv[(4 * i + g) * FMS + 16 * jb + c] = acc1[jb][i];
        __syncthreads();
        // ---- phase B: rows 2 eq + i; a pair beyond n computes on zeros, is
        // masked out of the sums and of r in LDS, and its stores go to the sink
        const int er = tile_of(j) * PT + 2 * eq;
        const bool ok = ecol && er < n;
        const double xs[2] = {vv[0].x, vv[0].y}, rs[2] = {vv[1].x, vv[1].y};
        const double ps[2] = {vv[2].x, vv[2].y}, ds[2] = {vv[3].x, vv[3].y};
        double ms[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int row = 2 * eq + i;
            ms[i] = ((slp[row * FMS + ej] + slp[PT * FLS + row * FMS + ej]) + slp[2 * PT * FLS + row * FMS + ej]) +
                    slp[3 * PT * FLS + row * FMS + ej];
        }
        // the mask is a factor, not a select: a select on a loaded value lets
        // the compiler move the load under a branch and wait for it there
        // (the clamped loads read finite rows, so the product is an exact zero)
        const double okf = ok ? 1.0 : 0.0;
        double xo[2], ro[2], po[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const double xv = xs[i] * okf, rv = rs[i] * okf, pv = ps[i] * okf, dv = ds[i] * okf;
            const double p = fma(eb, pv, rv);
            const double ap = fma(dv, p, 2.0 * ms[i]);
            const double rn = fma(-ea, ap, rv);
            const double rm = ok ? rn : 0.0;
            xo[i] = fma(ea, p, xv);
            ro[i] = rn;
            po[i] = p;
            srho = fma(rm, rm, srho);
            sa = fma(dv * rm, rm, sa);
            sb = fma(dv * rm, p, sb);
            srp[(2 * eq + i) * FMS + ej] = eact ? rm : 0.0;
        }
        {
            const bool real = eact && er < n;
            const int64_t o = (int64_t)ej * n + er;
            *reinterpret_cast<double2*>(real ? X + o : mysink) = double2{xo[0], xo[1]};
            *reinterpret_cast<double2*>(real ? R + o : mysink + 2) = double2{ro[0], ro[1]};
            *reinterpret_cast<double2*>(real ? P + o : mysink + 4) = double2{po[0], po[1]};
        }
        loadV(vv, j + 1);
        __syncthreads();
    };

    P2 la[4][2], lb[4][2];
#pragma unroll
    for (int s = 0; s < 4; ++s) lb[s][0] = lb[s][1] = P2{0, 0};
    loadL(la, 0);
    loadV(vv, 0);
    __syncthreads();
    // both pipelines pass the same number of barriers: the second one waits
    // one phase first, the shorter one pads at the end
    const int nbar = max(2 * ((tend - tbeg + 1) / 2), 1 + 2 * ((tend - tbeg) / 2));
    if (pp == 1) __syncthreads();
    int j = 0;
    for (; j + 1 < nj; j += 2) {
        tile_step(la, lb, j);
        tile_step(lb, la, j + 1);
    }
    if (j < nj) tile_step(la, lb, j);
    // the last tile's S term (its slice is in la when nj is odd, in lb when
    // nj is even; with no tile at all lb and r are zero)
    if (nj & 1) stage4(la);
    else stage4(lb);
    for (int b = pp + 2 * nj; b < nbar; ++b) __syncthreads();

    // hand-over: T is no longer read (every stage 2 lies before the barriers above)
    if (pp == 1) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int jb = 0; jb < 2; ++jb)
#pragma unroll
                for (int i = 0; i < 4; ++i) stt[srow(t, i) * 32 + 16 * jb + c] = acc2[t][jb][i];
        double* cs1 = sl + PSL + 3 * lt;
        cs1[0] = srho;
        cs1[1] = sa;
        cs1[2] = sb;
    }
    __syncthreads();
    if (pp == 1) return;
    double* out = rec + (int64_t)blockIdx.x * stride;
    if (hasL) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int jb = 0; jb < 2; ++jb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int idx = srow(t, i) * 32 + 16 * jb + c;
                    out[idx] = acc2[t][jb][i] + stt[idx];
                }
    }
    // column sums: the two pipelines, then the column's 8 threads
    // (consecutive lanes), each thread's own sum taken over its rows in tile order
    const double* cs1 = sl + PSL + 3 * lt;
    srho += cs1[0];
    sa += cs1[1];
    sb += cs1[2];
#pragma unroll
    for (int off = 1; off < 8; off <<= 1) {
        srho += __shfl_xor(srho, off, WAVE);
        sa += __shfl_xor(sa, off, WAVE);
        sb += __shfl_xor(sb, off, WAVE);
    }
    if (eq == 0) {
        double* cs = out + ldr * 32 + 4 * ej;
        cs[0] = srho;
        cs[1] = sa;
        cs[2] = sb;
        cs[3] = 0.0;
    }
}

// The same step for A = diag(delta): block (chunk, column j) over a row range
__global__ __launch_bounds__(256) void fcg_pass_K_kernel(int n, int nch, const double* __restrict__ delta,
                                                         double* __restrict__ X, double* __restrict__ R,
                                                         double* __restrict__ P, const double* __restrict__ alpha,
                                                         const double* __restrict__ beta,
                                                         const int* __restrict__ active, const int* __restrict__ any,
                                                         double* __restrict__ rec) {
    __shared__ double red[3][4];
    if (*any == 0) return;
    const int j = blockIdx.y, ch = blockIdx.x, tid = threadIdx.x;
    double* cs = rec + (int64_t)ch * FREC + 4 * j;
    if (!active[j]) {
        if (tid < 4) cs[tid] = 0.0;
        return;
    }
    const int rows = (n + nch - 1) / nch;
    const int r0 = ch * rows, r1 = min(n, r0 + rows);
    const int64_t off = (int64_t)j * n;
    const double a = alpha[j], b = beta[j];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int i = r0 + tid; i < r1; i += 256) {
        const double d = delta[i];
        const double p = fma(b, P[off + i], R[off + i]);
        const double rn = fma(-a, d * p, R[off + i]);
        X[off + i] = fma(a, p, X[off + i]);
        R[off + i] = rn;
        P[off + i] = p;
        s0 = fma(rn, rn, s0);
        s1 = fma(d * rn, rn, s1);
        s2 = fma(d * rn, p, s2);
    }
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    const int lane = tid % WAVE, wid = tid / WAVE;
    if (lane == 0) {
        red[0][wid] = s0;
        red[1][wid] = s1;
        red[2][wid] = s2;
    }
    __syncthreads();
    if (tid < 3) cs[tid] = ((red[tid][0] + red[tid][1]) + red[tid][2]) + red[tid][3];
    if (tid == 3) cs[3] = 0.0;
}

// Start of a fused CG: x = 0, r = p = b; column sums (|b|^2, b^T diag(delta) b)
__global__ __launch_bounds__(256) void fcg_init_kernel(int n, int nch, const double* __restrict__ delta,
                                                       const double* __restrict__ B, int64_t ldb,
                                                       double* __restrict__ X, double* __restrict__ R,
                                                       double* __restrict__ P, double* __restrict__ rec) {
    __shared__ double red[2][4];
    const int j = blockIdx.y, ch = blockIdx.x, tid = threadIdx.x;
    const int rows = (n + nch - 1) / nch;
    const int r0 = ch * rows, r1 = min(n, r0 + rows);
    const int64_t off = (int64_t)j * n;
    double s0 = 0.0, s1 = 0.0;
    for (int i = r0 + tid; i < r1; i += 256) {
        const double bv = B[(int64_t)j * ldb + i];
        X[off + i] = 0.0;
        R[off + i] = bv;
        P[off + i] = bv;
        s0 = fma(bv, bv, s0);
        s1 = fma(delta[i] * bv, bv, s1);
    }
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    const int lane = tid % WAVE, wid = tid / WAVE;
    if (lane == 0) {
        red[0][wid] = s0;
        red[1][wid] = s1;
    }
    __syncthreads();
    double* cs = rec + (int64_t)ch * FREC + 4 * j;
    if (tid < 2) cs[tid] = ((red[tid][0] + red[tid][1]) + red[tid][2]) + red[tid][3];
    if (tid == 2 || tid == 3) cs[tid] = 0.0;
}

// Fixed-order sum of the workgroup records (nrec records of `stride` doubles:
// S = L^T r in the first nS, then the column sums) into red; then the
// finishing step (fcg_finish_kernel): rho, beta, the relative residual test,
// T = S + beta T, c, alpha = rho / (c + 2 |T|^2) and any_active.  With init,
// the records hold (|b|^2, b^T diag(delta) b) and T = L^T b is already in place.
constexpr int FIN_PH = 32;   // record phases per element in fcg_reduce_kernel (<= 8 records each)

__global__ __launch_bounds__(32 * FIN_PH) void fcg_reduce_kernel(int nrec, int stride, const double* __restrict__ rec,
                                                                double* __restrict__ red, const int* __restrict__ any,
                                                                int init) {
    __shared__ double ph[FIN_PH][32];
    if (!init && *any == 0) return;
    const int tid = threadIdx.x, x = tid % 32, q = tid / 32;
    const int e = blockIdx.x * 32 + x;
    // records q, q + 32, ... (at most 8: nrec <= 256), all loads issued together
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int k = q + FIN_PH * u;
        v[u] = (e < stride && k < nrec) ? rec[(int64_t)k * stride + e] : 0.0;
    }
    ph[q][x] = ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
    __syncthreads();
    if (q == 0 && e < stride) {
        double t = ph[0][x];
#pragma unroll
        for (int p = 1; p < FIN_PH; ++p) t += ph[p][x];
        red[e] = t;
    }
}

// The finishing step from the reduced sums (one workgroup; the launch boundary
// after fcg_reduce_kernel makes its sums visible -- a last-arriving-block
// finish cost each of the 260 reducing workgroups a device-scope release)
__global__ __launch_bounds__(32 * FIN_PH) void fcg_finish_kernel(int w, int ldr, int nS,
                                                                const double* __restrict__ red, CgState s,
                                                                double tol, int init) {
    __shared__ double ph[FIN_PH][32];
    __shared__ double cb[32];
    __shared__ int cact[32];
    if (!init && *s.any_active == 0) return;
    const int tid = threadIdx.x, x = tid % 32, q = tid / 32;
    if (tid < 32) {
        const int j = tid;
        int act = 0, applied = 0;
        double bt = 0.0;
        if (j < w) {
            const double rn = red[nS + 4 * j], av = red[nS + 4 * j + 1], bv = red[nS + 4 * j + 2];
            if (init) {
                s.rr[j] = rn;
                s.bb[j] = rn;
                s.c[j] = av;
                act = rn > tol * tol * rn ? 1 : 0;
            } else if (s.active[j]) {
                applied = 1;
                bt = rn / s.rr[j];
                act = rn > tol * tol * s.bb[j] ? 1 : 0;
                s.c[j] = fma(bt * bt, s.c[j], fma(2.0 * bt, bv, av));
                s.rr[j] = rn;
            }
            s.beta[j] = bt;
        }
        cb[j] = bt;
        cact[j] = act;
        const unsigned long long na = __popcll(__ballot(applied));
        if (j == 0 && na) atomicAdd(s.napplies, na);
    }
    __syncthreads();
    // T = S + beta T and |T|^2 for the active columns: rows q, q + 32, ... (<= 8)
    double t2 = 0.0;
    if (ldr > 0 && x < w && cact[x]) {
        double tv[8], sv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = q + FIN_PH * u;
            tv[u] = k < ldr ? s.T[(int64_t)k * 32 + x] : 0.0;
            sv[u] = (!init && k < ldr) ? red[k * 32 + x] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = q + FIN_PH * u;
            if (k < ldr) {
                double tn = tv[u];
                if (!init) {
                    tn = fma(cb[x], tn, sv[u]);
                    s.T[(int64_t)k * 32 + x] = tn;
                }
                t2 = fma(tn, tn, t2);
            }
        }
    }
    ph[q][x] = t2;
    __syncthreads();
    if (tid < 32) {
        const int j = tid;
        double tt = ph[0][j];
#pragma unroll
        for (int p = 1; p < FIN_PH; ++p) tt += ph[p][j];
        int act = cact[j];
        double al = 0.0;
        if (act) {
            const double den = fma(2.0, tt, s.c[j]);
            if (den > 0.0)
                al = s.rr[j] / den;
            else
                act = 0;   // p^T A p <= 0: the column stops (singular operator)
        }
        if (j < w) {
            s.alpha[j] = al;
            s.active[j] = act;
        }
        const int anyv = __any(act) ? 1 : 0;
        if (j == 0) {
            *s.any_active = anyv;
            if (s.note)
                __hip_atomic_store(s.note, 2ull * s.seq + (unsigned long long)anyv, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

// the FP32 copy of the rows of L (each value rounded to nearest even once),
// padding columns included
__global__ __launch_bounds__(256) void rows_f32_kernel(int64_t count, const double* __restrict__ Lr,
                                                       float* __restrict__ Lr32) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256)
        Lr32[i] = (float)Lr[i];
}

}  // namespace

int64_t lowrank_row_ld(int64_t r) { return ((r + 63) / 64) * 64; }

hipError_t lowrank_rows_f32(hipStream_t st, int n, int r, const double* Lr, float* Lr32) {
    if (n < 1 || r < 1 || r > 256 || !Lr || !Lr32) return hipErrorInvalidValue;
    const int64_t count = (int64_t)n * lowrank_row_ld(r);
    hipLaunchKernelGGL(rows_f32_kernel, dim3((unsigned)std::min<int64_t>(4096, (count + 255) / 256)), dim3(256), 0,
                       st, count, Lr, Lr32);
    return hipGetLastError();
}

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


namespace {
// row chunks of the diagonal step and of the initialisation: a function of n
// alone, so that a column's sums are taken in the same order whatever the
// number of columns solved with it
int fcg_chunks(int n, int w) {
    (void)w;
    return std::max(1, std::min(32, n / 1024));
}
int fcg_groups(int n) {
    const int ntile = (n + PT - 1) / PT;
    return std::min(256, ntile);
}
// row chunk of the L^T b pass (a multiple of 2 RU, as in lowrank_apply_M_rows)
int fcg_lty_chunk(int n) {
    const int nchunk = std::max(1, std::min(512, n / 512));
    const int chunk = (n + nchunk - 1) / nchunk;
    return ((chunk + 2 * RU - 1) / (2 * RU)) * (2 * RU);
}
int fcg_lty_chunks(int n) { return (n + fcg_lty_chunk(n) - 1) / fcg_lty_chunk(n); }
}  // namespace

size_t fused_cg_work_elems(int n, int r, int w) {
    (void)w;
    const size_t ldr = r > 0 ? (size_t)lowrank_row_ld(r) : 0;
    const size_t stride = ldr * 32 + FREC;
    size_t need = (size_t)fcg_chunks(n, 32) * FREC + FREC;                       // init / diagonal steps
    if (r > 0) {
        // M steps: records, their reduction, the pass's store sink
        need = std::max(need, (size_t)fcg_groups(n) * stride + stride + (size_t)fcg_groups(n) * 512 * FSINK);
        need = std::max(need, (size_t)256 * 32 + (size_t)fcg_lty_chunks(n) * 8192 + FREC * 256);   // L^T b
    }
    return need;
}

hipError_t fused_cg_init(hipStream_t st, int n, int r, int w, const double* delta, const double* Lr, const CgState& s,
                         const double* B, int64_t ldb, double tol, double* work, size_t work_elems) {
    if (n < 64 || (n & 1) || w < 1 || w > 32 || (Lr && (r < 1 || r > 256)) ||
        work_elems < fused_cg_work_elems(n, Lr ? r : 0, w))
        return hipErrorInvalidValue;
    const int nch = fcg_chunks(n, w);
    double* rec = work;
    double* red = work + (size_t)nch * FREC;
    hipLaunchKernelGGL(fcg_init_kernel, dim3(nch, w), dim3(256), 0, st, n, nch, delta, B, ldb, s.X, s.R, s.P, rec);
    int ldr = 0;
    if (Lr) {
        // T = L^T b (the direction of the first step is b)
        ldr = (int)lowrank_row_ld(r);
        const int nchunk = fcg_lty_chunks(n);
        const int chunk = fcg_lty_chunk(n);
        double* part = red + FREC;
        hipLaunchKernelGGL(lr_lty_kernel, dim3(nchunk), dim3(256), 0, st, n, ldr, w, Lr, B, ldb, chunk, part,
                           nullptr);
        hipLaunchKernelGGL(lr_reduce_kernel, dim3(8192 / 32), dim3(32 * RED_PH), 0, st, ldr, nchunk, part, 1.0, s.T,
                           nullptr);
    }
    hipLaunchKernelGGL(fcg_reduce_kernel, dim3(FREC / 32), dim3(32 * FIN_PH), 0, st, nch, FREC, rec, red,
                       s.any_active, 1);
    hipLaunchKernelGGL(fcg_finish_kernel, dim3(1), dim3(32 * FIN_PH), 0, st, w, ldr, 0, red, s, tol, 1);
    return hipGetLastError();
}

hipError_t fused_cg_step(hipStream_t st, int n, int r, int w, const double* delta, const double* Lr,
                         const CgState& s, double tol, double* work, size_t work_elems, hipEvent_t* ev,
                         int* flag_log, const float* Lr32) {
    if (n < 64 || (n & 1) || w < 1 || w > 32 || (Lr && (r < 1 || r > 256)) ||
        work_elems < fused_cg_work_elems(n, Lr ? r : 0, w) || (reinterpret_cast<uintptr_t>(Lr) & 15) ||
        (reinterpret_cast<uintptr_t>(Lr32) & 7))
        return hipErrorInvalidValue;
    if (Lr) {
        const int ldr = (int)lowrank_row_ld(r);
        const int ntile = (n + PT - 1) / PT;
        const int nwg = fcg_groups(n);
        const int tpw = (ntile + nwg - 1) / nwg;
        const int ngrid = (ntile + tpw - 1) / tpw;
        const int stride = ldr * 32 + FREC;
        double* rec = work;
        double* red = work + (size_t)ngrid * stride;
        double* sink = red + stride;
        if (ev) (void)hipEventRecord(ev[0], st);
        if (Lr32)
            hipLaunchKernelGGL(fcg_pass_M_kernel<float>, dim3(ngrid), dim3(512), 0, st, n, ldr, w, tpw, Lr32, delta,
                               s.X, s.R, s.P, s.T, s.alpha, s.beta, s.active, s.any_active, rec, stride, sink,
                               flag_log);
        else
            hipLaunchKernelGGL(fcg_pass_M_kernel<double>, dim3(ngrid), dim3(512), 0, st, n, ldr, w, tpw, Lr, delta,
                               s.X, s.R, s.P, s.T, s.alpha, s.beta, s.active, s.any_active, rec, stride, sink,
                               flag_log);
        if (ev) (void)hipEventRecord(ev[1], st);
        hipLaunchKernelGGL(fcg_reduce_kernel, dim3((stride + 31) / 32), dim3(32 * FIN_PH), 0, st, ngrid, stride, rec,
                           red, s.any_active, 0);
        hipLaunchKernelGGL(fcg_finish_kernel, dim3(1), dim3(32 * FIN_PH), 0, st, w, ldr, ldr * 32, red, s, tol, 0);
    } else {
        const int nch = fcg_chunks(n, w);
        double* rec = work;
        double* red = work + (size_t)nch * FREC;
        hipLaunchKernelGGL(fcg_pass_K_kernel, dim3(nch, w), dim3(256), 0, st, n, nch, delta, s.X, s.R, s.P, s.alpha,
                           s.beta, s.active, s.any_active, rec);
        hipLaunchKernelGGL(fcg_reduce_kernel, dim3(FREC / 32), dim3(32 * FIN_PH), 0, st, nch, FREC, rec, red,
                           s.any_active, 0);
        hipLaunchKernelGGL(fcg_finish_kernel, dim3(1), dim3(32 * FIN_PH), 0, st, w, 0, 0, red, s, tol, 0);
    }
    return hipGetLastError();
}

}  // namespace lrep
