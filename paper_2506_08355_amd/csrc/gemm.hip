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

struct SegView {
    const double* p[kMaxSeg];
    int64_t ld[kMaxSeg];
    int start[kMaxSeg + 1];  // prefix of column counts
    int nseg;
};

__device__ __forceinline__ const double* seg_col(const SegView& s, int c, int64_t& ld) {
    int i = 0;
#pragma unroll
    for (int t = 1; t < kMaxSeg; ++t)
        if (t < s.nseg && c >= s.start[t]) i = t;
    ld = s.ld[i];
    return s.p[i] + (int64_t)(c - s.start[i]) * s.ld[i];
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
    // narrow tiles and one k chunk: these products (p = subspace size) are latency bound,
    // so the batch and the row tiles provide the parallelism
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
