// Streaming FP64 MFMA block apply Y = A X for a dense operator A (n x n,
// column-major) and a narrow block X (n x q, q <= 32): the CG inner solves of
// Step 6 (block Gauss-Seidel), where every launch reads the whole operator
// once and the product sits at the HBM/FP64-MFMA ridge (2 n^2 q flops over
// 8 n^2 bytes: q/4 flop/byte).
//
// Design for gfx950:
//  * no LDS and no barriers in the main loop.  Each wavefront owns 32 rows
//    and streams its A panel straight from HBM into registers with 16-byte
//    loads (two consecutive rows per lane), software-pipelined PF k-steps
//    ahead in two register halves, so that ~2 * PF KiB per wavefront are in
//    flight;
//  * the block X is first packed k-major (n x 32, zero-padded) so that the
//    MFMA B fragments are also contiguous 16-byte loads; the 2 KiB it takes
//    per k-step of 32 rows is reused by every wavefront through L1/L2;
//  * two row fragments x two column fragments = four v_mfma_f64_16x16x4
//    per k-step.  Fragment (fm, fn), row i, column c maps to row 2i + fm and
//    column 2c + fn of the wavefront tile (the interleave that the 16-byte
//    loads produce);
//  * the k dimension is split over workgroups for occupancy; each wavefront
//    writes its 32 x 32 partial tile in lane order (128 contiguous bytes per
//    lane) and a second kernel sums the splits in a fixed order (bitwise
//    reproducible) while scattering to the column-major result.
#include "device.hpp"
#include "kernels.hpp"

namespace lrep {

namespace {

constexpr int NT = 256;   // 4 wavefronts x 32 rows = 128 rows per workgroup
constexpr int PF = 4;     // k-steps (4 columns each) per prefetch half

__global__ __launch_bounds__(NT) void pack_kmajor_kernel(int n, int q, const double* __restrict__ X, int64_t ldx,
                                                         double* __restrict__ Pt, const int* __restrict__ flag) {
    if (flag && *flag == 0) return;
    const int64_t total = (int64_t)n * 32;
    for (int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * NT) {
        const int k = (int)(idx / 32), c = (int)(idx % 32);
        Pt[idx] = c < q ? X[(int64_t)c * ldx + k] : 0.0;
    }
}

__global__ __launch_bounds__(NT) void apply_stream_kernel(int m, int p, const double* __restrict__ A, int64_t lda,
                                                          const double* __restrict__ Pt, int kchunk,
                                                          double* __restrict__ part, const int* __restrict__ flag) {
    if (flag && *flag == 0) return;
    const int lane = threadIdx.x % WAVE, wid = threadIdx.x / WAVE;
    const int tile = blockIdx.x * (NT / WAVE) + wid;
    const int row0 = tile * 32;
    const int split = blockIdx.z;
    const int k_begin = split * kchunk;
    const int k_end = min(p, k_begin + kchunk);
    const int nsteps = (k_end - k_begin + 3) / 4;
    const int c = lane % 16, kq = lane / 16;
    const int arow = row0 + 2 * c;
    const bool full = (arow + 1 < m);
    d4 acc00 = {0, 0, 0, 0}, acc01 = acc00, acc10 = acc00, acc11 = acc00;
    double2 a0[PF], b0[PF], a1[PF], b1[PF];

    auto load = [&](double2 (&a)[PF], double2 (&b)[PF], int s0) {
#pragma unroll
        for (int j = 0; j < PF; ++j) {
            const int k = k_begin + (s0 + j) * 4 + kq;
            double2 av = {0.0, 0.0}, bv = {0.0, 0.0};
            if (k < k_end) {
                const double* ap = A + (int64_t)k * lda + arow;
                if (full) {
                    av = *reinterpret_cast<const double2*>(ap);
                } else if (arow < m) {
                    av.x = ap[0];
                }
                bv = *reinterpret_cast<const double2*>(Pt + (int64_t)k * 32 + 2 * c);
            }
            a[j] = av;
            b[j] = bv;
        }
    };
    auto compute = [&](const double2 (&a)[PF], const double2 (&b)[PF]) {
#pragma unroll
        for (int j = 0; j < PF; ++j) {
            acc00 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[j].x, b[j].x, acc00, 0, 0, 0);
            acc01 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[j].x, b[j].y, acc01, 0, 0, 0);
            acc10 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[j].y, b[j].x, acc10, 0, 0, 0);
            acc11 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[j].y, b[j].y, acc11, 0, 0, 0);
        }
    };

    if (row0 < m && nsteps > 0) {
        load(a0, b0, 0);
        for (int s = 0; s < nsteps; s += 2 * PF) {
            if (s + PF < nsteps) load(a1, b1, s + PF);
            compute(a0, b0);
            if (s + 2 * PF < nsteps) load(a0, b0, s + 2 * PF);
            if (s + PF < nsteps) compute(a1, b1);
        }
    }
    if (row0 < m) {
        const int ntiles = (m + 31) / 32;
        double* out = part + (((int64_t)split * ntiles + tile) * WAVE + lane) * 16;
        const d4 accs[4] = {acc00, acc01, acc10, acc11};
#pragma unroll
        for (int f = 0; f < 4; ++f)
            *reinterpret_cast<d4*>(out + 4 * f) = accs[f];
    }
}

// C = alpha * sum_split part + beta * C, un-interleaving the lane-order tiles.
__global__ __launch_bounds__(NT) void apply_reduce_kernel(int m, int q, int nsplit, const double* __restrict__ part,
                                                          double* __restrict__ C, int64_t ldc, double alpha,
                                                          double beta, const int* __restrict__ flag) {
    if (flag && *flag == 0) return;
    const int ntiles = (m + 31) / 32;
    const int64_t total = (int64_t)ntiles * WAVE * 16;
    for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
        const int v = (int)(e % 16);
        const int lane = (int)((e / 16) % WAVE);
        const int tile = (int)(e / (16 * WAVE));
        const int f = v / 4, r = v % 4;
        const int fm = f / 2, fn = f % 2;
        const int row = tile * 32 + 2 * (4 * r + lane / 16) + fm;
        const int col = 2 * (lane % 16) + fn;
        if (row >= m || col >= q) continue;
        double s = 0.0;
        for (int k = 0; k < nsplit; ++k) s += part[(int64_t)k * total + e];
        double o = alpha * s;
        if (beta != 0.0) o += beta * C[(int64_t)col * ldc + row];
        C[(int64_t)col * ldc + row] = o;
    }
}

}  // namespace

hipError_t dense_apply_narrow(hipStream_t st, int m, int q, int p, const double* A, int64_t lda, const double* X,
                              int64_t ldx, double* C, int64_t ldc, double alpha, double beta, double* work,
                              size_t work_elems, const int* active_flag, hipEvent_t* ev) {
    if (q < 1 || q > 32 || m < 1 || p < 1) return hipErrorInvalidValue;
    const int ntiles = (m + 31) / 32;
    const int wgs = (ntiles + 3) / 4;
    const int64_t tile_elems = (int64_t)ntiles * WAVE * 16;
    if (p > m || (size_t)m * 32 + (size_t)tile_elems > work_elems) return hipErrorInvalidValue;
    int ksplit = 1;
    while (wgs * ksplit < 1024 && p / (ksplit * 2) >= 256 && ksplit < 16 &&
           (size_t)m * 32 + (size_t)(2 * ksplit) * tile_elems <= work_elems)
        ksplit *= 2;
    int kchunk = (p + ksplit - 1) / ksplit;
    kchunk = ((kchunk + 3) / 4) * 4;
    ksplit = (p + kchunk - 1) / kchunk;
    double* Pt = work;
    double* part = work + (size_t)m * 32;
    const int pk_blocks = (int)std::min<int64_t>(2048, ((int64_t)p * 32 + NT - 1) / NT);
    hipLaunchKernelGGL(pack_kmajor_kernel, dim3(pk_blocks), dim3(NT), 0, st, p, q, X, ldx, Pt, active_flag);
    if (ev) (void)hipEventRecord(ev[0], st);
    hipLaunchKernelGGL(apply_stream_kernel, dim3(wgs, 1, ksplit), dim3(NT), 0, st, m, p, A, lda, Pt, kchunk, part,
                       active_flag);
    if (ev) (void)hipEventRecord(ev[1], st);
    const int rb = (int)std::min<int64_t>(4096, (tile_elems + NT - 1) / NT);
    hipLaunchKernelGGL(apply_reduce_kernel, dim3(rb), dim3(NT), 0, st, m, q, ksplit, part, C, ldc, alpha, beta,
                       active_flag);
    return hipGetLastError();
}

}  // namespace lrep
