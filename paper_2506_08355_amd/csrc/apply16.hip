// Mixed-precision CG apply for dense operators: the operator is held in a
// 16-bit copy (BF16 or FP16, FP64 values rounded once to nearest even) and the CG block in the
// same format, multiplied on the gfx950 v_mfma_f32_16x16x32_{bf16,f16} with
// FP32 accumulation; the result, the CG vectors and every other step of the
// solver stay FP64.  The CG of Step 6 only asks for a relative residual of
// cg_tol (1e-2 by default), well above the ~1e-3 relative error of a 16-bit
// product, and the operator images used by the Rayleigh-Ritz step and the
// residuals of Step 4 are always FP64 applies.
//
// Layout.  K and M are symmetric, so row i of the operator is column i of the
// stored matrix: the 16-bit copy keeps the column-major layout (ld n) and a
// wavefront reading output rows row0 .. row0 + 63 reads 64 stored columns,
// each a contiguous run along k.  The MFMA 16x16x32 operand layout
// (lane l: A[l % 16][8 (l / 16) + i], B[8 (l / 16) + i][l % 16], i = 0..7;
// D item i: D[4 (l / 16) + i][l % 16]) then takes one 16-byte load per lane
// and fragment.  The block is packed column-major (n x 32, 16-bit), so its
// fragments are 16-byte loads along k too.
//
// FP16 has a narrow exponent range: each CG column is scaled by a power of
// two 2^e_j ~ sqrt(n / |r_j|^2) before the conversion (elements of size
// about 1) and the product is scaled back exactly.  BF16 keeps FP32's range
// and needs no scaling.
//
// BF16x3 (precision 3): the operator and the block are each split into three
// BF16 parts, v = hi + mid + lo, every part the rounding of what the earlier
// ones leave (so hi + mid + lo carries 24 significant bits, FP32's), and the
// product sums the six part products of total order <= 2 (hi hi, hi mid,
// mid hi, hi lo, lo hi, mid mid) in FP32: an FP32-accurate product from BF16
// MFMAs, reading 6 n^2 bytes of operator (FP64: 8 n^2).
#include "device.hpp"
#include "kernels.hpp"

namespace lrep {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;

constexpr int WR = 64;   // output rows per wavefront
constexpr int KS = 32;   // k per MFMA step
constexpr int PF = 2;    // k-steps per prefetch half

// one rounding, to nearest even, from FP64 straight to the 16-bit format
// (no intermediate FP32 rounding)
template <int P>
__device__ __forceinline__ u16 to16(double v) {
    if constexpr (P == 1 || P == 3) return __builtin_bit_cast(u16, (__bf16)v);
    else return __builtin_bit_cast(u16, (_Float16)v);
}
// the three BF16 parts of v (each the rounding of the remainder, FP64 arithmetic)
__device__ __forceinline__ void split3(double v, u16& hi, u16& mid, u16& lo) {
    const __bf16 h = (__bf16)v;
    const double r1 = v - (double)h;
    const __bf16 m = (__bf16)r1;
    const double r2 = r1 - (double)m;
    hi = __builtin_bit_cast(u16, h);
    mid = __builtin_bit_cast(u16, m);
    lo = __builtin_bit_cast(u16, (__bf16)r2);
}

// out (16-bit, n x n, ld n) = 0.5 (A + A^T) rounded; 32 x 32 tiles through LDS.
// P = 3: three such matrices, hi, mid, lo parts, at out, out + n^2, out + 2 n^2.
template <int P>
__global__ __launch_bounds__(256) void convert16_kernel(int n, const double* __restrict__ A, int64_t lda,
                                                        u16* __restrict__ out) {
    __shared__ double t[32][33];
    const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;   // 32 x 8
    // t[a][b] = A(j0 + a, i0 + b), read along columns (coalesced over tx)
    for (int r = ty; r < 32; r += 8) {
        const int row = j0 + tx, col = i0 + r;
        t[tx][r] = (row < n && col < n) ? A[(int64_t)col * lda + row] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int i = i0 + tx, j = j0 + r;   // element (i, j)
        if (i < n && j < n) {
            const double a = A[(int64_t)j * lda + i];
            const double b = t[r][tx];          // A(j, i)
            if constexpr (P == 3) {
                const size_t nn = (size_t)n * n;
                u16 h, m, l;
                split3(0.5 * (a + b), h, m, l);
                out[(int64_t)j * n + i] = h;
                out[nn + (int64_t)j * n + i] = m;
                out[2 * nn + (int64_t)j * n + i] = l;
            } else {
                out[(int64_t)j * n + i] = to16<P>(0.5 * (a + b));
            }
        }
    }
}

// CG direction (p = r + beta p on the active columns unless `first`) and the
// 16-bit block Xh (n x 32, column-major, zero-padded), column j scaled by
// 2^e_j (FP16) where e_j = round(log2(sqrt(n / rr_j))); P = 3: the hi, mid,
// lo parts at Xh, Xh + 32 n, Xh + 64 n.
template <int P>
__global__ __launch_bounds__(256) void cg_dir_pack16_kernel(int n, int w, double* __restrict__ Pm,
                                                            const double* __restrict__ R,
                                                            const double* __restrict__ beta,
                                                            const int* __restrict__ active,
                                                            const double* __restrict__ rr, int first,
                                                            u16* __restrict__ Xh, const int* __restrict__ flag,
                                                            int* __restrict__ flag_log) {
    const int on = *flag;
    if (flag_log && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *flag_log = on;
    if (on == 0) return;
    const int c = blockIdx.y;
    double sc = 1.0;
    if (P == 2 && c < w && rr[c] > 0.0) sc = exp2(rint(0.5 * log2((double)n / rr[c])));
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        double v = 0.0;
        if (c < w) {
            v = Pm[(int64_t)c * n + i];
            if (!first && active[c]) {
                v = R[(int64_t)c * n + i] + beta[c] * v;
                Pm[(int64_t)c * n + i] = v;
            }
        }
        if constexpr (P == 3) {
            u16 h, m, l;
            split3(v, h, m, l);
            Xh[(int64_t)c * n + i] = h;
            Xh[(int64_t)(32 + c) * n + i] = m;
            Xh[(int64_t)(64 + c) * n + i] = l;
        } else {
            Xh[(int64_t)c * n + i] = to16<P>(v * sc);
        }
    }
}

template <int P>
__device__ __forceinline__ f4 mfma16(uint4 a, uint4 b, f4 c) {
    if constexpr (P == 1 || P == 3)
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                      c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c,
                                                     0, 0, 0);
}

// partial[split][tile][lane][32] (FP32, lane order) of A(rows of the tile) X
// over k in this split's chunk; A 16-bit n x n, X 16-bit n x 32, both
// column-major with ld n (n a multiple of 8, 16-byte aligned).
template <int P>
__global__ __launch_bounds__(64) void apply16_stream_kernel(int n, const u16* __restrict__ A,
                                                            const u16* __restrict__ X, int kchunk,
                                                            float* __restrict__ part,
                                                            const int* __restrict__ flag) {
    if (flag && *flag == 0) return;
    const int lane = threadIdx.x, tile = blockIdx.x, split = blockIdx.y;
    const int row0 = tile * WR;
    const int k_begin = split * kchunk;
    const int k_end = min(n, k_begin + kchunk);
    const int nfull = max(0, (k_end - k_begin) / KS);
    const int r = lane % 16, g = lane / 16;
    f4 acc[4][2];
#pragma unroll
    for (int f = 0; f < 4; ++f) acc[f][0] = acc[f][1] = f4{0.f, 0.f, 0.f, 0.f};
    // rows beyond n read row n - 1 (valid memory) and are dropped by the reduction
    const u16* ap[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) ap[f] = A + (int64_t)min(row0 + 16 * f + r, n - 1) * n + k_begin + 8 * g;
    const u16* bp0 = X + (int64_t)r * n + k_begin + 8 * g;
    const u16* bp1 = X + (int64_t)(16 + r) * n + k_begin + 8 * g;
    if (nfull > 0) {
        uint4 a0[PF][4], b0[PF][2], a1[PF][4], b1[PF][2];
        auto load = [&](uint4 (&a)[PF][4], uint4 (&b)[PF][2], int s0) {
#pragma unroll
            for (int j = 0; j < PF; ++j) {
                const int64_t o = (int64_t)min(s0 + j, nfull - 1) * KS;
#pragma unroll
                for (int f = 0; f < 4; ++f) a[j][f] = *reinterpret_cast<const uint4*>(ap[f] + o);
                b[j][0] = *reinterpret_cast<const uint4*>(bp0 + o);
                b[j][1] = *reinterpret_cast<const uint4*>(bp1 + o);
            }
        };
        auto compute = [&](const uint4 (&a)[PF][4], const uint4 (&b)[PF][2], int s0) {
#pragma unroll
            for (int j = 0; j < PF; ++j) {
                const bool live = s0 + j < nfull;
                const uint4 z = {0u, 0u, 0u, 0u};
                const uint4 bb0 = live ? b[j][0] : z, bb1 = live ? b[j][1] : z;
#pragma unroll
                for (int f = 0; f < 4; ++f) {
                    acc[f][0] = mfma16<P>(a[j][f], bb0, acc[f][0]);
                    acc[f][1] = mfma16<P>(a[j][f], bb1, acc[f][1]);
                }
            }
        };
        load(a0, b0, 0);
        for (int s = 0; s < nfull; s += 2 * PF) {
            load(a1, b1, s + PF);
            compute(a0, b0, s);
            load(a0, b0, s + 2 * PF);
            compute(a1, b1, s + PF);
        }
    }
    if (k_begin + KS * nfull < k_end) {
        // last partial k-step: per-element guards (n is a multiple of 8, so a
        // lane's 8 values are all in range or all out)
        const int64_t o = (int64_t)nfull * KS;
        const bool kin = k_begin + o + 8 * g < k_end;
        uint4 bb0 = {0u, 0u, 0u, 0u}, bb1 = bb0, aa[4] = {bb0, bb0, bb0, bb0};
        if (kin) {
            bb0 = *reinterpret_cast<const uint4*>(bp0 + o);
            bb1 = *reinterpret_cast<const uint4*>(bp1 + o);
#pragma unroll
            for (int f = 0; f < 4; ++f) aa[f] = *reinterpret_cast<const uint4*>(ap[f] + o);
        }
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            acc[f][0] = mfma16<P>(aa[f], bb0, acc[f][0]);
            acc[f][1] = mfma16<P>(aa[f], bb1, acc[f][1]);
        }
    }
    const int ntiles = (n + WR - 1) / WR;
    float* out = part + (((int64_t)split * ntiles + tile) * WAVE + lane) * 32;
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int u = 0; u < 2; ++u) *reinterpret_cast<f4*>(out + (f * 2 + u) * 4) = acc[f][u];
}

// The BF16x3 form of apply16_stream_kernel: the operator's hi, mid, lo parts
// at A, A + n^2, A + 2 n^2 and the block's at X, X + 32 n, X + 64 n; per
// k-step the six part products of order <= 2 into the one FP32 accumulator
// (smallest first).  One k-step per prefetch half (the parts triple the
// registers a step holds).
__global__ __launch_bounds__(64) void apply16x3_stream_kernel(int n, const u16* __restrict__ A,
                                                              const u16* __restrict__ X, int kchunk,
                                                              float* __restrict__ part,
                                                              const int* __restrict__ flag) {
    if (flag && *flag == 0) return;
    const int lane = threadIdx.x, tile = blockIdx.x, split = blockIdx.y;
    const int row0 = tile * WR;
    const int k_begin = split * kchunk;
    const int k_end = min(n, k_begin + kchunk);
    const int nfull = max(0, (k_end - k_begin) / KS);
    const int r = lane % 16, g = lane / 16;
    const int64_t nn = (int64_t)n * n, xn = (int64_t)32 * n;
    f4 acc[4][2];
#pragma unroll
    for (int f = 0; f < 4; ++f) acc[f][0] = acc[f][1] = f4{0.f, 0.f, 0.f, 0.f};
    // rows beyond n read row n - 1 (valid memory) and are dropped by the reduction
    const u16* ap[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) ap[f] = A + (int64_t)min(row0 + 16 * f + r, n - 1) * n + k_begin + 8 * g;
    const u16* bp0 = X + (int64_t)r * n + k_begin + 8 * g;
    const u16* bp1 = X + (int64_t)(16 + r) * n + k_begin + 8 * g;
    // a[part][f], b[part][u] of one k-step (part 0 hi, 1 mid, 2 lo)
    auto load = [&](uint4 (&a)[3][4], uint4 (&b)[3][2], int s, bool in) {
        const int64_t o = (int64_t)s * KS;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            if (in) {
#pragma unroll
                for (int f = 0; f < 4; ++f) a[q][f] = *reinterpret_cast<const uint4*>(ap[f] + q * nn + o);
                b[q][0] = *reinterpret_cast<const uint4*>(bp0 + q * xn + o);
                b[q][1] = *reinterpret_cast<const uint4*>(bp1 + q * xn + o);
            } else {
                const uint4 z = {0u, 0u, 0u, 0u};
#pragma unroll
                for (int f = 0; f < 4; ++f) a[q][f] = z;
                b[q][0] = b[q][1] = z;
            }
        }
    };
    auto compute = [&](const uint4 (&a)[3][4], const uint4 (&b)[3][2]) {
        // (operator part, block part): lo hi, hi lo, mid mid, mid hi, hi mid, hi hi
        constexpr int pa[6] = {2, 0, 1, 1, 0, 0}, pb[6] = {0, 2, 1, 0, 1, 0};
#pragma unroll
        for (int t = 0; t < 6; ++t)
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                acc[f][0] = mfma16<3>(a[pa[t]][f], b[pb[t]][0], acc[f][0]);
                acc[f][1] = mfma16<3>(a[pa[t]][f], b[pb[t]][1], acc[f][1]);
            }
    };
    if (nfull > 0) {
        uint4 a0[3][4], b0[3][2], a1[3][4], b1[3][2];
        load(a0, b0, 0, true);
        for (int s = 0; s < nfull; s += 2) {
            load(a1, b1, min(s + 1, nfull - 1), true);
            compute(a0, b0);
            load(a0, b0, min(s + 2, nfull - 1), true);
            if (s + 1 < nfull) compute(a1, b1);
        }
    }
    if (k_begin + KS * nfull < k_end) {
        // last partial k-step: a lane's 8 values are all in range or all out (n % 8 == 0)
        const bool kin = k_begin + (int64_t)nfull * KS + 8 * g < k_end;
        uint4 aa[3][4], bb[3][2];
        load(aa, bb, nfull, kin);
        compute(aa, bb);
    }
    const int ntiles = (n + WR - 1) / WR;
    float* out = part + (((int64_t)split * ntiles + tile) * WAVE + lane) * 32;
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int u = 0; u < 2; ++u) *reinterpret_cast<f4*>(out + (f * 2 + u) * 4) = acc[f][u];
}

// Q (FP64, n x w, ld n) = 2^-e_j * sum_split part, fixed split order, and
// pq[tile * 32 + j] = sum over the tile's rows of P[:, j] Q[:, j].  Block
// (tile, col group) of 256 threads: thread = (row, column pair).
template <int P>
__global__ __launch_bounds__(256) void apply16_reduce_kernel(int n, int w, int nsplit, const float* __restrict__ part,
                                                             const double* __restrict__ rr,
                                                             double* __restrict__ Q,
                                                             const double* __restrict__ Pm,
                                                             double* __restrict__ pq,
                                                             const int* __restrict__ flag) {
    if (flag && *flag == 0) return;
    const int tile = blockIdx.x, grp = blockIdx.y;
    const int ntiles = (n + WR - 1) / WR;
    const int64_t total = (int64_t)ntiles * WAVE * 32;
    const int row = threadIdx.x % WR, cp = threadIdx.x / WR;
    const int col0 = 8 * grp + 2 * cp;
    const int f = row / 16, rr16 = row % 16, g = rr16 / 4, it = rr16 % 4;
    double prod[2] = {0.0, 0.0};
    const int grow = tile * WR + row;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int col = col0 + h, u = col / 16, c = col % 16;
        const int lane = 16 * g + c;
        const float* src = part + ((int64_t)tile * WAVE + lane) * 32 + (f * 2 + u) * 4 + it;
        double s = 0.0;
        for (int k = 0; k < nsplit; ++k) s += (double)src[(int64_t)k * total];
        if (grow < n && col < w) {
            double sc = 1.0;
            if (P == 2 && rr[col] > 0.0) sc = exp2(-rint(0.5 * log2((double)n / rr[col])));
            const double o = s * sc;
            Q[(int64_t)col * n + grow] = o;
            prod[h] = Pm[(int64_t)col * n + grow] * o;
        }
    }
    prod[0] = wave_sum(prod[0]);
    prod[1] = wave_sum(prod[1]);
    if (row == 0) {
        pq[(int64_t)tile * 32 + col0] = prod[0];
        pq[(int64_t)tile * 32 + col0 + 1] = prod[1];
    }
}

}  // namespace

hipError_t convert_operator16(hipStream_t st, int precision, int n, const double* A, int64_t lda, uint16_t* out) {
    dim3 grid((n + 31) / 32, (n + 31) / 32);
    if (precision == 1)
        hipLaunchKernelGGL(convert16_kernel<1>, grid, dim3(256), 0, st, n, A, lda, out);
    else if (precision == 2)
        hipLaunchKernelGGL(convert16_kernel<2>, grid, dim3(256), 0, st, n, A, lda, out);
    else if (precision == 3)
        hipLaunchKernelGGL(convert16_kernel<3>, grid, dim3(256), 0, st, n, A, lda, out);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t cg_dense_apply16(hipStream_t st, int precision, int n, int w, const uint16_t* A16, double* P,
                            const double* R, const double* beta, const int* active, const double* rr, int first,
                            double* Q, double* pq, double* work, size_t work_elems, const int* any_active,
                            hipEvent_t* ev, int* flag_log) {
    if (w < 1 || w > 32 || n < 64 || (n % 8) != 0 || precision < 1 || precision > 3 ||
        (reinterpret_cast<uintptr_t>(A16) & 15))
        return hipErrorInvalidValue;
    const int ntiles = (n + WR - 1) / WR;
    int ksplit = 1;
    while (ntiles * ksplit < 2048 && n / (ksplit * 2) >= 1024 && ksplit < 16) ksplit *= 2;
    int kchunk = (n + ksplit - 1) / ksplit;
    kchunk = ((kchunk + KS * 2 * PF - 1) / (KS * 2 * PF)) * (KS * 2 * PF);
    ksplit = (n + kchunk - 1) / kchunk;
    // workspace: Xh (n x 32 16-bit; three parts for BF16x3) then the FP32 partial tiles
    const size_t parts = precision == 3 ? 3 : 1;
    const size_t xh_elems = (parts * n * 32 * sizeof(uint16_t) + 15) / 16 * 2;   // in doubles, 16-byte units
    const size_t part_floats = (size_t)ksplit * ntiles * WAVE * 32;
    if (xh_elems + (part_floats + 1) / 2 > work_elems) return hipErrorInvalidValue;
    uint16_t* Xh = reinterpret_cast<uint16_t*>(work);
    float* part = reinterpret_cast<float*>(work + xh_elems);
    const dim3 pgrid((n + 255) / 256 < 64 ? (n + 255) / 256 : 64, 32);
    if (precision == 3) {
        hipLaunchKernelGGL(cg_dir_pack16_kernel<3>, pgrid, dim3(256), 0, st, n, w, P, R, beta, active, rr, first, Xh,
                           any_active, flag_log);
        if (ev) (void)hipEventRecord(ev[0], st);
        hipLaunchKernelGGL(apply16x3_stream_kernel, dim3(ntiles, ksplit), dim3(64), 0, st, n, A16, Xh, kchunk, part,
                           any_active);
        if (ev) (void)hipEventRecord(ev[1], st);
        hipLaunchKernelGGL(apply16_reduce_kernel<3>, dim3(ntiles, 4), dim3(256), 0, st, n, w, ksplit, part, rr, Q, P,
                           pq, any_active);
    } else if (precision == 1) {
        hipLaunchKernelGGL(cg_dir_pack16_kernel<1>, pgrid, dim3(256), 0, st, n, w, P, R, beta, active, rr, first, Xh,
                           any_active, flag_log);
        if (ev) (void)hipEventRecord(ev[0], st);
        hipLaunchKernelGGL(apply16_stream_kernel<1>, dim3(ntiles, ksplit), dim3(64), 0, st, n, A16, Xh, kchunk, part,
                           any_active);
        if (ev) (void)hipEventRecord(ev[1], st);
        hipLaunchKernelGGL(apply16_reduce_kernel<1>, dim3(ntiles, 4), dim3(256), 0, st, n, w, ksplit, part, rr, Q, P,
                           pq, any_active);
    } else {
        hipLaunchKernelGGL(cg_dir_pack16_kernel<2>, pgrid, dim3(256), 0, st, n, w, P, R, beta, active, rr, first, Xh,
                           any_active, flag_log);
        if (ev) (void)hipEventRecord(ev[0], st);
        hipLaunchKernelGGL(apply16_stream_kernel<2>, dim3(ntiles, ksplit), dim3(64), 0, st, n, A16, Xh, kchunk, part,
                           any_active);
        if (ev) (void)hipEventRecord(ev[1], st);
        hipLaunchKernelGGL(apply16_reduce_kernel<2>, dim3(ntiles, 4), dim3(256), 0, st, n, w, ksplit, part, rr, Q, P,
                           pq, any_active);
    }
    return hipGetLastError();
}

}  // namespace lrep
