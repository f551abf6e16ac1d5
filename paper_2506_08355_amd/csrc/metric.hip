// Metric of a generalized LREP (K x = lambda B y, M y = lambda B x, B SPD;
// the remark on the generalized LREP in Section 3.2).  With B = C C^T and
// x^ = C^T x, y^ = C^T y the pencil is the standard LREP of C^-1 K C^-T and
// C^-1 M C^-T, and the Euclidean inner product of transformed vectors is the
// B inner product of the originals (x^T B y = x^^T y^).
//   diagonal B = diag(b):  C = B^1/2; one-time elementwise HBM passes with
//                          S = B^-1/2 (coalesced column sweeps);
//   dense B (dense operators only): C = L, the Cholesky factor, by a blocked
//                          right-looking factorisation (64-wide diagonal
//                          blocks in LDS, panel and trailing updates as MFMA
//                          block products), L^-1 by blocked forward
//                          substitution on I, then two n^3 products per
//                          operator.  L^T and L^-T are kept for the
//                          coordinate changes of start blocks, null-space
//                          bases and results.
#include <algorithm>
#include <cfloat>

#include "device.hpp"
#include "internal.hpp"
#include "kernels.hpp"

namespace lrep {

namespace {

constexpr int NT = 256;

__global__ __launch_bounds__(NT) void metric_prepare_kernel(int64_t n, const double* __restrict__ b,
                                                            double* __restrict__ s, int* __restrict__ bad) {
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        const double v = b[i];
        if (v > 0.0 && v <= DBL_MAX) {
            s[i] = 1.0 / sqrt(v);
        } else {   // zero, negative, infinite or NaN
            s[i] = 1.0;
            *bad = 1;
        }
    }
}

// one column per blockIdx.y step: A[i, j] <- (s_i s_j) A[i, j]
__global__ __launch_bounds__(NT) void metric_scale_sym_kernel(int64_t n, double* __restrict__ A, int64_t ld,
                                                              const double* __restrict__ s) {
    for (int64_t j = blockIdx.y; j < n; j += gridDim.y) {
        const double sj = s[j];
        double* col = A + j * ld;
        for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
            col[i] *= s[i] * sj;
    }
}

__global__ __launch_bounds__(NT) void metric_scale_diag_kernel(int64_t n, double* __restrict__ d,
                                                               const double* __restrict__ s) {
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
        d[i] *= s[i] * s[i];
}

__global__ __launch_bounds__(NT) void metric_scale_rows_kernel(int64_t n, int cols, double* __restrict__ X,
                                                               int64_t ldx, const double* __restrict__ s,
                                                               int inverse) {
    for (int64_t j = blockIdx.y; j < cols; j += gridDim.y) {
        double* col = X + j * ldx;
        for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
            col[i] = inverse ? col[i] / s[i] : col[i] * s[i];
    }
}

unsigned row_blocks(int64_t n) { return (unsigned)std::min<int64_t>((n + NT - 1) / NT, 1024); }

constexpr int CB = 64;   // diagonal block of the dense factorisation

// Cholesky of the diagonal block A (kb x kb, kb <= 64, ld lda) in LDS, in place
// (lower triangle; the strict upper triangle is zeroed), and its inverse:
// V = L11^-1 and W = L11^-T (both 64 x 64, column-major, ld 64, zero outside
// kb x kb).  A pivot that is not positive and finite sets *bad (the
// factorisation then continues with pivot 1 so that every access stays in
// range).
__global__ __launch_bounds__(256) void chol_block_kernel(int kb, double* __restrict__ A, int64_t lda,
                                                         double* __restrict__ V, double* __restrict__ W,
                                                         int* __restrict__ bad) {
    __shared__ double a[CB][CB + 1];
    __shared__ double v[CB][CB + 1];
    const int tid = threadIdx.x;
    for (int idx = tid; idx < CB * CB; idx += 256) {
        const int i = idx % CB, c = idx / CB;
        a[i][c] = (i < kb && c < kb && i >= c) ? A[(int64_t)c * lda + i] : 0.0;
    }
    __syncthreads();
    for (int j = 0; j < kb; ++j) {
        double piv = a[j][j];
        if (!(piv > 0.0 && piv <= DBL_MAX)) {
            if (tid == 0) *bad = 1;
            piv = 1.0;
        }
        const double d = sqrt(piv);
        __syncthreads();   // every thread has read a[j][j]
        if (tid < kb) {
            if (tid > j) a[tid][j] /= d;
            else if (tid == j) a[j][j] = d;
        }
        __syncthreads();
        for (int idx = tid; idx < kb * kb; idx += 256) {
            const int i = idx % kb, c = idx / kb;
            if (c > j && i >= c) a[i][c] -= a[i][j] * a[c][j];
        }
        __syncthreads();
    }
    for (int idx = tid; idx < kb * kb; idx += 256) {
        const int i = idx % kb, c = idx / kb;
        A[(int64_t)c * lda + i] = (i >= c) ? a[i][c] : 0.0;
    }
    // column c of L11^-1 by forward substitution (thread c)
    if (tid < CB) {
        const int c = tid;
        for (int i = 0; i < CB; ++i) {
            double x = 0.0;
            if (c < kb && i < kb && i >= c) {
                double sacc = (i == c) ? 1.0 : 0.0;
                for (int k = c; k < i; ++k) sacc -= a[i][k] * v[k][c];
                x = sacc / a[i][i];
            }
            v[i][c] = x;
        }
    }
    __syncthreads();
    for (int idx = tid; idx < CB * CB; idx += 256) {
        const int i = idx % CB, c = idx / CB;
        V[c * CB + i] = v[i][c];
        W[c * CB + i] = v[c][i];
    }
}

// out (cols x rows, ld ldo) = in^T for in (rows x cols, ld ldi); 64 x 64 tiles through LDS
__global__ __launch_bounds__(256) void transpose_kernel(int64_t rows, int64_t cols, const double* __restrict__ in,
                                                        int64_t ldi, double* __restrict__ out, int64_t ldo) {
    __shared__ double t[64][65];
    const int64_t r0 = (int64_t)blockIdx.x * 64, c0 = (int64_t)blockIdx.y * 64;
    for (int idx = threadIdx.x; idx < 64 * 64; idx += 256) {
        const int i = idx % 64, c = idx / 64;
        t[c][i] = (r0 + i < rows && c0 + c < cols) ? in[(c0 + c) * ldi + r0 + i] : 0.0;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < 64 * 64; idx += 256) {
        const int c = idx % 64, i = idx / 64;   // out row c0 + c, out column r0 + i
        if (r0 + i < rows && c0 + c < cols) out[(r0 + i) * ldo + c0 + c] = t[c][i];
    }
}

// strict upper triangle of A (n x n, ld n) = 0
__global__ __launch_bounds__(NT) void zero_upper_kernel(int64_t n, double* __restrict__ A) {
    for (int64_t j = blockIdx.y; j < n; j += gridDim.y)
        for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < j; i += (int64_t)gridDim.x * NT) A[j * n + i] = 0.0;
}

// X (n x n, ld n) = I
__global__ __launch_bounds__(NT) void identity_kernel(int64_t n, double* __restrict__ X) {
    for (int64_t j = blockIdx.y; j < n; j += gridDim.y)
        for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
            X[j * n + i] = (i == j) ? 1.0 : 0.0;
}

// A (n x n) <- (A + A^T) / 2, each pair (i, j), i > j, by one thread
__global__ __launch_bounds__(NT) void symmetrize_kernel(int64_t n, double* __restrict__ A, int64_t lda) {
    for (int64_t j = blockIdx.y; j < n; j += gridDim.y)
        for (int64_t i = j + 1 + (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
            const double m = 0.5 * (A[j * lda + i] + A[i * lda + j]);
            A[j * lda + i] = m;
            A[i * lda + j] = m;
        }
}

hipError_t transpose(hipStream_t st, int64_t rows, int64_t cols, const double* in, int64_t ldi, double* out,
                     int64_t ldo) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)((rows + 63) / 64), (unsigned)((cols + 63) / 64)), dim3(256),
                       0, st, rows, cols, in, ldi, out, ldo);
    return hipGetLastError();
}

}  // namespace

hipError_t metric_prepare(hipStream_t st, int64_t n, const double* b, double* s, int* bad) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(metric_prepare_kernel, dim3(row_blocks(n)), dim3(NT), 0, st, n, b, s, bad);
    return hipGetLastError();
}

hipError_t metric_scale_sym(hipStream_t st, int64_t n, double* A, int64_t ld, const double* s) {
    if (n <= 0) return hipSuccess;
    const unsigned gx = (unsigned)std::min<int64_t>((n + NT - 1) / NT, 64);
    const unsigned gy = (unsigned)std::min<int64_t>(n, 4096);
    hipLaunchKernelGGL(metric_scale_sym_kernel, dim3(gx, gy), dim3(NT), 0, st, n, A, ld, s);
    return hipGetLastError();
}

hipError_t metric_scale_diag(hipStream_t st, int64_t n, double* d, const double* s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(metric_scale_diag_kernel, dim3(row_blocks(n)), dim3(NT), 0, st, n, d, s);
    return hipGetLastError();
}

hipError_t metric_scale_rows(hipStream_t st, int64_t n, int cols, double* X, int64_t ldx, const double* s,
                             bool inverse) {
    if (n <= 0 || cols <= 0) return hipSuccess;
    const unsigned gx = (unsigned)std::min<int64_t>((n + NT - 1) / NT, 256);
    const unsigned gy = (unsigned)std::min(cols, 4096);
    hipLaunchKernelGGL(metric_scale_rows_kernel, dim3(gx, gy), dim3(NT), 0, st, n, cols, X, ldx, s,
                       inverse ? 1 : 0);
    return hipGetLastError();
}

hipError_t metric_dense_setup(hipStream_t st, int64_t n, double* Lb, double* Xb, double* Tb, double* LT,
                              double* LinvT, double* Vall, double* Wb, double* Pt, double* work, size_t work_elems,
                              int* bad) {
    // 1. B = L L^T in place in Lb (n x n, ld n); Vall keeps every L_kk^-1
    for (int64_t k0 = 0; k0 < n; k0 += CB) {
        const int kb = (int)std::min<int64_t>(CB, n - k0);
        const int64_t m2 = n - k0 - kb;
        double* A11 = Lb + k0 * n + k0;
        double* Vk = Vall + k0 * CB;
        hipLaunchKernelGGL(chol_block_kernel, dim3(1), dim3(256), 0, st, kb, A11, n, Vk, Wb, bad);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess || m2 == 0) {
            if (e != hipSuccess) return e;
            continue;
        }
        double* A21 = A11 + kb;
        double* A22 = A11 + (int64_t)kb * n + kb;
        const Seg a21{A21, n, kb};
        // L21 = A21 L11^-T, through the panel buffer
        e = gemm_nn(st, (int)m2, kb, kb, &a21, 1, Wb, CB, Tb, m2, 1.0, 0.0, work, work_elems);
        if (e == hipSuccess) e = copy_cols(st, (int)m2, kb, Tb, m2, A21, n);
        // A22 -= L21 L21^T (the whole square; only its lower part is used later)
        if (e == hipSuccess) e = transpose(st, m2, kb, A21, n, Pt, kb);
        if (e == hipSuccess)
            e = gemm_nn(st, (int)m2, (int)m2, kb, &a21, 1, Pt, kb, A22, n, -1.0, 1.0, work, work_elems);
        if (e != hipSuccess) return e;
    }
    // the strict upper triangle of Lb still holds B's (partly updated) entries
    const dim3 sq((unsigned)std::min<int64_t>((n + NT - 1) / NT, 64), (unsigned)std::min<int64_t>(n, 4096));
    hipLaunchKernelGGL(zero_upper_kernel, sq, dim3(NT), 0, st, n, Lb);
    // 2. Linv = L^-1 by blocked forward substitution on I (in Xb)
    hipLaunchKernelGGL(identity_kernel, sq, dim3(NT), 0, st, n, Xb);
    hipError_t e = hipGetLastError();
    for (int64_t k0 = 0; k0 < n && e == hipSuccess; k0 += CB) {
        const int kb = (int)std::min<int64_t>(CB, n - k0);
        const int64_t m2 = n - k0 - kb;
        const Seg vk{Vall + k0 * CB, CB, kb};
        // X_k = L_kk^-1 X_k (rows k0 .. k0 + kb, all n columns)
        e = gemm_nn(st, kb, (int)n, kb, &vk, 1, Xb + k0, n, Tb, kb, 1.0, 0.0, work, work_elems);
        if (e == hipSuccess) e = copy_cols(st, kb, (int)n, Tb, kb, Xb + k0, n);
        if (e == hipSuccess && m2 > 0) {
            const Seg l21{Lb + k0 * n + k0 + kb, n, kb};
            e = gemm_nn(st, (int)m2, (int)n, kb, &l21, 1, Xb + k0, n, Xb + k0 + kb, n, -1.0, 1.0, work, work_elems);
        }
    }
    // 3. LT = L^T (upper: the lower triangle of Lb transposed, zeros below)
    //    and LinvT = (L^-1)^T
    if (e == hipSuccess) e = transpose(st, n, n, Lb, n, LT, n);
    if (e == hipSuccess) e = transpose(st, n, n, Xb, n, LinvT, n);
    return e;
}

hipError_t metric_dense_apply(hipStream_t st, int64_t n, double* A, int64_t lda, const double* Linv,
                              const double* LinvT, double* Tb, double* work, size_t work_elems) {
    // A <- L^-1 A L^-T, then symmetrised
    const Seg li{Linv, n, (int)n};
    hipError_t e = gemm_nn(st, (int)n, (int)n, (int)n, &li, 1, A, lda, Tb, n, 1.0, 0.0, work, work_elems);
    const Seg tb{Tb, n, (int)n};
    if (e == hipSuccess)
        e = gemm_nn(st, (int)n, (int)n, (int)n, &tb, 1, LinvT, n, A, lda, 1.0, 0.0, work, work_elems);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(symmetrize_kernel, dim3((unsigned)std::min<int64_t>((n + NT - 1) / NT, 64),
                                                   (unsigned)std::min<int64_t>(n, 4096)), dim3(NT), 0, st, n, A, lda);
        e = hipGetLastError();
    }
    return e;
}

int op_metric_transform(Op* op, hipStream_t st, bool to_hat, int cols, double* X, int64_t ldx, double* tmp,
                        double* work, size_t work_elems) {
    if (cols <= 0) return LREP_OK;
    hipError_t e = hipSuccess;
    const int64_t n = op->n;
    if (op->Sv) {
        e = metric_scale_rows(st, n, cols, X, ldx, op->Sv, to_hat);
    } else if (op->MetLT.p) {
        const Seg t{to_hat ? op->MetLT.p : op->MetLinvT.p, n, (int)n};
        e = gemm_nn(st, (int)n, cols, (int)n, &t, 1, X, ldx, tmp, n, 1.0, 0.0, work, work_elems);
        if (e == hipSuccess) e = copy_cols(st, (int)n, cols, tmp, n, X, ldx);
    }
    return e == hipSuccess ? LREP_OK : LREP_EDEVICE;
}

}  // namespace lrep
