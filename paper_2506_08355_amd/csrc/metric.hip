// Diagonal metric of a generalized LREP (K x = lambda B y, M y = lambda B x,
// B = diag(b); the remark on the generalized LREP in Section 3.2).  With
// S = B^-1/2 the pencil is the standard LREP of S K S and S M S, and the
// Euclidean inner product of scaled vectors is the B inner product of the
// originals.  These are one-time, elementwise HBM passes: coalesced column
// sweeps, no reuse to exploit.
#include <algorithm>
#include <cfloat>

#include "device.hpp"
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

}  // namespace lrep
