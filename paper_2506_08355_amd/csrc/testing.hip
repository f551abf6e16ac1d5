// Kernel-level entry points for the library's unit tests (include/lrep_testing.h).
#include "../../include/lrep_testing.h"
#include "internal.hpp"

using namespace lrep;

struct lrep_ctx_s : public Ctx {};
struct lrep_op_s : public Op {};

namespace lrep {
int block_mgs_standalone(Ctx* c, hipStream_t st, int64_t n, int m, double* X, double* Y, int* kept);
int cg_standalone(Op* op, hipStream_t st, int which, int nw, const double* B, double* X, double tol, int maxit,
                  int fused, int64_t* applies);
}

namespace {
__global__ __launch_bounds__(256) void copy_kernel(const double2* __restrict__ src, double2* __restrict__ dst,
                                                  int64_t pairs) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < pairs; i += (int64_t)gridDim.x * 256)
        dst[i] = src[i];
}

// plain streaming read: out[block] = sum of the block's grid-stride share of
// src (16-byte loads), the reference for the achievable HBM read rate
__global__ __launch_bounds__(256) void read_sum_kernel(const double2* __restrict__ src, int64_t pairs,
                                                       double* __restrict__ out) {
    __shared__ double red[256];
    double s0 = 0.0, s1 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < pairs; i += (int64_t)gridDim.x * 256) {
        const double2 v = src[i];
        s0 += v.x;
        s1 += v.y;
    }
    red[threadIdx.x] = s0 + s1;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

int finish(Ctx* c, hipError_t e) {
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        c->set_error(hipGetErrorString(e));
        return LREP_EDEVICE;
    }
    return LREP_OK;
}
}  // namespace

extern "C" {

int lrep_test_gemm_nn(lrep_ctx_t ctx, int m, int q, int p, const double* A, int64_t lda, const double* B,
                      int64_t ldb, double* C, int64_t ldc, double alpha, double beta, int ksplit) {
    if (!ctx || m < 0 || q < 0 || p < 0 || lda < m || ldb < p || ldc < m) return LREP_EINVAL;
    (void)hipSetDevice(ctx->device);
    DevBuf work;
    const size_t welems = (size_t)std::max(ksplit, 64) * m * q + 1;
    int rc = work.alloc(ctx, welems * sizeof(double));
    if (rc != LREP_OK) return rc;
    Seg a{A, lda, p};
    return finish(ctx, gemm_nn(ctx->stream, m, q, p, &a, 1, B, ldb, C, ldc, alpha, beta, work.p, welems, nullptr,
                               nullptr, 0, ksplit));
}

int lrep_test_gemm_tn(lrep_ctx_t ctx, int n, int p, int q, const double* A, int64_t lda, const double* B,
                      int64_t ldb, double* C, int64_t ldc, int symmetrize) {
    if (!ctx || n < 0 || p < 0 || q < 0 || lda < n || ldb < n || ldc < p) return LREP_EINVAL;
    (void)hipSetDevice(ctx->device);
    DevBuf work;
    const size_t welems = (size_t)1024 * p * q + 1;
    int rc = work.alloc(ctx, welems * sizeof(double));
    if (rc != LREP_OK) return rc;
    Seg a{A, lda, p}, b{B, ldb, q};
    return finish(ctx, gemm_tn(ctx->stream, n, p, q, &a, 1, &b, 1, C, ldc, 1.0, symmetrize, work.p, welems));
}

int lrep_test_small_lrep(lrep_ctx_t ctx, int d, const double* Kh, const double* Mh, int64_t ldh, double* lam,
                         double* Xh, double* Yh) {
    if (!ctx || d < 1 || d > kMaxD || ldh < d) return LREP_EINVAL;
    (void)hipSetDevice(ctx->device);
    DevBuf scr, st, work;
    const size_t welems = size_t(1) << 20;
    int rc = scr.alloc(ctx, 4 * kMaxD * kMaxD * sizeof(double));
    if (rc == LREP_OK) rc = st.alloc(ctx, ST_COUNT * sizeof(int));
    if (rc == LREP_OK) rc = work.alloc(ctx, welems * sizeof(double));
    if (rc != LREP_OK) return rc;
    int* status = reinterpret_cast<int*>(st.p);
    hipError_t e = hipMemsetAsync(status, 0, ST_COUNT * sizeof(int), ctx->stream);
    if (e == hipSuccess) e = small_lrep(ctx->stream, d, Kh, Mh, ldh, lam, Xh, Yh, scr.p, status, work.p, welems);
    rc = finish(ctx, e);
    if (rc != LREP_OK) return rc;
    int hs[ST_COUNT];
    if (hipMemcpy(hs, status, sizeof(hs), hipMemcpyDeviceToHost) != hipSuccess) return LREP_EDEVICE;
    return hs[ST_NOTSPD] ? LREP_ENOTSPD : LREP_OK;
}

int lrep_test_block_mgs(lrep_ctx_t ctx, int n, int m, double* X, double* Y, int* kept) {
    if (!ctx || n < 1 || m < 0 || m > kMaxD || !kept) return LREP_EINVAL;
    (void)hipSetDevice(ctx->device);
    return block_mgs_standalone(ctx, ctx->stream, n, m, X, Y, kept);
}

int lrep_test_apply(lrep_op_t op, int which, int cols, const double* X, double* Y) {
    if (!op || cols < 0 || (which != 0 && which != 1)) return LREP_EINVAL;
    Ctx* c = op->ctx;
    (void)hipSetDevice(c->device);
    DevBuf work, small;
    const size_t welems = size_t(8) << 20;
    int rc = work.alloc(c, welems * sizeof(double));
    if (rc == LREP_OK) rc = small.alloc(c, (size_t)std::max<int64_t>(op->rank, 1) * std::max(cols, 1) * sizeof(double));
    if (rc != LREP_OK) return rc;
    rc = op_apply(op, c->stream, which, X, op->n, cols, Y, op->n, work.p, welems, small.p, nullptr);
    if (rc != LREP_OK) return rc;
    return finish(c, hipSuccess);
}

int lrep_test_cg(lrep_op_t op, int which, int nw, const double* B, double* X, double tol, int maxit, int fused,
                 int64_t* applies) {
    if (!op || (which != 0 && which != 1) || nw < 1 || nw > 32 || !B || !X || (fused < -1 || fused > 1))
        return LREP_EINVAL;
    Ctx* c = op->ctx;
    (void)hipSetDevice(c->device);
    return cg_standalone(op, c->stream, which, nw, B, X, tol, maxit, fused, applies);
}

int lrep_test_convert16(lrep_ctx_t ctx, int precision, int n, const double* A, int64_t lda, uint16_t* out) {
    if (!ctx || precision < 1 || precision > 3 || n < 1 || lda < n || !A || !out) return LREP_EINVAL;
    (void)hipSetDevice(ctx->device);
    return finish(ctx, convert_operator16(ctx->stream, precision, n, A, lda, out));
}

int lrep_test_apply16(lrep_ctx_t ctx, int precision, int n, int cols, const uint16_t* A16, const double* X,
                      const double* rr, double* Y) {
    if (!ctx || cols < 1 || cols > 32 || precision < 1 || precision > 3 || n < 64 || (n % 8) != 0 || !A16 ||
        !X || !rr || !Y)
        return LREP_EINVAL;
    (void)hipSetDevice(ctx->device);
    DevBuf work, pq, flag;
    const size_t welems = size_t(8) << 20;
    int rc = work.alloc(ctx, welems * sizeof(double));
    if (rc == LREP_OK) rc = pq.alloc(ctx, stream_tiles(n) * 32 * sizeof(double));
    if (rc == LREP_OK) rc = flag.alloc(ctx, sizeof(int));
    if (rc != LREP_OK) return rc;
    const int one = 1;
    hipError_t e = hipMemcpyAsync(flag.p, &one, sizeof(int), hipMemcpyHostToDevice, ctx->stream);
    // first step of a CG: the direction is X as given (not written), no beta / active read
    if (e == hipSuccess)
        e = cg_dense_apply16(ctx->stream, precision, n, cols, A16, const_cast<double*>(X), nullptr, nullptr, nullptr,
                             rr, 1, Y, pq.p, work.p, welems, reinterpret_cast<const int*>(flag.p), nullptr, nullptr);
    return finish(ctx, e);
}

int lrep_test_read(lrep_ctx_t ctx, const double* src, int64_t count, int blocks, int iters, double* out,
                   double* ms) {
    if (!ctx || !src || !out || !ms || count < 0 || (count & 1) || blocks < 1 || blocks > 65536 || iters < 1 ||
        (reinterpret_cast<uintptr_t>(src) & 15))
        return LREP_EINVAL;
    (void)hipSetDevice(ctx->device);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipEventRecord(e0, ctx->stream);
    for (int i = 0; i < iters && e == hipSuccess; ++i) {
        hipLaunchKernelGGL(read_sum_kernel, dim3(blocks), dim3(256), 0, ctx->stream,
                           reinterpret_cast<const double2*>(src), count / 2, out);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    *ms = (double)t;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return finish(ctx, e);
}

int lrep_test_copy(lrep_ctx_t ctx, const double* src, double* dst, int64_t count) {
    if (!ctx || !src || !dst || count < 0 || (count & 1) || (reinterpret_cast<uintptr_t>(src) & 15) ||
        (reinterpret_cast<uintptr_t>(dst) & 15))
        return LREP_EINVAL;
    (void)hipSetDevice(ctx->device);
    const int64_t pairs = count / 2;
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(8192, (pairs + 255) / 256));
    hipLaunchKernelGGL(copy_kernel, dim3(blocks), dim3(256), 0, ctx->stream, reinterpret_cast<const double2*>(src),
                       reinterpret_cast<double2*>(dst), pairs);
    return finish(ctx, hipGetLastError());
}

}  // extern "C"
