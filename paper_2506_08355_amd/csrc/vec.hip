// Streaming (HBM-bound) kernels of the BOSP iteration on gfx950: fused
// residual norms (Step 4), the block CG of Step 6, right-hand sides of the
// block Gauss-Seidel sweep, and small utilities.  Every reduction is two
// stage with a fixed summation order (bitwise reproducible).
#include "device.hpp"
#include "kernels.hpp"

namespace lrep {

namespace {
constexpr int NT = 256;

inline int chunks_for(int n, int cols, int rows_per_block = 4096, int max_chunks = 256) {
    int c = (n + rows_per_block - 1) / rows_per_block;
    // keep at least ~512 workgroups in flight when the problem is big enough
    while (c * cols < 512 && c < max_chunks && (n + 2 * c - 1) / (2 * c) >= 1024) c *= 2;
    return std::max(1, std::min(c, max_chunks));
}

__global__ __launch_bounds__(NT) void diag_scale_kernel(int n, int cols, const double* __restrict__ delta,
                                                        const double* __restrict__ X, int64_t ldx,
                                                        double* __restrict__ Y, int64_t ldy,
                                                        const int* __restrict__ active_flag) {
    if (active_flag && *active_flag == 0) return;
    const int j = blockIdx.y;
    for (int i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT)
        Y[(int64_t)j * ldy + i] = delta[i] * X[(int64_t)j * ldx + i];
}

// block (tile of 64 rows) x 256 threads: thread = (row, column group of 8);
// per column the tile's sum of x y, rows in wave-sum order
__global__ __launch_bounds__(NT) void diag_scale_pq_kernel(int n, int cols, const double* __restrict__ delta,
                                                           const double* __restrict__ X, int64_t ldx,
                                                           double* __restrict__ Y, int64_t ldy,
                                                           double* __restrict__ pq,
                                                           const int* __restrict__ active_flag) {
    if (active_flag && *active_flag == 0) return;
    const int i = threadIdx.x % 64, grp = threadIdx.x / 64;
    const int row = blockIdx.x * 64 + i;
    const double dv = row < n ? delta[row] : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int col = grp * 8 + u;
        double s = 0.0;
        if (col < cols && row < n) {
            const double x = X[(int64_t)col * ldx + row];
            const double y = dv * x;
            Y[(int64_t)col * ldy + row] = y;
            s = x * y;
        }
        s = wave_sum(s);
        if (i == 0 && col < cols) pq[(int64_t)blockIdx.x * 32 + col] = s;
    }
}

// the same with the CG's pending direction update folded in: for the active
// columns p = r + beta p (written back), then q = delta o p and the tile sums
// of p . q; the arithmetic of each entry is that of cg_direction_kernel
__global__ __launch_bounds__(NT) void diag_dir_scale_pq_kernel(int n, int cols, const double* __restrict__ delta,
                                                               double* __restrict__ P, const double* __restrict__ R,
                                                               const double* __restrict__ beta,
                                                               const int* __restrict__ active,
                                                               double* __restrict__ Q, double* __restrict__ pq,
                                                               const int* __restrict__ active_flag) {
    if (active_flag && *active_flag == 0) return;
    const int i = threadIdx.x % 64, grp = threadIdx.x / 64;
    const int row = blockIdx.x * 64 + i;
    const double dv = row < n ? delta[row] : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int col = grp * 8 + u;
        double s = 0.0;
        if (col < cols && row < n) {
            const int64_t o = (int64_t)col * n + row;
            double x = P[o];
            if (active[col]) {
                x = R[o] + beta[col] * x;
                P[o] = x;
            }
            const double y = dv * x;
            Q[o] = y;
            s = x * y;
        }
        s = wave_sum(s);
        if (i == 0 && col < cols) pq[(int64_t)blockIdx.x * 32 + col] = s;
    }
}

// ---------------------------------------------------------------- residuals
__global__ __launch_bounds__(NT) void residual_kernel(int n, int cols, int nchunks, const double* __restrict__ X,
                                                      const double* __restrict__ Y, const double* __restrict__ KX,
                                                      const double* __restrict__ MY, int64_t ld,
                                                      const double* __restrict__ lam, double* __restrict__ eps,
                                                      double* __restrict__ part, unsigned* ticket) {
    __shared__ double red[NT / WAVE];
    const int j = blockIdx.y, ch = blockIdx.x;
    const int rows = (n + nchunks - 1) / nchunks;
    const int r0 = ch * rows, r1 = min(n, r0 + rows);
    const double l = lam[j];
    const int64_t off = (int64_t)j * ld;
    double s1 = 0, s2 = 0, sx = 0, sy = 0;
    for (int i = r0 + threadIdx.x; i < r1; i += NT) {
        const double x = X[off + i], y = Y[off + i];
        const double a = KX[off + i] - l * y;
        const double b = MY[off + i] - l * x;
        s1 += a * a;
        s2 += b * b;
        sx += x * x;
        sy += y * y;
    }
    s1 = block_sum<NT>(s1, red);
    s2 = block_sum<NT>(s2, red);
    sx = block_sum<NT>(sx, red);
    sy = block_sum<NT>(sy, red);
    if (threadIdx.x == 0) {
        double* p = part + ((int64_t)j * nchunks + ch) * 4;
        p[0] = s1;
        p[1] = s2;
        p[2] = sx;
        p[3] = sy;
    }
}

__global__ __launch_bounds__(NT) void residual_fin_kernel(int cols, int nchunks, const double* __restrict__ part,
                                                          const double* __restrict__ lam, double* __restrict__ eps) {
    for (int c = threadIdx.x; c < cols; c += NT) {
        double t1 = 0, t2 = 0, tx = 0, ty = 0;
        const double* p = part + (int64_t)c * nchunks * 4;
        for (int k = 0; k < nchunks; ++k) {
            t1 += p[4 * k];
            t2 += p[4 * k + 1];
            tx += p[4 * k + 2];
            ty += p[4 * k + 3];
        }
        const double lc = lam[c];
        eps[c] = sqrt(t1 + t2) / ((1.0 + lc) * sqrt(tx + ty));
    }
}

// ---------------------------------------------------------------- CG
// Called by every block of a CG launch after its chunk sum is stored: true in
// the block that arrives last (device-scope counter s.ticket, reset by that
// block), which then runs the finishing step in its first wavefront.  Every
// other block has read rr / active / any_active before it arrived, so the
// finishing step may overwrite them.
__device__ bool cg_arrive_last(const CgState& s) {
    __shared__ int last;
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned total = gridDim.x * gridDim.y;
        last = atomicAdd(s.ticket, 1u) == total - 1 ? 1 : 0;
    }
    __syncthreads();
    if (!last) return false;
    __threadfence();
    if (threadIdx.x == 0) *s.ticket = 0u;
    return true;
}

// one wavefront: rr = bb = |b|^2, active = rr > tol^2 bb, any_active
__device__ void cg_init_fin_wave(int w, int nchunks, const CgState& s, double tol) {
    int any = 0;
    for (int c = threadIdx.x; c < w; c += 64) {
        double t = 0;
        for (int k = 0; k < nchunks; ++k) t += s.part[(int64_t)c * nchunks + k];
        s.rr[c] = t;
        s.bb[c] = t;
        const int a = t > tol * tol * t ? 1 : 0;
        s.active[c] = a;
        any |= a;
    }
    any = __any(any) ? 1 : 0;
    if (threadIdx.x == 0) {
        *s.any_active = any;
        if (s.note) __hip_atomic_store(s.note, 2ull * s.seq + (unsigned long long)any, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// one wavefront: alpha = rr / (p . q); a column with p^T A p <= 0 stops
__device__ void cg_alpha_fin_wave(int w, int nchunks, const CgState& s) {
    int na = 0;
    for (int c = threadIdx.x; c < w; c += 64) {
        double a = 0.0;
        if (s.active[c]) {
            ++na;
            double pq = 0;
            for (int k = 0; k < nchunks; ++k) pq += s.part[(int64_t)c * nchunks + k];
            if (pq > 0.0)
                a = s.rr[c] / pq;
            else
                s.active[c] = 0;   // breakdown: p^T A p <= 0 (singular operator)
        }
        s.alpha[c] = a;
    }
    // count the columns that received an apply (fixed-order wave sum of ints)
    for (int off = 32; off >= 1; off >>= 1) na += __shfl_xor(na, off, 64);
    if (threadIdx.x == 0) *s.napplies += (unsigned long long)na;
}

// finishing steps as launches of their own, for grids too large for one
// device-scope arrival counter
__global__ __launch_bounds__(64) void cg_init_fin_kernel(int w, int nchunks, CgState s, double tol) {
    cg_init_fin_wave(w, nchunks, s, tol);
}
__global__ __launch_bounds__(64) void cg_alpha_fin_kernel(int w, int nchunks, CgState s) {
    if (*s.any_active == 0) return;
    cg_alpha_fin_wave(w, nchunks, s);
}

__global__ __launch_bounds__(NT) void cg_init_kernel(int n, int w, int nchunks, CgState s,
                                                     const double* __restrict__ B, int64_t ldb, double tol,
                                                     int fin) {
    __shared__ double red[NT / WAVE];
    const int j = blockIdx.y, ch = blockIdx.x;
    const int rows = (n + nchunks - 1) / nchunks;
    const int r0 = ch * rows, r1 = min(n, r0 + rows);
    const int64_t off = (int64_t)j * n;
    double acc = 0;
    for (int i = r0 + threadIdx.x; i < r1; i += NT) {
        const double b = B[(int64_t)j * ldb + i];
        s.X[off + i] = 0.0;
        s.R[off + i] = b;
        s.P[off + i] = b;
        acc += b * b;
    }
    acc = block_sum<NT>(acc, red);
    if (threadIdx.x == 0) s.part[(int64_t)j * nchunks + ch] = acc;
    if (fin && cg_arrive_last(s) && threadIdx.x < 64) cg_init_fin_wave(w, nchunks, s, tol);
}

__global__ __launch_bounds__(NT) void cg_alpha_kernel(int n, int w, int nchunks, CgState s, int fin) {
    __shared__ double red[NT / WAVE];
    if (*s.any_active == 0) return;
    const int j = blockIdx.y, ch = blockIdx.x;
    const int rows = (n + nchunks - 1) / nchunks;
    const int r0 = ch * rows, r1 = min(n, r0 + rows);
    const int64_t off = (int64_t)j * n;
    double acc = 0;
    if (s.active[j])
        for (int i = r0 + threadIdx.x; i < r1; i += NT) acc += s.P[off + i] * s.Q[off + i];
    acc = block_sum<NT>(acc, red);
    if (threadIdx.x == 0) s.part[(int64_t)j * nchunks + ch] = acc;
    if (fin && cg_arrive_last(s) && threadIdx.x < 64) cg_alpha_fin_wave(w, nchunks, s);
}

// beta, rr, active and any_active from the per-chunk sums of |r|^2, run by
// one wavefront (lanes over columns)
__device__ void cg_fin_wave(int w, int nchunks, const CgState& s, double tol) {
    int any = 0;
    for (int c = threadIdx.x; c < w; c += 64) {
        if (s.active[c]) {
            double t = 0;
            for (int k = 0; k < nchunks; ++k) t += s.part[(int64_t)c * nchunks + k];
            s.beta[c] = t / s.rr[c];
            s.rr[c] = t;
            const int a = t > tol * tol * s.bb[c] ? 1 : 0;
            s.active[c] = a;
            any |= a;
        }
    }
    any = __any(any) ? 1 : 0;
    if (threadIdx.x == 0) {
        *s.any_active = any;
        if (s.note) __hip_atomic_store(s.note, 2ull * s.seq + (unsigned long long)any, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

__global__ __launch_bounds__(64) void cg_update_fin_kernel(int w, int nchunks, CgState s, double tol) {
    if (*s.any_active == 0) return;
    cg_fin_wave(w, nchunks, s, tol);
}

constexpr int kFold = 128;   // tiles per block of cg_fold_pq_kernel

// folded[b * 32 + j] = sum of pq[k * 32 + j] over tiles k in [128 b, 128 b + 128):
// thread (j = t % 32, s = t / 32) sums k = 128 b + s, + 8, ..., the eight
// partial sums are then added in order of s
__global__ __launch_bounds__(NT) void cg_fold_pq_kernel(int ntiles, const double* __restrict__ pq,
                                                        double* __restrict__ folded, const int* __restrict__ any) {
    static_assert(NT == 256, "32 columns x 8 tile phases");
    __shared__ double red[8][32];
    if (*any == 0) return;
    const int j = threadIdx.x % 32, sub = threadIdx.x / 32;
    const int k0 = blockIdx.x * kFold;
    double acc = 0.0;
    for (int k = k0 + sub; k < min(ntiles, k0 + kFold); k += 8) acc += pq[(int64_t)k * 32 + j];
    red[sub][j] = acc;
    __syncthreads();
    if (threadIdx.x < 32) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) t += red[q][j];
        folded[(int64_t)blockIdx.x * 32 + j] = t;
    }
}

__global__ __launch_bounds__(NT) void cg_update_tiles_kernel(int n, int w, int nchunks, int ntiles,
                                                             const double* __restrict__ pq, CgState s, double tol,
                                                             int fin) {
    __shared__ double red[NT / WAVE];
    if (*s.any_active == 0) return;
    const int j = blockIdx.y, ch = blockIdx.x;
    const int rows = (n + nchunks - 1) / nchunks;
    const int r0 = ch * rows, r1 = min(n, r0 + rows);
    const int64_t off = (int64_t)j * n;
    double acc = 0;
    if (s.active[j]) {
        double t = 0.0;
        for (int k = threadIdx.x; k < ntiles; k += NT) t += pq[(int64_t)k * 32 + j];
        t = block_sum<NT>(t, red);
        if (ch == 0 && threadIdx.x == 0) atomicAdd(s.napplies, 1ull);
        if (t > 0.0) {
            const double a = s.rr[j] / t;
            if (ch == 0 && threadIdx.x == 0) s.alpha[j] = a;
            for (int i = r0 + threadIdx.x; i < r1; i += NT) {
                s.X[off + i] += a * s.P[off + i];
                const double r = s.R[off + i] - a * s.Q[off + i];
                s.R[off + i] = r;
                acc += r * r;
            }
        } else {
            // breakdown: p^T A p <= 0 (singular operator); the column stops and
            // cg_update_fin leaves it inactive
            if (ch == 0 && threadIdx.x == 0) s.alpha[j] = 0.0;
            acc = -1.0;
        }
    }
    acc = block_sum<NT>(acc, red);
    if (threadIdx.x == 0) s.part[(int64_t)j * nchunks + ch] = acc;
    if (fin && cg_arrive_last(s) && threadIdx.x < 64) cg_fin_wave(w, nchunks, s, tol);
}

__global__ __launch_bounds__(NT) void cg_update_kernel(int n, int w, int nchunks, CgState s, double tol, int fin) {
    __shared__ double red[NT / WAVE];
    if (*s.any_active == 0) return;
    const int j = blockIdx.y, ch = blockIdx.x;
    const int rows = (n + nchunks - 1) / nchunks;
    const int r0 = ch * rows, r1 = min(n, r0 + rows);
    const int64_t off = (int64_t)j * n;
    double acc = 0;
    if (s.active[j]) {
        const double a = s.alpha[j];
        for (int i = r0 + threadIdx.x; i < r1; i += NT) {
            s.X[off + i] += a * s.P[off + i];
            const double r = s.R[off + i] - a * s.Q[off + i];
            s.R[off + i] = r;
            acc += r * r;
        }
    }
    acc = block_sum<NT>(acc, red);
    if (threadIdx.x == 0) s.part[(int64_t)j * nchunks + ch] = acc;
    if (fin && cg_arrive_last(s) && threadIdx.x < 64) cg_fin_wave(w, nchunks, s, tol);
}

// one block: beta, rr, active (relative residual test), any_active
__global__ __launch_bounds__(NT) void cg_direction_kernel(int n, int w, CgState s) {
    if (*s.any_active == 0) return;
    const int j = blockIdx.y;
    if (!s.active[j]) return;
    const double b = s.beta[j];
    const int64_t off = (int64_t)j * n;
    for (int i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT)
        s.P[off + i] = s.R[off + i] + b * s.P[off + i];
}

// Coefficients of the first-order biorthogonality correction of returned
// pairs: with G = X^T Y (c x c, ld ldg), Bx = I - (G - I)^T / 2 and
// By = I - (G - I) / 2, so that (X Bx)^T (Y By) = I + O(|G - I|^2).
__global__ __launch_bounds__(NT) void biorth_fix_kernel(int c, const double* __restrict__ G, int64_t ldg,
                                                        double* __restrict__ Bx, double* __restrict__ By,
                                                        int64_t ldb) {
    for (int idx = blockIdx.x * NT + threadIdx.x; idx < c * c; idx += gridDim.x * NT) {
        const int i = idx % c, j = idx / c;
        const double d = (i == j) ? 1.0 : 0.0;
        Bx[(int64_t)j * ldb + i] = d - 0.5 * (G[(int64_t)i * ldg + j] - d);
        By[(int64_t)j * ldb + i] = d - 0.5 * (G[(int64_t)j * ldg + i] - d);
    }
}

__global__ __launch_bounds__(NT) void gs_rhs_kernel(int n, const double* __restrict__ S, int64_t lds,
                                                    const double* __restrict__ T, const double* __restrict__ U,
                                                    int64_t ldt, const int* __restrict__ win,
                                                    const double* __restrict__ lam_w, double* __restrict__ out,
                                                    int64_t ldo) {
    const int j = blockIdx.y;
    const int g = win[j];
    const double l = lam_w[j];
    for (int i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT) {
        const double sv = S ? S[(int64_t)j * lds + i] : 0.0;
        out[(int64_t)j * ldo + i] = l * (sv + T[(int64_t)g * ldt + i]) - U[(int64_t)g * ldt + i];
    }
}

__global__ __launch_bounds__(NT) void copy_cols_kernel(int n, const double* __restrict__ in, int64_t ldi,
                                                       double* __restrict__ out, int64_t ldo) {
    const int j = blockIdx.y;
    for (int i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT)
        out[(int64_t)j * ldo + i] = in[(int64_t)j * ldi + i];
}

__global__ __launch_bounds__(NT) void sub_cols_kernel(int n, const double* __restrict__ A, int64_t lda,
                                                      const double* __restrict__ B, int64_t ldb,
                                                      double* __restrict__ C, int64_t ldc) {
    const int j = blockIdx.y;
    for (int i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT)
        C[(int64_t)j * ldc + i] = A[(int64_t)j * lda + i] - B[(int64_t)j * ldb + i];
}

// U = Y + X, V = Y - X (n x cols)
__global__ __launch_bounds__(NT) void xy_to_uv_kernel(int n, const double* __restrict__ X, const double* __restrict__ Y,
                                                      int64_t ldxy, double* __restrict__ U, double* __restrict__ V,
                                                      int64_t lduv) {
    const int j = blockIdx.y;
    for (int i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT) {
        const double x = X[(int64_t)j * ldxy + i], y = Y[(int64_t)j * ldxy + i];
        U[(int64_t)j * lduv + i] = y + x;
        V[(int64_t)j * lduv + i] = y - x;
    }
}

__global__ __launch_bounds__(1024) void max_offidentity_kernel(int d, const double* __restrict__ S, int64_t lds,
                                                               double* out) {
    __shared__ double red[1024 / WAVE];
    double m = 0.0;
    for (int idx = threadIdx.x; idx < d * d; idx += 1024) {
        const int i = idx % d, j = idx / d;
        const double v = S[(int64_t)j * lds + i] - (i == j ? 1.0 : 0.0);
        m = fmax(m, fabs(v));
        if (!(v == v)) m = INFINITY;   // NaN -> force a restore / error path
    }
    m = wave_max(m);
    const int lane = threadIdx.x % WAVE, wid = threadIdx.x / WAVE;
    if (lane == 0) red[wid] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < 1024 / WAVE; ++i) t = fmax(t, red[i]);
        *out = t;
    }
}

// Philox4x32-10 (Salmon et al., "Parallel random numbers: as easy as 1, 2, 3", SC'11)
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)M0 * c[0];
        const uint64_t p1 = (uint64_t)M1 * c[2];
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += W0;
        k1 += W1;
    }
}

__global__ __launch_bounds__(NT) void philox_normal_kernel(int n, uint64_t seed, double* __restrict__ out,
                                                           int64_t ld) {
    const int j = blockIdx.y;
    for (int i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT) {
        const uint64_t ctr = (uint64_t)i + (uint64_t)j * (uint64_t)n;
        uint32_t c[4] = {(uint32_t)ctr, (uint32_t)(ctr >> 32), 0u, 0u};
        philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
        const double u1 = ((double)(c[0] >> 5) * 67108864.0 + (double)(c[1] >> 6) + 0.5) * (1.0 / 9007199254740992.0);
        const double u2 = ((double)(c[2] >> 5) * 67108864.0 + (double)(c[3] >> 6)) * (1.0 / 9007199254740992.0);
        out[(int64_t)j * ld + i] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
    }
}

__global__ __launch_bounds__(NT) void sign_normalise_kernel(int n, double* __restrict__ X, double* __restrict__ Y,
                                                            int64_t ld) {
    __shared__ double sv[NT];
    __shared__ int si[NT];
    const int j = blockIdx.x;
    double best = -1.0;
    int bi = 0x7fffffff;
    double sgn = 1.0;
    for (int i = threadIdx.x; i < n; i += NT) {
        const double v = X[(int64_t)j * ld + i];
        const double a = fabs(v);
        if (a > best) {
            best = a;
            bi = i;
            sgn = v < 0 ? -1.0 : 1.0;
        }
    }
    sv[threadIdx.x] = best * sgn;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const double a = fabs(sv[threadIdx.x]), b = fabs(sv[threadIdx.x + s]);
            if (b > a || (b == a && si[threadIdx.x + s] < si[threadIdx.x])) {
                sv[threadIdx.x] = sv[threadIdx.x + s];
                si[threadIdx.x] = si[threadIdx.x + s];
            }
        }
        __syncthreads();
    }
    const double f = sv[0] < 0 ? -1.0 : 1.0;
    if (f < 0)
        for (int i = threadIdx.x; i < n; i += NT) {
            X[(int64_t)j * ld + i] = -X[(int64_t)j * ld + i];
            Y[(int64_t)j * ld + i] = -Y[(int64_t)j * ld + i];
        }
}

__global__ __launch_bounds__(NT) void combine_ab_kernel(int64_t total, double* __restrict__ K, double* __restrict__ M) {
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < total; i += (int64_t)gridDim.x * NT) {
        const double a = K[i], b = M[i];
        K[i] = a - b;
        M[i] = a + b;
    }
}

inline dim3 grid_rows(int n, int cols, int max_x = 1024) {
    return dim3(std::max(1, std::min(max_x, (n + NT - 1) / NT)), cols);
}
}  // namespace

hipError_t diag_scale(hipStream_t st, int n, int cols, const double* delta, const double* X, int64_t ldx,
                      double* Y, int64_t ldy, const int* active_flag) {
    if (cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(diag_scale_kernel, grid_rows(n, cols, 512), dim3(NT), 0, st, n, cols, delta, X, ldx, Y, ldy,
                       active_flag);
    return hipGetLastError();
}

hipError_t diag_scale_pq(hipStream_t st, int n, int cols, const double* delta, const double* X, int64_t ldx,
                         double* Y, int64_t ldy, double* pq, const int* active_flag) {
    if (cols <= 0) return hipSuccess;
    if (cols > 32) return hipErrorInvalidValue;
    hipLaunchKernelGGL(diag_scale_pq_kernel, dim3((n + 63) / 64), dim3(NT), 0, st, n, cols, delta, X, ldx, Y, ldy, pq,
                       active_flag);
    return hipGetLastError();
}

hipError_t diag_dir_scale_pq(hipStream_t st, int n, int cols, const double* delta, double* P, const double* R,
                             const double* beta, const int* active, double* Q, double* pq, const int* active_flag) {
    if (cols <= 0) return hipSuccess;
    if (cols > 32) return hipErrorInvalidValue;
    hipLaunchKernelGGL(diag_dir_scale_pq_kernel, dim3((n + 63) / 64), dim3(NT), 0, st, n, cols, delta, P, R, beta,
                       active, Q, pq, active_flag);
    return hipGetLastError();
}

hipError_t residual_eps(hipStream_t st, int n, int cols, const double* X, const double* Y, const double* KX,
                        const double* MY, int64_t ld, const double* lam, double* eps, double* part,
                        size_t part_elems, unsigned* ticket) {
    if (cols <= 0) return hipSuccess;
    int nch = chunks_for(n, cols);
    while ((size_t)nch * cols * 4 > part_elems && nch > 1) nch /= 2;
    hipLaunchKernelGGL(residual_kernel, dim3(nch, cols), dim3(NT), 0, st, n, cols, nch, X, Y, KX, MY, ld, lam, eps,
                       part, ticket);
    hipLaunchKernelGGL(residual_fin_kernel, dim3(1), dim3(NT), 0, st, cols, nch, part, lam, eps);
    return hipGetLastError();
}

// relative drift of carried operator images: per column of two pairs
// (A1 vs B1, A2 vs B2) the partial sums of |a - b|^2 and |b|^2 over a chunk
__global__ __launch_bounds__(NT) void drift_kernel(int n, int cols, int nchunks, const double* __restrict__ A1,
                                                   const double* __restrict__ B1, const double* __restrict__ A2,
                                                   const double* __restrict__ B2, int64_t ld,
                                                   double* __restrict__ part) {
    __shared__ double red[NT / WAVE];
    const int j = blockIdx.y, ch = blockIdx.x, side = blockIdx.z;
    const double* Aa = side ? A2 : A1;
    const double* Bb = side ? B2 : B1;
    const int rows = (n + nchunks - 1) / nchunks;
    const int r0 = ch * rows, r1 = min(n, r0 + rows);
    double dd = 0.0, bb = 0.0;
    for (int i = r0 + threadIdx.x; i < r1; i += NT) {
        const double b = Bb[(int64_t)j * ld + i];
        const double e = Aa[(int64_t)j * ld + i] - b;
        dd += e * e;
        bb += b * b;
    }
    dd = block_sum<NT>(dd, red);
    bb = block_sum<NT>(bb, red);
    if (threadIdx.x == 0) {
        double* p = part + (((int64_t)side * cols + j) * nchunks + ch) * 2;
        p[0] = dd;
        p[1] = bb;
    }
}

__global__ __launch_bounds__(64) void drift_fin_kernel(int cols, int nchunks, const double* __restrict__ part,
                                                       double* __restrict__ out) {
    double mx = 0.0;
    for (int c = threadIdx.x; c < 2 * cols; c += 64) {
        double dd = 0.0, bb = 0.0;
        for (int k = 0; k < nchunks; ++k) {
            dd += part[((int64_t)c * nchunks + k) * 2];
            bb += part[((int64_t)c * nchunks + k) * 2 + 1];
        }
        const double r = bb > 0.0 ? sqrt(dd / bb) : (dd > 0.0 ? INFINITY : 0.0);
        mx = fmax(mx, r != r ? INFINITY : r);
    }
    mx = wave_max(mx);
    if (threadIdx.x == 0) *out = mx;
}

// the last-arriving block finishes a CG launch of up to 512 blocks; larger
// grids (the arrivals on one counter would serialise) take a separate launch
static int fuse_fin(int nch, int w) { return nch * w <= 512 ? 1 : 0; }

static int cg_chunks(int n, int w, const CgState& s) {
    int nch = chunks_for(n, w);
    while ((size_t)nch * w > s.part_elems && nch > 1) nch /= 2;
    return nch;
}

hipError_t cg_init(hipStream_t st, int n, int w, const CgState& s, const double* B, int64_t ldb, double tol) {
    const int nch = cg_chunks(n, w, s);
    const int fin = fuse_fin(nch, w);
    hipLaunchKernelGGL(cg_init_kernel, dim3(nch, w), dim3(NT), 0, st, n, w, nch, s, B, ldb, tol, fin);
    if (!fin) hipLaunchKernelGGL(cg_init_fin_kernel, dim3(1), dim3(64), 0, st, w, nch, s, tol);
    return hipGetLastError();
}
hipError_t cg_alpha(hipStream_t st, int n, int w, const CgState& s) {
    const int nch = cg_chunks(n, w, s);
    const int fin = fuse_fin(nch, w);
    hipLaunchKernelGGL(cg_alpha_kernel, dim3(nch, w), dim3(NT), 0, st, n, w, nch, s, fin);
    if (!fin) hipLaunchKernelGGL(cg_alpha_fin_kernel, dim3(1), dim3(64), 0, st, w, nch, s);
    return hipGetLastError();
}
size_t cg_pq_elems(int ntiles) { return (size_t)(ntiles + (ntiles + kFold - 1) / kFold) * 32; }

hipError_t cg_update_tiles(hipStream_t st, int n, int w, int ntiles, double* pq, const CgState& s, double tol) {
    if (ntiles > 8 * kFold) {
        // every update block would otherwise walk the whole strided tile list
        // (thousands of tiles at n = 262144; at n <= 65536 that walk costs less
        // than the extra launch)
        const int nb = (ntiles + kFold - 1) / kFold;
        double* folded = pq + (size_t)ntiles * 32;
        hipLaunchKernelGGL(cg_fold_pq_kernel, dim3(nb), dim3(NT), 0, st, ntiles, pq, folded, s.any_active);
        pq = folded;
        ntiles = nb;
    }
    const int nch = cg_chunks(n, w, s);
    const int fin = fuse_fin(nch, w);
    hipLaunchKernelGGL(cg_update_tiles_kernel, dim3(nch, w), dim3(NT), 0, st, n, w, nch, ntiles, pq, s, tol, fin);
    if (!fin) hipLaunchKernelGGL(cg_update_fin_kernel, dim3(1), dim3(64), 0, st, w, nch, s, tol);
    return hipGetLastError();
}
hipError_t cg_update(hipStream_t st, int n, int w, const CgState& s, double tol) {
    const int nch = cg_chunks(n, w, s);
    const int fin = fuse_fin(nch, w);
    hipLaunchKernelGGL(cg_update_kernel, dim3(nch, w), dim3(NT), 0, st, n, w, nch, s, tol, fin);
    if (!fin) hipLaunchKernelGGL(cg_update_fin_kernel, dim3(1), dim3(64), 0, st, w, nch, s, tol);
    return hipGetLastError();
}
hipError_t cg_direction(hipStream_t st, int n, int w, const CgState& s) {
    hipLaunchKernelGGL(cg_direction_kernel, grid_rows(n, w, 256), dim3(NT), 0, st, n, w, s);
    return hipGetLastError();
}

hipError_t biorth_fix_coef(hipStream_t st, int c, const double* G, int64_t ldg, double* Bx, double* By, int64_t ldb) {
    if (c <= 0) return hipSuccess;
    hipLaunchKernelGGL(biorth_fix_kernel, dim3((c * c + NT - 1) / NT), dim3(NT), 0, st, c, G, ldg, Bx, By, ldb);
    return hipGetLastError();
}

hipError_t gs_rhs(hipStream_t st, int n, int w, const double* S, int64_t lds, const double* T, const double* U,
                  int64_t ldt, const int* win, const double* lam_w, double* out, int64_t ldo) {
    if (w <= 0) return hipSuccess;
    hipLaunchKernelGGL(gs_rhs_kernel, grid_rows(n, w, 256), dim3(NT), 0, st, n, S, lds, T, U, ldt, win, lam_w, out,
                       ldo);
    return hipGetLastError();
}

hipError_t copy_cols(hipStream_t st, int n, int cols, const double* in, int64_t ldi, double* out, int64_t ldo) {
    if (cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(copy_cols_kernel, grid_rows(n, cols, 256), dim3(NT), 0, st, n, in, ldi, out, ldo);
    return hipGetLastError();
}

hipError_t xy_to_uv(hipStream_t st, int n, int cols, const double* X, const double* Y, int64_t ldxy, double* U,
                    double* V, int64_t lduv) {
    if (cols <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL(xy_to_uv_kernel, grid_rows(n, cols, 256), dim3(NT), 0, st, n, X, Y, ldxy, U, V, lduv);
    return hipGetLastError();
}

hipError_t sub_cols(hipStream_t st, int n, int cols, const double* A, int64_t lda, const double* B, int64_t ldb,
                    double* C, int64_t ldc) {
    if (cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(sub_cols_kernel, grid_rows(n, cols, 256), dim3(NT), 0, st, n, A, lda, B, ldb, C, ldc);
    return hipGetLastError();
}

hipError_t combine_ab(hipStream_t st, int64_t n, double* K, double* M) {
    const int64_t total = n * n;
    hipLaunchKernelGGL(combine_ab_kernel, dim3((unsigned)std::min<int64_t>(8192, (total + NT - 1) / NT)), dim3(NT), 0,
                       st, total, K, M);
    return hipGetLastError();
}

hipError_t max_offidentity(hipStream_t st, int d, const double* S, int64_t lds, double* out) {
    hipLaunchKernelGGL(max_offidentity_kernel, dim3(1), dim3(1024), 0, st, d, S, lds, out);
    return hipGetLastError();
}

hipError_t philox_normal(hipStream_t st, int n, int cols, uint64_t seed, double* out, int64_t ld) {
    if (cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(philox_normal_kernel, grid_rows(n, cols, 256), dim3(NT), 0, st, n, seed, out, ld);
    return hipGetLastError();
}

hipError_t sign_normalise(hipStream_t st, int n, int cols, double* X, double* Y, int64_t ld) {
    if (cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(sign_normalise_kernel, dim3(cols), dim3(NT), 0, st, n, X, Y, ld);
    return hipGetLastError();
}

hipError_t image_drift(hipStream_t st, int n, int cols, const double* A1, const double* B1, const double* A2,
                       const double* B2, int64_t ld, double* part, size_t part_elems, double* out) {
    if (cols <= 0) return hipSuccess;
    int nch = chunks_for(n, cols);
    while ((size_t)nch * cols * 4 > part_elems && nch > 1) nch /= 2;
    hipLaunchKernelGGL(drift_kernel, dim3(nch, cols, 2), dim3(NT), 0, st, n, cols, nch, A1, B1, A2, B2, ld, part);
    hipLaunchKernelGGL(drift_fin_kernel, dim3(1), dim3(64), 0, st, cols, nch, part, out);
    return hipGetLastError();
}

}  // namespace lrep
