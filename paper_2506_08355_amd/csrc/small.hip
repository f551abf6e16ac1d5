// One-workgroup FP64 kernels on the small (d <= 128) matrices of the BOSP
// iteration, for gfx950:
//
//  small_lrep  the projected structured LREP of Step 3: two Cholesky
//              factorisations and one SVD (Section 3.2 / cost discussion of
//              Section 3.3).  The SVD of B = L2^T L1 is a one-sided
//              (Hestenes) Jacobi iteration with the round-robin pair ordering;
//              the stacked columns [B; L1] live in registers, 8 per wavefront,
//              and only the two columns that cross a wavefront boundary move
//              through LDS at each step.  At convergence column c holds
//              [psi_c sigma_c; L1 phi_c], so
//                  Y^_c = L1 phi_c / sqrt(sigma_c),
//                  X^_c = L2 psi_c / sqrt(sigma_c) = L2 (B phi_c) / sigma_c^(3/2).
//  step5_pq    Step 5 in coefficient space (equation for P^, Q^) with the
//              small MGS-Biorth.
//  coef_mgs    the coefficient pass of block MGS-Biorth: the recurrence of
//              Algorithm MGS-Biorth run on coefficient vectors with every
//              inner product taken from the Gram matrix of [X Y].
#include "device.hpp"
#include "kernels.hpp"

namespace lrep {

namespace {

constexpr double JACOBI_TOL = 1e-15;
constexpr int JACOBI_MAX_SWEEPS = 40;

// Cholesky of the symmetric part of A (d x d, lda) into L (lower, ld kMaxD,
// strict upper part zeroed).  LDS matrix `S` has room for kMaxD x (kMaxD+1).
// Returns false (uniformly) if a pivot is not positive.
__device__ bool chol_lds(int d, const double* __restrict__ A, int64_t lda, double* __restrict__ L,
                         double* S, int* flag) {
    const int tid = threadIdx.x, nt = blockDim.x;
    constexpr int LD = kMaxD + 1;
    for (int idx = tid; idx < d * d; idx += nt) {
        const int i = idx % d, j = idx / d;
        S[i * LD + j] = 0.5 * (A[(int64_t)j * lda + i] + A[(int64_t)i * lda + j]);
    }
    if (tid == 0) *flag = 0;
    __syncthreads();
    for (int k = 0; k < d; ++k) {
        if (tid == 0) {
            const double v = S[k * LD + k];
            if (!(v > 0.0)) *flag = 1;
            else S[k * LD + k] = sqrt(v);
        }
        __syncthreads();
        if (*flag) return false;
        const double piv = S[k * LD + k];
        for (int i = k + 1 + tid; i < d; i += nt) S[i * LD + k] /= piv;
        __syncthreads();
        const int m = d - k - 1;
        for (int idx = tid; idx < m * m; idx += nt) {
            const int i = k + 1 + idx % m, j = k + 1 + idx / m;
            if (j <= i) S[i * LD + j] -= S[i * LD + k] * S[j * LD + k];
        }
        __syncthreads();
    }
    for (int idx = tid; idx < kMaxD * kMaxD; idx += nt) {
        const int i = idx % kMaxD, j = idx / kMaxD;
        L[(int64_t)j * kMaxD + i] = (i < d && j < d && j <= i) ? S[i * LD + j] : 0.0;
    }
    __syncthreads();
    return true;
}

template <int D>
__global__ __launch_bounds__(D * 8) void small_lrep_kernel(int d, const double* __restrict__ Kh,
                                                          const double* __restrict__ Mh, int64_t ldh,
                                                          double* __restrict__ lam, double* __restrict__ Xh,
                                                          double* __restrict__ Yh, double* __restrict__ scratch,
                                                          int* __restrict__ status) {
    constexpr int NW = D / 8;            // wavefronts
    constexpr int NTH = NW * WAVE;
    constexpr int E = (2 * D) / WAVE;    // stacked elements per lane per column
    constexpr int M = D / 2;             // pairs
    constexpr size_t CHOL = (size_t)kMaxD * (kMaxD + 1);
    constexpr size_t XCH = (size_t)2 * 2 * NW * 2 * D;
    constexpr size_t LDSN = CHOL > XCH ? CHOL : XCH;
    __shared__ double lds[LDSN];
    __shared__ double sig[D];
    __shared__ double bnorm[D];
    __shared__ int rank_of[D];
    __shared__ int flag;
    __shared__ double wmax[NW];

    const int tid = threadIdx.x, lane = tid % WAVE, w = tid / WAVE;
    double* L1 = scratch;
    double* L2 = scratch + kMaxD * kMaxD;
    double* T = scratch + 2 * kMaxD * kMaxD;

    if (!chol_lds(d, Kh, ldh, L1, lds, &flag) || !chol_lds(d, Mh, ldh, L2, lds, &flag)) {
        if (tid == 0) status[ST_NOTSPD] = 1;
        return;
    }

    // ---- load stacked columns [B; L1], B = L2^T L1 (upper-times-lower) -------
    // slots 0..3 = T[4w..4w+3] (tournament "top" row), 4..7 = Bt[4w..4w+3]
    double col[8][E];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const int k = 4 * w + (s & 3);
        const int c = (s < 4) ? 2 * k : 2 * k + 1;   // initial column in this slot
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int row = e * WAVE + lane;
            double v = 0.0;
            if (c < d) {
                if (row < D) {
                    if (row < d) {
                        // B[row][c] = sum_k L2[k][row] L1[k][c], k >= max(row, c)
                        const int k0 = row > c ? row : c;
                        for (int kk = k0; kk < d; ++kk)
                            v += L2[(int64_t)row * kMaxD + kk] * L1[(int64_t)c * kMaxD + kk];
                    }
                } else {
                    const int r = row - D;
                    if (r < d) v = L1[(int64_t)c * kMaxD + r];
                }
            }
            col[s][e] = v;
        }
    }
    __syncthreads();   // LDS (Cholesky) is reused below

    double* xT = lds;                       // [2][NW][2D]
    double* xB = lds + 2 * NW * 2 * D;      // [2][NW][2D]

    for (int sweep = 0; sweep < JACOBI_MAX_SWEEPS; ++sweep) {
        double offmax = 0.0;
        for (int step = 0; step < D - 1; ++step) {
            // rotate the four pairs (slot i, slot 4+i)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                double al = 0, be = 0, ga = 0;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    if (e * WAVE + lane < D) {
                        const double a = col[i][e], b = col[4 + i][e];
                        al += a * a;
                        be += b * b;
                        ga += a * b;
                    }
                }
                al = wave_sum(al);
                be = wave_sum(be);
                ga = wave_sum(ga);
                if (ga != 0.0) {
                    const double rel = fabs(ga) / sqrt(al * be);
                    offmax = fmax(offmax, rel);
                    if (rel > JACOBI_TOL) {
                        const double zeta = (be - al) / (2.0 * ga);
                        const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                        const double c = 1.0 / sqrt(1.0 + t * t);
                        const double s = c * t;
#pragma unroll
                        for (int e = 0; e < E; ++e) {
                            const double a = col[i][e], b = col[4 + i][e];
                            col[i][e] = c * a - s * b;
                            col[4 + i][e] = s * a + c * b;
                        }
                    }
                }
            }
            // round-robin move; only boundary columns cross wavefronts
            const int par = step & 1;
            double* oT = xT + ((size_t)par * NW + w) * 2 * D;
            double* oB = xB + ((size_t)par * NW + w) * 2 * D;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                oT[e * WAVE + lane] = col[3][e];   // T[4w+3] -> wave w+1
                oB[e * WAVE + lane] = col[4][e];   // Bt[4w]  -> wave w-1
            }
            __syncthreads();
            const double* iT = xT + ((size_t)par * NW + (w > 0 ? w - 1 : 0)) * 2 * D;
            const double* iB = xB + ((size_t)par * NW + (w < NW - 1 ? w + 1 : 0)) * 2 * D;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const double t0 = col[0][e], t1 = col[1][e], t2 = col[2][e], t3 = col[3][e];
                const double b0 = col[4][e], b1 = col[5][e], b2 = col[6][e], b3 = col[7][e];
                if (w == 0) {
                    col[0][e] = t0;        // fixed
                    col[1][e] = b0;
                } else {
                    col[0][e] = iT[e * WAVE + lane];
                    col[1][e] = t0;
                }
                col[2][e] = t1;
                col[3][e] = t2;
                col[4][e] = b1;
                col[5][e] = b2;
                col[6][e] = b3;
                col[7][e] = (w == NW - 1) ? t3 : iB[e * WAVE + lane];
            }
        }
        // sweep convergence (uniform decision)
        if (lane == 0) wmax[w] = offmax;
        __syncthreads();
        double om = 0.0;
#pragma unroll
        for (int i = 0; i < NW; ++i) om = fmax(om, wmax[i]);
        __syncthreads();
        if (om <= JACOBI_TOL) break;
    }

    // ---- singular values, ordering, outputs --------------------------------
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        double tn = 0, bn = 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const double v = col[s][e];
            if (e * WAVE + lane < D) tn += v * v;
            else bn += v * v;
        }
        tn = wave_sum(tn);
        bn = wave_sum(bn);
        const int slot = 8 * w + s;
        if (lane == 0) {
            sig[slot] = sqrt(tn);
            bnorm[slot] = bn;
        }
    }
    __syncthreads();
    // rank among live (non-padding) columns: ascending sigma, ties by slot
    for (int a = tid; a < D; a += NTH) {
        int r = -1;
        if (bnorm[a] > 0.0) {
            r = 0;
            for (int b = 0; b < D; ++b)
                if (bnorm[b] > 0.0 && (sig[b] < sig[a] || (sig[b] == sig[a] && b < a))) ++r;
        }
        rank_of[a] = r;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const int slot = 8 * w + s;
        const int r = rank_of[slot];
        if (r < 0 || r >= d) continue;
        const double sg = sig[slot];
        const double isq = 1.0 / sqrt(sg);
        const double i32 = isq / sg;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int row = e * WAVE + lane;
            if (row < D) {
                if (row < d) T[(int64_t)r * kMaxD + row] = col[s][e] * i32;
            } else if (row - D < d) {
                Yh[(int64_t)r * kMaxD + (row - D)] = col[s][e] * isq;
            }
        }
        if (lane == 0) lam[r] = sg;
    }
    __syncthreads();
    __threadfence_block();
    // X^ = L2 T (L2 lower triangular)
    for (int idx = tid; idx < d * d; idx += NTH) {
        const int i = idx % d, c = idx / d;
        double v = 0.0;
        for (int k = 0; k <= i; ++k) v += L2[(int64_t)k * kMaxD + i] * T[(int64_t)c * kMaxD + k];
        Xh[(int64_t)c * kMaxD + i] = v;
    }
}

// ---------------------------------------------------------------------------
// Step 5.  256 threads.  V, U columns (d x nw) live in LDS.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void step5_kernel(int d, int hi, const double* __restrict__ Xh,
                                                    const double* __restrict__ Yh, const int* __restrict__ win,
                                                    int nw, double* __restrict__ Ph, double* __restrict__ Qh,
                                                    double* __restrict__ C, int* __restrict__ status,
                                                    double cos_tol, double dep_tol) {
    __shared__ double V[kMaxD * 64];
    __shared__ double U[kMaxD * 64];
    __shared__ double n0v[64], n0u[64];
    __shared__ int live[64];
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int idx = tid; idx < d * nw; idx += nt) {
        const int i = idx % d, j = idx / d;
        const int g = win[j];
        const double e = (i == g) ? 1.0 : 0.0;
        V[j * kMaxD + i] = Xh[(int64_t)g * kMaxD + i] - e;
        U[j * kMaxD + i] = Yh[(int64_t)g * kMaxD + i] - e;
    }
    __syncthreads();
    for (int j = tid; j < nw; j += nt) {
        double a = 0, b = 0;
        for (int i = 0; i < d; ++i) {
            a += V[j * kMaxD + i] * V[j * kMaxD + i];
            b += U[j * kMaxD + i] * U[j * kMaxD + i];
        }
        n0v[j] = sqrt(a);
        n0u[j] = sqrt(b);
    }
    __syncthreads();
    // two applications of each projector; C (global scratch) holds hi x nw coefficients
    for (int side = 0; side < 2; ++side) {
        double* Vs = side == 0 ? V : U;
        const double* Pb = side == 0 ? Xh : Yh;   // basis
        const double* Pd = side == 0 ? Yh : Xh;   // dual
        for (int pass = 0; pass < 2; ++pass) {
            for (int idx = tid; idx < hi * nw; idx += nt) {
                const int i = idx % hi, j = idx / hi;
                double s = 0;
                for (int k = 0; k < d; ++k) s += Pd[(int64_t)i * kMaxD + k] * Vs[j * kMaxD + k];
                C[(int64_t)j * kMaxD + i] = s;
            }
            __syncthreads();
            __threadfence_block();
            for (int idx = tid; idx < d * nw; idx += nt) {
                const int k = idx % d, j = idx / d;
                double s = 0;
                for (int i = 0; i < hi; ++i) s += Pb[(int64_t)i * kMaxD + k] * C[(int64_t)j * kMaxD + i];
                Vs[j * kMaxD + k] -= s;
            }
            __syncthreads();
        }
    }
    for (int j = tid; j < nw; j += nt) {
        double a = 0, b = 0;
        for (int i = 0; i < d; ++i) {
            a += V[j * kMaxD + i] * V[j * kMaxD + i];
            b += U[j * kMaxD + i] * U[j * kMaxD + i];
        }
        live[j] = (sqrt(a) > dep_tol * n0v[j]) && (sqrt(b) > dep_tol * n0u[j]);
    }
    __syncthreads();
    // MGS-Biorth on live columns, one wavefront (lanes over rows)
    if (tid < WAVE) {
        const int lane = tid;
        int np = 0;
        for (int l = 0; l < nw; ++l) {
            if (!live[l]) continue;
            double* p = V + l * kMaxD;
            double* q = U + l * kMaxD;
            double xn = 0, yn = 0;
            for (int i = lane; i < d; i += WAVE) {
                xn += p[i] * p[i];
                yn += q[i] * q[i];
            }
            xn = sqrt(wave_sum(xn));
            yn = sqrt(wave_sum(yn));
            for (int j = 0; j < np; ++j) {
                const double* pj = Ph + (int64_t)j * kMaxD;
                const double* qj = Qh + (int64_t)j * kMaxD;
                double r = 0;
                for (int i = lane; i < d; i += WAVE) r += qj[i] * p[i];
                r = wave_sum(r);
                for (int i = lane; i < d; i += WAVE) p[i] -= r * pj[i];
                double s = 0;
                for (int i = lane; i < d; i += WAVE) s += pj[i] * q[i];
                s = wave_sum(s);
                for (int i = lane; i < d; i += WAVE) q[i] -= s * qj[i];
            }
            double eta = 0, pn = 0, qn = 0;
            for (int i = lane; i < d; i += WAVE) {
                eta += p[i] * q[i];
                pn += p[i] * p[i];
                qn += q[i] * q[i];
            }
            eta = wave_sum(eta);
            pn = sqrt(wave_sum(pn));
            qn = sqrt(wave_sum(qn));
            if (eta == 0.0 || fabs(eta) <= cos_tol * pn * qn || pn <= dep_tol * xn || qn <= dep_tol * yn) continue;
            const double sl = sqrt(fabs(eta));
            const double rl = eta < 0 ? -sl : sl;
            for (int i = lane; i < d; i += WAVE) {
                Ph[(int64_t)np * kMaxD + i] = p[i] / rl;
                Qh[(int64_t)np * kMaxD + i] = q[i] / sl;
            }
            ++np;
        }
        if (lane == 0) status[ST_NP] = np;
    }
}

// ---------------------------------------------------------------------------
// coefficient pass of block MGS-Biorth.  One wavefront does the recurrence;
// lanes run over the m coefficients.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void coef_mgs_kernel(int m, const double* __restrict__ G, int64_t ldg,
                                                      double* __restrict__ A, double* __restrict__ B,
                                                      int* __restrict__ status, double cos_tol, double dep_tol) {
    // G = [[Gxx, Gxy], [Gyx, Gyy]] of [X Y];  a_l, b_l: coefficients of p_l, q_l
    __shared__ double a[kMaxD], b[kMaxD];
    __shared__ double hq[kMaxD * kMaxD];   // row j: b_j^T Gyx  (so q_j . X c = hq_j . c)
    // hp_j = a_j^T Gxy is stored in the output slot region of A's spare space;
    // kept in global scratch B + kMaxD*kMaxD (caller provides 2 kMaxD^2 doubles for B)
    double* hp = B + (int64_t)kMaxD * kMaxD;
    const int lane = threadIdx.x;
    auto gxx = [&](int i, int j) { return G[(int64_t)j * ldg + i]; };
    auto gxy = [&](int i, int j) { return G[(int64_t)(m + j) * ldg + i]; };
    auto gyy = [&](int i, int j) { return G[(int64_t)(m + j) * ldg + (m + i)]; };
    int np = 0;
    for (int l = 0; l < m; ++l) {
        for (int i = lane; i < m; i += WAVE) {
            a[i] = (i == l) ? 1.0 : 0.0;
            b[i] = a[i];
        }
        __syncthreads();
        for (int j = 0; j < np; ++j) {
            // r = q_j . p  = hq_j . a
            double r = 0;
            for (int i = lane; i < m; i += WAVE) r += hq[j * kMaxD + i] * a[i];
            r = wave_sum(r);
            for (int i = lane; i < m; i += WAVE) a[i] -= r * A[(int64_t)j * kMaxD + i];
            __syncthreads();
            // s = p_j . q  = hp_j . b
            double s = 0;
            for (int i = lane; i < m; i += WAVE) s += hp[(int64_t)j * kMaxD + i] * b[i];
            s = wave_sum(s);
            for (int i = lane; i < m; i += WAVE) b[i] -= s * B[(int64_t)j * kMaxD + i];
            __syncthreads();
        }
        // eta = a^T Gxy b, |p|^2 = a^T Gxx a, |q|^2 = b^T Gyy b
        double eta = 0, pn = 0, qn = 0;
        for (int i = lane; i < m; i += WAVE) {
            double ty = 0, tx = 0, tq = 0;
            for (int k = 0; k < m; ++k) {
                ty += gxy(i, k) * b[k];
                tx += gxx(i, k) * a[k];
                tq += gyy(i, k) * b[k];
            }
            eta += a[i] * ty;
            pn += a[i] * tx;
            qn += b[i] * tq;
        }
        eta = wave_sum(eta);
        pn = sqrt(fmax(wave_sum(pn), 0.0));
        qn = sqrt(fmax(wave_sum(qn), 0.0));
        const double xn = sqrt(gxx(l, l)), yn = sqrt(gyy(l, l));
        if (eta == 0.0 || fabs(eta) <= cos_tol * pn * qn || pn <= dep_tol * xn || qn <= dep_tol * yn) {
            __syncthreads();
            continue;
        }
        const double sl = sqrt(fabs(eta));
        const double rl = eta < 0 ? -sl : sl;
        for (int i = lane; i < m; i += WAVE) {
            a[i] /= rl;
            b[i] /= sl;
            A[(int64_t)np * kMaxD + i] = a[i];
            B[(int64_t)np * kMaxD + i] = b[i];
        }
        __syncthreads();
        // hq_np[i] = sum_k Gxy(i,k) b_k  (q_np . x_i);  hp_np[i] = sum_k a_k Gxy(k,i)  (p_np . y_i)
        for (int i = lane; i < m; i += WAVE) {
            double t1 = 0, t2 = 0;
            for (int k = 0; k < m; ++k) {
                t1 += gxy(i, k) * b[k];
                t2 += a[k] * gxy(k, i);
            }
            hq[np * kMaxD + i] = t1;
            hp[(int64_t)np * kMaxD + i] = t2;
        }
        __syncthreads();
        ++np;
    }
    if (lane == 0) status[ST_NKEPT] = np;
}

}  // namespace

hipError_t small_lrep(hipStream_t st, int d, const double* Kh, const double* Mh, int64_t ldh, double* lam,
                      double* Xh, double* Yh, double* scratch, int* status) {
    if (d < 1 || d > kMaxD) return hipErrorInvalidValue;
    if (d <= 32)
        hipLaunchKernelGGL(small_lrep_kernel<32>, dim3(1), dim3(32 * 8), 0, st, d, Kh, Mh, ldh, lam, Xh, Yh, scratch,
                           status);
    else if (d <= 64)
        hipLaunchKernelGGL(small_lrep_kernel<64>, dim3(1), dim3(64 * 8), 0, st, d, Kh, Mh, ldh, lam, Xh, Yh, scratch,
                           status);
    else
        hipLaunchKernelGGL(small_lrep_kernel<128>, dim3(1), dim3(128 * 8), 0, st, d, Kh, Mh, ldh, lam, Xh, Yh,
                           scratch, status);
    return hipGetLastError();
}

hipError_t step5_pq(hipStream_t st, int d, int hi, const double* Xh, const double* Yh, const int* win, int nw,
                    double* Ph, double* Qh, double* scratch, int* status, double cos_tol, double dep_tol) {
    if (nw > 64 || d > kMaxD) return hipErrorInvalidValue;
    hipLaunchKernelGGL(step5_kernel, dim3(1), dim3(256), 0, st, d, hi, Xh, Yh, win, nw, Ph, Qh, scratch, status,
                       cos_tol, dep_tol);
    return hipGetLastError();
}

hipError_t coef_mgs(hipStream_t st, int m, const double* G, int64_t ldg, double* A, double* B, int* status,
                    double cos_tol, double dep_tol) {
    if (m > kMaxD) return hipErrorInvalidValue;
    hipLaunchKernelGGL(coef_mgs_kernel, dim3(1), dim3(64), 0, st, m, G, ldg, A, B, status, cos_tol, dep_tol);
    return hipGetLastError();
}

}  // namespace lrep
