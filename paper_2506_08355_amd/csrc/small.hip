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
//              The dense products B = L2^T L1 and X^ = L2 T run as MFMA
//              block products (gemm.hip); the Cholesky factorisations and
//              the Jacobi sweeps are one-workgroup kernels.
//  step5_pq    Step 5 in coefficient space (equation for P^, Q^): the two
//              projector applications are block products, followed by the
//              small MGS-Biorth on explicit d-vectors.
//  coef_mgs    the coefficient pass of block MGS-Biorth: the recurrence of
//              Algorithm MGS-Biorth run on coefficient vectors with every
//              inner product taken from the Gram matrix of [X Y].
// The MGS-Biorth recurrences run right-looking (after p_l, q_l are final,
// every later column is updated against them); each pair (l, j) sees the
// same coefficients, in the same order, as in the column-by-column form.
#include "device.hpp"
#include "kernels.hpp"

namespace lrep {

namespace {

// convergence: every pair's cosine below ~ sqrt(d) eps (the usual one-sided
// Jacobi criterion)
constexpr double JACOBI_TOL = 4e-15;
constexpr int JACOBI_MAX_SWEEPS = 40;
constexpr int LD = kMaxD + 1;
constexpr size_t D2 = (size_t)kMaxD * kMaxD;

// ---- cross-lane sums with DPP (row-local) and readlane (across rows) ------
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
    int2 p = __builtin_bit_cast(int2, v);
    p.x = __builtin_amdgcn_update_dpp(0, p.x, CTRL, 0xF, 0xF, false);
    p.y = __builtin_amdgcn_update_dpp(0, p.y, CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, p);
}
__device__ __forceinline__ double readlane(double v, int l) {
    int2 p = __builtin_bit_cast(int2, v);
    p.x = __builtin_amdgcn_readlane(p.x, l);
    p.y = __builtin_amdgcn_readlane(p.y, l);
    return __builtin_bit_cast(double, p);
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_rows(double v) {
    int2 p = __builtin_bit_cast(int2, v);
    p.x = __builtin_amdgcn_update_dpp(0, p.x, CTRL, ROWMASK, 0xF, false);
    p.y = __builtin_amdgcn_update_dpp(0, p.y, CTRL, ROWMASK, 0xF, false);
    return __builtin_bit_cast(double, p);
}
// Sum over the 64 lanes.  Within each row of 16 lanes: xor-1 and xor-2 quad
// permutes, then half-mirror and mirror (each stage adds two equal partial
// sums in either order, so all 16 lanes hold bitwise the same row sum); then
// row 1 += row 0 and row 3 += row 2 (row_bcast:15), row 3 += row 1
// (row_bcast:31), and lane 63's total is broadcast from a scalar register.
// Every lane returns bitwise the same total.
__device__ __forceinline__ double wsum(double v) {
    v += dpp<0xB1>(v);
    v += dpp<0x4E>(v);
    v += dpp<0x141>(v);
    v += dpp<0x140>(v);
    v += dpp_rows<0x142, 0xA>(v);
    v += dpp_rows<0x143, 0xC>(v);
    return readlane(v, 63);
}

// stacked row e * 64 + lane lies in the top (B) part: rows < D = 32 E
template <int E>
__device__ __forceinline__ bool is_top(int e, int lane) {
    if constexpr (E >= 2) return e < E / 2;
    else return lane < 32;
}

// 1 / x to full precision from the hardware estimate and one Newton step
__device__ __forceinline__ double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    const double e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
// 1 / sqrt(x) from the hardware estimate and one Newton step
__device__ __forceinline__ double rsq_nr(double x) {
    double r = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x * r;
    return fma(r, fma(-h, r, 0.5), r);
}

// ---------------------------------------------------------------------------
// Cholesky of the symmetric parts of K^ (block 0) and M^ (block 1), d <= 128.
// Right-looking on an LDS copy; one barrier per column: at step k every
// thread reads the final pivot S[k][k] and column k (unscaled), writes the
// scaled column of L to global memory and updates its own trailing entries
// with S[i][j] -= S[i][k] S[j][k] / S[k][k].
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void chol2_kernel(int d, const double* __restrict__ Kh,
                                                    const double* __restrict__ Mh, int64_t ldh,
                                                    double* __restrict__ scratch, int* __restrict__ status) {
    __shared__ double S[kMaxD * LD];
    const double* A = blockIdx.x == 0 ? Kh : Mh;
    double* L = scratch + (size_t)blockIdx.x * D2;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int idx = tid; idx < d * d; idx += nt) {
        const int i = idx % d, j = idx / d;
        S[i * LD + j] = 0.5 * (A[(int64_t)j * ldh + i] + A[(int64_t)i * ldh + j]);
    }
    for (int idx = tid; idx < (int)D2; idx += nt) L[idx] = 0.0;
    __syncthreads();
    for (int k = 0; k < d; ++k) {
        const double v = S[k * LD + k];
        if (!(v > 0.0)) {
            if (tid == 0) status[ST_NOTSPD] = 1;
            return;   // uniform: every thread read the same pivot
        }
        const double piv = sqrt(v);
        const double inv = 1.0 / v;
        for (int i = k + tid; i < d; i += nt) L[(int64_t)k * kMaxD + i] = (i == k) ? piv : S[i * LD + k] / piv;
        const int m = d - k - 1;
        for (int idx = tid; idx < m * m; idx += nt) {
            const int i = k + 1 + idx % m, j = k + 1 + idx / m;
            if (j <= i) S[i * LD + j] -= S[i * LD + k] * S[j * LD + k] * inv;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// One-sided Jacobi on the stacked columns [B; L1] (B = L2^T L1, both d x d,
// ld kMaxD), round-robin ordering.  Wavefront w owns tournament slots
// T[4w..4w+3] (register slots 0..3) and Bt[4w..4w+3] (slots 4..7); lane l
// holds stacked rows e*64 + l.  Outputs lam (ascending), Yh = L1 phi /
// sqrt(sigma) and T = (B phi) / sigma^(3/2) (so that X^ = L2 T).
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(D * 8) void jacobi_kernel(int d, const double* __restrict__ scratch,
                                                      double* __restrict__ lam, double* __restrict__ Yh,
                                                      double* __restrict__ T, int* __restrict__ status) {
    constexpr int NW = D / 8;
    constexpr int NTH = NW * WAVE;
    constexpr int E = (2 * D) / WAVE;
    __shared__ double xT[2 * NW * (2 * D + 2)];
    __shared__ double xB[2 * NW * (2 * D + 2)];
    __shared__ double sig[D];
    __shared__ double bnorm[D];
    __shared__ int rank_of[D];
    __shared__ double wmax[NW];
    const double* L1 = scratch;
    const double* Bm = scratch + 3 * D2;
    const int tid = threadIdx.x, lane = tid % WAVE, w = tid / WAVE;

    double col[8][E];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const int k = 4 * w + (s & 3);
        const int c = (s < 4) ? 2 * k : 2 * k + 1;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int row = e * WAVE + lane;
            double v = 0.0;
            if (c < d) {
                if (row < D) {
                    if (row < d) v = Bm[(int64_t)c * kMaxD + row];
                } else if (row - D < d) {
                    v = L1[(int64_t)c * kMaxD + (row - D)];
                }
            }
            col[s][e] = v;
        }
    }

    // squared norms of the top parts travel with their columns (uniform per
    // wave); they are recomputed exactly at the start of every sweep and
    // updated by the rotation formulas in between (alpha' = alpha - t gamma,
    // beta' = beta + t gamma), so each pair needs one cross-lane sum only.
    double nrm[8];
    int sweeps = 0;
    for (int sweep = 0; sweep < JACOBI_MAX_SWEEPS; ++sweep) {
        ++sweeps;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            double t = 0.0;
#pragma unroll
            for (int e = 0; e < E; ++e)
                if (is_top<E>(e, lane)) t += col[s][e] * col[s][e];
            nrm[s] = wsum(t);
        }
        double offmax = 0.0;
        for (int step = 0; step < D - 1; ++step) {
            double ga[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                ga[i] = 0.0;
#pragma unroll
                for (int e = 0; e < E; ++e)
                    if (is_top<E>(e, lane)) ga[i] += col[i][e] * col[4 + i][e];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) ga[i] = wsum(ga[i]);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const double al = nrm[i], be = nrm[4 + i];
                if (ga[i] != 0.0) {
                    const double rel = fabs(ga[i]) * rsq_nr(al * be);
                    offmax = fmax(offmax, rel);
                    if (rel > JACOBI_TOL) {
                        // Rutishauser's rotation: zeta = (beta - alpha) / (2 gamma),
                        // t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), c = 1/sqrt(1+t^2), s = c t
                        const double zeta = (be - al) * rcp_nr(2.0 * ga[i]);
                        const double az = fabs(zeta);
                        const double root = az < 1e150 ? (1.0 + zeta * zeta) * rsq_nr(1.0 + zeta * zeta) : az;
                        const double t = copysign(rcp_nr(az + root), zeta);
                        const double c = rsq_nr(1.0 + t * t);
                        const double s = c * t;
#pragma unroll
                        for (int e = 0; e < E; ++e) {
                            const double a = col[i][e], b = col[4 + i][e];
                            col[i][e] = c * a - s * b;
                            col[4 + i][e] = s * a + c * b;
                        }
                        nrm[i] = al - t * ga[i];
                        nrm[4 + i] = be + t * ga[i];
                        if (nrm[i] < 1e-2 * al) {   // heavy cancellation: recompute exactly
                            double t2 = 0.0;
#pragma unroll
                            for (int e = 0; e < E; ++e)
                                if (is_top<E>(e, lane)) t2 += col[i][e] * col[i][e];
                            nrm[i] = wsum(t2);
                        }
                    }
                }
            }
            // round-robin move: only T[4w+3] and Bt[4w] cross wavefronts
            const int par = step & 1;
            double* oT = xT + ((size_t)par * NW + w) * (2 * D + 2);
            double* oB = xB + ((size_t)par * NW + w) * (2 * D + 2);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                oT[e * WAVE + lane] = col[3][e];
                oB[e * WAVE + lane] = col[4][e];
            }
            if (lane == 0) {
                oT[2 * D] = nrm[3];
                oB[2 * D] = nrm[4];
            }
            __syncthreads();
            const double* iT = xT + ((size_t)par * NW + (w > 0 ? w - 1 : 0)) * (2 * D + 2);
            const double* iB = xB + ((size_t)par * NW + (w < NW - 1 ? w + 1 : 0)) * (2 * D + 2);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const double t0 = col[0][e], t1 = col[1][e], t2 = col[2][e], t3 = col[3][e];
                const double b0 = col[4][e], b1 = col[5][e], b2 = col[6][e], b3 = col[7][e];
                if (w == 0) {
                    col[0][e] = t0;
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
            {
                const double t0 = nrm[0], t1 = nrm[1], t2 = nrm[2], t3 = nrm[3];
                const double b0 = nrm[4], b1 = nrm[5], b2 = nrm[6], b3 = nrm[7];
                if (w == 0) {
                    nrm[1] = b0;
                } else {
                    nrm[0] = iT[2 * D];
                    nrm[1] = t0;
                }
                nrm[2] = t1;
                nrm[3] = t2;
                nrm[4] = b1;
                nrm[5] = b2;
                nrm[6] = b3;
                nrm[7] = (w == NW - 1) ? t3 : iB[2 * D];
            }
        }
        if (lane == 0) wmax[w] = offmax;
        __syncthreads();
        double om = 0.0;
#pragma unroll
        for (int i = 0; i < NW; ++i) om = fmax(om, wmax[i]);
        __syncthreads();
        if (om <= JACOBI_TOL) break;
    }
    if (tid == 0 && status) status[ST_SWEEPS] = sweeps;

#pragma unroll
    for (int s = 0; s < 8; ++s) {
        double tn = 0, bn = 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const double v = col[s][e];
            if (is_top<E>(e, lane)) tn += v * v;
            else bn += v * v;
        }
        tn = wsum(tn);
        bn = wsum(bn);
        if (lane == 0) {
            sig[8 * w + s] = sqrt(tn);
            bnorm[8 * w + s] = bn;
        }
    }
    __syncthreads();
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
}

// ---------------------------------------------------------------------------
// Step 5, gather:  V = Xh[:, win] - E, U = Yh[:, win] - E (d x nw, ld kMaxD)
// and their column norms (for the "annihilated by the projector" test).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void step5_gather_kernel(int d, const double* __restrict__ Xh,
                                                           const double* __restrict__ Yh, const int* __restrict__ win,
                                                           int nw, double* __restrict__ V, double* __restrict__ U,
                                                           double* __restrict__ n0) {
    __shared__ double red[256 / WAVE];
    const int j = blockIdx.x;
    const int g = win[j];
    double sv = 0, su = 0;
    for (int i = threadIdx.x; i < d; i += 256) {
        const double e = (i == g) ? 1.0 : 0.0;
        const double v = Xh[(int64_t)g * kMaxD + i] - e;
        const double u = Yh[(int64_t)g * kMaxD + i] - e;
        V[(int64_t)j * kMaxD + i] = v;
        U[(int64_t)j * kMaxD + i] = u;
        sv += v * v;
        su += u * u;
    }
    sv = block_sum<256>(sv, red);
    su = block_sum<256>(su, red);
    if (threadIdx.x == 0) {
        n0[j] = sqrt(sv);
        n0[64 + j] = sqrt(su);
    }
}

// ---------------------------------------------------------------------------
// MGS-Biorth of explicit small vectors (d x nw, ld kMaxD, in place in LDS),
// right-looking, with the oracle's breakdown rule; columns whose norm the
// projector reduced below dep_tol * n0 are skipped first.  Writes the kept
// columns compacted to Ph, Qh and status[ST_NP].
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void small_mgs_kernel(int d, int nw, const double* __restrict__ Vin,
                                                        const double* __restrict__ Uin,
                                                        const double* __restrict__ n0, double* __restrict__ Ph,
                                                        double* __restrict__ Qh, int* __restrict__ status,
                                                        double cos_tol, double dep_tol) {
    __shared__ double P[kMaxD * 64];
    __shared__ double Q[kMaxD * 64];
    __shared__ double xn[64], yn[64], rr[64], ss[64];
    __shared__ int live[64];
    __shared__ double red[256 / WAVE];
    __shared__ double sc[4];
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid % WAVE, wid = tid / WAVE;
    for (int idx = tid; idx < d * nw; idx += nt) {
        const int i = idx % d, j = idx / d;
        P[j * kMaxD + i] = Vin[(int64_t)j * kMaxD + i];
        Q[j * kMaxD + i] = Uin[(int64_t)j * kMaxD + i];
    }
    __syncthreads();
    // column norms of the projected inputs (x_l, y_l of the MGS) and liveness
    for (int j = wid; j < nw; j += nt / WAVE) {
        double a = 0, b = 0;
        for (int i = lane; i < d; i += WAVE) {
            a += P[j * kMaxD + i] * P[j * kMaxD + i];
            b += Q[j * kMaxD + i] * Q[j * kMaxD + i];
        }
        a = sqrt(wsum(a));
        b = sqrt(wsum(b));
        if (lane == 0) {
            xn[j] = a;
            yn[j] = b;
            live[j] = (a > dep_tol * n0[j]) && (b > dep_tol * n0[64 + j]);
        }
    }
    __syncthreads();
    int np = 0;
    for (int l = 0; l < nw; ++l) {
        if (!live[l]) continue;
        const double* p = P + l * kMaxD;
        const double* q = Q + l * kMaxD;
        double eta = 0, pn = 0, qn = 0;
        for (int i = tid; i < d; i += nt) {
            eta += p[i] * q[i];
            pn += p[i] * p[i];
            qn += q[i] * q[i];
        }
        eta = block_sum<256>(eta, red);
        pn = sqrt(block_sum<256>(pn, red));
        qn = sqrt(block_sum<256>(qn, red));
        if (eta == 0.0 || fabs(eta) <= cos_tol * pn * qn || pn <= dep_tol * xn[l] || qn <= dep_tol * yn[l]) continue;
        const double sl = sqrt(fabs(eta));
        const double rl = eta < 0 ? -sl : sl;
        for (int i = tid; i < d; i += nt) {
            const double pv = p[i] / rl, qv = q[i] / sl;
            P[l * kMaxD + i] = pv;
            Q[l * kMaxD + i] = qv;
            Ph[(int64_t)np * kMaxD + i] = pv;
            Qh[(int64_t)np * kMaxD + i] = qv;
        }
        ++np;
        __syncthreads();
        // coefficients for every later column: r_j = q_l . p_j, s_j = p_l . q_j
        for (int j = l + 1 + wid; j < nw; j += nt / WAVE) {
            double r = 0, s = 0;
            for (int i = lane; i < d; i += WAVE) {
                r += q[i] * P[j * kMaxD + i];
                s += p[i] * Q[j * kMaxD + i];
            }
            r = wsum(r);
            s = wsum(s);
            if (lane == 0) {
                rr[j] = r;
                ss[j] = s;
            }
        }
        __syncthreads();
        for (int idx = tid; idx < d * (nw - l - 1); idx += nt) {
            const int i = idx % d, j = l + 1 + idx / d;
            P[j * kMaxD + i] -= rr[j] * p[i];
            Q[j * kMaxD + i] -= ss[j] * q[i];
        }
        __syncthreads();
    }
    if (tid == 0) status[ST_NP] = np;
    (void)sc;
}

// ---------------------------------------------------------------------------
// Coefficient pass of block MGS-Biorth (right-looking).  G = [[Gxx, Gxy],
// [Gyx, Gyy]] is the Gram of [X Y] (2m x 2m, ld ldg).  a_j, b_j (columns of
// A, B, m x m in global scratch, ld kMaxD) are the coefficients of the
// current p~_j = X a_j, q~_j = Y b_j.  Per step l:
//   eta = a_l^T Gxy b_l, |p~_l|^2 = a_l^T Gxx a_l, |q~_l|^2 = b_l^T Gyy b_l;
//   scale, then for j > l: r_j = (Gxy b_l) . a_j, a_j -= r_j a_l;
//                          s_j = (Gxy^T a_l) . b_j, b_j -= s_j b_l.
// Kept columns are copied compacted to Aout, Bout.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void coef_mgs_kernel(int m, const double* __restrict__ G, int64_t ldg,
                                                       double* __restrict__ A, double* __restrict__ B,
                                                       double* __restrict__ Aout, double* __restrict__ Bout,
                                                       int* __restrict__ status, double cos_tol, double dep_tol) {
    __shared__ double txy[kMaxD], txx[kMaxD], tyy[kMaxD], u[kMaxD], rr[kMaxD], ss[kMaxD];
    __shared__ double red[256 / WAVE];
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid % WAVE, wid = tid / WAVE;
    auto gxx = [&](int i, int j) { return G[(int64_t)j * ldg + i]; };
    auto gxy = [&](int i, int j) { return G[(int64_t)(m + j) * ldg + i]; };
    auto gyy = [&](int i, int j) { return G[(int64_t)(m + j) * ldg + (m + i)]; };
    for (int idx = tid; idx < m * m; idx += nt) {
        const int i = idx % m, j = idx / m;
        A[(int64_t)j * kMaxD + i] = (i == j) ? 1.0 : 0.0;
        B[(int64_t)j * kMaxD + i] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    int np = 0;
    for (int l = 0; l < m; ++l) {
        const double* al = A + (int64_t)l * kMaxD;
        const double* bl = B + (int64_t)l * kMaxD;
        // a_l, b_l are supported on rows 0..l
        for (int t = tid; t < 4 * m; t += nt) {
            const int which = t / m, i = t % m;
            double s = 0;
            if (which == 0)
                for (int k = 0; k <= l; ++k) s += gxy(i, k) * bl[k];
            else if (which == 1)
                for (int k = 0; k <= l; ++k) s += gxx(i, k) * al[k];
            else if (which == 2)
                for (int k = 0; k <= l; ++k) s += gyy(i, k) * bl[k];
            else
                for (int k = 0; k <= l; ++k) s += gxy(k, i) * al[k];
            (which == 0 ? txy : which == 1 ? txx : which == 2 ? tyy : u)[i] = s;
        }
        __syncthreads();
        double eta = 0, pn = 0, qn = 0;
        for (int i = tid; i <= l; i += nt) {
            eta += al[i] * txy[i];
            pn += al[i] * txx[i];
            qn += bl[i] * tyy[i];
        }
        eta = block_sum<256>(eta, red);
        pn = sqrt(fmax(block_sum<256>(pn, red), 0.0));
        qn = sqrt(fmax(block_sum<256>(qn, red), 0.0));
        const double xn = sqrt(gxx(l, l)), yn = sqrt(gyy(l, l));
        if (eta == 0.0 || fabs(eta) <= cos_tol * pn * qn || pn <= dep_tol * xn || qn <= dep_tol * yn) continue;
        const double sl = sqrt(fabs(eta));
        const double rl = eta < 0 ? -sl : sl;
        for (int i = tid; i < m; i += nt) {
            const double av = (i <= l) ? al[i] / rl : 0.0, bv = (i <= l) ? bl[i] / sl : 0.0;
            Aout[(int64_t)np * kMaxD + i] = av;
            Bout[(int64_t)np * kMaxD + i] = bv;
            txy[i] /= sl;   // Gxy b_l with the scaled b_l
            u[i] /= rl;     // Gxy^T a_l with the scaled a_l
        }
        __syncthreads();
        for (int i = tid; i <= l; i += nt) {
            A[(int64_t)l * kMaxD + i] = al[i] / rl;
            B[(int64_t)l * kMaxD + i] = bl[i] / sl;
        }
        ++np;
        __syncthreads();
        for (int j = l + 1 + wid; j < m; j += nt / WAVE) {
            double r = 0, s = 0;
            for (int i = lane; i <= j; i += WAVE) {
                r += txy[i] * A[(int64_t)j * kMaxD + i];
                s += u[i] * B[(int64_t)j * kMaxD + i];
            }
            r = wsum(r);
            s = wsum(s);
            if (lane == 0) {
                rr[j] = r;
                ss[j] = s;
            }
        }
        __syncthreads();
        for (int idx = tid; idx < (l + 1) * (m - l - 1); idx += nt) {
            const int i = idx % (l + 1), j = l + 1 + idx / (l + 1);
            A[(int64_t)j * kMaxD + i] -= rr[j] * A[(int64_t)l * kMaxD + i];
            B[(int64_t)j * kMaxD + i] -= ss[j] * B[(int64_t)l * kMaxD + i];
        }
        __syncthreads();
    }
    if (tid == 0) status[ST_NKEPT] = np;
}

}  // namespace

hipError_t small_lrep(hipStream_t st, int d, const double* Kh, const double* Mh, int64_t ldh, double* lam,
                      double* Xh, double* Yh, double* scratch, int* status, double* work, size_t work_elems) {
    if (d < 1 || d > kMaxD) return hipErrorInvalidValue;
    hipLaunchKernelGGL(chol2_kernel, dim3(2), dim3(1024), 0, st, d, Kh, Mh, ldh, scratch, status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // B = L2^T L1 into scratch + 3 D2
    Seg a{scratch + D2, kMaxD, d}, b{scratch, kMaxD, d};
    e = gemm_tn(st, d, d, d, &a, 1, &b, 1, scratch + 3 * D2, kMaxD, 1.0, 0, work, work_elems);
    if (e != hipSuccess) return e;
    double* T = scratch + 2 * D2;
    if (d <= 32)
        hipLaunchKernelGGL(jacobi_kernel<32>, dim3(1), dim3(32 * 8), 0, st, d, scratch, lam, Yh, T, status);
    else if (d <= 64)
        hipLaunchKernelGGL(jacobi_kernel<64>, dim3(1), dim3(64 * 8), 0, st, d, scratch, lam, Yh, T, status);
    else
        hipLaunchKernelGGL(jacobi_kernel<128>, dim3(1), dim3(128 * 8), 0, st, d, scratch, lam, Yh, T, status);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // X^ = L2 T
    Seg l2{scratch + D2, kMaxD, d};
    return gemm_nn(st, d, d, d, &l2, 1, T, kMaxD, Xh, kMaxD, 1.0, 0.0, work, work_elems);
}

hipError_t step5_pq(hipStream_t st, int d, int hi, const double* Xh, const double* Yh, const int* win, int nw,
                    double* Ph, double* Qh, double* scratch, int* status, double cos_tol, double dep_tol,
                    double* work, size_t work_elems) {
    if (nw > 64 || nw < 1 || d > kMaxD || hi > d) return hipErrorInvalidValue;
    double* V = scratch;
    double* U = scratch + kMaxD * 64;
    double* C = scratch + 2 * kMaxD * 64;
    double* n0 = scratch + 3 * kMaxD * 64;
    hipLaunchKernelGGL(step5_gather_kernel, dim3(nw), dim3(256), 0, st, d, Xh, Yh, win, nw, V, U, n0);
    hipError_t e = hipGetLastError();
    for (int side = 0; side < 2 && e == hipSuccess && hi > 0; ++side) {
        double* Vs = side == 0 ? V : U;
        Seg basis{side == 0 ? Xh : Yh, kMaxD, hi};
        Seg dual{side == 0 ? Yh : Xh, kMaxD, hi};
        Seg vs{Vs, kMaxD, nw};
        for (int pass = 0; pass < 2 && e == hipSuccess; ++pass) {
            e = gemm_tn(st, d, hi, nw, &dual, 1, &vs, 1, C, kMaxD, 1.0, 0, work, work_elems);
            if (e == hipSuccess)
                e = gemm_nn(st, d, nw, hi, &basis, 1, C, kMaxD, Vs, kMaxD, -1.0, 1.0, work, work_elems);
        }
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(small_mgs_kernel, dim3(1), dim3(256), 0, st, d, nw, V, U, n0, Ph, Qh, status, cos_tol,
                       dep_tol);
    return hipGetLastError();
}

hipError_t coef_mgs(hipStream_t st, int m, const double* G, int64_t ldg, double* A, double* B, int* status,
                    double cos_tol, double dep_tol, double* scratch) {
    if (m > kMaxD) return hipErrorInvalidValue;
    hipLaunchKernelGGL(coef_mgs_kernel, dim3(1), dim3(256), 0, st, m, G, ldg, scratch, scratch + D2, A, B, status,
                       cos_tol, dep_tol);
    return hipGetLastError();
}

}  // namespace lrep
