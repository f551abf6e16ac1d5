// One-workgroup FP64 kernels on the small (d <= 128) matrices of the BOSP
// iteration, for gfx950:
//
//  small_lrep  the projected structured LREP of Step 3: two Cholesky
//              factorisations and one SVD (Section 3.2 / cost discussion of
//              Section 3.3).  With K^ = L1 L1^T, M^ = L2 L2^T and the SVD
//              B = L2^T L1 = Psi Sigma Phi^T, the Ritz pairs are
//                  X^_c = L2 psi_c / sqrt(sigma_c),
//                  Y^_c = L1 phi_c / sqrt(sigma_c) = sqrt(sigma_c) L2^{-T} psi_c.
//              The SVD is a one-sided (Hestenes) Jacobi iteration on the
//              columns of B, register resident (jacobi_kernel); at
//              convergence column c is sigma_c psi_c.  B = L2^T L1 and
//              X^ = L2 T are MFMA block products (gemm.hip) and Y^ a
//              triangular solve with L2^T.
//  step5_pq    Step 5 in coefficient space (equation for P^, Q^): the two
//              projector applications are block products, followed by the
//              small MGS-Biorth on explicit d-vectors.
//  coef_mgs    the coefficient pass of block MGS-Biorth: the recurrence of
//              Algorithm MGS-Biorth run on coefficient vectors with every
//              inner product taken from the Gram matrix of [X Y].
// The MGS-Biorth recurrences run right-looking (after p_l, q_l are final,
// every later column is updated against them); each pair (l, j) sees the
// same coefficients, in the same order, as in the column-by-column form.
#include <type_traits>

#include "device.hpp"
#include "kernels.hpp"

namespace lrep {

namespace {

// convergence: every pair's cosine below ~ sqrt(d) eps (the usual one-sided
// Jacobi criterion)
constexpr double JACOBI_TOL = 1e-14;
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

// ---------------------------------------------------------------------------
// Cholesky of the symmetric parts of K^ (block 0) and M^ (block 1), d <= 128,
// blocked right-looking on an LDS copy (blocks of CB = 16 columns), 256
// threads per matrix:
//   (a) the diagonal block is factored by one wavefront in registers, lane i
//       holding row i, the pivot broadcast with readlane and each scaled
//       column through LDS (L(k,k) = a_kk / sqrt(a_kk) with a full-precision
//       reciprocal square root);
//   (b) the panel below it is solved row by row (L_pd = A_pd L_dd^{-T}), one
//       thread per row, multiplying by the reciprocals 1 / L(k,k);
//   (c) the trailing matrix takes the rank-CB update A -= L_pd L_pd^T in
//       4 x 4 register tiles.
// A non-positive pivot sets status[ST_NOTSPD].
// ---------------------------------------------------------------------------
constexpr int CB = 16;

// 1/x and 1/sqrt(x) to full FP64 precision: the hardware estimates are good
// to ~2^-24, two Newton steps bring them to rounding level.
__device__ __forceinline__ double rcp2(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ double rsq2(double x) {
    double r = __builtin_amdgcn_rsq(x);
    double h = 0.5 * x * r;
    r = fma(r, fma(-h, r, 0.5), r);
    h = 0.5 * x * r;
    return fma(r, fma(-h, r, 0.5), r);
}


__device__ __forceinline__ double rdlane(double v, int l) {
    int2 p = __builtin_bit_cast(int2, v);
    p.x = __builtin_amdgcn_readlane(p.x, l);
    p.y = __builtin_amdgcn_readlane(p.y, l);
    return __builtin_bit_cast(double, p);
}

__global__ __launch_bounds__(256) void chol2_kernel(int d, const double* __restrict__ Kh,
                                                   const double* __restrict__ Mh, int64_t ldh,
                                                   double* __restrict__ scratch, int* __restrict__ status) {
    __shared__ double S[kMaxD * LD];
    __shared__ double colb[CB], dinv[CB];
    __shared__ int fail;
    const double* A = blockIdx.x == 0 ? Kh : Mh;
    double* L = scratch + (size_t)blockIdx.x * D2;
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid % WAVE, wid = tid / WAVE;
    // column c of A into row c of S (S[c LD + r] = A(r, c)): coalesced reads,
    // eight columns in flight per wavefront
    constexpr int NW = 256 / WAVE;
    for (int c0 = wid; c0 < d; c0 += 8 * NW) {
        double v0[8], v1[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int c = c0 + k * NW;
            const double* col = A + (int64_t)c * ldh;
            v0[k] = (c < d && lane < d) ? col[lane] : 0.0;
            v1[k] = (c < d && lane + WAVE < d) ? col[lane + WAVE] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int c = c0 + k * NW;
            if (c < d) {
                S[c * LD + lane] = v0[k];
                S[c * LD + lane + WAVE] = v1[k];
            }
        }
    }
    if (tid == 0) fail = 0;
    __syncthreads();
    // the symmetric part into the lower triangle: for i > j, S[i LD + j]
    // holds A(j, i) and S[j LD + i] holds A(i, j) (never written here); the
    // diagonal is already A(i, i)
    for (int i = 1 + wid; i < d; i += NW)
        for (int j = lane; j < i; j += WAVE) S[i * LD + j] = 0.5 * (S[i * LD + j] + S[j * LD + i]);
    __syncthreads();
    for (int kb = 0; kb < d; kb += CB) {
        const int nb = min(CB, d - kb);
        // (a) diagonal block, one wavefront: lane i holds row i; at step k the
        //     pivot comes from lane k (readlane), the scaled column k goes
        //     through LDS to every lane (a wavefront sees its own LDS writes
        //     in order), and 1 / L(k,k) is kept for the panel solve
        if (wid == 0) {
            // rows past nb (a short last block) are padded with the identity,
            // so every step runs unpredicated
            double r[CB];
#pragma unroll
            for (int j = 0; j < CB; ++j)
                r[j] = lane < nb ? (j <= lane ? S[(kb + lane) * LD + kb + j] : 0.0) : (j == lane ? 1.0 : 0.0);
            bool bad = false;
#pragma unroll
            for (int k = 0; k < CB; ++k) {
                const double piv = rdlane(r[k], k);
                bad = bad || !(piv > 0.0);   // uniform; later steps may run on NaN, never stored
                const double inv = rsq2(piv);
                const double lk = (lane == k) ? piv * inv : r[k] * inv;
                r[k] = (lane >= k) ? lk : r[k];
                if (lane < CB) colb[lane] = lk;
                if (lane == 0) dinv[k] = inv;
                __builtin_amdgcn_wave_barrier();
                // entries above the diagonal (j > lane) take values that are never
                // read or stored
#pragma unroll
                for (int j = k + 1; j < CB; ++j) r[j] = fma(-lk, colb[j], r[j]);
                __builtin_amdgcn_wave_barrier();
            }
            if (bad) {
                if (lane == 0) {
                    fail = 1;
                    status[ST_NOTSPD] = 1;
                }
            } else if (lane < nb) {
#pragma unroll
                for (int j = 0; j < CB; ++j)
                    if (j <= lane) S[(kb + lane) * LD + kb + j] = r[j];
            }
        }
        __syncthreads();
        if (fail) return;   // uniform
        // rows below the block exist only under a full block (nb == CB: a
        // short block is the last one), so (b) and (c) run with compile-time
        // trip counts
        const int m = d - kb - nb;
        if (m <= 0) break;   // uniform: the last block
        // (b) panel rows below the block
        for (int t = tid; t < m; t += nt) {
            const int i = kb + CB + t;
            double x[CB];
#pragma unroll
            for (int j = 0; j < CB; ++j) x[j] = S[i * LD + kb + j];
#pragma unroll
            for (int j = 0; j < CB; ++j) {
                double v = x[j];
#pragma unroll
                for (int l = 0; l < j; ++l) v = fma(-x[l], S[(kb + j) * LD + kb + l], v);
                x[j] = v * dinv[j];
            }
#pragma unroll
            for (int j = 0; j < CB; ++j) S[i * LD + kb + j] = x[j];
        }
        __syncthreads();
        // (c) trailing update on 4 x 4 tiles (ti >= tj); rows past d are read
        // clamped and never stored
        const int mt = (m + 3) / 4;
        const int ntile = mt * (mt + 1) / 2;
        for (int tt = tid; tt < ntile; tt += nt) {
            int ti = (int)((sqrt(8.0 * tt + 1.0) - 1.0) * 0.5);
            while ((ti + 1) * (ti + 2) / 2 <= tt) ++ti;
            while (ti * (ti + 1) / 2 > tt) --ti;
            const int tj = tt - ti * (ti + 1) / 2;
            const int i0 = kb + CB + 4 * ti, j0 = kb + CB + 4 * tj;
            const double* rowi[4];
            const double* rowj[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                rowi[u] = S + min(i0 + u, d - 1) * LD + kb;
                rowj[u] = S + min(j0 + u, d - 1) * LD + kb;
            }
            double acc[4][4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
#pragma unroll
            for (int l = 0; l < CB; ++l) {
                double pi[4], pj[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    pi[u] = rowi[u][l];
                    pj[u] = rowj[u][l];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[u][v] = fma(pi[u], pj[v], acc[u][v]);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = i0 + u, j = j0 + v;
                    if (i < d && j <= i) S[i * LD + j] -= acc[u][v];
                }
        }
        __syncthreads();
    }
    for (int idx = tid; idx < (int)D2; idx += nt) {
        const int i = idx % kMaxD, j = idx / kMaxD;
        L[idx] = (i < d && j <= i) ? S[i * LD + j] : 0.0;
    }
}

// ---------------------------------------------------------------------------
// One-sided (Hestenes) Jacobi on the columns of B = L2^T L1 (d x d, ld kMaxD,
// zero-padded to D), register resident, one workgroup of D / 32 wavefronts.
//
// Layout: the D columns form S = D / 2 slots of two columns (a, b).  Slot
// s = 16 w + i lives in wavefront w, lane column i: lanes i, i + 16, i + 32,
// i + 48 hold rows [q R, q R + R) of both columns (q = lane / 16, R = D / 4).
// A pair's inner product is a 4-lane sum (two permlane swaps), and the
// rotation parameters are computed once per lane, i.e. the 16 pairs of a
// wavefront in parallel.
//
// Pair ordering: a recursive split.  Level 0 pairs every a with every b
// (S steps, b moving between slots); level L >= 1 first swaps, for slot pairs
// (s, s ^ G) with G = S >> L, the b of the lower slot with the a of the upper
// one, then pairs within groups of G slots (G steps).  Every pair of columns
// meets exactly once per sweep (D - 1 steps).  The b moves are a rotation by
// one lane inside the 16-lane rows (DPP row_ror:1) and, every 16 steps of the
// levels with G >= 16, an exchange between wavefronts through LDS; groups of
// fewer than 16 slots use XOR moves in Gray-code order (DPP quad_perm and
// mirrors).  The squared norms travel with their columns and are recomputed
// exactly at the start of every sweep (and after heavy cancellation), so a
// pair costs one cross-lane sum.
//
// Outputs, ranked by ascending sigma:  lam = sigma, T = col / sigma^(3/2)
// (so X^ = L2 T) and Z = col / sigma^(1/2) (so Y^ = L2^{-T} Z).
// ---------------------------------------------------------------------------

template <int CTRL>
__device__ __forceinline__ double dmov(double v) {   // patterns where every lane reads a valid lane
    int2 p = __builtin_bit_cast(int2, v);
    p.x = __builtin_amdgcn_mov_dpp(p.x, CTRL, 0xF, 0xF, true);
    p.y = __builtin_amdgcn_mov_dpp(p.y, CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, p);
}
// value of lane i ^ k inside each 16-lane row, k in {1, 2, 4, 8}
template <int K>
__device__ __forceinline__ double xperm(double v) {
    if constexpr (K == 1) return dmov<0xB1>(v);                // quad_perm [1,0,3,2]
    else if constexpr (K == 2) return dmov<0x4E>(v);           // quad_perm [2,3,0,1]
    else if constexpr (K == 4) return dmov<0x1B>(dmov<0x141>(v));   // i^7 then i^3
    else return dmov<0x141>(dmov<0x140>(v));                   // i^15 then i^7
}
// sum over the 4 lanes l, l^16, l^32, l^48; every lane gets bitwise the same value
__device__ __forceinline__ double qsum(double v) {
    int2 p = __builtin_bit_cast(int2, v);
    auto lo = __builtin_amdgcn_permlane32_swap(p.x, p.x, false, false);
    auto hi = __builtin_amdgcn_permlane32_swap(p.y, p.y, false, false);
    double y = __builtin_bit_cast(double, int2{(int)lo[0], (int)hi[0]}) +
               __builtin_bit_cast(double, int2{(int)lo[1], (int)hi[1]});
    p = __builtin_bit_cast(int2, y);
    lo = __builtin_amdgcn_permlane16_swap(p.x, p.x, false, false);
    hi = __builtin_amdgcn_permlane16_swap(p.y, p.y, false, false);
    return __builtin_bit_cast(double, int2{(int)lo[0], (int)hi[0]}) +
           __builtin_bit_cast(double, int2{(int)lo[1], (int)hi[1]});
}

template <int R>
__device__ __forceinline__ double sumsq(const double (&x)[R]) {
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int e = 0; e < R; e += 2) {
        s0 = fma(x[e], x[e], s0);
        s1 = fma(x[e + 1], x[e + 1], s1);
    }
    return qsum(s0 + s1);
}

// 1/x and 1/sqrt(x) after one Newton step (relative error ~1e-15): enough
// where the value only steers the iteration
__device__ __forceinline__ double rcp1(double x) {
    const double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ double rsq1(double x) {
    const double r = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x * r;
    return fma(r, fma(-h, r, 0.5), r);
}

// One rotation of the slot's pair.  The columns are kept scaled (Rutishauser's
// fast form): the true columns are A = sa a and B = sb b, na and nb their
// squared norms.  The rotation  A' = c (A - t B),  B' = c (B + t A)  is taken
// as two in-place shears of the stored vectors and a change of the scales:
//   b <- b + v a          with v = t sa / sb,      sb <- c sb,
//   a <- a - u b (new b)  with u = t c^2 sb / sa,  sa <- sa sqrt(1 + t^2),
// which gives exactly the rotated columns (substitute the new b into the
// second shear: the coefficient of A is c (1 + t^2) (1 - t^2 c^2) = c).  Each
// row costs two FMAs and no register copies.  The angle t is the root of
// t^2 + 2 zeta t - 1 = 0 of smaller magnitude, zeta = (nb - na) / (2 gamma),
// written as  t = sign(zeta) |2 gamma| / (|nb - na| + sqrt((nb - na)^2 + 4 gamma^2))
// (no division by gamma); t itself needs no full precision, since the map is
// an exact rotation for whatever t is used once c = 1 / sqrt(1 + t^2) is
// exact for it, so only c takes two Newton steps.
template <int R>
__device__ __forceinline__ void jacobi_rotate(double (&a)[R], double (&b)[R], double& na, double& nb, double& sa,
                                              double& sb, double& offmax) {
    double g0 = 0.0, g1 = 0.0, g2 = 0.0, g3 = 0.0;
#pragma unroll
    for (int e = 0; e < R; e += 4) {
        g0 = fma(a[e], b[e], g0);
        g1 = fma(a[e + 1], b[e + 1], g1);
        g2 = fma(a[e + 2], b[e + 2], g2);
        g3 = fma(a[e + 3], b[e + 3], g3);
    }
    const double ga = qsum((g0 + g1) + (g2 + g3)) * (sa * sb);
    const double al = na, be = nb;
    const double rel = (ga != 0.0) ? fabs(ga) * rsq1(al * be) : 0.0;
    offmax = fmax(offmax, rel);
    const bool rot = rel > JACOBI_TOL;
    if (!__any(rot)) return;
    // lanes whose pair needs no rotation apply the identity (u = v = 0,
    // scale factors 1, exact), so that the update below runs unpredicated
    double u = 0.0, v = 0.0, fa = 1.0, c = 1.0, tg = 0.0;
    if (rot) {
        const double diff = be - al, h = 2.0 * ga;
        const double x = fma(diff, diff, h * h);
        const double tm = fabs(h) * rcp1(fabs(diff) + x * rsq1(x));
        const double t = ((diff >= 0.0) == (h >= 0.0)) ? tm : -tm;
        const double w = fma(t, t, 1.0);
        c = rsq2(w);
        v = t * sa * rcp2(sb);
        u = t * (c * c) * sb * rcp2(sa);
        fa = w * c;
        tg = t * ga;
    }
#pragma unroll
    for (int e = 0; e < R; ++e) b[e] = fma(v, a[e], b[e]);
#pragma unroll
    for (int e = 0; e < R; ++e) a[e] = fma(-u, b[e], a[e]);
    sa *= fa;
    sb *= c;
    na = al - tg;
    nb = be + tg;
    const bool need = rot && ((na < 1e-2 * al) || (nb < 1e-2 * be));
    if (__any(need)) {   // heavy cancellation somewhere in the wavefront: exact norms
        const double ea = sumsq<R>(a) * (sa * sa), eb = sumsq<R>(b) * (sb * sb);
        if (need) {
            na = ea;
            nb = eb;
        }
    }
}

template <int D>
__global__ __launch_bounds__(D * 2) void jacobi_kernel(int d, const double* __restrict__ Bm,
                                                      double* __restrict__ lam, double* __restrict__ Z,
                                                      double* __restrict__ T, int* __restrict__ status) {
    constexpr int NW = D / 32;   // wavefronts
    constexpr int S = D / 2;     // slots
    constexpr int R = D / 4;     // rows per lane and column
    constexpr int NTH = NW * WAVE;
    __shared__ double xbuf[NW * R * WAVE];
    __shared__ double xnrm[NW * WAVE];
    __shared__ double xscl[NW * WAVE];
    __shared__ double sig[D];
    __shared__ int rank_of[D];
    __shared__ double wmax[NW];
    const int tid = threadIdx.x, lane = tid % WAVE, w = tid / WAVE;
    const int li = lane % 16, q = lane / 16;
    const int slot = 16 * w + li;

    double a[R], b[R];
#pragma unroll
    for (int e = 0; e < R; ++e) {
        const int row = q * R + e;
        const int ca = slot, cb = slot + S;
        a[e] = (ca < d && row < d) ? Bm[(int64_t)ca * kMaxD + row] : 0.0;
        b[e] = (cb < d && row < d) ? Bm[(int64_t)cb * kMaxD + row] : 0.0;
    }

    // exchange of b (with its norm and scale) with wavefront w ^ kw
    auto xwave_b = [&](int kw, double& nb, double& sb) {
        double* mine = xbuf + (size_t)w * R * WAVE;
#pragma unroll
        for (int e = 0; e < R; ++e) mine[e * WAVE + lane] = b[e];
        xnrm[w * WAVE + lane] = nb;
        xscl[w * WAVE + lane] = sb;
        __syncthreads();
        const double* src = xbuf + (size_t)(w ^ kw) * R * WAVE;
#pragma unroll
        for (int e = 0; e < R; ++e) b[e] = src[e * WAVE + lane];
        nb = xnrm[(w ^ kw) * WAVE + lane];
        sb = xscl[(w ^ kw) * WAVE + lane];
        __syncthreads();
    };
    // level start: the lower slot's b <-> the upper slot's a (slots s, s ^ m)
    auto relayout = [&](int m, double& na, double& nb, double& ca, double& cb) {
        const double sa = na, sb = nb, fa = ca, fb = cb;
        if (m >= 16) {
            const int kw = m / 16;
            const bool up = (w & kw) != 0;
            double* mine = xbuf + (size_t)w * R * WAVE;
#pragma unroll
            for (int e = 0; e < R; ++e) {
                const double va = a[e], vb = b[e];
                mine[e * WAVE + lane] = up ? va : vb;
            }
            xnrm[w * WAVE + lane] = up ? sa : sb;
            xscl[w * WAVE + lane] = up ? fa : fb;
            __syncthreads();
            const double* src = xbuf + (size_t)(w ^ kw) * R * WAVE;
#pragma unroll
            for (int e = 0; e < R; ++e) {
                const double v = src[e * WAVE + lane], va = a[e], vb = b[e];
                a[e] = up ? v : va;
                b[e] = up ? vb : v;
            }
            const double vn = xnrm[(w ^ kw) * WAVE + lane];
            const double vs = xscl[(w ^ kw) * WAVE + lane];
            na = up ? vn : sa;
            nb = up ? sb : vn;
            ca = up ? vs : fa;
            cb = up ? fb : vs;
            __syncthreads();
        } else {
            const bool up = (li & m) != 0;
            auto swap_with = [&](auto kconst) {
                constexpr int K = decltype(kconst)::value;
#pragma unroll
                for (int e = 0; e < R; ++e) {
                    const double va = a[e], vb = b[e];
                    const double v = xperm<K>(up ? va : vb);
                    a[e] = up ? v : va;
                    b[e] = up ? vb : v;
                }
                const double vn = xperm<K>(up ? sa : sb);
                na = up ? vn : sa;
                nb = up ? sb : vn;
                const double vs = xperm<K>(up ? fa : fb);
                ca = up ? vs : fa;
                cb = up ? fb : vs;
            };
            if (m == 8) swap_with(std::integral_constant<int, 8>{});
            else if (m == 4) swap_with(std::integral_constant<int, 4>{});
            else if (m == 2) swap_with(std::integral_constant<int, 2>{});
            else swap_with(std::integral_constant<int, 1>{});
        }
    };

    int sweeps = 0;
    double sa = 1.0, sb = 1.0;   // column scales (fast rotations)
    for (int sweep = 0; sweep < JACOBI_MAX_SWEEPS; ++sweep) {
        ++sweeps;
        // fold the scales back in and take exact norms at every sweep start
#pragma unroll
        for (int e = 0; e < R; ++e) {
            a[e] *= sa;
            b[e] *= sb;
        }
        sa = sb = 1.0;
        double na = sumsq<R>(a), nb = sumsq<R>(b);
        double offmax = 0.0;
        auto rot = [&]() { jacobi_rotate<R>(a, b, na, nb, sa, sb, offmax); };
        auto mv = [&](auto kconst) {
            constexpr int K = decltype(kconst)::value;
#pragma unroll
            for (int e = 0; e < R; ++e) b[e] = xperm<K>(b[e]);
            nb = xperm<K>(nb);
            sb = xperm<K>(sb);
        };
        // levels with groups of 16 slots or more: b rotates by one lane inside
        // the 16-lane rows, and moves between wavefronts every 16 steps
        int L = 0;
        for (int G = S; G >= 16; G >>= 1, ++L) {
            if (L > 0) relayout(G, na, nb, sa, sb);
            for (int blk = 0; blk < G / 16; ++blk) {
                if (blk > 0) xwave_b(1 << __builtin_ctz(blk), nb, sb);
                rot();
                for (int u = 1; u < 16; ++u) {
#pragma unroll
                    for (int e = 0; e < R; ++e) b[e] = dmov<0x121>(b[e]);   // row_ror:1
                    nb = dmov<0x121>(nb);
                    sb = dmov<0x121>(sb);
                    rot();
                }
            }
        }
        // groups of 8, 4, 2, 1 slots: XOR moves in Gray-code order
        using I1 = std::integral_constant<int, 1>;
        using I2 = std::integral_constant<int, 2>;
        using I4 = std::integral_constant<int, 4>;
        relayout(8, na, nb, sa, sb);
        rot(); mv(I1{}); rot(); mv(I2{}); rot(); mv(I1{}); rot();
        mv(I4{}); rot(); mv(I1{}); rot(); mv(I2{}); rot(); mv(I1{}); rot();
        relayout(4, na, nb, sa, sb);
        rot(); mv(I1{}); rot(); mv(I2{}); rot(); mv(I1{}); rot();
        relayout(2, na, nb, sa, sb);
        rot(); mv(I1{}); rot();
        relayout(1, na, nb, sa, sb);
        rot();
        const double wm = wave_max(offmax);
        if (lane == 0) wmax[w] = wm;
        __syncthreads();
        double om = 0.0;
#pragma unroll
        for (int k = 0; k < NW; ++k) om = fmax(om, wmax[k]);
        __syncthreads();
        if (om <= JACOBI_TOL) break;
    }
#pragma unroll
    for (int e = 0; e < R; ++e) {
        a[e] *= sa;
        b[e] *= sb;
    }
    if (tid == 0 && status) status[ST_SWEEPS] = sweeps;

    // singular values, ranks (ascending sigma, position breaks ties), outputs
    const double siga = sqrt(sumsq<R>(a)), sigb = sqrt(sumsq<R>(b));
    if (q == 0) {
        sig[slot] = siga;
        sig[S + slot] = sigb;
    }
    __syncthreads();
    for (int p = tid; p < D; p += NTH) {
        int r = -1;
        if (sig[p] > 0.0) {
            r = 0;
            for (int o = 0; o < D; ++o)
                if (sig[o] > 0.0 && (sig[o] < sig[p] || (sig[o] == sig[p] && o < p))) ++r;
        }
        rank_of[p] = r;
    }
    __syncthreads();
    if (tid == 0) {
        int nv = 0;
        for (int p = 0; p < D; ++p) nv += rank_of[p] >= 0;
        if (nv != d && status) status[ST_NOTSPD] = 1;   // singular B: cannot happen for SPD K^, M^
    }
    auto emit = [&](const double (&x)[R], int pos) {
        const int r = rank_of[pos];
        if (r < 0 || r >= d) return;
        const double sg = sig[pos];
        const double isq = 1.0 / sqrt(sg);
        const double i32 = isq / sg;
#pragma unroll
        for (int e = 0; e < R; ++e) {
            const int row = q * R + e;
            if (row < d) {
                T[(int64_t)r * kMaxD + row] = x[e] * i32;
                Z[(int64_t)r * kMaxD + row] = x[e] * isq;
            }
        }
        if (q == 0) lam[r] = sg;
    };
    emit(a, slot);
    emit(b, S + slot);
}

// ---------------------------------------------------------------------------
// Y <- L^{-T} Y for the lower-triangular L (d x d, ld kMaxD, zeros above the
// diagonal) and d right-hand sides (ld kMaxD): back substitution in the
// column (right-looking) form.  A workgroup of 16 wavefronts holds the rows
// of L in LDS (row i contiguous, diagonal kept apart as reciprocals) and
// solves 16 right-hand sides, one per wavefront, lane l holding rows l and
// l + 64: at step i (descending) x_i = y_i / L(i,i) is broadcast from its
// lane and every row k < i takes y_k -= L(i,k) x_i.
// ---------------------------------------------------------------------------
constexpr int TRSM_W = 16;   // right-hand sides (wavefronts) per workgroup

__global__ __launch_bounds__(TRSM_W * WAVE) void trsm_lt_kernel(int d, const double* __restrict__ L,
                                                               double* __restrict__ Y) {
    __shared__ double Lr[kMaxD * LD];   // Lr[i LD + k] = L(i, k), k < i; 0 elsewhere
    __shared__ double rdiag[kMaxD];
    const int tid = threadIdx.x, lane = tid % WAVE, w = tid / WAVE;
    // column c of L (rows r = tid % 128, coalesced) into row r of Lr; 8 loads
    // in flight per thread
    constexpr int NT = TRSM_W * WAVE;
    const int r = tid % kMaxD;
    for (int c0 = tid / kMaxD; c0 < d; c0 += 8 * (NT / kMaxD)) {
        double v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int c = c0 + k * (NT / kMaxD);
            v[k] = (c < d && r < d) ? L[(int64_t)c * kMaxD + r] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int c = c0 + k * (NT / kMaxD);
            if (c < d) {
                Lr[r * LD + c] = (r == c) ? 0.0 : v[k];
                if (r == c) rdiag[r] = 1.0 / v[k];
            }
        }
    }
    __syncthreads();
    const int col = blockIdx.x * TRSM_W + w;
    if (col >= d) return;   // no barrier follows
    double* y = Y + (int64_t)col * kMaxD;
    const int j0 = lane, j1 = lane + 64;
    double y0 = j0 < d ? y[j0] : 0.0, y1 = j1 < d ? y[j1] : 0.0;
    for (int i = d - 1; i >= 0; --i) {
        const double xi = readlane(i < 64 ? y0 : y1, i & 63) * rdiag[i];
        if (lane == (i & 63)) {
            if (i < 64) y0 = xi;
            else y1 = xi;
        }
        const double* li = Lr + i * LD;
        y0 = fma(-li[j0], xi, y0);   // L(i, k) = 0 for k >= i
        if (i > 64) y1 = fma(-li[j1], xi, y1);
    }
    if (j0 < d) y[j0] = y0;
    if (j1 < d) y[j1] = y1;
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
    // d <= kMaxD = 128: a wavefront covers a column with two entries per lane.
    // Every wavefront forms the pivot quantities of column l itself (same
    // data, same order: bitwise the same decisions everywhere, no barrier),
    // the wavefronts then update the later columns they own, and one barrier
    // per kept column orders that against the next pivot.  Column l stays
    // unscaled in LDS (later steps never read it); its scaled form goes to
    // Ph, Qh.
    __shared__ double P[kMaxD * 64];
    __shared__ double Q[kMaxD * 64];
    __shared__ double xn[64], yn[64];
    __shared__ int live[64];
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid % WAVE, wid = tid / WAVE;
    constexpr int NWV = 256 / WAVE;
    for (int idx = tid; idx < d * nw; idx += nt) {
        const int i = idx % d, j = idx / d;
        P[j * kMaxD + i] = Vin[(int64_t)j * kMaxD + i];
        Q[j * kMaxD + i] = Uin[(int64_t)j * kMaxD + i];
    }
    __syncthreads();
    // column norms of the projected inputs (x_l, y_l of the MGS) and liveness
    for (int j = wid; j < nw; j += NWV) {
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
    const int i0 = lane, i1 = lane + WAVE;
    int np = 0;
    for (int l = 0; l < nw; ++l) {
        if (!live[l]) continue;
        const double* p = P + l * kMaxD;
        const double* q = Q + l * kMaxD;
        const double p0 = i0 < d ? p[i0] : 0.0, p1 = i1 < d ? p[i1] : 0.0;
        const double q0 = i0 < d ? q[i0] : 0.0, q1 = i1 < d ? q[i1] : 0.0;
        const double eta = wsum(p0 * q0 + p1 * q1);
        const double pn = sqrt(wsum(p0 * p0 + p1 * p1));
        const double qn = sqrt(wsum(q0 * q0 + q1 * q1));
        if (eta == 0.0 || fabs(eta) <= cos_tol * pn * qn || pn <= dep_tol * xn[l] || qn <= dep_tol * yn[l]) continue;
        const double sl = sqrt(fabs(eta));
        const double rl = eta < 0 ? -sl : sl;
        const double irl = 1.0 / rl, isl = 1.0 / sl;
        const double pv0 = p0 * irl, pv1 = p1 * irl, qv0 = q0 * isl, qv1 = q1 * isl;
        if (wid == (l % NWV)) {
            if (i0 < d) {
                Ph[(int64_t)np * kMaxD + i0] = pv0;
                Qh[(int64_t)np * kMaxD + i0] = qv0;
            }
            if (i1 < d) {
                Ph[(int64_t)np * kMaxD + i1] = pv1;
                Qh[(int64_t)np * kMaxD + i1] = qv1;
            }
        }
        // later columns: r_j = q_l . p_j, p_j -= r_j p_l; s_j = p_l . q_j, q_j -= s_j q_l
        for (int j = l + 1 + wid; j < nw; j += NWV) {
            double* pj = P + j * kMaxD;
            double* qj = Q + j * kMaxD;
            const double a0 = i0 < d ? pj[i0] : 0.0, a1 = i1 < d ? pj[i1] : 0.0;
            const double b0 = i0 < d ? qj[i0] : 0.0, b1 = i1 < d ? qj[i1] : 0.0;
            const double r = wsum(qv0 * a0 + qv1 * a1);
            const double sj = wsum(pv0 * b0 + pv1 * b1);
            if (i0 < d) {
                pj[i0] = a0 - r * pv0;
                qj[i0] = b0 - sj * qv0;
            }
            if (i1 < d) {
                pj[i1] = a1 - r * pv1;
                qj[i1] = b1 - sj * qv1;
            }
        }
        ++np;
        __syncthreads();
    }
    if (tid == 0) status[ST_NP] = np;
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

// Coefficient pass of block MGS-Biorth for m <= CM columns: the recurrence of
// coef_mgs_kernel (every inner product taken against the original Gram
// blocks, which keeps the column form's accuracy on ill-conditioned inputs)
// with the three Gram blocks and the coefficient vectors resident in LDS.
// Four wavefronts: in each step wavefront p forms one of the four Gram
// products (lane = row), wavefront 0 the pivot and norms, wavefronts 0 and 1
// the coefficients r_j and s_j of the later columns (lane = j), and all
// threads the right-looking update.
constexpr int CM = 56;
constexpr int CL = CM + 1;

__global__ __launch_bounds__(256) void coef_mgs_lds_kernel(int m, const double* __restrict__ G, int64_t ldg,
                                                           double* __restrict__ Aout, double* __restrict__ Bout,
                                                           int* __restrict__ status, double cos_tol,
                                                           double dep_tol) {
    __shared__ double gxx[CM * CL], gxy[CM * CL], gyy[CM * CL];   // g[i * CL + k] = G(i, k)
    __shared__ double A[CM * CL], B[CM * CL];                      // A[j * CL + i] = a_j[i]
    __shared__ double tv[4][CM];                                   // Gxy b_l, Gxx a_l, Gyy b_l, Gxy^T a_l
    __shared__ double rs[2][CM];
    __shared__ double sc[4];
    const int tid = threadIdx.x, lane = tid % WAVE, wid = tid / WAVE;
    for (int idx = tid; idx < m * m; idx += 256) {
        const int i = idx % m, k = idx / m;
        gxx[i * CL + k] = G[(int64_t)k * ldg + i];
        gxy[i * CL + k] = G[(int64_t)(m + k) * ldg + i];
        gyy[i * CL + k] = G[(int64_t)(m + k) * ldg + (m + i)];
        A[k * CL + i] = (i == k) ? 1.0 : 0.0;
        B[k * CL + i] = (i == k) ? 1.0 : 0.0;
    }
    __syncthreads();
    int np = 0;
    for (int l = 0; l < m; ++l) {
        const double* al = A + l * CL;
        const double* bl = B + l * CL;
        // a_l, b_l are supported on rows 0..l
        if (lane < m) {
            const int i = lane;
            const double* v = (wid == 1 || wid == 3) ? al : bl;
            double s0 = 0.0, s1 = 0.0;
            int k = 0;
            if (wid == 3) {
                for (; k + 1 <= l; k += 2) {
                    s0 += gxy[k * CL + i] * v[k];
                    s1 += gxy[(k + 1) * CL + i] * v[k + 1];
                }
                if (k == l) s0 += gxy[k * CL + i] * v[k];
            } else {
                const double* g = (wid == 0) ? gxy : (wid == 1 ? gxx : gyy);
                for (; k + 1 <= l; k += 2) {
                    s0 += g[i * CL + k] * v[k];
                    s1 += g[i * CL + k + 1] * v[k + 1];
                }
                if (k == l) s0 += g[i * CL + k] * v[k];
            }
            tv[wid][i] = s0 + s1;
        }
        __syncthreads();
        if (wid == 0) {
            double e = 0.0, p = 0.0, q = 0.0;
            if (lane <= l) {
                e = al[lane] * tv[0][lane];
                p = al[lane] * tv[1][lane];
                q = bl[lane] * tv[2][lane];
            }
            e = wave_sum(e);
            p = wave_sum(p);
            q = wave_sum(q);
            if (lane == 0) {
                sc[0] = e;
                sc[1] = sqrt(fmax(p, 0.0));
                sc[2] = sqrt(fmax(q, 0.0));
            }
        }
        __syncthreads();
        const double e = sc[0], pn = sc[1], qn = sc[2];
        const double xn = sqrt(gxx[l * CL + l]), yn = sqrt(gyy[l * CL + l]);
        if (e == 0.0 || fabs(e) <= cos_tol * pn * qn || pn <= dep_tol * xn || qn <= dep_tol * yn) continue;
        const double sl = sqrt(fabs(e));
        const double rl = e < 0 ? -sl : sl;
        __syncthreads();   // all threads have read sc before it is reused
        if (tid < m) {
            const int i = tid;
            const double av = (i <= l) ? al[i] / rl : 0.0, bv = (i <= l) ? bl[i] / sl : 0.0;
            Aout[(int64_t)np * kMaxD + i] = av;
            Bout[(int64_t)np * kMaxD + i] = bv;
            if (i <= l) {
                A[l * CL + i] = av;
                B[l * CL + i] = bv;
            }
            tv[0][i] /= sl;   // Gxy b_l with the scaled b_l
            tv[3][i] /= rl;   // Gxy^T a_l with the scaled a_l
        }
        ++np;
        __syncthreads();
        // r_j = (Gxy b_l) . a_j (wavefront 0), s_j = (Gxy^T a_l) . b_j (wavefront 1), j > l
        if (wid < 2 && lane > l && lane < m) {
            const int j = lane;
            const double* t = (wid == 0) ? tv[0] : tv[3];
            const double* c = (wid == 0) ? (A + j * CL) : (B + j * CL);
            double s0 = 0.0, s1 = 0.0;
            int i = 0;
            for (; i + 1 <= j; i += 2) {
                s0 += t[i] * c[i];
                s1 += t[i + 1] * c[i + 1];
            }
            if (i == j) s0 += t[i] * c[i];
            rs[wid][j] = s0 + s1;
        }
        __syncthreads();
        for (int idx = tid; idx < (l + 1) * (m - l - 1); idx += 256) {
            const int i = idx % (l + 1), j = l + 1 + idx / (l + 1);
            A[j * CL + i] -= rs[0][j] * A[l * CL + i];
            B[j * CL + i] -= rs[1][j] * B[l * CL + i];
        }
        __syncthreads();
    }
    if (tid == 0) status[ST_NKEPT] = np;
}

}  // namespace

hipError_t small_lrep(hipStream_t st, int d, const double* Kh, const double* Mh, int64_t ldh, double* lam,
                      double* Xh, double* Yh, double* scratch, int* status, double* work, size_t work_elems) {
    if (d < 1 || d > kMaxD) return hipErrorInvalidValue;
    hipLaunchKernelGGL(chol2_kernel, dim3(2), dim3(256), 0, st, d, Kh, Mh, ldh, scratch, status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // B = L2^T L1 into scratch + 3 D2
    Seg a{scratch + D2, kMaxD, d}, b{scratch, kMaxD, d};
    e = gemm_tn(st, d, d, d, &a, 1, &b, 1, scratch + 3 * D2, kMaxD, 1.0, 0, work, work_elems);
    if (e != hipSuccess) return e;
    double* T = scratch + 2 * D2;
    const double* Bm = scratch + 3 * D2;
    if (d <= 32)
        hipLaunchKernelGGL(jacobi_kernel<32>, dim3(1), dim3(64), 0, st, d, Bm, lam, Yh, T, status);
    else if (d <= 64)
        hipLaunchKernelGGL(jacobi_kernel<64>, dim3(1), dim3(128), 0, st, d, Bm, lam, Yh, T, status);
    else
        hipLaunchKernelGGL(jacobi_kernel<128>, dim3(1), dim3(256), 0, st, d, Bm, lam, Yh, T, status);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // X^ = L2 T, Y^ = L2^{-T} Z (Z written to Yh by the Jacobi kernel)
    Seg l2{scratch + D2, kMaxD, d};
    e = gemm_nn(st, d, d, d, &l2, 1, T, kMaxD, Xh, kMaxD, 1.0, 0.0, work, work_elems);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(trsm_lt_kernel, dim3((d + TRSM_W - 1) / TRSM_W), dim3(TRSM_W * WAVE), 0, st, d,
                       scratch + D2, Yh);
    return hipGetLastError();
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
    if (m <= CM) {
        hipLaunchKernelGGL(coef_mgs_lds_kernel, dim3(1), dim3(256), 0, st, m, G, ldg, A, B, status, cos_tol,
                           dep_tol);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(coef_mgs_kernel, dim3(1), dim3(256), 0, st, m, G, ldg, scratch, scratch + D2, A, B, status,
                       cos_tol, dep_tol);
    return hipGetLastError();
}

}  // namespace lrep
