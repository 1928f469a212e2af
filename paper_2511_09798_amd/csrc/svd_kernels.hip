// svd_kernels.hip -- SVD of the projected bidiagonal C_l (Algorithm 2 step 2,
// Algorithm 4 step 2) on the device, by multisection for the singular values
// and twisted factorisations for the vectors, with the implicit QR iteration
// (k_bidiag_svd) as the fallback for spectra the fast path does not resolve.
//
// Steps, one problem per grid row (blockIdx.y, or blockIdx.x for the
// per-problem kernels):
//  1. k_msvd_setup: the left rotations that take C_l to the upper bidiagonal
//     B (d, e) while carrying beta_1 e_1 (g, and f~_{l+1}); the eigenvalue
//     bound and the pivot floor of the qd transforms.
//  2. k_msvd_values: one workgroup per singular value s_j (the j-th largest):
//     256 counts of the eigenvalues of B^T B below 256 points of the current
//     bracket per round (multisection), about eight rounds to a bracket of two
//     ulps.  Each s_j to high relative accuracy, independently of the others.
//  3. k_msvd_vectors: one wave per j: twisted factorisations of B^T B - s_j^2 I
//     (right vector v_j) and B B^T - s_j^2 I (left vector u_j), the sign of
//     u_j from u_j^T B v_j > 0, the residuals of both relations, h_j = u_j^T g.
//  4. k_msvd_gram: E = V^T V - I (kept) and the largest |U^T U - I| (tile maxima).
//  5. k_msvd_finish: the acceptance test (Gram matrices within 1e-9 of I,
//     residuals within 1e-9 s_j plus a rounding floor); on success V <- V (I - E/2) and
//     f~ = (I - E_U/2) h, which make the vectors orthonormal to second order
//     in E; otherwise the problem is flagged for the fallback.
//  6. k_bidiag_svd (QR) runs for flagged problems only.
// The vectors of singular values with relative gap g are determined by the
// data to about eps/g; the symmetric correction of step 5 restores the
// orthogonality without moving them further than that.
#include <float.h>

#include "bidiag_svd.hpp"
#include "kernels.hpp"
#include "msvd.hpp"

namespace mqh {

namespace {

constexpr int kFinRows = 4;    // rows of V updated per workgroup in k_msvd_finish
constexpr int kGramTile = 32;  // k_msvd_gram tile edge

// |x| with NaN taken as +inf (a maximum that a NaN cannot hide in)
__device__ __forceinline__ double abs_or_inf(double x) { return x == x ? fabs(x) : INFINITY; }

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double w = __shfl_xor(v, o, kWave);
        v = w > v ? w : v;
    }
    return v;
}

template <int NT>
__device__ __forceinline__ double block_max(double v, double* lds) {
    v = wave_max(v);
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) lds[w] = v;
    __syncthreads();
    double m = lds[0];
#pragma unroll
    for (int i = 1; i < NT / kWave; ++i) m = lds[i] > m ? lds[i] : m;
    __syncthreads();
    return m;
}

}  // namespace

// ---------------------------------------------------------------------------
// 1. Setup (one workgroup per problem)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_msvd_setup(const double* __restrict__ alpha,
                                                       const double* __restrict__ beta, int32_t L,
                                                       const int32_t* __restrict__ l_ptr, double* __restrict__ ws,
                                                       double* __restrict__ ftil, int32_t* __restrict__ status,
                                                       ProjBatch pb) {
    const int64_t z = blockIdx.x;
    alpha += z * pb.vec;
    beta += z * pb.vec;
    ftil += z * pb.vec;
    if (l_ptr != nullptr) l_ptr += z * pb.lstr;
    if (status != nullptr) status += z;
    const SvdWs w = svd_ws(ws + z * pb.ws, L);
    const int l = l_ptr != nullptr ? *l_ptr : L;
    __shared__ double sa[kMaxEll], sb[kMaxEll + 1], sd[kMaxEll], se[kMaxEll], sg[kMaxEll];
    __shared__ double red[kBlock / kWave];
    const int tid = threadIdx.x;
    if (l <= 0) {
        if (tid == 0) {
            ftil[0] = beta[0];
            w.flag[0] = 0;
            w.flag[1] = 0;
            if (status != nullptr) status[0] = 0;
        }
        return;
    }
    for (int i = tid; i < l; i += kBlock) {
        sa[i] = alpha[i];
        se[i] = 0.0;
    }
    for (int i = tid; i <= l; i += kBlock) sb[i] = beta[i];
    __syncthreads();
    if (tid == 0) ftil[l] = bsvd::reduce_lower(sa, sb, l, sd, se, sg);
    __syncthreads();
    double emax = 0.0, bad = 0.0;
    for (int i = tid; i < l; i += kBlock) {
        w.d[i] = sd[i];
        w.e[i] = se[i];
        w.g[i] = sg[i];
        const double e2 = se[i] * se[i];
        emax = e2 > emax ? e2 : emax;
        // a zero or non-finite pivot of B (an exactly singular bidiagonal)
        // leaves the relative-accuracy transforms undefined: fallback
        bad = (!(sd[i] > 0.0) || !isfinite(sd[i]) || !isfinite(se[i]) || !isfinite(sg[i])) ? 1.0 : bad;
    }
    emax = block_max<kBlock>(emax, red);
    bad = block_max<kBlock>(bad, red);
    if (tid == 0) {
        w.misc[0] = msvd::eig_bound(sd, se, l);
        w.misc[1] = DBL_MIN * (emax > 1.0 ? emax : 1.0);
        w.flag[0] = bad > 0.0 ? 1 : 0;
        w.flag[1] = 0;
    }
}

// ---------------------------------------------------------------------------
// 2. Values: workgroup j of problem z brackets lambda_j = s_j^2, the j-th
// largest eigenvalue of B^T B, by rounds of kSections counts.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_msvd_values(int32_t L, const int32_t* __restrict__ l_ptr,
                                                        double* __restrict__ ws, double* __restrict__ sv,
                                                        ProjBatch pb) {
    static_assert(msvd::kSections == kBlock, "one multisection point per thread");
    const int64_t z = blockIdx.y;
    sv += z * pb.vec;
    if (l_ptr != nullptr) l_ptr += z * pb.lstr;
    const SvdWs w = svd_ws(ws + z * pb.ws, L);
    const int l = l_ptr != nullptr ? *l_ptr : L;
    const int j = blockIdx.x;
    if (j >= l) return;
    __shared__ double d2[kMaxEll], e2[kMaxEll];
    __shared__ double xs[kBlock];
    __shared__ unsigned long long masks[kBlock / kWave];
    const int tid = threadIdx.x;
    for (int i = tid; i < l; i += kBlock) {
        const double di = w.d[i], ei = w.e[i];
        d2[i] = di * di;
        e2[i] = ei * ei;
    }
    const double pivmin = w.misc[1];
    double lo = 0.0, hi = w.misc[0];
    const int k = l - 1 - j;  // lambda_j is the k-th smallest (0-based)
    __syncthreads();
    for (int round = 0; round < 64; ++round) {
        if (hi - lo <= 2.0 * DBL_EPSILON * hi) break;
        const double x = msvd::section_point(lo, hi, tid, kBlock);
        const int c = msvd::negcount(d2, 1, e2, 1, l, x, pivmin);
        xs[tid] = x;
        const unsigned long long m = __ballot(c <= k);
        if ((tid & (kWave - 1)) == 0) masks[tid / kWave] = m;
        __syncthreads();
        // the largest point with at most k eigenvalues below it
        int ts = -1;
        for (int q = kBlock / kWave - 1; q >= 0 && ts < 0; --q)
            if (masks[q] != 0ull) ts = q * kWave + 63 - __clzll(masks[q]);
        const double nlo = ts >= 0 ? xs[ts] : lo;
        const double nhi = ts + 1 < kBlock ? xs[ts + 1] : hi;
        __syncthreads();
        if (nlo == lo && nhi == hi) break;
        lo = nlo;
        hi = nhi;
    }
    if (tid == 0) {
        const double lam = lo + 0.5 * (hi - lo);
        w.lam[j] = lam;
        sv[j] = sqrt(lam);
        // s_j below 2^-500 of the bound: not bracketed from below
        if (!(lo > 0.0)) w.flag[0] = 1;
    }
}

// ---------------------------------------------------------------------------
// 3. Vectors: one wave per (j, problem).  LDS: d, e and two arrays per side
// (side 0 = B^T B on (d, e), side 1 = B B^T on the reversed sequences).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kWave) void k_msvd_vectors(int32_t L, const int32_t* __restrict__ l_ptr,
                                                        double* __restrict__ ws, const double* __restrict__ sv,
                                                        double* __restrict__ V, int64_t ldv, ProjBatch pb) {
    const int64_t z = blockIdx.y;
    sv += z * pb.vec;
    V += z * pb.mat;
    if (l_ptr != nullptr) l_ptr += z * pb.lstr;
    const SvdWs w = svd_ws(ws + z * pb.ws, L);
    const int l = l_ptr != nullptr ? *l_ptr : L;
    const int j = blockIdx.x;
    if (j >= l) return;
    extern __shared__ double sh[];
    double* Ld = sh;
    double* Le = sh + L;
    double* A[2] = {sh + 2 * L, sh + 4 * L};  // L+ then z
    double* Bv[2] = {sh + 3 * L, sh + 5 * L};  // s then U-
    __shared__ int s_r[2];
    const int lane = threadIdx.x;
    for (int i = lane; i < l; i += kWave) {
        Ld[i] = w.d[i];
        Le[i] = w.e[i];
    }
    const double lam = w.lam[j];
    const double sig = sv[j];
    const double pivmin = w.misc[1];
    __syncthreads();
    if (lane < 2) {
        // both lanes run the same instructions on their own sequences
        const int side = lane;
        const double* dp = side ? Ld + (l - 1) : Ld;
        const double* ep = (side && l >= 2) ? Le + (l - 2) : Le;
        const int st = side ? -1 : 1;
        msvd::stationary(dp, st, ep, st, l, lam, pivmin, A[side], Bv[side]);
        double gr;
        s_r[side] = msvd::progressive_twist(dp, st, ep, st, l, lam, pivmin, Bv[side], &gr);
    }
    __syncthreads();
    if (lane < 4) {
        const int side = lane >> 1;
        const int dir = (lane & 1) ? 1 : -1;
        const int r = s_r[side];
        msvd::twisted_solve(A[side], Bv[side], l, r, dir);
        if (dir < 0) A[side][r] = 1.0;
    }
    __syncthreads();
    // norms; side 1 holds u in reversed order: u_k = A[1][l-1-k]
    double nv = 0.0, nu = 0.0;
    for (int k = lane; k < l; k += kWave) {
        nv = fma(A[0][k], A[0][k], nv);
        nu = fma(A[1][k], A[1][k], nu);
    }
    nv = wave_sum(nv);
    nu = wave_sum(nu);
    const double iv = 1.0 / sqrt(nv), iu = 1.0 / sqrt(nu);
    // sign of u from u^T B v > 0
    double t = 0.0;
    for (int k = lane; k < l; k += kWave) {
        const double vk1 = k + 1 < l ? Le[k] * A[0][k + 1] : 0.0;
        t = fma(A[1][l - 1 - k], fma(Ld[k], A[0][k], vk1), t);
    }
    t = wave_sum(t);
    const double su = t < 0.0 ? -iu : iu;
    // residuals of B v = s u and B^T u = s v; h = u^T g
    double r1 = 0.0, r2 = 0.0, hg = 0.0;
    for (int k = lane; k < l; k += kWave) {
        const double vk = A[0][k] * iv;
        const double vk1 = k + 1 < l ? A[0][k + 1] * iv : 0.0;
        const double uk = A[1][l - 1 - k] * su;
        const double ukm = k > 0 ? A[1][l - k] * su : 0.0;
        const double a = msvd::resid_row(Ld[k], vk, k + 1 < l ? Le[k] : 0.0, vk1, sig, uk);
        const double b = msvd::resid_row(Ld[k], uk, k > 0 ? Le[k - 1] : 0.0, ukm, sig, vk);
        hg = fma(uk, w.g[k], hg);
        r1 = fma(a, a, r1);
        r2 = fma(b, b, r2);
    }
    r1 = wave_sum(r1);
    r2 = wave_sum(r2);
    hg = wave_sum(hg);
    for (int k = lane; k < l; k += kWave) {
        V[(int64_t)j * ldv + k] = A[0][k] * iv;
        w.U[(int64_t)j * L + k] = A[1][l - 1 - k] * su;
    }
    if (lane == 0) {
        w.h[j] = hg;
        const double rr = sqrt(r1 > r2 ? r1 : r2) / msvd::resid_bound(sig, sv[0], l);
        w.res[j] = rr == rr ? rr : INFINITY;
    }
}

// ---------------------------------------------------------------------------
// 4. Gram matrices: tile (bx, by) of V^T V - I (which = 0, kept in E) or of
// U^T U - I (which = 1, only its largest entry), 2 x 2 entries per thread.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_msvd_gram(int32_t L, const int32_t* __restrict__ l_ptr,
                                                      double* __restrict__ ws, const double* __restrict__ V,
                                                      int64_t ldv, ProjBatch pb) {
    const int which = blockIdx.z & 1;
    const int64_t z = blockIdx.z >> 1;
    V += z * pb.mat;
    if (l_ptr != nullptr) l_ptr += z * pb.lstr;
    const SvdWs w = svd_ws(ws + z * pb.ws, L);
    const int l = l_ptr != nullptr ? *l_ptr : L;
    const int ntl = (l + kGramTile - 1) / kGramTile;
    const int bi = blockIdx.x, bj = blockIdx.y;
    if (bi >= ntl || bj >= ntl) return;
    const double* M = which ? w.U : V;
    const int64_t ld = which ? (int64_t)L : ldv;
    __shared__ double Xi[kGramTile][kGramTile + 1], Xj[kGramTile][kGramTile + 1];
    __shared__ double red[kBlock / kWave];
    const int tid = threadIdx.x;
    const int ty = tid / 16, tx = tid % 16;
    double acc00 = 0.0, acc01 = 0.0, acc10 = 0.0, acc11 = 0.0;
    for (int k0 = 0; k0 < l; k0 += kGramTile) {
        for (int q = tid; q < kGramTile * kGramTile; q += kBlock) {
            const int c = q / kGramTile, kk = q % kGramTile;
            const int ci = bi * kGramTile + c, cj = bj * kGramTile + c, kr = k0 + kk;
            Xi[c][kk] = (ci < l && kr < l) ? M[(int64_t)ci * ld + kr] : 0.0;
            Xj[c][kk] = (cj < l && kr < l) ? M[(int64_t)cj * ld + kr] : 0.0;
        }
        __syncthreads();
#pragma unroll 8
        for (int kk = 0; kk < kGramTile; ++kk) {
            const double a0 = Xi[2 * ty][kk], a1 = Xi[2 * ty + 1][kk];
            const double b0 = Xj[2 * tx][kk], b1 = Xj[2 * tx + 1][kk];
            acc00 = fma(a0, b0, acc00);
            acc01 = fma(a0, b1, acc01);
            acc10 = fma(a1, b0, acc10);
            acc11 = fma(a1, b1, acc11);
        }
        __syncthreads();
    }
    double m = 0.0;
    const double acc[2][2] = {{acc00, acc01}, {acc10, acc11}};
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int i = bi * kGramTile + 2 * ty + a, jj = bj * kGramTile + 2 * tx + b;
            if (i < l && jj < l) {
                const double v = acc[a][b] - (i == jj ? 1.0 : 0.0);
                if (!which) w.E[(int64_t)i * L + jj] = v;
                const double av = abs_or_inf(v);
                m = av > m ? av : m;
            }
        }
    m = block_max<kBlock>(m, red);
    if (tid == 0) w.tmax[which * kSvdTiles + bi * (kSvdTiles / 32) + bj] = m;
}

// ---------------------------------------------------------------------------
// 5. Acceptance test and the symmetric correction.  Workgroup b updates rows
// b*kFinRows .. of V and computes f~_j for the same j; every workgroup takes
// the same decision from the tile maxima and residuals.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_msvd_finish(int32_t L, const int32_t* __restrict__ l_ptr,
                                                        double* __restrict__ ws, double* __restrict__ V,
                                                        int64_t ldv, double* __restrict__ ftil,
                                                        int32_t* __restrict__ status, ProjBatch pb) {
    const int64_t z = blockIdx.y;
    V += z * pb.mat;
    ftil += z * pb.vec;
    if (l_ptr != nullptr) l_ptr += z * pb.lstr;
    if (status != nullptr) status += z;
    const SvdWs w = svd_ws(ws + z * pb.ws, L);
    const int l = l_ptr != nullptr ? *l_ptr : L;
    const int r0 = blockIdx.x * kFinRows;
    if (r0 >= l) return;
    __shared__ double vr[kFinRows][kMaxEll];
    __shared__ double hs[kMaxEll], wv[kMaxEll];
    __shared__ double red[kBlock / kWave];
    const int tid = threadIdx.x;
    const int ntl = (l + kGramTile - 1) / kGramTile;
    double mo = 0.0, mr = 0.0;
    for (int q = tid; q < 2 * ntl * ntl; q += kBlock) {
        const int which = q / (ntl * ntl), rem = q % (ntl * ntl);
        const double v = abs_or_inf(w.tmax[which * kSvdTiles + (rem / ntl) * (kSvdTiles / 32) + rem % ntl]);
        mo = v > mo ? v : mo;
    }
    for (int i = tid; i < l; i += kBlock) {
        const double v = abs_or_inf(w.res[i]);
        mr = v > mr ? v : mr;
    }
    mo = block_max<kBlock>(mo, red);
    mr = block_max<kBlock>(mr, red);
    const bool ok = w.flag[0] == 0 && mo <= msvd::kOrthTol && mr <= 1.0;
    if (!ok) {
        if (blockIdx.x == 0 && tid == 0) {
            w.flag[1] = 1;
            if (status != nullptr) status[0] = 2;
        }
        return;
    }
    const int nr = l - r0 < kFinRows ? l - r0 : kFinRows;
    for (int i = tid; i < l; i += kBlock) {
#pragma unroll
        for (int q = 0; q < kFinRows; ++q) vr[q][i] = q < nr ? V[(int64_t)i * ldv + r0 + q] : 0.0;
        hs[i] = w.h[i];
    }
    __syncthreads();
    // w = U h (every workgroup: the f~ of its rows need all of it)
    for (int r = tid; r < l; r += kBlock) {
        double a = 0.0;
        for (int jj = 0; jj < l; ++jj) a = fma(w.U[(int64_t)jj * L + r], hs[jj], a);
        wv[r] = a;
    }
    // rows of V (I - E/2); E is symmetric, read along its rows
    for (int jj = tid; jj < l; jj += kBlock) {
        double acc[kFinRows] = {};
        for (int i = 0; i < l; ++i) {
            const double eij = w.E[(int64_t)i * L + jj];
#pragma unroll
            for (int q = 0; q < kFinRows; ++q) acc[q] = fma(vr[q][i], eij, acc[q]);
        }
#pragma unroll
        for (int q = 0; q < kFinRows; ++q)
            if (q < nr) V[(int64_t)jj * ldv + r0 + q] = fma(-0.5, acc[q], vr[q][jj]);
    }
    __syncthreads();
    // f~_j = h_j - ((U^T U - I) h)_j / 2 = 1.5 h_j - u_j^T w / 2, one wave per j
    const int wid = tid / kWave, lane = tid % kWave;
    if (wid < nr) {
        const int jj = r0 + wid;
        double a = 0.0;
        for (int r = lane; r < l; r += kWave) a = fma(w.U[(int64_t)jj * L + r], wv[r], a);
        a = wave_sum(a);
        if (lane == 0) ftil[jj] = fma(1.5, hs[jj], -0.5 * a);
    }
    if (blockIdx.x == 0 && tid == 0 && status != nullptr) status[0] = 0;
}

// ---------------------------------------------------------------------------
// Host launcher: the fast path, then the QR iteration for flagged problems
// (mode 0); the QR iteration alone (mode 1); the fast path alone, a failed
// acceptance test leaving status 2 (mode 2).
// ---------------------------------------------------------------------------
void launch_bidiag_svd(const double* alpha, const double* beta, int32_t l, const int32_t* l_ptr, double* ws,
                       double* sv, double* ftil, double* V, int64_t ldv, int32_t* status, int mode, hipStream_t s,
                       int nz, ProjBatch pb) {
    if (mode != 1) {
        k_msvd_setup<<<nz, kBlock, 0, s>>>(alpha, beta, l, l_ptr, ws, ftil, status, pb);
        k_msvd_values<<<dim3(l, nz), kBlock, 0, s>>>(l, l_ptr, ws, sv, pb);
        k_msvd_vectors<<<dim3(l, nz), kWave, 6 * (size_t)l * sizeof(double), s>>>(l, l_ptr, ws, sv, V, ldv, pb);
        const int nt = (l + kGramTile - 1) / kGramTile;
        k_msvd_gram<<<dim3(nt, nt, 2 * nz), kBlock, 0, s>>>(l, l_ptr, ws, V, ldv, pb);
        k_msvd_finish<<<dim3((l + kFinRows - 1) / kFinRows, nz), kBlock, 0, s>>>(l, l_ptr, ws, V, ldv, ftil,
                                                                                 status, pb);
    }
    if (mode != 2) launch_bidiag_qr(alpha, beta, l, l_ptr, ws, sv, ftil, V, ldv, status, mode == 0, s, nz, pb);
}

void launch_msvd_core(int32_t l, double* ws, double* sv, double* ftil, double* V, int64_t ldv, int32_t* status,
                      hipStream_t s) {
    const ProjBatch pb{};
    k_msvd_values<<<dim3(l, 1), kBlock, 0, s>>>(l, nullptr, ws, sv, pb);
    k_msvd_vectors<<<dim3(l, 1), kWave, 6 * (size_t)l * sizeof(double), s>>>(l, nullptr, ws, sv, V, ldv, pb);
    const int nt = (l + kGramTile - 1) / kGramTile;
    k_msvd_gram<<<dim3(nt, nt, 2), kBlock, 0, s>>>(l, nullptr, ws, V, ldv, pb);
    k_msvd_finish<<<dim3((l + kFinRows - 1) / kFinRows, 1), kBlock, 0, s>>>(l, nullptr, ws, V, ldv, ftil, status, pb);
}

}  // namespace mqh
