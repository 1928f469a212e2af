// band_kernels.hip -- the projected problem of the block Golub-Kahan path
// (Algorithm 4 per source on the shared block Krylov space) through the SVD
// of its block bidiagonal C: a Householder bulge chase takes C^T to a scalar
// bidiagonal (band.hpp), the multisection / twisted-factorisation kernels of
// svd_kernels.hip give its SVD, and the data and the solutions of the s
// sources go through the chase's reflectors.
//
// Kernels, one problem per call:
//  1. k_band_chase (one workgroup): C^T in LDS as a band (3 b + 1 doubles per
//     row), the chase in pipelined steps, one task per wave and step; the
//     reflectors to HBM in step order, the bidiagonal (d, e) at the end.
//  2. k_band_data (one workgroup): the s data columns (E_1 e_k; 0) through
//     the right reflectors (replayed in step order from chunks staged in
//     LDS), then through the rotations that take the (N + 1) x N lower
//     bidiagonal (alpha = d, beta_{j+1} = e_j) to the upper bidiagonal B
//     whose SVD the multisection kernels compute; B and the rotated data go
//     to the SVD workspace, ||b_k||^2 beside them.
//  3. the multisection path on B (values, vectors, Gram matrices, acceptance
//     test and symmetric correction of V).
//  4. k_band_mm: F~ = (I - E_U/2) U^T g for the s data columns (three small
//     products), and after the parameter choice yhat_k = V diag(s_j /
//     (s_j^2 + lambda_k^2)) F~_k.
//  5. k_band_solve (one workgroup): the solutions through the left
//     reflectors, last step first.
// A problem the acceptance test rejects is left flagged (status 2) for the
// caller's Jacobi path.
#include <float.h>

#include "band.hpp"
#include "kernels.hpp"
#include "msvd.hpp"

namespace mqh {

namespace {

constexpr int kBandThreads = 1024;  // the replay kernels
constexpr int kBandWaves = kBandThreads / kWave;
constexpr int kChaseThreads = 512;  // the chase: two tasks per wave, 16 per pass (LDS holds the band)
constexpr int kChaseWaves = kChaseThreads / kWave;
constexpr int kStageDoubles = 8192;  // reflectors staged per chunk in the replay kernels (64 KiB)
constexpr int kMmRows = 16;          // output rows per workgroup of k_band_mm

// Orders a wave's LDS accesses across its lanes: what one lane wrote before
// this point is seen by every lane's reads after it.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Tree sum and maximum of |a| over 16 values (short dependency chains).
__device__ __forceinline__ double tree_sum16(const double (&a)[band::kMaxB]) {
    double t[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) t[k] = a[2 * k] + a[2 * k + 1];
#pragma unroll
    for (int k = 0; k < 4; ++k) t[k] = t[2 * k] + t[2 * k + 1];
    return (t[0] + t[1]) + (t[2] + t[3]);
}
__device__ __forceinline__ double tree_absmax16(const double (&a)[band::kMaxB], int k_from) {
    double t[8];
#pragma unroll
    for (int k = 0; k < 8; ++k)
        t[k] = fmax(2 * k >= k_from ? fabs(a[2 * k]) : 0.0, 2 * k + 1 >= k_from ? fabs(a[2 * k + 1]) : 0.0);
#pragma unroll
    for (int k = 0; k < 4; ++k) t[k] = fmax(t[2 * k], t[2 * k + 1]);
    return fmax(fmax(t[0], t[1]), fmax(t[2], t[3]));
}

// The reflector of band.hpp for x_0 .. x_15 (0 past the reflector's length),
// computed alike in every lane: tau, beta and sc (v_k = x_k sc for k >= 1,
// v_0 = 1; sc = 0 when tau = 0).  NaN data make tau NaN, which the
// acceptance test downstream rejects.
__device__ __forceinline__ double local_reflector(const double (&x)[band::kMaxB], double* beta, double* sc) {
    const double amax = tree_absmax16(x, 0), tmax = tree_absmax16(x, 1);
    if (!(tmax > 0.0)) {
        *beta = x[0];
        *sc = 0.0;
        return 0.0;
    }
    const double inv = 1.0 / amax;
    double a[band::kMaxB];
#pragma unroll
    for (int k = 0; k < band::kMaxB; ++k) {
        const double y = x[k] * inv;
        a[k] = y * y;
    }
    const double nrm = amax * sqrt(tree_sum16(a));
    const double bt = x[0] >= 0.0 ? -nrm : nrm;
    *sc = 1.0 / (x[0] - bt);
    *beta = bt;
    return (bt - x[0]) / bt;
}

// y <- (I - tau v v^T) y on n <= 16 entries at y[k * ys], v_k = x_k sc
// (v_0 = 1, v_k = 0 for k >= n); tree dot product.  No branch per entry:
// entries k >= n are read at y[(n - 1) ys] (their v_k is 0) and written to
// the scratch slot sink.
__device__ __forceinline__ void local_apply(const double (&x)[band::kMaxB], double sc, double tau, int n, double* y,
                                            int64_t ys, double* sink) {
    double yv[band::kMaxB], pr[band::kMaxB];
#pragma unroll
    for (int k = 0; k < band::kMaxB; ++k) {
        yv[k] = y[(k < n ? k : n - 1) * ys];
        pr[k] = (k == 0 ? 1.0 : x[k] * sc) * yv[k];
    }
    const double tw = tau * tree_sum16(pr);
#pragma unroll
    for (int k = 0; k < band::kMaxB; ++k) {
        double* dst = k < n ? y + k * ys : sink;
        *dst = fma(-tw, k == 0 ? 1.0 : x[k] * sc, yv[k]);
    }
}

// y[0] = beta, y[k * ys] = 0 for 0 < k < n (entries k >= n to sink).
__device__ __forceinline__ void local_set(double beta, int n, double* y, int64_t ys, double* sink) {
#pragma unroll
    for (int k = 0; k < band::kMaxB; ++k) {
        double* dst = k < n ? y + k * ys : sink;
        *dst = k == 0 ? beta : 0.0;
    }
}

// Up to two tasks of the chase per wave, one per half-wave (hl = lane % 32):
// task (i, t) when on, its reflectors to rr and ll (b + 1 doubles each:
// v_0 .. v_{b-1}, tau); vsh: the half-wave's 16 doubles of LDS, through
// which its lanes get the reflector's data.  One lane per row (right
// reflector) or column (left reflector), at most 2 b <= 32 of them.
__device__ void chase_task(double* B, int N, int Mc, int b, bool on, int i, int t, double* __restrict__ rr,
                           double* __restrict__ ll, double* vsh, double* sink, int hl) {
    int r0 = 0, c0 = 0, c1 = 0;
    if (on) band::task_cols(i, t, b, Mc, r0, c0, c1);
    const int nj = on ? c1 - c0 + 1 : 0, r1 = c1 < N - 1 ? c1 : N - 1;
    const int64_t cs = band::width(b) - 1;  // from (r, c) to (r + 1, c)
    double x[band::kMaxB], beta, sc;
    // right reflector from row r0
    double xk = 0.0;
    if (hl < band::kMaxB) {
        xk = hl < nj ? B[band::at(r0, c0 + hl, b)] : 0.0;
        vsh[hl] = xk;
    }
    wave_sync();
#pragma unroll
    for (int k = 0; k < band::kMaxB; ++k) x[k] = vsh[k];
    const double tau = local_reflector(x, &beta, &sc);
    if (on) {
        if (hl < b) rr[hl] = hl == 0 ? 1.0 : xk * sc;
        if (hl == b) rr[b] = tau;
    }
    if (on && tau != 0.0 && hl <= r1 - r0) {
        if (hl == 0)
            local_set(beta, nj, B + band::at(r0, c0, b), 1, sink);
        else
            local_apply(x, sc, tau, nj, B + band::at(r0 + hl, c0, b), 1, sink);
    }
    wave_sync();
    // left reflector from column c0, rows c0 .. r1
    const int ni = on ? r1 - c0 + 1 : 0;
    xk = 0.0;
    if (hl < band::kMaxB) {
        xk = hl < ni ? B[band::at(c0 + hl, c0, b)] : 0.0;
        vsh[hl] = xk;
    }
    wave_sync();
#pragma unroll
    for (int k = 0; k < band::kMaxB; ++k) x[k] = vsh[k];
    const double tau2 = ni >= 2 ? local_reflector(x, &beta, &sc) : 0.0;
    if (on) {
        if (hl < b) ll[hl] = hl == 0 ? 1.0 : (ni >= 2 ? xk * sc : 0.0);
        if (hl == b) ll[b] = tau2;
    }
    const int ce = c1 + b < Mc - 1 ? c1 + b : Mc - 1;
    if (on && tau2 != 0.0 && hl <= ce - c0) {
        if (hl == 0)
            local_set(beta, ni, B + band::at(c0, c0, b), cs, sink);
        else
            local_apply(x, sc, tau2, ni, B + band::at(c0, c0 + hl, b), cs, sink);
    }
    wave_sync();
}

// One reflector of a replay on the s columns of X (row-major, leading
// dimension lx): rows r .. r + n - 1, the reflector (v_0 .. v_{b-1}, tau) at
// rf.  Lane l takes column l % 16 and rows 4 (l / 16) .. + 3 of the n <= 16;
// the four partial products of a column are added across the wave.
__device__ __forceinline__ void replay_apply(double* X, int lx, int s, int r, int n, const double* rf, int b,
                                             double* sink, int lane) {
    const double tau = rf[b];
    if (tau == 0.0) return;
    const int k = lane & 15, g = lane >> 4, j0 = 4 * g;
    const int kk = k < s ? k : s - 1;
    double vv[4], y[4];
    double* x[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const bool in = j0 + j < n;
        vv[j] = rf[in ? j0 + j : b - 1] * (in ? 1.0 : 0.0);
        y[j] = X[(int64_t)(r + (in ? j0 + j : n - 1)) * lx + kk];
        x[j] = (in && k < s) ? X + (int64_t)(r + j0 + j) * lx + k : sink;
    }
    double p = fma(vv[0], y[0], vv[1] * y[1]) + fma(vv[2], y[2], vv[3] * y[3]);
    p += __shfl_xor(p, 16, kWave);
    p += __shfl_xor(p, 32, kWave);
    const double tw = tau * p;
#pragma unroll
    for (int j = 0; j < 4; ++j) *x[j] = fma(-tw, vv[j], y[j]);
}

// Loads steps [s0, s1) of the reflectors (tasks toff[s0] .. toff[s1]) into
// the stage; the caller has synchronised.
__device__ void stage_chunk(const double* __restrict__ R, const int32_t* toff, int s0, int s1, int b,
                            double* stage) {
    const int64_t q0 = toff[s0], q1 = toff[s1];
    const int64_t len = (q1 - q0) * (b + 1);
    const double* src = R + q0 * (b + 1);
    for (int64_t k = threadIdx.x; k < len; k += blockDim.x) stage[k] = src[k];
}

// The chunks of the replay: from step s0, the last step s1 > s0 whose tasks
// fit the stage (at least one step; a step's tasks always fit, see
// band_fits).
__device__ int chunk_end(const int32_t* toff, int s0, int T, int cap) {
    int s1 = s0 + 1;
    while (s1 < T && toff[s1 + 1] - toff[s0] <= cap) ++s1;
    return s1;
}
__device__ int chunk_begin(const int32_t* toff, int s1, int cap) {
    int s0 = s1 - 1;
    while (s0 > 0 && toff[s1] - toff[s0 - 1] <= cap) --s0;
    return s0;
}

}  // namespace

// ---------------------------------------------------------------------------
// 1. The chase.  C: (Mc) x N row-major, leading dimension ldc; b = s.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kChaseThreads) void k_band_chase(const double* __restrict__ C, int64_t ldc, int N, int Mc,
                                                             int b, int T, double* __restrict__ RR,
                                                             double* __restrict__ LL, int32_t* __restrict__ toff,
                                                             double* __restrict__ d, double* __restrict__ e) {
    __shared__ double B[kBandLdsDoubles];
    __shared__ int32_t cntw[2][kChaseWaves];
    __shared__ double vsh[kChaseWaves][2][band::kMaxB];
    __shared__ double sink[kChaseWaves];  // written, never read
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const int half = lane >> 5, hl = lane & 31;
    const int W = band::width(b);
    for (int64_t idx = tid; idx < (int64_t)N * W; idx += kChaseThreads) {
        const int r = (int)(idx / W), o = (int)(idx - (int64_t)r * W);
        const int c = r + o - (b - 1);
        B[idx] = (c >= r && c <= r + b && c < Mc) ? C[(int64_t)c * ldc + r] : 0.0;
    }
    __syncthreads();
    int q0 = 0;
    for (int s = 0; s < T; ++s) {
        // the step's sweeps are ihi, ihi - 1, ... while they have a task at
        // this step (a contiguous range of ranks q = ihi - i); wave wv takes
        // ranks 2 wv, 2 wv + 1, then 2 kChaseWaves further on, one per half-wave
        const int ihi = band::step_top(s, N, Mc);
        int mine = 0;
        for (int p = wv;; p += kChaseWaves) {
            bool on[2];
            int ii[2], tt[2];
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int q = 2 * p + e;
                ii[e] = ihi - q;
                tt[e] = s - band::kLag * ii[e];
                on[e] = ii[e] >= 0 && tt[e] < band::ntasks(ii[e], N, Mc, b);
            }
            if (!on[0]) break;
            const int q = 2 * p + half;
            chase_task(B, N, Mc, b, on[half], ii[half], tt[half], RR + (int64_t)(q0 + q) * (b + 1),
                       LL + (int64_t)(q0 + q) * (b + 1), vsh[wv][half], &sink[wv], hl);
            mine += on[1] ? 2 : 1;
            if (!on[1]) break;
        }
        if (lane == 0) cntw[s & 1][wv] = mine;
        if (tid == 0) toff[s] = q0;
        __syncthreads();
        int cnt = 0;
#pragma unroll
        for (int q = 0; q < kChaseWaves; ++q) cnt += cntw[s & 1][q];
        q0 += cnt;
    }
    if (tid == 0) toff[T] = q0;
    for (int i = tid; i < N; i += kChaseThreads) {
        d[i] = B[band::at(i, i, b)];
        e[i] = B[band::at(i, i + 1, b)];
    }
}

// ---------------------------------------------------------------------------
// 2. The data.  E1: s x s row-major (b_k = (E1 e_k; 0)); G (N x 16 row-major):
// the rotated data of the upper bidiagonal B; fn2[k] = ||b_k||^2; the SVD
// workspace's d, e, g, bounds and flags.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBandThreads) void k_band_data(const double* __restrict__ E1, int N, int Mc, int b,
                                                            const double* __restrict__ RR,
                                                            const int32_t* __restrict__ toff_g, int T,
                                                            const double* __restrict__ d, const double* __restrict__ e,
                                                            double* __restrict__ ws, double* __restrict__ G,
                                                            double* __restrict__ fn2) {
    __shared__ double X[kBandDataDoubles];
    __shared__ double stage[kStageDoubles];
    __shared__ int32_t toff[kBandMaxSteps + 1];
    __shared__ double red[kBandThreads / kWave];
    __shared__ double sink[kBandWaves];  // written, never read
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const int s = b;       // data columns
    const int lx = s + 1;  // X's leading dimension (padded against LDS bank conflicts)
    for (int idx = tid; idx < Mc * lx; idx += kBandThreads) {
        const int r = idx / lx, k = idx - r * lx;
        X[idx] = (r < s && k < s) ? E1[r * s + k] : 0.0;
    }
    for (int k = tid; k <= T; k += kBandThreads) toff[k] = toff_g[k];
    if (tid < s) {
        double a = 0.0;
        for (int r = 0; r < s; ++r) a = fma(E1[r * s + tid], E1[r * s + tid], a);
        fn2[tid] = a;
    }
    __syncthreads();
    const int cap = kStageDoubles / (b + 1);
    for (int s0 = 0; s0 < T;) {
        const int s1 = chunk_end(toff, s0, T, cap);
        stage_chunk(RR, toff, s0, s1, b, stage);
        __syncthreads();
        // two steps per barrier: tasks that touch a common data row lie at
        // least two steps apart
        for (int st = s0; st < s1; st += 2) {
            const int st2 = st + 2 < s1 ? st + 2 : s1;
            for (int q = toff[st] + wv; q < toff[st2]; q += kBandWaves) {
                const int sq = q < toff[st + 1] ? st : st + 1;
                const int i = band::step_top(sq, N, Mc) - (q - toff[sq]);
                int r0, c0, c1;
                band::task_cols(i, sq - band::kLag * i, b, Mc, r0, c0, c1);
                replay_apply(X, lx, s, c0, c1 - c0 + 1, stage + (int64_t)(q - toff[s0]) * (b + 1), b, &sink[wv], lane);
            }
            __syncthreads();
        }
        s0 = s1;
    }
    // the lower-to-upper rotations: d, e to LDS (the stage), then one lane per
    // data column runs the whole chain (lane 0 also keeps B)
    double* sd = stage;
    double* se = stage + N;
    double* du = stage + 2 * N;
    double* eu = stage + 3 * N;
    for (int i = tid; i < N; i += kBandThreads) {
        sd[i] = d[i];
        se[i] = e[i];
    }
    __syncthreads();
    if (wv == 0 && lane < (s > 1 ? s : 1)) {
        double a = sd[0];
        for (int j = 0; j < N; ++j) {
            double c, sn;
            const double r = band::givens(a, se[j], &c, &sn);
            const double an = j + 1 < N ? sd[j + 1] : 0.0;
            if (lane == 0) {
                du[j] = r;
                eu[j] = sn * an;
            }
            a = c * an;
            if (lane < s) {
                const double g0 = X[j * lx + lane], g1 = X[(j + 1) * lx + lane];
                X[j * lx + lane] = fma(c, g0, sn * g1);
                X[(j + 1) * lx + lane] = fma(-sn, g0, c * g1);
            }
        }
    }
    __syncthreads();
    const SvdWs w = svd_ws(ws, N);
    double emax = 0.0, bad = 0.0;
    for (int i = tid; i < N; i += kBandThreads) {
        const double di = du[i], ei = i + 1 < N ? eu[i] : 0.0;
        w.d[i] = di;
        w.e[i] = ei;
        w.g[i] = 0.0;
        emax = ei * ei > emax ? ei * ei : emax;
        bad = (!(di > 0.0) || !isfinite(di) || !isfinite(ei)) ? 1.0 : bad;
    }
    for (int idx = tid; idx < N * kBlkRhs; idx += kBandThreads) {
        const int r = idx / kBlkRhs, k = idx - r * kBlkRhs;
        const double g = k < s ? X[r * lx + k] : 0.0;
        G[idx] = g;
        bad = isfinite(g) ? bad : 1.0;
    }
    // maxima over the workgroup
    {
        double m1 = emax, m2 = bad;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double x1 = __shfl_xor(m1, o, kWave), x2 = __shfl_xor(m2, o, kWave);
            m1 = x1 > m1 ? x1 : m1;
            m2 = x2 > m2 ? x2 : m2;
        }
        __syncthreads();  // the stage's du / eu are still read below by thread 0 only
        if (lane == 0) red[wv] = m1;
        __syncthreads();
        if (tid == 0) {
            double mm = 0.0;
            for (int q = 0; q < kBandWaves; ++q) mm = red[q] > mm ? red[q] : mm;
            w.misc[1] = DBL_MIN * (mm > 1.0 ? mm : 1.0);
        }
        __syncthreads();
        if (lane == 0) red[wv] = m2;
        __syncthreads();
        if (tid == 0) {
            double mm = 0.0;
            for (int q = 0; q < kBandWaves; ++q) mm = red[q] > mm ? red[q] : mm;
            eu[N - 1] = 0.0;
            w.misc[0] = msvd::eig_bound(du, eu, N);
            w.flag[0] = mm > 0.0 ? 1 : 0;
            w.flag[1] = 0;
        }
    }
}

// ---------------------------------------------------------------------------
// 4. Small products over the N x N matrices of the SVD (rows j of A = the
// vectors: A[j * lda + i]) and N x 16 row-major operands:
//  mode 0: out[j][k] = sum_i A[j][i] X[i][k]                      (H = U g)
//  mode 1: out[i][k] = sum_j A[j][i] X[j][k]                      (U^T H)
//  mode 2: Fcol[k N + j] = 1.5 X2[j][k] - 0.5 sum_i A[j][i] X[i][k]  (F~)
//  mode 3: out[i][k] = sum_j A[j][i] phi_jk Fcol[k N + j],
//          phi_jk = s_j / (s_j^2 + lambda_k^2)                    (yhat)
// k >= s: 0.  One thread per output (16 rows x 16 columns per workgroup).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_band_mm(int mode, const double* __restrict__ A, int64_t lda, int N, int s,
                                                    const double* __restrict__ X, const double* __restrict__ X2,
                                                    const double* __restrict__ sv, const ParamOut* __restrict__ po,
                                                    double* __restrict__ out) {
    const int k = threadIdx.x % kBlkRhs;
    const int row = blockIdx.x * kMmRows + threadIdx.x / kBlkRhs;
    if (row >= N) return;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    if (k < s) {
        if (mode == 0 || mode == 2) {
            const double* ar = A + (int64_t)row * lda;
            int i = 0;
            for (; i + 3 < N; i += 4) {
                a0 = fma(ar[i], X[(int64_t)i * kBlkRhs + k], a0);
                a1 = fma(ar[i + 1], X[(int64_t)(i + 1) * kBlkRhs + k], a1);
                a2 = fma(ar[i + 2], X[(int64_t)(i + 2) * kBlkRhs + k], a2);
                a3 = fma(ar[i + 3], X[(int64_t)(i + 3) * kBlkRhs + k], a3);
            }
            for (; i < N; ++i) a0 = fma(ar[i], X[(int64_t)i * kBlkRhs + k], a0);
        } else {
            const double lam = mode == 3 ? po[k].lambda : 0.0;
            const double l2 = lam * lam;
            const double* fc = X + (int64_t)k * N;
            auto x_of = [&](int j) -> double {
                if (mode == 1) return X[(int64_t)j * kBlkRhs + k];
                const double sj = sv[j];
                return sj / fma(sj, sj, l2) * fc[j];
            };
            int j = 0;
            for (; j + 3 < N; j += 4) {
                a0 = fma(A[(int64_t)j * lda + row], x_of(j), a0);
                a1 = fma(A[(int64_t)(j + 1) * lda + row], x_of(j + 1), a1);
                a2 = fma(A[(int64_t)(j + 2) * lda + row], x_of(j + 2), a2);
                a3 = fma(A[(int64_t)(j + 3) * lda + row], x_of(j + 3), a3);
            }
            for (; j < N; ++j) a0 = fma(A[(int64_t)j * lda + row], x_of(j), a0);
        }
    }
    const double acc = (a0 + a1) + (a2 + a3);
    if (mode == 2) {
        if (k < s) out[(int64_t)k * N + row] = fma(1.5, X2[(int64_t)row * kBlkRhs + k], -0.5 * acc);
    } else {
        out[(int64_t)row * kBlkRhs + k] = acc;
    }
}

// ---------------------------------------------------------------------------
// 5. The solutions: Yh (N x 16 row-major) through the left reflectors, last
// step first, into Y (N x 16 row-major).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBandThreads) void k_band_solve(const double* __restrict__ Yh, int N, int Mc, int b,
                                                             const double* __restrict__ LL,
                                                             const int32_t* __restrict__ toff_g, int T,
                                                             double* __restrict__ Y) {
    __shared__ double X[kBandDataDoubles];  // N x b, row-major, leading dimension b + 1
    __shared__ double stage[kStageDoubles];
    __shared__ int32_t toff[kBandMaxSteps + 1];
    __shared__ double sink[kBandWaves];  // written, never read
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const int lx = b + 1;
    for (int idx = tid; idx < N * lx; idx += kBandThreads) {
        const int r = idx / lx, k = idx - r * lx;
        X[idx] = k < b ? Yh[(int64_t)r * kBlkRhs + k] : 0.0;
    }
    for (int k = tid; k <= T; k += kBandThreads) toff[k] = toff_g[k];
    __syncthreads();
    const int cap = kStageDoubles / (b + 1);
    for (int s1 = T; s1 > 0;) {
        const int s0 = chunk_begin(toff, s1, cap);
        stage_chunk(LL, toff, s0, s1, b, stage);
        __syncthreads();
        // two steps per barrier, last step first (as in the data replay)
        for (int st = s1; st > s0; st -= 2) {
            const int sb = st - 2 > s0 ? st - 2 : s0;
            for (int q = toff[sb] + wv; q < toff[st]; q += kBandWaves) {
                const int sq = q < toff[sb + 1] ? sb : sb + 1;
                const int i = band::step_top(sq, N, Mc) - (q - toff[sq]);
                int r0, c0, c1;
                band::task_cols(i, sq - band::kLag * i, b, Mc, r0, c0, c1);
                const int r1 = c1 < N - 1 ? c1 : N - 1;
                if (r1 > c0)
                    replay_apply(X, lx, b, c0, r1 - c0 + 1, stage + (int64_t)(q - toff[s0]) * (b + 1), b, &sink[wv],
                                 lane);
            }
            __syncthreads();
        }
        s1 = s0;
    }
    for (int idx = tid; idx < N * kBlkRhs; idx += kBandThreads) {
        const int r = idx / kBlkRhs, k = idx - r * kBlkRhs;
        Y[idx] = k < b ? X[r * lx + k] : 0.0;
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
bool band_fits(int N, int s) {
    if (s < 1 || s > band::kMaxB || N < 1 || N > kMaxEll || N > kBandMaxN) return false;
    const int Mc = N + s;
    if ((int64_t)N * band::width(s) > kBandLdsDoubles || (int64_t)Mc * (s + 1) > kBandDataDoubles) return false;
    const int T = band::nsteps(N, Mc, s);
    if (T > kBandMaxSteps) return false;
    // every step's reflectors fit the replay stage
    for (int st = 0; st < T; ++st) {
        int ihi;
        if ((int64_t)band::step_tasks(st, N, Mc, s, ihi) * (s + 1) > kStageDoubles) return false;
    }
    return true;
}

int band_ntasks(int N, int s, int* nsteps) {
    const int Mc = N + s;
    const int T = band::nsteps(N, Mc, s);
    int tot = 0;
    for (int st = 0; st < T; ++st) {
        int ihi;
        tot += band::step_tasks(st, N, Mc, s, ihi);
    }
    *nsteps = T;
    return tot;
}

void launch_band_chase(const double* C, int64_t ldc, int N, int s, int T, double* RR, double* LL, int32_t* toff,
                       double* d, double* e, hipStream_t st) {
    k_band_chase<<<1, kChaseThreads, 0, st>>>(C, ldc, N, N + s, s, T, RR, LL, toff, d, e);
}

void launch_band_data(const double* E1, int N, int s, const double* RR, const int32_t* toff, int T, const double* d,
                      const double* e, double* ws, double* G, double* fn2, hipStream_t st) {
    k_band_data<<<1, kBandThreads, 0, st>>>(E1, N, N + s, s, RR, toff, T, d, e, ws, G, fn2);
}

void launch_band_mm(int mode, const double* A, int64_t lda, int N, int s, const double* X, const double* X2,
                    const double* sv, const ParamOut* po, double* out, hipStream_t st) {
    k_band_mm<<<(N + kMmRows - 1) / kMmRows, kBlock, 0, st>>>(mode, A, lda, N, s, X, X2, sv, po, out);
}

void launch_band_solve(const double* Yh, int N, int s, const double* LL, const int32_t* toff, int T, double* Y,
                       hipStream_t st) {
    k_band_solve<<<1, kBandThreads, 0, st>>>(Yh, N, N + s, s, LL, toff, T, Y);
}

}  // namespace mqh
