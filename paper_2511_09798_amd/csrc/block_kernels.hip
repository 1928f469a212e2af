// block_kernels.hip -- the block Golub-Kahan process for s <= 16 right-hand
// sides that share one Krylov space (Algorithm 1 with an n x s starting
// block) on gfx950, FP64.
//
// Two tall-skinny contractions carry the reorthogonalisation against a
// shared basis of m columns (m = s j at step j) and the block QR:
//   c = V^T P   (m x s, K = n rows)        -- k_blk_gemvt + k_blk_reduce
//   P -= V c, or P = V c                   -- k_blk_update
// both on the FP64 matrix cores (v_mfma_f64_16x16x4f64: lane l supplies
// A[l%16][l/16] and B[l/16][l%16] and receives D[4r + l/16][l%16]).  The
// block QR is shifted Cholesky QR applied three times (the shift in the
// first pass keeps the Cholesky factorisation defined for nearly dependent
// columns; the two unshifted passes restore orthogonality to rounding):
// k_blk_chol factors one 16 x 16 Gram matrix on one workgroup.

#include <float.h>
#include <math.h>

#include "common.hpp"
#include "kernels.hpp"

namespace mqh {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kBt = 64;        // rows of a staged tile; basis columns per workgroup of k_blk_gemvt
constexpr int kBtLd = kBt + 1;  // padded LDS row of the basis tile
constexpr int kPLd = kBlkRhs + 1;

// part[(chunk m + col) 16 + k] = sum over the rows i of the chunk (i < n) of
// V[col][i] P[k][i], for col < m and all 16 k (zero for k >= s).  V: column
// col at V + col ldv; P: column k at P + k ldp.  Grid (chunks, ceil(m / 64)),
// chunk a multiple of 64; wave w forms columns 64 y + 16 w .. + 15.
__global__ __launch_bounds__(kBlock) void k_blk_gemvt(const double* __restrict__ V, int64_t ldv, int64_t n,
                                                      int32_t m, const double* __restrict__ P, int64_t ldp,
                                                      int32_t s, int64_t chunk, double* __restrict__ part) {
    __shared__ double tV[kBt * kBtLd];
    __shared__ double tP[kBt * kPLd];
    const int64_t r0 = (int64_t)blockIdx.x * chunk;
    const int64_t r1 = r0 + chunk < n ? r0 + chunk : n;
    const int c0 = blockIdx.y * kBt;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int li = lane & 15, lk = lane >> 4;
    const int rr = threadIdx.x & (kBt - 1), rq = threadIdx.x / kBt;  // staging: row rr, column rq + 4 q
    v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
    for (int64_t rb = r0; rb < r1; rb += kBt) {
        __syncthreads();  // the previous tile's reads are done
        const int64_t row = rb + rr;
        const bool rok = row < r1;
#pragma unroll
        for (int q = 0; q < kBt / (kBlock / kBt); ++q) {
            const int cc = rq + (kBlock / kBt) * q;
            const int col = c0 + cc;
            tV[rr * kBtLd + cc] = (rok && col < m) ? V[(int64_t)col * ldv + row] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < kBlkRhs / (kBlock / kBt); ++q) {
            const int k = rq + (kBlock / kBt) * q;
            tP[rr * kPLd + k] = (rok && k < s) ? P[(int64_t)k * ldp + row] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < kBt; kk += 4) {
            // A[i][k'] = V[col 16 w + i][row kk + k'], B[k'][j] = P[rhs j][row kk + k']
            const double a = tV[(kk + lk) * kBtLd + 16 * w + li];
            const double b = tP[(kk + lk) * kPLd + li];
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int col = c0 + 16 * w + 4 * r + lk;
        if (col < m) part[((int64_t)blockIdx.x * m + col) * kBlkRhs + li] = acc[r];
    }
}

// c[col 16 + k] = sum over chunks of part[(chunk m + col) 16 + k]: one wave
// per entry, lane l summing chunks l, l + 64, ... in order, then a fixed
// shuffle tree (deterministic).
__global__ __launch_bounds__(kBlock) void k_blk_reduce(const double* __restrict__ part, int chunks, int32_t m,
                                                       double* __restrict__ c) {
    const int64_t e = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (e >= (int64_t)m * kBlkRhs) return;  // wave-uniform
    const int lane = threadIdx.x & (kWave - 1);
    double v = 0.0;
    for (int q = lane; q < chunks; q += kWave) v += part[(int64_t)q * m * kBlkRhs + e];
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    if (lane == 0) c[e] = v;
}

// Rows [16 (4 x + w), + 16) of the s output columns, per wave:
//   sub = 1: P[k][i] -= sum_col V[col][i] c[col cs + k ks]
//   sub = 0: P[k][i]  = sum_col V[col][i] c[col cs + k ks]
// (V may be P itself for sub = 0: a wave reads all its rows before it
// writes them, and no two waves share a row).  No barrier: waves past n
// return at once.
__global__ __launch_bounds__(kBlock) void k_blk_update(const double* V, int64_t ldv, int64_t n, int32_t m,
                                                       const double* __restrict__ c, int64_t cs, int64_t ks,
                                                       double* P, int64_t ldp, int32_t s, int32_t sub) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t row0 = ((int64_t)blockIdx.x * (kBlock / kWave) + w) * 16;
    if (row0 >= n) return;
    const int64_t row = row0 + li;
    const bool rok = row < n;
    v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
    for (int kk = 0; kk < m; kk += 4) {
        const int col = kk + lk;
        const bool cok = col < m;
        // A[i][k'] = V[col kk + k'][row0 + i], B[k'][j] = c[col kk + k'][j]
        const double a = (rok && cok) ? V[(int64_t)col * ldv + row] : 0.0;
        const double b = (cok && li < s) ? c[(int64_t)col * cs + (int64_t)li * ks] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    if (li >= s) return;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t rr = row0 + 4 * r + lk;
        if (rr < n) {
            double* dst = P + (int64_t)li * ldp + rr;
            *dst = sub ? *dst - acc[r] : acc[r];
        }
    }
}

// One pass of (shifted) Cholesky QR on one workgroup of 256 threads, thread
// (i, j) = (t / 16, t % 16) owning entry (i, j) of the 16 x 16 tiles in LDS:
// G (c layout, G[i 16 + j] = P_i . P_j, i, j < s) plus, if shifted,
// 11 (n s + s (s + 1)) eps trace(G) on the diagonal is factored as R^T R
// (R upper triangular, right-looking: per column a pivot, a row of R, a
// rank-one update of the trailing block); Rinv = R^{-1} (back substitution,
// column j by thread j) in the c layout of k_blk_update (Rinv[col 16 + k]);
// Racc <- R Racc (row-major 16 x 16, the accumulated triangular factor).
// status <- 1 if a pivot is not positive and finite (Racc and Rinv are then
// left as they were).
__global__ __launch_bounds__(kBlock) void k_blk_chol(const double* __restrict__ G, int32_t s, int64_t n,
                                                     int32_t shifted, double* __restrict__ Rinv,
                                                     double* __restrict__ Racc, int32_t* __restrict__ status) {
    __shared__ double M[kBlkRhs][kBlkRhs];  // the trailing matrix, then R
    __shared__ double X[kBlkRhs][kBlkRhs];  // R^{-1}
    __shared__ double red[kBlock / kWave];
    __shared__ int bad;
    const int i = threadIdx.x / kBlkRhs, j = threadIdx.x % kBlkRhs;
    const bool in = i < s && j < s;
    const double g = in ? G[i * kBlkRhs + j] : 0.0;
    double tr = (in && i == j) ? g : 0.0;
    tr = block_sum<kBlock>(tr, red);
    const double shift = shifted ? 11.0 * ((double)n * s + (double)s * (s + 1)) * DBL_EPSILON * tr : 0.0;
    M[i][j] = in ? g + (i == j ? shift : 0.0) : 0.0;
    X[i][j] = 0.0;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    for (int c = 0; c < s; ++c) {
        if (threadIdx.x == 0) {
            const double d = M[c][c];
            if (!(d > 0.0) || !isfinite(d)) bad = 1;
            M[c][c] = (d > 0.0 && isfinite(d)) ? sqrt(d) : 1.0;
        }
        __syncthreads();
        if (i == c && j > c && j < s) M[c][j] /= M[c][c];  // row c of R
        __syncthreads();
        if (i > c && j >= i && j < s) M[i][j] -= M[c][i] * M[c][j];  // trailing upper triangle
        __syncthreads();
    }
    if (bad) {
        if (threadIdx.x == 0) *status = 1;
        return;
    }
    // R = upper triangle of M; R^{-1} column by column (thread j < s)
    if (threadIdx.x < s) {
        const int cj = threadIdx.x;
        for (int r = cj; r >= 0; --r) {
            double v = (r == cj) ? 1.0 : 0.0;
            for (int k = r + 1; k <= cj; ++k) v -= M[r][k] * X[k][cj];
            X[r][cj] = v / M[r][r];
        }
    }
    __syncthreads();
    Rinv[i * kBlkRhs + j] = X[i][j];
    // Racc <- R Racc (upper triangular), entry (i, j) by thread (i, j)
    double v = 0.0;
    if (in && j >= i)
        for (int k = i; k <= j; ++k) v += M[i][k] * Racc[k * kBlkRhs + j];
    __syncthreads();  // every thread has read Racc
    if (in) Racc[i * kBlkRhs + j] = j >= i ? v : 0.0;
}

// Racc <- identity (row-major 16 x 16), status <- 0.
__global__ void k_blk_eye(double* __restrict__ Racc, int32_t* __restrict__ status) {
    const int e = threadIdx.x;
    if (e < kBlkRhs * kBlkRhs) Racc[e] = (e / kBlkRhs == e % kBlkRhs) ? 1.0 : 0.0;
    if (e == 0) *status = 0;
}

// The breakdown test of a block QR on the device (no host round trip per
// step).  kind 0: E_1 (the data's factor, kept in E1; a diagonal entry at
// most tau times its largest, or a failed factorisation, marks the sources
// invalid); kind 1: D_j = R^T of step j; kind 2: E_{j+1} = R.  For kinds 1
// and 2 the running scale is the largest diagonal entry of the D and E blocks
// so far; a failed factorisation or a diagonal entry at most tau times the
// scale stops the run (ell_done = j - 1 at a D block, j at an E block, flag =
// kind).  Otherwise the block goes into C (row-major, ld ldc) and its
// transpose (16 x 16, the update kernel's coefficient layout) into mat, the
// coefficients of the next shift.  Once stopped, nothing is written.
__global__ __launch_bounds__(kBlkRhs * kBlkRhs) void k_blk_check(const double* __restrict__ Racc,
                                                                 const int32_t* __restrict__ status, int32_t s,
                                                                 int32_t kind, int32_t j, double tau,
                                                                 BlkState* __restrict__ bs, double* __restrict__ C,
                                                                 int64_t ldc, double* __restrict__ E1,
                                                                 double* __restrict__ mat) {
    __shared__ int s_ok;
    if (threadIdx.x == 0) {
        int ok = bs->stopped ? 0 : 1;
        if (ok) {
            double mn = HUGE_VAL, mx = 0.0;
            for (int i = 0; i < s; ++i) {
                const double d = fabs(Racc[i * kBlkRhs + i]);
                mn = d < mn ? d : mn;
                mx = d > mx ? d : mx;
            }
            const bool bad = *status != 0;
            if (kind == 0) {
                if (bad || !(mn > tau * mx)) {
                    bs->invalid = 1;
                    bs->stopped = 1;
                    bs->ell_done = 0;
                    ok = 0;
                }
            } else {
                const double sc = mx > bs->scale ? mx : bs->scale;
                if (bad || !(mn > tau * sc)) {
                    bs->stopped = 1;
                    bs->ell_done = kind == 1 ? j - 1 : j;
                    bs->flag = kind;
                    ok = 0;
                } else {
                    bs->scale = sc;
                }
            }
        }
        s_ok = ok;
    }
    __syncthreads();
    if (!s_ok) return;
    const int r = threadIdx.x / kBlkRhs, c = threadIdx.x % kBlkRhs;
    const double v = Racc[r * kBlkRhs + c];
    const bool in = r < s && c < s;
    mat[c * kBlkRhs + r] = in ? v : 0.0;
    if (!in) return;
    if (kind == 0)
        E1[r * s + c] = v;
    else if (kind == 1)
        C[(int64_t)((j - 1) * s + c) * ldc + (j - 1) * s + r] = v;  // D_j = R^T
    else
        C[(int64_t)(j * s + r) * ldc + (j - 1) * s + c] = v;  // E_{j+1} = R
}

}  // namespace

int blk_chunks(int64_t n, int32_t m, int64_t* chunk) {
    const int64_t tiles = (m + kBt - 1) / kBt;
    int64_t want = (1024 + tiles - 1) / tiles;
    const int64_t cmax = (n + kBt - 1) / kBt;
    if (want > cmax) want = cmax;
    if (want < 1) want = 1;
    int64_t ch = (n + want - 1) / want;
    ch = (ch + kBt - 1) / kBt * kBt;
    *chunk = ch;
    return (int)((n + ch - 1) / ch);
}

void launch_blk_gemvt(const double* V, int64_t ldv, int64_t n, int32_t m, const double* P, int64_t ldp, int32_t s,
                      double* part, double* c, hipStream_t st) {
    int64_t chunk;
    const int chunks = blk_chunks(n, m, &chunk);
    k_blk_gemvt<<<dim3((unsigned)chunks, (unsigned)((m + kBt - 1) / kBt)), kBlock, 0, st>>>(V, ldv, n, m, P, ldp, s,
                                                                                           chunk, part);
    const int64_t waves = (int64_t)m * kBlkRhs, per = kBlock / kWave;
    k_blk_reduce<<<(unsigned)((waves + per - 1) / per), kBlock, 0, st>>>(part, chunks, m, c);
}

void launch_blk_update(const double* V, int64_t ldv, int64_t n, int32_t m, const double* c, int64_t cs, int64_t ks,
                       double* P, int64_t ldp, int32_t s, int32_t sub, hipStream_t st) {
    const int64_t rows_per_block = 16 * (kBlock / kWave);
    k_blk_update<<<(unsigned)((n + rows_per_block - 1) / rows_per_block), kBlock, 0, st>>>(V, ldv, n, m, c, cs, ks, P,
                                                                                         ldp, s, sub);
}

void launch_blk_chol(const double* G, int32_t s, int64_t n, int32_t shifted, double* Rinv, double* Racc,
                     int32_t* status, hipStream_t st) {
    k_blk_chol<<<1, kBlock, 0, st>>>(G, s, n, shifted, Rinv, Racc, status);
}

void launch_blk_check(const double* Racc, const int32_t* status, int32_t s, int32_t kind, int32_t j, double tau,
                      BlkState* bs, double* C, int64_t ldc, double* E1, double* mat, hipStream_t st) {
    k_blk_check<<<1, kBlkRhs * kBlkRhs, 0, st>>>(Racc, status, s, kind, j, tau, bs, C, ldc, E1, mat);
}

// The Jacobi route's work matrix of the projected problem from the device
// copies: G[i][j] = C[i][j] (m x ls, leading dimension ldc) and the data
// columns G[i][m + k] = E1[i][k] for i < s (rows i >= s stay zero).  G is
// zero on entry (full_reset).
__global__ __launch_bounds__(kBlock) void k_blk_fill_g(const double* __restrict__ C, int64_t ldc, int64_t m,
                                                       int64_t ls, const double* __restrict__ E1, int32_t s,
                                                       double* __restrict__ G, int64_t ldg) {
    const int64_t i = blockIdx.y;
    const double* ci = C + i * ldc;
    double* gi = G + i * ldg;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < ls; j += (int64_t)gridDim.x * kBlock) gi[j] = ci[j];
    if (blockIdx.x == 0 && i < s && (int)threadIdx.x < s) gi[m + threadIdx.x] = E1[i * s + threadIdx.x];
}

void launch_blk_fill_g(const double* C, int64_t ldc, int64_t m, int64_t ls, const double* E1, int32_t s, double* G,
                       int64_t ldg, hipStream_t st) {
    const unsigned gx = (unsigned)((ls + kBlock - 1) / kBlock);
    k_blk_fill_g<<<dim3(gx, (unsigned)m), kBlock, 0, st>>>(C, ldc, m, ls, E1, s, G, ldg);
}

void launch_blk_eye(double* Racc, int32_t* status, hipStream_t st) {
    k_blk_eye<<<1, kBlkRhs * kBlkRhs, 0, st>>>(Racc, status);
}

}  // namespace mqh
