// full_kernels.hip -- full SVD of the collocation matrix on gfx950 (FP64) and
// the classical regularised solutions built on it: Tikhonov with the GCV of
// the full problem (Algorithm 3, eq. (25)) and truncated SVD (eq. (14)).
//
// One-sided block Jacobi on the rows of the work matrix G = [A | f]
// (row-major, leading dimension ldg >= n + 1, rows padded with zero rows to a
// whole number of 32-row blocks).  Each sweep first orders the rows by
// decreasing norm (de Rijk's ordering; blocks are runs of 32 rows in that
// order, through an index, the rows stay in place); a round pairs the blocks
// (a round-robin tournament, so a sweep meets every pair once); for a pair, X = the 64 rows
// of its two blocks, M = X_A X_A^T is their Gram matrix over the A columns,
// M = P diag P^T its eigendecomposition (cyclic Jacobi in LDS), and X <- P^T X
// makes the 64 rows mutually orthogonal.  The rotations act on the f column
// too.  At convergence G = Q [A | f] with Q orthogonal and the rows of Q A
// orthogonal: A = Q^T Sigma Ubar^T, so the singular values are the row norms
// sigma_i of Q A, U^T f = Q f is the last column (f^_i), and the Tikhonov
// solution is sum_i f^_i / (sigma_i^2 + lambda^2) (row i of Q A)^T: neither U
// nor V is ever formed.
//
// The two products of a round (the Gram matrices and the update) run on the
// FP64 matrix cores (v_mfma_f64_16x16x4f64: lane l supplies A[l%16][l/16]
// and B[l/16][l%16] and receives D[4r + l/16][l%16], r = 0..3).
#include <float.h>
#include <math.h>

#include "kernels.hpp"

namespace mqh {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kFsRows = 2 * kFsBlock;  // rows of a pair (64)
constexpr int kFsLd = kFsRows + 1;     // LDS row of a 64 x 64 FP64 tile (padded)
static_assert(kFsRows % (kBlock / kWave) == 0 && kFsRows == kWave, "tile loader: one row per wave and load");

// Row of the work matrix holding row r (0..63) of pair (bi, bj): block b
// consists of the rows rowidx[32 b .. 32 b + 31] (the sweep's order).
__device__ __forceinline__ int64_t pair_row(const int32_t* __restrict__ rowidx, int2 pr, int r) {
    return rowidx[r < kFsBlock ? pr.x * kFsBlock + r : pr.y * kFsBlock + (r - kFsBlock)];
}

// Columns [c0, c0 + 64) of the pair's 64 rows into an LDS tile (zeros past cend).
__device__ __forceinline__ void load_tile(const double* __restrict__ G, int64_t ldg, const int32_t* __restrict__ rowidx,
                                          int2 pr, int64_t c0, int64_t cend, double* __restrict__ t) {
    // a wave reads 64 consecutive doubles of one row per load (512 B, aligned
    // when ldg and c0 are multiples of 64)
    const int c = threadIdx.x & (kWave - 1), r0 = threadIdx.x / kWave;
    const bool ok = c0 + c < cend;
#pragma unroll
    for (int q = 0; q < kFsRows / (kBlock / kWave); ++q) {
        const int r = r0 + (kBlock / kWave) * q;
        t[r * kFsLd + c] = ok ? G[pair_row(rowidx, pr, r) * ldg + c0 + c] : 0.0;
    }
}

// Whether the pair in schedule slot `slot` (blocks pr.x, pr.y) can be left
// out this round: with the row order unchanged (same != 0), its blocks were
// both last rotated before the round at which this pair was last found
// orthogonal (pair_ok[slot] >= 0), so its rows, and its Gram matrix, are
// exactly as they were then.  blk_stamp: per block the global round of its
// last rotation (-1: none).
__device__ __forceinline__ bool pair_unchanged(const int32_t* __restrict__ pair_ok,
                                               const int32_t* __restrict__ blk_stamp, int2 pr, int64_t slot,
                                               int same) {
    if (!same) return false;
    const int32_t g0 = pair_ok[slot];
    return g0 >= 0 && blk_stamp[pr.x] < g0 && blk_stamp[pr.y] < g0;
}

// The 16 x 16 tiles (tr, tc), tr <= tc, of a 64 x 64 Gram matrix's upper
// triangle: tile u = 0..9 is (0,0) (0,1) (0,2) (0,3) (1,1) (1,2) (1,3) (2,2)
// (2,3) (3,3).
__device__ __forceinline__ int gram_tr(int u) { return u < 4 ? 0 : u < 7 ? 1 : u < 9 ? 2 : 3; }
__device__ __forceinline__ int gram_tc(int u) { return u < 4 ? u : u < 7 ? u - 3 : u < 9 ? u - 5 : 3; }
constexpr int kGramTiles = 10;

// Partial Gram matrices: Pg[(pair * S + chunk)][a][b] = sum over the chunk's
// columns c < ncol of X[a][c] X[b][c], for the entries of the upper-triangle
// tiles (a / 16 <= b / 16) only: the lower tiles are left unwritten (the
// reader takes M[a][b] = M[b][a] there).  Grid (S, pairs), 256 threads.
// Per staged 64-column tile, wave w takes columns 16 w .. 16 w + 15 and
// forms all 10 tiles over them: its four operand loads per 4 columns feed
// 10 independent matrix-core chains (the operands of A and B are the same
// rows, lane l supplying X[16 t + l % 16][k + l / 16] for tile row or
// column t).  At the end the four waves' sums are added in LDS in wave
// order.  Pairs left out this round (pair_unchanged) write nothing.
__global__ __launch_bounds__(kBlock, 2) void k_fs_gram(const double* __restrict__ G, int64_t ldg, int64_t ncol,
                                                    const int32_t* __restrict__ rowidx,
                                                    const int2* __restrict__ pairs, int64_t chunk,
                                                    double* __restrict__ Pg, const int32_t* __restrict__ pair_ok,
                                                    const int32_t* __restrict__ blk_stamp, int64_t slot0, int same) {
    __shared__ double t[kFsRows * kFsLd];
    const int2 pr = pairs[blockIdx.y];
    if (pair_unchanged(pair_ok, blk_stamp, pr, slot0 + blockIdx.y, same)) return;  // block-uniform
    const int S = gridDim.x;
    const int64_t c0 = (int64_t)blockIdx.x * chunk;
    const int64_t c1 = c0 + chunk < ncol ? c0 + chunk : ncol;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int li = lane & 15, lk = lane >> 4;
    v4d acc[kGramTiles];
#pragma unroll
    for (int u = 0; u < kGramTiles; ++u) acc[u] = v4d{0.0, 0.0, 0.0, 0.0};
    // software pipeline: the next tile's loads are in flight (registers) while
    // this tile's products run from LDS
    constexpr int kQ = kFsRows / (kBlock / kWave);  // rows loaded per lane
    const int lc = threadIdx.x & (kWave - 1), lr = threadIdx.x / kWave;
    int64_t rowoff[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) rowoff[q] = pair_row(rowidx, pr, lr + (kBlock / kWave) * q) * ldg;
    double nxt[kQ];
    auto fetch = [&](int64_t cc) {
        const bool ok = cc < c1 && cc + lc < c1;
#pragma unroll
        for (int q = 0; q < kQ; ++q) nxt[q] = ok ? G[rowoff[q] + cc + lc] : 0.0;
    };
    fetch(c0);
    for (int64_t c = c0; c < c1; c += kFsRows) {
        __syncthreads();  // the previous tile has been consumed
#pragma unroll
        for (int q = 0; q < kQ; ++q) t[(lr + (kBlock / kWave) * q) * kFsLd + lc] = nxt[q];
        __syncthreads();
        fetch(c + kFsRows);
#pragma unroll
        for (int kk = 16 * w; kk < 16 * w + 16; kk += 4) {
            double v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = t[(16 * q + li) * kFsLd + kk + lk];
#pragma unroll
            for (int u = 0; u < kGramTiles; ++u)
                acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[gram_tr(u)], v[gram_tc(u)], acc[u], 0, 0, 0);
        }
    }
    // sum over the waves in LDS (wave order), then the partial Gram's upper tiles to Pg
    double* out = Pg + ((int64_t)blockIdx.y * S + blockIdx.x) * (kFsRows * kFsRows);
    for (int src = 0; src < kBlock / kWave; ++src) {
        __syncthreads();  // t free (the last tile consumed) / the previous wave's sums stored
        if (w == src) {
#pragma unroll
            for (int u = 0; u < kGramTiles; ++u)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int e = (16 * gram_tr(u) + 4 * r + lk) * kFsLd + 16 * gram_tc(u) + li;
                    const double s = src == 0 ? acc[u][r] : t[e] + acc[u][r];
                    if (src + 1 < kBlock / kWave)
                        t[e] = s;
                    else
                        out[(16 * gram_tr(u) + 4 * r + lk) * kFsRows + 16 * gram_tc(u) + li] = s;
                }
        }
    }
}

// Threads of the pair eigensolver: the rotation steps are chains of LDS
// accesses, so more threads per pair shorten each step (one 2 x 2 block of M
// and two column pairs of P per thread).
constexpr int kEigThreads = 1024;

// Largest |M_ab| / (max(||x_a||, ||x_b||) F) over a != b, F = ||A||_F given as
// inv_f = 1 / F (block-wide, every thread gets it): the component of the
// smaller row along the larger one relative to the matrix's norm.  Below
// c sqrt(n) eps the rows are orthogonal to the rounding level of a dense
// SVD (singular values to a small multiple of c sqrt(n) eps ||A||_F); a
// relative cosine test cannot be met by rows near that level, which every
// sweep renews.  M in LDS with row length kFsLd.
__device__ double offdiag(const double* __restrict__ M, double inv_f, double* __restrict__ red) {
    double mx = 0.0;
    for (int e = threadIdx.x; e < kFsRows * kFsRows; e += kEigThreads) {
        const int a = e / kFsRows, b = e % kFsRows;
        if (a == b) continue;
        const double ma = M[a * kFsLd + a], mb = M[b * kFsLd + b];
        const double mm = ma > mb ? ma : mb;
        if (mm > 0.0) {
            const double v = fabs(M[a * kFsLd + b]) / sqrt(mm) * inv_f;
            mx = v > mx ? v : mx;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double y = __shfl_xor(mx, o, kWave);
        mx = y > mx ? y : mx;
    }
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = mx;
    __syncthreads();
    double r = 0.0;
    for (int i = 0; i < kEigThreads / kWave; ++i) r = red[i] > r ? red[i] : r;
    __syncthreads();
    return r;
}

// One workgroup per pair (schedule slot slot0 + pair, global round g): pairs
// left out (pair_unchanged) only clear their flag; otherwise M = sum of the
// S partial Grams, off[pair] = its off-diagonal measure (offdiag), and at or
// below tol the slot is marked orthogonal at round g (pair_ok), while above
// tol both blocks are stamped with g and a cyclic Jacobi (round-robin
// order, 32 disjoint rotations per step, 63 steps per sweep, rotations
// skipped when |M_pq| <= eps/4 sqrt(M_pp M_qq); until the measure is below
// eps or max_inner sweeps) gives P^T M P (nearly) diagonal, and P goes to
// Pout[pair] with flag[pair] = 1; else flag 0.
__global__ __launch_bounds__(kEigThreads) void k_fs_eig(const double* __restrict__ Pg, int S, double tol, double inv_f,
                                                   int max_inner, double* __restrict__ Pout,
                                                   int32_t* __restrict__ flag, double* __restrict__ off,
                                                   const int2* __restrict__ pairs, int32_t* __restrict__ pair_ok,
                                                   int32_t* __restrict__ blk_stamp, int64_t slot0, int32_t g,
                                                   int same) {
    __shared__ double M[kFsRows * kFsLd];
    __shared__ double P[kFsRows * kFsLd];
    __shared__ double red[kEigThreads / kWave];
    __shared__ double rc[kFsRows / 2], rs[kFsRows / 2];
    __shared__ int rp[kFsRows / 2], rq[kFsRows / 2];
    const int pair = blockIdx.x;
    const int2 pr = pairs[pair];
    const int64_t slot = slot0 + pair;
    if (pair_unchanged(pair_ok, blk_stamp, pr, slot, same)) {
        // left out: off[pair] keeps the value this slot had when it was found orthogonal
        if (threadIdx.x == 0) flag[pair] = 0;
        return;
    }
    const double* src = Pg + (int64_t)pair * S * (kFsRows * kFsRows);
    for (int e = threadIdx.x; e < kFsRows * kFsRows; e += kEigThreads) {
        const int a = e / kFsRows, b = e % kFsRows;
        const int es = a / 16 > b / 16 ? b * kFsRows + a : e;  // k_fs_gram writes the upper tiles only
        double v = 0.0;
        for (int s = 0; s < S; ++s) v += src[(int64_t)s * (kFsRows * kFsRows) + es];
        M[a * kFsLd + b] = v;
        P[a * kFsLd + b] = a == b ? 1.0 : 0.0;
    }
    __syncthreads();
    const double o0 = offdiag(M, inv_f, red);
    if (threadIdx.x == 0) off[pair] = o0;
    if (!(o0 > tol)) {
        if (threadIdx.x == 0) {
            flag[pair] = 0;
            pair_ok[slot] = g;
        }
        return;
    }
    if (threadIdx.x == 0) {
        pair_ok[slot] = -1;
        blk_stamp[pr.x] = g;
        blk_stamp[pr.y] = g;
    }
    const double tol_in = DBL_EPSILON;
    for (int sweep = 0; sweep < max_inner; ++sweep) {
        for (int step = 0; step < kFsRows - 1; ++step) {
            if (threadIdx.x < kFsRows / 2) {
                // round-robin: position 0 fixed, the others rotate by one per step
                const int k = threadIdx.x;
                const int ia = k == 0 ? 0 : 1 + (k - 1 + step) % (kFsRows - 1);
                const int ib = 1 + (kFsRows - 2 - k + step) % (kFsRows - 1);
                const int p = ia < ib ? ia : ib, q = ia < ib ? ib : ia;
                const double a = M[p * kFsLd + p], d = M[q * kFsLd + q], b = M[p * kFsLd + q];
                double c = 1.0, s = 0.0;
                if (b != 0.0 && fabs(b) > DBL_EPSILON * 0.25 * sqrt(fabs(a * d))) {
                    const double tau = (d - a) / (2.0 * b);
                    const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + t * t);
                    s = t * c;
                }
                rp[k] = p;
                rq[k] = q;
                rc[k] = c;
                rs[k] = s;
            }
            __syncthreads();
            // M <- J^T M J in one pass: the 32 disjoint rotations split M into
            // 2 x 2 blocks (rows {p_a, q_a}, columns {p_b, q_b}), each updated on
            // its own (rows first, then columns, as two separate passes would);
            // P <- P J beside it
            for (int e = threadIdx.x; e < (kFsRows / 2) * (kFsRows / 2); e += kEigThreads) {
                const int ka = e / (kFsRows / 2), kb = e % (kFsRows / 2);
                const int pa = rp[ka], qa = rq[ka], pb = rp[kb], qb = rq[kb];
                const double ca = rc[ka], sa = rs[ka], cb = rc[kb], sb = rs[kb];
                const double m00 = M[pa * kFsLd + pb], m01 = M[pa * kFsLd + qb];
                const double m10 = M[qa * kFsLd + pb], m11 = M[qa * kFsLd + qb];
                const double r00 = ca * m00 - sa * m10, r01 = ca * m01 - sa * m11;
                const double r10 = sa * m00 + ca * m10, r11 = sa * m01 + ca * m11;
                M[pa * kFsLd + pb] = cb * r00 - sb * r01;
                M[pa * kFsLd + qb] = sb * r00 + cb * r01;
                M[qa * kFsLd + pb] = cb * r10 - sb * r11;
                M[qa * kFsLd + qb] = sb * r10 + cb * r11;
            }
            for (int e = threadIdx.x; e < (kFsRows / 2) * kFsRows; e += kEigThreads) {
                const int k = e / kFsRows, i = e % kFsRows;
                const int p = rp[k], q = rq[k];
                const double c = rc[k], s = rs[k];
                const double pp = P[i * kFsLd + p], pq = P[i * kFsLd + q];
                P[i * kFsLd + p] = c * pp - s * pq;
                P[i * kFsLd + q] = s * pp + c * pq;
            }
            __syncthreads();
        }
        if (sweep + 1 < max_inner && !(offdiag(M, inv_f, red) > tol_in)) break;
    }
    double* dst = Pout + (int64_t)pair * (kFsRows * kFsRows);
    for (int e = threadIdx.x; e < kFsRows * kFsRows; e += kEigThreads)
        dst[e] = P[(e / kFsRows) * kFsLd + e % kFsRows];
    if (threadIdx.x == 0) flag[pair] = 1;
}

// X <- P^T X on the pair's 64 rows, column tiles [kFsUpdTiles bx, kFsUpdTiles
// (bx + 1)) of 64 columns each, of ncol (all columns, the f column included).
// Each lane holds the 16 entries of P it supplies as the A operand in
// registers for all the workgroup's tiles, so LDS holds only the staged
// tile.  Skipped when flag[pair] = 0.
__global__ __launch_bounds__(kBlock, 3) void k_fs_update(double* __restrict__ G, int64_t ldg, int64_t ncol,
                                                      const int32_t* __restrict__ rowidx,
                                                      const int2* __restrict__ pairs,
                                                      const double* __restrict__ Pin,
                                                      const int32_t* __restrict__ flag) {
    __shared__ double t[kFsRows * kFsLd];
    const int pair = blockIdx.y;
    if (flag[pair] == 0) return;  // block-uniform
    const int2 pr = pairs[pair];
    const double* P = Pin + (int64_t)pair * (kFsRows * kFsRows);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int li = lane & 15, lk = lane >> 4;
    // Y[i][c] = sum_k P[k][i] X[k][c]: A[i][k] = P[k][i] (lane: k = kk + lk, i = 16 w + li)
    double pa[kFsRows / 4];
#pragma unroll
    for (int s = 0; s < kFsRows / 4; ++s) pa[s] = P[(4 * s + lk) * kFsRows + 16 * w + li];
    // the four output rows of this lane, fixed over the tiles
    int64_t orow[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) orow[r] = (int64_t)pair_row(rowidx, pr, 16 * w + 4 * r + lk) * ldg;
    const int64_t ntile = (ncol + kFsRows - 1) / kFsRows;
    const int64_t tb = (int64_t)blockIdx.x * kFsUpdTiles;
    const int64_t te = tb + kFsUpdTiles < ntile ? tb + kFsUpdTiles : ntile;
    // software pipeline: the next tile's loads are in flight (registers) while
    // this tile's products run from LDS (the tiles' columns are disjoint, so
    // the in-place stores never meet a pending load)
    constexpr int kQ = kFsRows / (kBlock / kWave);  // rows loaded per lane
    const int lc = threadIdx.x & (kWave - 1), lr = threadIdx.x / kWave;
    int64_t rowoff[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) rowoff[q] = pair_row(rowidx, pr, lr + (kBlock / kWave) * q) * ldg;
    double nxt[kQ];
    auto fetch = [&](int64_t tl) {
        const int64_t cc = tl * kFsRows;
        const bool ok = tl < te && cc + lc < ncol;
#pragma unroll
        for (int q = 0; q < kQ; ++q) nxt[q] = ok ? G[rowoff[q] + cc + lc] : 0.0;
    };
    fetch(tb);
    for (int64_t tile = tb; tile < te; ++tile) {
        const int64_t c0 = tile * kFsRows;
        __syncthreads();  // the previous tile's reads of t done
#pragma unroll
        for (int q = 0; q < kQ; ++q) t[(lr + (kBlock / kWave) * q) * kFsLd + lc] = nxt[q];
        __syncthreads();
        fetch(tile + 1);
        v4d acc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < kFsRows / 4; ++s) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double bv = t[(4 * s + lk) * kFsLd + 16 * q + li];
                acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[s], bv, acc[q], 0, 0, 0);
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t col = c0 + 16 * q + li;
            if (col >= ncol) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) G[orow[r] + col] = acc[q][r];
        }
    }
}

// Largest entry of off[0 .. count) into out[0] and the number of entries
// above tol into out[1] (one workgroup).
__global__ __launch_bounds__(kBlock) void k_fs_maxoff(const double* __restrict__ off, int64_t count, double tol,
                                                      double* __restrict__ out) {
    __shared__ double red[kBlock / kWave];
    __shared__ double cnt[kBlock / kWave];
    double mx = 0.0, c = 0.0;
    for (int64_t i = threadIdx.x; i < count; i += kBlock) {
        mx = off[i] > mx ? off[i] : mx;
        c += off[i] > tol ? 1.0 : 0.0;
    }
    c = block_sum<kBlock>(c, cnt);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double y = __shfl_xor(mx, o, kWave);
        mx = y > mx ? y : mx;
    }
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = 0.0;
        for (int i = 0; i < kBlock / kWave; ++i) r = red[i] > r ? red[i] : r;
        out[0] = r;
        out[1] = c;
    }
}

// sigma_i = ||row i of Q A|| (columns < n), fhat_i = G[i][n]; one workgroup per row.
__global__ __launch_bounds__(kBlock) void k_fs_norms(const double* __restrict__ G, int64_t ldg, int64_t n,
                                                     double* __restrict__ sig, double* __restrict__ fh) {
    // grid: one workgroup per row (any number of rows; columns < n)
    __shared__ double lds[kBlock / kWave];
    const int64_t i = blockIdx.x;
    const double* row = G + i * ldg;
    double s = 0.0;
    for (int64_t j = threadIdx.x; j < n; j += kBlock) s = fma(row[j], row[j], s);
    s = block_sum<kBlock>(s, lds);
    if (threadIdx.x == 0) {
        sig[i] = sqrt(s);
        fh[i] = row[n];
    }
}

// Descending order: rank[i] = #{j : sig_j > sig_i or (sig_j == sig_i and j < i)};
// sv[rank] = sig_i, fs[rank] = fh_i, order[rank] = i.
__global__ __launch_bounds__(kBlock) void k_fs_rank(const double* __restrict__ sig, const double* __restrict__ fh,
                                                    int64_t n, int32_t* __restrict__ rank, double* __restrict__ sv,
                                                    double* __restrict__ fs, int32_t* __restrict__ order) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double si = sig[i];
    int64_t rk = 0;
    for (int64_t j = 0; j < n; ++j) {
        const double sj = sig[j];
        rk += (sj > si || (sj == si && j < i)) ? 1 : 0;
    }
    rank[i] = (int32_t)rk;
    sv[rk] = si;
    fs[rk] = fh[i];
    order[rk] = (int32_t)i;
}

// ---------------------------------------------------------------------------
// Parameter choice on the full problem (eq. (25)): sv descending (n values;
// the first r, r = the number of positive ones but at most rcap, are used),
// fs = U^T f in the same order, s_perp = ||f||^2 - sum_{i < r} fs_i^2
// (clamped at 0), N = n in the denominator.  One workgroup per source.  Tikhonov: GCV(lambda) on J log-spaced points on
// [max(sigma_r, 16 eps sigma_1), sigma_1], golden-section refinement of
// log lambda over the two cells around the grid minimum (ties to the larger
// lambda, a minimum at an end kept with the edge flag) -- the rule of the
// projected problem with N in the denominator.  TSVD: k minimising
// (sum_{i>k} fs_i^2 + s_perp) / (N - k)^2 over k = 1 .. min(r, N - 1), ties to
// the smaller k.  FIXED: lambda_fixed or k_fixed.  One workgroup.
// ---------------------------------------------------------------------------

__device__ double full_gcv(const double* __restrict__ sv, const double* __restrict__ fs, int64_t r, int64_t n,
                           double sperp, double lam, double* __restrict__ lds) {
    const double l2 = lam * lam;
    double a = 0.0, t = 0.0;
    for (int64_t i = threadIdx.x; i < r; i += kBlock) {
        const double s2 = sv[i] * sv[i];
        const double den = s2 + l2;
        const double x = l2 / den * fs[i];
        a = fma(x, x, a);
        t += s2 / den;
    }
    a = block_sum<kBlock>(a, lds);
    t = block_sum<kBlock>(t, lds);
    const double d = (double)n - t;
    return (a + sperp) / (d * d);
}

__global__ __launch_bounds__(kBlock) void k_full_param(const double* __restrict__ sv, const double* __restrict__ fs,
                                                       int64_t n, int64_t rcap, const double* __restrict__ fnorm2v,
                                                       int64_t vs, int32_t method, int32_t rule, int32_t J,
                                                       double lambda_fixed, int32_t k_fixed,
                                                       double* __restrict__ tail, ParamOut* __restrict__ out) {
    __shared__ double lds[kBlock / kWave];
    // source z = blockIdx.x: its data at fs + z vs, its tail at + z (n + 1), its choice at out + z
    const int64_t z = blockIdx.x;
    fs += z * vs;
    tail += z * (n + 1);
    out += z;
    const double fnorm2 = fnorm2v[z];
    __shared__ double vals[kMaxGrid];
    __shared__ int64_t s_r;
    if (threadIdx.x == 0) {
        int64_t r = 0;
        while (r < n && r < rcap && sv[r] > 0.0) ++r;
        s_r = r;
    }
    __syncthreads();
    const int64_t r = s_r;
    // s_perp: what the r retained components leave of ||f||^2
    double ssum = 0.0;
    for (int64_t i = threadIdx.x; i < r; i += kBlock) ssum = fma(fs[i], fs[i], ssum);
    ssum = block_sum<kBlock>(ssum, lds);
    const double sperp = fnorm2 - ssum > 0.0 ? fnorm2 - ssum : 0.0;
    uint32_t flags = 0;
    if (method == 0) {  // TSVD
        int64_t k = 1;
        double crit = 0.0;
        const int64_t kmax = r < n - 1 ? r : n - 1;
        if (threadIdx.x == 0) {
            // tail[k] = sum_{i >= k} fs_i^2 over the r retained values, k = 0 .. r
            double acc = 0.0;
            tail[r] = 0.0;
            for (int64_t i = r - 1; i >= 0; --i) {
                acc = fma(fs[i], fs[i], acc);
                tail[i] = acc;
            }
        }
        __syncthreads();
        if (rule == 2) {
            k = k_fixed < 1 ? 1 : (k_fixed > r ? r : k_fixed);
            const double d = (double)(n - k);
            crit = d > 0.0 ? (tail[k] + sperp) / (d * d) : 0.0;
        } else if (kmax >= 1) {
            // argmin over k = 1 .. kmax, ties to the smaller k
            double best = 0.0;
            int64_t bk = -1;
            for (int64_t kk = 1 + threadIdx.x; kk <= kmax; kk += kBlock) {
                const double d = (double)(n - kk);
                const double g = (tail[kk] + sperp) / (d * d);
                if (bk < 0 || g < best) {
                    best = g;
                    bk = kk;
                }
            }
            __shared__ double bv[kBlock];
            __shared__ int64_t bi[kBlock];
            bv[threadIdx.x] = best;
            bi[threadIdx.x] = bk;
            __syncthreads();
            if (threadIdx.x == 0) {
                double b = 0.0;
                int64_t kb = -1;
                for (int q = 0; q < kBlock; ++q) {
                    if (bi[q] < 0) continue;
                    if (kb < 0 || bv[q] < b || (bv[q] == b && bi[q] < kb)) {
                        b = bv[q];
                        kb = bi[q];
                    }
                }
                s_r = kb;
                lds[0] = b;
            }
            __syncthreads();
            k = s_r;
            crit = lds[0];
            if (k == 1 || k == kmax) flags |= 2u;
        }
        if (threadIdx.x == 0) {
            double eta2 = 0.0;
            for (int64_t i = 0; i < k; ++i) eta2 += (fs[i] / sv[i]) * (fs[i] / sv[i]);
            out->lambda = 0.0;
            out->k = (int32_t)k;
            out->crit = crit;
            out->flags = flags;
            out->rho = sqrt(tail[k] + sperp);
            out->eta = sqrt(eta2);
        }
        return;
    }
    // Tikhonov
    double lam;
    double crit;
    if (rule == 2 || r == 0) {
        lam = r == 0 ? 0.0 : lambda_fixed;
        crit = r == 0 ? 0.0 : full_gcv(sv, fs, r, n, sperp, lam, lds);
    } else {
        const double s1 = sv[0];
        double lo = sv[r - 1];
        if (lo < 16.0 * DBL_EPSILON * s1) lo = 16.0 * DBL_EPSILON * s1;
        if (!(lo < s1)) lo = 16.0 * DBL_EPSILON * s1;
        const double llo = log(lo), lhi = log(s1);
        for (int j = 0; j < J; ++j) {
            const double lj = exp(llo + (lhi - llo) * j / (J - 1));
            const double g = full_gcv(sv, fs, r, n, sperp, lj, lds);
            if (threadIdx.x == 0) vals[j] = g;
        }
        __syncthreads();
        int jb = 0;
        for (int j = 1; j < J; ++j)
            if (vals[j] <= vals[jb]) jb = j;  // ties to the larger lambda
        lam = exp(llo + (lhi - llo) * jb / (J - 1));
        crit = vals[jb];
        if (jb == 0 || jb == J - 1) {
            flags |= 2u;
        } else {
            // golden section on log lambda over [grid jb-1, grid jb+1]
            double a = llo + (lhi - llo) * (jb - 1) / (J - 1), b = llo + (lhi - llo) * (jb + 1) / (J - 1);
            const double gr = 0.5 * (sqrt(5.0) - 1.0);
            double x1 = b - gr * (b - a), x2 = a + gr * (b - a);
            double f1 = full_gcv(sv, fs, r, n, sperp, exp(x1), lds), f2 = full_gcv(sv, fs, r, n, sperp, exp(x2), lds);
            for (int it = 0; it < 200 && (b - a) > 1e-10; ++it) {
                if (f1 <= f2) {
                    b = x2;
                    x2 = x1;
                    f2 = f1;
                    x1 = b - gr * (b - a);
                    f1 = full_gcv(sv, fs, r, n, sperp, exp(x1), lds);
                } else {
                    a = x1;
                    x1 = x2;
                    f1 = f2;
                    x2 = a + gr * (b - a);
                    f2 = full_gcv(sv, fs, r, n, sperp, exp(x2), lds);
                }
            }
            const double xm = 0.5 * (a + b);
            const double gm = full_gcv(sv, fs, r, n, sperp, exp(xm), lds);
            if (gm <= crit) {
                lam = exp(xm);
                crit = gm;
            }
        }
    }
    // residual and solution norms at lambda
    const double l2 = lam * lam;
    double rho2 = 0.0, eta2 = 0.0;
    for (int64_t i = threadIdx.x; i < r; i += kBlock) {
        const double s2 = sv[i] * sv[i];
        const double den = s2 + l2;
        const double x = l2 / den * fs[i];
        const double y = sv[i] / den * fs[i];
        rho2 = fma(x, x, rho2);
        eta2 = fma(y, y, eta2);
    }
    rho2 = block_sum<kBlock>(rho2, lds);
    eta2 = block_sum<kBlock>(eta2, lds);
    if (threadIdx.x == 0) {
        out->lambda = lam;
        out->k = 0;
        out->crit = crit;
        out->flags = flags;
        out->rho = sqrt(rho2 + sperp);
        out->eta = sqrt(eta2);
    }
}

// The solutions.  With G = Q A (Q orthogonal), the Tikhonov solution is
// exactly x = G^T y with (G G^T + lambda^2 I) y = Q f = f^; the TSVD solution
// of rank k is x = G_k^T y with G_k G_k^T y = f^_k over the k rows of the
// largest sigma.  Neither needs the rows to be orthogonal, only Q to be.
// G G^T = diag(sigma^2) + E, E the rows' remaining off-diagonal products:
// the convergence test bounds E_ij by tol ||A||_F max(sigma_i, sigma_j), so
// rows with sigma near lambda keep couplings of order tol ||A||_F / lambda
// after scaling, which the solution's large cancelling coefficients do not
// forgive.  The system is solved by conjugate gradients preconditioned with
// its diagonal d_i = sigma_i^2 + lambda^2 (resp. sigma_i^2 on the k rows),
// from y = 0, until sqrt(r^T D^-1 r) <= 1e-15 of its start (the attainable
// level) or an iteration cap.  One iteration: x = G^T q (split over row
// chunks), w = G x + lambda^2 q, two dot products, the updates.

// d_i of row i (0: row not in the solution; rows of rank >= rcap, past the
// retained singular values, never are).
__device__ __forceinline__ double sol_diag(double sig, int32_t rank, int32_t method, double l2, int64_t k,
                                           int64_t rcap) {
    const double s2 = sig * sig;
    if (rank >= rcap) return 0.0;
    if (method == 0) return (rank < k && s2 > 0.0) ? s2 : 0.0;
    return s2 + l2;
}

__device__ __forceinline__ double sol_l2(int32_t method, const ParamOut* po) {
    return method == 0 ? 0.0 : po->lambda * po->lambda;
}

// Every solution kernel serves nz data columns at once (source z from the
// grid, see each kernel): its vectors for source z start at + z vs, its
// scalars pc at + 4 z, its choice at po + z.

// y = 0, r = b (active rows), q = D^-1 r, t_i = r_i q_i.  Grid (rows, nz).
__global__ __launch_bounds__(kBlock) void k_fs_pcg_start(const double* __restrict__ sig,
                                                         const double* __restrict__ fh,
                                                         const int32_t* __restrict__ rank, int64_t n, int32_t method,
                                                         int64_t rcap, const ParamOut* __restrict__ po, int64_t vs,
                                                         double* __restrict__ y, double* __restrict__ r,
                                                         double* __restrict__ q, double* __restrict__ t) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t z = blockIdx.y, o = z * vs + i;
    po += z;
    const double d = sol_diag(sig[i], rank[i], method, sol_l2(method, po), po->k, rcap);
    const double b = d > 0.0 ? fh[o] : 0.0;
    y[o] = 0.0;
    r[o] = b;
    q[o] = d > 0.0 ? b / d : 0.0;
    t[o] = d > 0.0 ? b * b / d : 0.0;
}

// part[z][c][j] = sum over the rows i of chunk c (rows < n) of q_z[i] G[i][j];
// grid (columns / kBlock, chunks, nz), one thread per column.
__global__ __launch_bounds__(kBlock) void k_fs_gemvt_part(const double* __restrict__ G, int64_t ldg, int64_t n,
                                                          int64_t rows_per_chunk, const double* __restrict__ q,
                                                          int64_t vs, double* __restrict__ part) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    q += (int64_t)blockIdx.z * vs;
    const int64_t i0 = (int64_t)blockIdx.y * rows_per_chunk;
    const int64_t i1 = i0 + rows_per_chunk < n ? i0 + rows_per_chunk : n;
    double s0 = 0.0, s1 = 0.0;
    int64_t i = i0;
    for (; i + 1 < i1; i += 2) {
        s0 = fma(q[i], G[i * ldg + j], s0);
        s1 = fma(q[i + 1], G[(i + 1) * ldg + j], s1);
    }
    if (i < i1) s0 = fma(q[i], G[i * ldg + j], s0);
    part[((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * n + j] = s0 + s1;
}

// x_z[j] = sum_c part[z][c][j], chunks in order; grid (columns / kBlock, nz).
__global__ __launch_bounds__(kBlock) void k_fs_colsum(const double* __restrict__ part, int chunks, int64_t n,
                                                      int64_t vs, double* __restrict__ x) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    const int64_t z = blockIdx.y;
    part += z * chunks * n;
    double s = 0.0;
    for (int c = 0; c < chunks; ++c) s += part[(int64_t)c * n + j];
    x[z * vs + j] = s;
}

// w_i = G[i] . x + lambda^2 q_i on active rows (0 elsewhere), t_i = q_i w_i;
// grid (rows, nz), one workgroup per row.
__global__ __launch_bounds__(kBlock) void k_fs_pcg_matvec(const double* __restrict__ G, int64_t ldg, int64_t n,
                                                          const double* __restrict__ x,
                                                          const double* __restrict__ sig,
                                                          const int32_t* __restrict__ rank, int32_t method,
                                                          int64_t rcap, const ParamOut* __restrict__ po, int64_t vs,
                                                          const double* __restrict__ q, double* __restrict__ w,
                                                          double* __restrict__ t) {
    __shared__ double lds[kBlock / kWave];
    const int64_t i = blockIdx.x, z = blockIdx.y;
    x += z * vs;
    const double* row = G + i * ldg;
    double s = 0.0;
    for (int64_t j = threadIdx.x; j < n; j += kBlock) s = fma(row[j], x[j], s);
    s = block_sum<kBlock>(s, lds);
    if (threadIdx.x == 0) {
        po += z;
        const int64_t o = z * vs + i;
        const double l2 = sol_l2(method, po);
        const double d = sol_diag(sig[i], rank[i], method, l2, po->k, rcap);
        const double wi = d > 0.0 ? s + l2 * q[o] : 0.0;
        w[o] = wi;
        t[o] = q[o] * wi;
    }
}

// pc[4 z + slot] = sum_i t_z[i] (one workgroup per source, fixed order).
__global__ __launch_bounds__(kBlock) void k_fs_pcg_sum(const double* __restrict__ t, int64_t n, int64_t vs,
                                                       double* __restrict__ pc, int slot) {
    __shared__ double lds[kBlock / kWave];
    const int64_t z = blockIdx.x;
    t += z * vs;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kBlock) s += t[i];
    s = block_sum<kBlock>(s, lds);
    if (threadIdx.x == 0) pc[4 * z + slot] = s;
}

// a = pc[cur] / pc[0] (r^T D^-1 r over q^T B q); y += a q; r -= a w;
// t_i = r_i^2 / d_i.  Grid (rows, nz).
__global__ __launch_bounds__(kBlock) void k_fs_pcg_step(const double* __restrict__ sig,
                                                        const int32_t* __restrict__ rank, int64_t n, int32_t method,
                                                        int64_t rcap, const ParamOut* __restrict__ po, int64_t vs,
                                                        const double* __restrict__ pc, int cur,
                                                        const double* __restrict__ q, const double* __restrict__ w,
                                                        double* __restrict__ y, double* __restrict__ r,
                                                        double* __restrict__ t) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t z = blockIdx.y, o = z * vs + i;
    po += z;
    pc += 4 * z;
    const double qw = pc[0];
    const double a = qw > 0.0 ? pc[cur] / qw : 0.0;
    const double d = sol_diag(sig[i], rank[i], method, sol_l2(method, po), po->k, rcap);
    y[o] = fma(a, q[o], y[o]);
    const double ri = fma(-a, w[o], r[o]);
    r[o] = ri;
    t[o] = d > 0.0 ? ri * ri / d : 0.0;
}

// q = D^-1 r + (pc[nxt] / pc[cur]) q.  Grid (rows, nz).
__global__ __launch_bounds__(kBlock) void k_fs_pcg_dir(const double* __restrict__ sig,
                                                       const int32_t* __restrict__ rank, int64_t n, int32_t method,
                                                       int64_t rcap, const ParamOut* __restrict__ po, int64_t vs,
                                                       const double* __restrict__ pc, int cur, int nxt,
                                                       const double* __restrict__ r, double* __restrict__ q) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t z = blockIdx.y, o = z * vs + i;
    po += z;
    pc += 4 * z;
    const double beta = pc[cur] > 0.0 ? pc[nxt] / pc[cur] : 0.0;
    const double d = sol_diag(sig[i], rank[i], method, sol_l2(method, po), po->k, rcap);
    q[o] = d > 0.0 ? fma(beta, q[o], r[o] / d) : 0.0;
}

// Norms of the returned solution: t_i = (G[i] . x - fh_i)^2 (one workgroup
// per row; with Q orthogonal sum_i t_i = ||A x - f||^2, the padding rows
// staying exactly zero), and w_i = x_i^2.  Grid (rows, nz).
__global__ __launch_bounds__(kBlock) void k_fs_resid(const double* __restrict__ G, int64_t ldg, int64_t n,
                                                     const double* __restrict__ x, const double* __restrict__ fh,
                                                     int64_t vs, double* __restrict__ t, double* __restrict__ w) {
    __shared__ double lds[kBlock / kWave];
    const int64_t i = blockIdx.x, z = blockIdx.y;
    x += z * vs;
    const double* row = G + i * ldg;
    double s = 0.0;
    for (int64_t j = threadIdx.x; j < n; j += kBlock) s = fma(row[j], x[j], s);
    s = block_sum<kBlock>(s, lds);
    if (threadIdx.x == 0) {
        const double d = s - fh[z * vs + i];
        t[z * vs + i] = d * d;
        w[z * vs + i] = x[i] * x[i];
    }
}

// po[z].rho = sqrt(pc[4 z + 1]), po[z].eta = sqrt(pc[4 z]), z < nz.
__global__ void k_fs_set_norms(const double* __restrict__ pc, ParamOut* __restrict__ po, int nz) {
    const int z = threadIdx.x;
    if (z < nz) {
        po[z].rho = sqrt(pc[4 * z + 1]);
        po[z].eta = sqrt(pc[4 * z]);
    }
}

// fs_z[rank[i]] = fh_z[i] (the data columns in descending singular-value
// order); grid (rows, nz).
__global__ __launch_bounds__(kBlock) void k_fs_gather(const int32_t* __restrict__ rank, const double* __restrict__ fh,
                                                      int64_t n, int64_t vs, double* __restrict__ fs) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t z = blockIdx.y;
    fs[z * vs + rank[i]] = fh[z * vs + i];
}

// out[z vs + i] = G[i][col0 + z], i < rows; grid (rows, nz).
__global__ __launch_bounds__(kBlock) void k_fs_col(const double* __restrict__ G, int64_t ldg, int64_t rows,
                                                   int64_t col0, int64_t vs, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t z = blockIdx.y;
    if (i < rows) out[z * vs + i] = G[i * ldg + col0 + z];
}

// G[i][n] = f_i for i < n (the f column of the work matrix).
__global__ __launch_bounds__(kBlock) void k_fs_setf(double* __restrict__ G, int64_t ldg, int64_t n,
                                                    const double* __restrict__ f) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) G[i * ldg + n] = f != nullptr ? f[i] : 0.0;
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------

void launch_fs_setf(double* G, int64_t ldg, int64_t n, const double* f, hipStream_t s) {
    k_fs_setf<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(G, ldg, n, f);
}

void launch_fs_gram(const double* G, int64_t ldg, int64_t ncol, const int32_t* rowidx, const int2* pairs, int npairs,
                    int S, int64_t chunk, double* Pg, const int32_t* pair_ok, const int32_t* blk_stamp, int64_t slot0,
                    int same, hipStream_t s) {
    k_fs_gram<<<dim3((unsigned)S, (unsigned)npairs), kBlock, 0, s>>>(G, ldg, ncol, rowidx, pairs, chunk, Pg, pair_ok,
                                                                     blk_stamp, slot0, same);
}

void launch_fs_eig(const double* Pg, int S, int npairs, double tol, double inv_f, int max_inner, double* Pout,
                   int32_t* flag, double* off, const int2* pairs, int32_t* pair_ok, int32_t* blk_stamp, int64_t slot0,
                   int32_t g, int same, hipStream_t s) {
    k_fs_eig<<<(unsigned)npairs, kEigThreads, 0, s>>>(Pg, S, tol, inv_f, max_inner, Pout, flag, off, pairs, pair_ok,
                                                 blk_stamp, slot0, g, same);
}

void launch_fs_update(double* G, int64_t ldg, int64_t ncol, const int32_t* rowidx, const int2* pairs, int npairs,
                      const double* Pin, const int32_t* flag, hipStream_t s) {
    const int64_t ntile = (ncol + kFsRows - 1) / kFsRows;
    k_fs_update<<<dim3((unsigned)((ntile + kFsUpdTiles - 1) / kFsUpdTiles), (unsigned)npairs), kBlock, 0, s>>>(
        G, ldg, ncol, rowidx, pairs, Pin, flag);
}

void launch_fs_maxoff(const double* off, int64_t count, double tol, double* out, hipStream_t s) {
    k_fs_maxoff<<<1, kBlock, 0, s>>>(off, count, tol, out);
}

void launch_fs_norms(const double* G, int64_t ldg, int64_t rows, int64_t n, double* sig, double* fh, hipStream_t s) {
    k_fs_norms<<<(unsigned)rows, kBlock, 0, s>>>(G, ldg, n, sig, fh);
}

void launch_fs_rank(const double* sig, const double* fh, int64_t n, int32_t* rank, double* sv, double* fs,
                    int32_t* order, hipStream_t s) {
    k_fs_rank<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(sig, fh, n, rank, sv, fs, order);
}

void launch_full_param(const double* sv, const double* fs, int64_t n, int64_t rcap, const double* fnorm2v,
                       int64_t vs, int32_t method, int32_t rule, int32_t J, double lambda_fixed, int32_t k_fixed,
                       double* tail, ParamOut* out, int nz, hipStream_t s) {
    k_full_param<<<(unsigned)nz, kBlock, 0, s>>>(sv, fs, n, rcap, fnorm2v, vs, method, rule, J, lambda_fixed, k_fixed,
                                                 tail, out);
}

int fs_gemvt_chunks(int64_t n) {
    // enough workgroups to cover the chip: columns / kBlock x chunks >= 1024
    const int64_t cols = (n + kBlock - 1) / kBlock;
    int64_t c = (1024 + cols - 1) / cols;
    const int64_t cmax = (n + 63) / 64;  // at least 64 rows per chunk
    if (c > cmax) c = cmax;
    if (c > kFsMaxChunks) c = kFsMaxChunks;
    return (int)(c < 1 ? 1 : c);
}

void launch_fs_gemvt(const double* G, int64_t ldg, int64_t n, const double* q, int64_t vs, double* part, double* x,
                     int nz, hipStream_t s) {
    const int c = fs_gemvt_chunks(n);
    const int64_t rows = (n + c - 1) / c;
    const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
    k_fs_gemvt_part<<<dim3(nb, (unsigned)c, (unsigned)nz), kBlock, 0, s>>>(G, ldg, n, rows, q, vs, part);
    k_fs_colsum<<<dim3(nb, (unsigned)nz), kBlock, 0, s>>>(part, c, n, vs, x);
}

void launch_fs_pcg_start(const double* sig, const double* fh, const int32_t* rank, int64_t n, int32_t method,
                         int64_t rcap, const ParamOut* po, int64_t vs, double* y, double* r, double* q, double* t,
                         double* pc, int slot, int nz, hipStream_t s) {
    const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
    k_fs_pcg_start<<<dim3(nb, (unsigned)nz), kBlock, 0, s>>>(sig, fh, rank, n, method, rcap, po, vs, y, r, q, t);
    k_fs_pcg_sum<<<(unsigned)nz, kBlock, 0, s>>>(t, n, vs, pc, slot);
}

void launch_fs_pcg_iter(const double* G, int64_t ldg, int64_t n, const double* sig, const int32_t* rank,
                        int32_t method, int64_t rcap, const ParamOut* po, int64_t vs, double* pc, int cur, int nxt,
                        double* y, double* r, const double* q, double* w, double* t, double* part, double* x, int nz,
                        hipStream_t s) {
    const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
    launch_fs_gemvt(G, ldg, n, q, vs, part, x, nz, s);
    k_fs_pcg_matvec<<<dim3((unsigned)n, (unsigned)nz), kBlock, 0, s>>>(G, ldg, n, x, sig, rank, method, rcap, po, vs,
                                                                       q, w, t);
    k_fs_pcg_sum<<<(unsigned)nz, kBlock, 0, s>>>(t, n, vs, pc, 0);
    k_fs_pcg_step<<<dim3(nb, (unsigned)nz), kBlock, 0, s>>>(sig, rank, n, method, rcap, po, vs, pc, cur, q, w, y, r,
                                                           t);
    k_fs_pcg_sum<<<(unsigned)nz, kBlock, 0, s>>>(t, n, vs, pc, nxt);
}

void launch_fs_solution_norms(const double* G, int64_t ldg, int64_t n, const double* x, const double* fh, int64_t vs,
                              double* t, double* w, double* pc, ParamOut* po, int nz, hipStream_t s) {
    k_fs_resid<<<dim3((unsigned)n, (unsigned)nz), kBlock, 0, s>>>(G, ldg, n, x, fh, vs, t, w);
    k_fs_pcg_sum<<<(unsigned)nz, kBlock, 0, s>>>(t, n, vs, pc, 1);
    k_fs_pcg_sum<<<(unsigned)nz, kBlock, 0, s>>>(w, n, vs, pc, 0);
    k_fs_set_norms<<<1, 64, 0, s>>>(pc, po, nz);
}

void launch_fs_pcg_dir(const double* sig, const int32_t* rank, int64_t n, int32_t method, int64_t rcap,
                       const ParamOut* po, int64_t vs, const double* pc, int cur, int nxt, const double* r, double* q,
                       int nz, hipStream_t s) {
    k_fs_pcg_dir<<<dim3((unsigned)((n + kBlock - 1) / kBlock), (unsigned)nz), kBlock, 0, s>>>(
        sig, rank, n, method, rcap, po, vs, pc, cur, nxt, r, q);
}

void launch_fs_col(const double* G, int64_t ldg, int64_t rows, int64_t col0, int64_t vs, double* out, int nz,
                   hipStream_t s) {
    k_fs_col<<<dim3((unsigned)((rows + kBlock - 1) / kBlock), (unsigned)nz), kBlock, 0, s>>>(G, ldg, rows, col0, vs,
                                                                                            out);
}

void launch_fs_gather(const int32_t* rank, const double* fh, int64_t n, int64_t vs, double* fs, int nz,
                      hipStream_t s) {
    k_fs_gather<<<dim3((unsigned)((n + kBlock - 1) / kBlock), (unsigned)nz), kBlock, 0, s>>>(rank, fh, n, vs, fs);
}

}  // namespace mqh
