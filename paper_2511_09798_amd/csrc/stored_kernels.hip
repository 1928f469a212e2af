// stored_kernels.hip -- the stored FP64 Kansa matrix on gfx950: assembly
// (tiled, and dense row-major for the full-SVD reference), the products
// A x and A^T x on the tiles with their fixed-order reduction, and rows of A.
//
// Vectors have a leading dimension ldn (multiple of 64, >= n) and are zero
// past n; nodes are double4 records (centred, scaled by eps).
#include "kernels.hpp"

namespace mqh {

// ---------------------------------------------------------------------------
// Stored FP64 operator in symmetric-block tiles.
//
// The interior-interior block of A (L phi rows against interior centres) and
// the boundary-boundary block (phi rows against boundary centres) are
// symmetric, since their entries depend on |X_i - X_j| only.  Node indices are
// cut into tiles of kTile per class (interior tiles 0 .. nti-1, boundary tiles
// nti .. nt-1, each class zero-padded to whole tiles), and A is stored as
// kTile x kTile tiles, row-major inside a tile:
//   interior tile row R: tiles (R, C) for C = R .. nt-1   (upper part of the
//                        interior block, then the interior-boundary block);
//   boundary tile row R: tiles (R, C) for C = 0 .. nti-1, then C = R .. nt-1
//                        (boundary-interior block, upper part of the
//                        boundary block).
// Tile rows follow each other (tile_base[R] = first tile of row R).  A tile
// below the diagonal of a symmetric block is the transpose of a stored one.
// A product visits every stored tile once and uses it as T x_C for y_R (row
// use) and/or T^T x_R for y_C (column use):
//   A x:    row use everywhere; column use for off-diagonal symmetric tiles;
//   A^T x:  row use for symmetric tiles; column use for every tile off the
//           diagonal (the mixed tiles enter A^T transposed).
// ---------------------------------------------------------------------------

// Dense row-major A (n rows, leading dimension lda, zero columns past n), for
// the full-SVD reference's work matrix: one block = RB rows x 512 columns
// (two columns per lane, 16-byte non-temporal stores); the column records stay
// in registers across rows.
template <int RB>
__global__ __launch_bounds__(kBlock) void k_assemble(const double4* __restrict__ X, int64_t n, int64_t n_int,
                                                     int64_t lda, EntryConst c, double* __restrict__ A) {
    const int64_t c0 = (int64_t)blockIdx.x * (2 * kBlock) + 2 * threadIdx.x;
    if (c0 >= lda) return;  // no barriers below
    const bool va = c0 < n, vb = c0 + 1 < n;
    const double4 qa = X[va ? c0 : 0];
    const double4 qb = X[vb ? c0 + 1 : 0];
    const int64_t r0 = (int64_t)blockIdx.y * RB;
    const int64_t r1 = r0 + RB < n ? r0 + RB : n;
    for (int64_t i = r0; i < r1; ++i) {
        const double4 p = X[i];
        const double ta = t_of(p.x, p.y, p.z, qa.x, qa.y, qa.z);
        const double tb = t_of(p.x, p.y, p.z, qb.x, qb.y, qb.z);
        double ea, eb;
        if (i < n_int) {
            ea = entry_interior(ta, c);
            eb = entry_interior(tb, c);
        } else {
            ea = entry_boundary(ta, c);
            eb = entry_boundary(tb, c);
        }
        v2d v;
        v.x = va ? ea : 0.0;
        v.y = vb ? eb : 0.0;
        store_nt(A + i * lda + c0, v);
    }
}

__device__ __forceinline__ int64_t pk_start(const PackedLayout& L, int T) {
    return T < L.nti ? (int64_t)T * kTile : L.n_int + (int64_t)(T - L.nti) * kTile;
}
__device__ __forceinline__ int64_t pk_end(const PackedLayout& L, int T) { return T < L.nti ? L.n_int : L.n; }
// column tile of position p in tile row R, and the position of tile (R, C)
__device__ __forceinline__ int pk_col(const PackedLayout& L, int R, int p) {
    return R < L.nti ? R + p : (p < L.nti ? p : R + (p - L.nti));
}
__device__ __forceinline__ int pk_pos(const PackedLayout& L, int R, int C) {
    return R < L.nti ? C - R : (C < L.nti ? C : L.nti + (C - R));
}

// A[tile (R, C)][i][j] = A(node R_i, node C_j): one workgroup per stored tile
// (blockIdx.y = R, blockIdx.x = position in the row), four rows at a time,
// two columns per lane, 16-byte non-temporal stores; padding rows and
// columns are zero.
__global__ __launch_bounds__(kBlock) void k_assemble_packed(const double4* __restrict__ X, PackedLayout L,
                                                            EntryConst c, double* __restrict__ A) {
    const int R = blockIdx.y, p = blockIdx.x;
    const int ntr = R < L.nti ? L.nt - R : L.nti + (L.nt - R);
    if (p >= ntr) return;  // whole workgroup; no barriers in this kernel
    const int C = pk_col(L, R, p);
    const int64_t r0 = pk_start(L, R), rend = pk_end(L, R);
    const int64_t c0 = pk_start(L, C), cend = pk_end(L, C);
    const bool interior = R < L.nti;
    const int lane2 = 2 * (threadIdx.x & (kWave - 1));
    const int64_t ja = c0 + lane2, jb = ja + 1;
    const bool va = ja < cend, vb = jb < cend;
    const double4 qa = X[va ? ja : 0];
    const double4 qb = X[vb ? jb : 0];
    double* T = A + (L.tile_base[R] + p) * kTileElems + lane2;
    for (int i = threadIdx.x / kWave; i < kTile; i += kBlock / kWave) {
        const int64_t g = r0 + i;
        v2d v;
        v.x = 0.0;
        v.y = 0.0;
        if (g < rend) {
            const double4 q = X[g];
            const double ta = t_of(q.x, q.y, q.z, qa.x, qa.y, qa.z);
            const double tb = t_of(q.x, q.y, q.z, qb.x, qb.y, qb.z);
            const double ea = interior ? entry_interior(ta, c) : entry_boundary(ta, c);
            const double eb = interior ? entry_interior(tb, c) : entry_boundary(tb, c);
            v.x = va ? ea : 0.0;
            v.y = vb ? eb : 0.0;
        }
        store_nt(T + (int64_t)i * kTile, v);
    }
}

// One work item = up to kTileChunk consecutive tiles of one tile row R, all
// four waves on the same tile at once (wave w: rows 32 w .. 32 w + 31, lane
// l: columns 2l, 2l+1, 1 KB per wave load, so a workgroup reads 32 KB runs),
// the next 8-row group's loads always in flight.  Column use: per-lane sums
// over the wave's rows, added over the waves through LDS, one partial per
// tile, PC[tile index][0 .. kTile).  Row use: the per-lane products of 8 rows
// go through LDS and are summed by groups of 8 lanes (no per-row wave
// reduction); one partial per item, PR[item][0 .. kTile).
template <int TRANS>
__global__ __launch_bounds__(kBlock) void k_packed_product(const double* __restrict__ A, PackedLayout L,
                                                           const double* __restrict__ x, double* __restrict__ PR,
                                                           double* __restrict__ PC,
                                                           const GkbState* __restrict__ st) {
    if (st != nullptr && st->stopped) return;  // uniform over the grid
    constexpr int GR = 8;
    constexpr int kWaves = kBlock / kWave;
    constexpr int kRows = kTile / kWaves;   // rows of a tile per wave (32)
    constexpr int kGpw = kRows / GR;        // groups per wave and tile (4)
    constexpr int kRed = GR * (kWave + 1);
    constexpr int kLpr = kWave / GR;
    __shared__ double xr[kTile];
    __shared__ double rsum[kTile];
    __shared__ double red[kWaves][kRed];
    __shared__ double csum[2][kWaves][kTile];  // double-buffered: one barrier per tile
    const int4 it = L.items[blockIdx.x];
    const int R = it.x, p0 = it.y, cnt = it.z;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
    const int total = cnt * kGpw;
    const double* A0 = A + (L.tile_base[R] + p0) * kTileElems + (int64_t)(w * kRows) * kTile + 2 * lane;
    auto gptr = [&](int G) { return A0 + (G / kGpw) * kTileElems + (int64_t)(GR * (G % kGpw)) * kTile; };
    v2d a0[GR], a1[GR];
    {
        const double* T = gptr(0);
#pragma unroll
        for (int r = 0; r < GR; ++r) a0[r] = load_nt(T + (int64_t)r * kTile);
    }
    const int64_t r0 = pk_start(L, R), rend = pk_end(L, R);
    if (tid < kTile) {
        xr[tid] = r0 + tid < rend ? x[r0 + tid] : 0.0;
        rsum[tid] = 0.0;
    }
    __syncthreads();
    double* buf = red[w];
    const int rq = lane / kLpr, qq = lane % kLpr;
    bool use_row = false, use_col = false;
    double xc0 = 0.0, xc1 = 0.0, cs0 = 0.0, cs1 = 0.0;
    int64_t tix = 0;
    auto setup = [&](int q) {
        const int p = p0 + q;
        const int C = pk_col(L, R, p);
        const bool sym = (R < L.nti) == (C < L.nti);
        const bool diag = C == R;
        use_row = TRANS ? sym : true;
        use_col = TRANS ? !diag : (sym && !diag);
        const int64_t c0 = pk_start(L, C), cend = pk_end(L, C);
        const int64_t ca = c0 + 2 * lane, cb = ca + 1;
        xc0 = ca < cend ? x[ca] : 0.0;
        xc1 = cb < cend ? x[cb] : 0.0;
        tix = L.tile_base[R] + p;
        cs0 = 0.0;
        cs1 = 0.0;
    };
    // all waves reach finish (uniform trip count); tile q uses buffer q % 2,
    // whose previous readers (tile q - 2) finished before the barrier of
    // tile q - 1
    auto finish = [&](int q) {
        double* cb = &csum[q & 1][0][0];
        if (use_col) {
            cb[w * kTile + 2 * lane] = cs0;
            cb[w * kTile + 2 * lane + 1] = cs1;
        }
        __syncthreads();
        if (use_col && tid < kTile) {
            double sm = cb[tid];
#pragma unroll
            for (int v = 1; v < kWaves; ++v) sm += cb[v * kTile + tid];
            PC[tix * kTile + tid] = sm;
        }
    };
    auto group = [&](int g, const v2d* a) {  // g: group of this wave within the tile
        const int rbase = w * kRows + GR * g;
        double rp[GR];
#pragma unroll
        for (int r = 0; r < GR; ++r) {
            if (use_col) {
                const double xi = xr[rbase + r];
                cs0 = fma(a[r].x, xi, cs0);
                cs1 = fma(a[r].y, xi, cs1);
            }
            rp[r] = fma(a[r].y, xc1, a[r].x * xc0);
        }
        if (use_row) {
#pragma unroll
            for (int r = 0; r < GR; ++r) buf[r * (kWave + 1) + lane] = rp[r];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
            double sm = 0.0;
#pragma unroll
            for (int k = 0; k < GR; ++k) sm += buf[rq * (kWave + 1) + qq * GR + k];
#pragma unroll
            for (int o = 1; o < kLpr; o <<= 1) sm += __shfl_xor(sm, o, kWave);
            if (qq == 0) rsum[rbase + rq] += sm;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
        }
    };
    for (int G = 0; G < total; G += 2) {  // kGpw is even: G and G + 1 in the same tile
        {
            const double* T = gptr(G + 1);
#pragma unroll
            for (int r = 0; r < GR; ++r) a1[r] = load_nt(T + (int64_t)r * kTile);
        }
        if (G % kGpw == 0) setup(G / kGpw);
        group(G % kGpw, a0);
        if (G + 2 < total) {
            const double* T = gptr(G + 2);
#pragma unroll
            for (int r = 0; r < GR; ++r) a0[r] = load_nt(T + (int64_t)r * kTile);
        }
        group((G + 1) % kGpw, a1);
        if ((G + 2) % kGpw == 0) finish(G / kGpw);
    }
    __syncthreads();
    if (tid < kTile) PR[(int64_t)blockIdx.x * kTile + tid] = rsum[tid];
}

// y_X = sum over the items of tile row X (row use, item order) + sum over the
// tiles (R, X) with a column use (R ascending) - shift z; one workgroup per
// output tile X, four groups of kTile threads taking every fourth source,
// combined in group order.
template <int TRANS>
__global__ __launch_bounds__(4 * kTile) void k_packed_reduce(PackedLayout L, const double* __restrict__ PR,
                                                             const double* __restrict__ PC,
                                                             const double* __restrict__ shift_ptr, double shift_val,
                                                             const double* __restrict__ z, double* __restrict__ y,
                                                             const GkbState* __restrict__ st) {
    if (st != nullptr && st->stopped) return;
    __shared__ double part[4][kTile];
    const int X = blockIdx.x;
    const int t = threadIdx.x & (kTile - 1), grp = threadIdx.x / kTile;
    const int i0 = L.item_first[X], nrow = L.item_first[X + 1] - i0;
    // sources of the column use: R in [a0, a1) and then [b0, b1)
    int a0, a1, b0 = 0, b1 = 0;
    if (X < L.nti) {
        a0 = 0;
        a1 = X;
        if (TRANS) {
            b0 = L.nti;
            b1 = L.nt;
        }
    } else {
        a0 = TRANS ? 0 : L.nti;
        a1 = X;
    }
    const int na = a1 - a0;
    const int total = nrow + na + (b1 - b0);
    double s = 0.0;
#pragma unroll 4
    for (int k = grp; k < total; k += 4) {
        const double* src;
        if (k < nrow) {
            src = PR + (int64_t)(i0 + k) * kTile;
        } else {
            const int c = k - nrow;
            const int Rs = c < na ? a0 + c : b0 + (c - na);
            src = PC + (L.tile_base[Rs] + pk_pos(L, Rs, X)) * kTile;
        }
        s += src[t];
    }
    part[grp][t] = s;
    __syncthreads();
    if (grp == 0) {
        s = (part[0][t] + part[1][t]) + (part[2][t] + part[3][t]);
        const int64_t o = pk_start(L, X) + t;
        if (o < pk_end(L, X)) {
            if (z != nullptr) {
                const double sh = shift_ptr != nullptr ? *shift_ptr : shift_val;
                s -= sh * z[o];
            }
            y[o] = s;
        }
    }
}

// Rows [row0, row0 + gridDim.y) of the stored tiled matrix, row-major with
// leading dimension n (an entry below the diagonal of a symmetric block is
// read from the transposed stored tile).
__global__ __launch_bounds__(kBlock) void k_packed_rows(const double* __restrict__ A, PackedLayout L, int64_t row0,
                                                        double* __restrict__ out) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t i = row0 + blockIdx.y;
    if (j >= L.n) return;
    const int R = i < L.n_int ? (int)(i / kTile) : L.nti + (int)((i - L.n_int) / kTile);
    const int ir = (int)(i - pk_start(L, R));
    const int C = j < L.n_int ? (int)(j / kTile) : L.nti + (int)((j - L.n_int) / kTile);
    const int jc = (int)(j - pk_start(L, C));
    const bool sym = (R < L.nti) == (C < L.nti);
    double v;
    if (sym && C < R)
        v = A[(L.tile_base[C] + pk_pos(L, C, R)) * kTileElems + (int64_t)jc * kTile + ir];
    else
        v = A[(L.tile_base[R] + pk_pos(L, R, C)) * kTileElems + (int64_t)ir * kTile + jc];
    out[(int64_t)blockIdx.y * L.n + j] = v;
}

void launch_assemble(const double4* X, int64_t n, int64_t n_int, int64_t lda, const EntryConst& c, double* A,
                     hipStream_t s) {
    constexpr int RB = 64;
    dim3 grid((unsigned)((lda + 2 * kBlock - 1) / (2 * kBlock)), (unsigned)((n + RB - 1) / RB));
    k_assemble<RB><<<grid, kBlock, 0, s>>>(X, n, n_int, lda, c, A);
}

void launch_assemble_packed(const double4* X, const PackedLayout& L, int32_t max_row_tiles, const EntryConst& c,
                            double* A, hipStream_t s) {
    dim3 grid((unsigned)max_row_tiles, (unsigned)L.nt);
    k_assemble_packed<<<grid, kBlock, 0, s>>>(X, L, c, A);
}

void launch_packed_product(int trans, const double* A, const PackedLayout& L, const double* x, double* PR, double* PC,
                           const GkbState* st, hipStream_t s) {
    if (trans)
        k_packed_product<1><<<(unsigned)L.nitems, kBlock, 0, s>>>(A, L, x, PR, PC, st);
    else
        k_packed_product<0><<<(unsigned)L.nitems, kBlock, 0, s>>>(A, L, x, PR, PC, st);
}

void launch_packed_reduce(int trans, const PackedLayout& L, const double* PR, const double* PC,
                          const double* shift_ptr, double shift_val, const double* z, double* y, const GkbState* st,
                          hipStream_t s) {
    if (trans)
        k_packed_reduce<1><<<(unsigned)L.nt, 4 * kTile, 0, s>>>(L, PR, PC, shift_ptr, shift_val, z, y, st);
    else
        k_packed_reduce<0><<<(unsigned)L.nt, 4 * kTile, 0, s>>>(L, PR, PC, shift_ptr, shift_val, z, y, st);
}

void launch_packed_rows(const double* A, const PackedLayout& L, int64_t row0, int64_t count, double* out,
                        hipStream_t s) {
    dim3 grid((unsigned)((L.n + kBlock - 1) / kBlock), (unsigned)count);
    k_packed_rows<<<grid, kBlock, 0, s>>>(A, L, row0, out);
}

}  // namespace mqh
