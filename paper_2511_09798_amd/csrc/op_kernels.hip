// op_kernels.hip -- the Kansa operator on gfx950: assembly of the stored
// matrix, stored FP64 products, matrix-free products (FP64 or FP32 entries
// with FP64 accumulation), the deterministic split-K reduction and the
// evaluation of the RBF expansion.
//
// Layout: n nodes as double4/float4 records (centred, scaled by eps; the
// 4th lane is padding).  Vectors have a leading dimension ldn (multiple of
// 64, >= n) and are zero past n.  The stored matrix is row-major with
// lda = ldn and zero columns past n.
#include "kernels.hpp"

namespace mqh {

// ---------------------------------------------------------------------------
// Matrix-free products.  One lane per output element; the loop index is
// wave-uniform, so the loop node's record and weight are scalar loads and
// each entry costs only VALU work (entry + one FP64 FMA).  The loop range is
// cut into S slices (split-K, blockIdx.y) whose partial sums go to
// P[slice * ldp + out]; k_reduce_slices adds them in slice order.
// ---------------------------------------------------------------------------

template <typename R, int KIND>
__device__ __forceinline__ void mf_span(const typename NodeOf<R>::type* __restrict__ X,
                                        const double* __restrict__ w, int64_t j0, int64_t j1, R px, R py,
                                        R pz, const EntryConst& c, double& acc0, double& acc1) {
    int64_t j = j0;
    for (; j + 1 < j1; j += 2) {
        const auto q0 = X[j];
        const auto q1 = X[j + 1];
        const double w0 = w[j], w1 = w[j + 1];
        const R t0 = t_of(px, py, pz, q0.x, q0.y, q0.z);
        const R t1 = t_of(px, py, pz, q1.x, q1.y, q1.z);
        const R e0 = KIND == 0 ? entry_interior(t0, c) : entry_boundary(t0, c);
        const R e1 = KIND == 0 ? entry_interior(t1, c) : entry_boundary(t1, c);
        acc0 = fma((double)e0, w0, acc0);
        acc1 = fma((double)e1, w1, acc1);
    }
    if (j < j1) {
        const auto q0 = X[j];
        const R t0 = t_of(px, py, pz, q0.x, q0.y, q0.z);
        const R e0 = KIND == 0 ? entry_interior(t0, c) : entry_boundary(t0, c);
        acc0 = fma((double)e0, w[j], acc0);
    }
}

// y = A x partials.  Blocks [0, nb_int) cover interior rows, the rest the
// boundary rows, so the row kind is uniform per block.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_mf_rows(const typename NodeOf<R>::type* __restrict__ X,
                                                    const double* __restrict__ x, int64_t n, int64_t n_int,
                                                    int64_t nb_int, int64_t slice_len, EntryConst c,
                                                    double* __restrict__ P, int64_t ldp,
                                                    const GkbState* __restrict__ st) {
    if (st != nullptr && st->stopped) return;
    const int64_t b = blockIdx.x;
    const bool interior = b < nb_int;
    const int64_t row = interior ? b * kBlock + threadIdx.x : n_int + (b - nb_int) * kBlock + threadIdx.x;
    const int64_t row_end = interior ? n_int : n;
    const bool valid = row < row_end;
    const auto p = X[valid ? row : 0];
    const int64_t j0 = (int64_t)blockIdx.y * slice_len;
    const int64_t j1 = j0 + slice_len < n ? j0 + slice_len : n;
    double a0 = 0.0, a1 = 0.0;
    if (interior)
        mf_span<R, 0>(X, x, j0, j1, p.x, p.y, p.z, c, a0, a1);
    else
        mf_span<R, 1>(X, x, j0, j1, p.x, p.y, p.z, c, a0, a1);
    if (valid) P[(int64_t)blockIdx.y * ldp + row] = a0 + a1;
}

// y = A^T x partials: one lane per column; the loop runs over rows, first
// the interior ones (L phi), then the boundary ones (phi).
template <typename R>
__global__ __launch_bounds__(kBlock) void k_mf_cols(const typename NodeOf<R>::type* __restrict__ X,
                                                    const double* __restrict__ x, int64_t n, int64_t n_int,
                                                    int64_t slice_len, EntryConst c, double* __restrict__ P,
                                                    int64_t ldp, const GkbState* __restrict__ st) {
    if (st != nullptr && st->stopped) return;
    const int64_t col = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool valid = col < n;
    const auto p = X[valid ? col : 0];
    const int64_t i0 = (int64_t)blockIdx.y * slice_len;
    const int64_t i1 = i0 + slice_len < n ? i0 + slice_len : n;
    double a0 = 0.0, a1 = 0.0;
    const int64_t m1 = i1 < n_int ? i1 : n_int;
    if (i0 < m1) mf_span<R, 0>(X, x, i0, m1, p.x, p.y, p.z, c, a0, a1);
    const int64_t m0 = i0 > n_int ? i0 : n_int;
    if (m0 < i1) mf_span<R, 1>(X, x, m0, i1, p.x, p.y, p.z, c, a0, a1);
    if (valid) P[(int64_t)blockIdx.y * ldp + col] = a0 + a1;
}

// y_i = sum_s P[s][i] - shift * z_i  (shift from *shift_ptr when given);
// the slices are summed in four interleaved groups combined in a fixed order.
__global__ __launch_bounds__(kBlock) void k_reduce_slices(const double* __restrict__ P, int64_t ldp, int S,
                                                          int64_t n, const double* __restrict__ shift_ptr,
                                                          double shift_val, const double* __restrict__ z,
                                                          double* __restrict__ y,
                                                          const GkbState* __restrict__ st) {
    if (st != nullptr && st->stopped) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int k = 0;
    for (; k + 3 < S; k += 4) {
        a0 += P[(int64_t)k * ldp + i];
        a1 += P[(int64_t)(k + 1) * ldp + i];
        a2 += P[(int64_t)(k + 2) * ldp + i];
        a3 += P[(int64_t)(k + 3) * ldp + i];
    }
    for (; k < S; ++k) a0 += P[(int64_t)k * ldp + i];
    double s = (a0 + a1) + (a2 + a3);
    if (z != nullptr) {
        const double sh = shift_ptr != nullptr ? *shift_ptr : shift_val;
        s -= sh * z[i];
    }
    y[i] = s;
}

// ---------------------------------------------------------------------------
// FP32-evaluated matrix-free products.  On gfx950 an FP32 VALU instruction
// can be issued together with another one only when it reads no scalar
// register, so the loop nodes are staged through LDS (broadcast reads into
// vector registers) instead of scalar loads.  Each lane owns R outputs; the
// weight w_j of a loop node is folded into the entry coefficients
// (interior: (w kappa^2 t + 2 w eps^2 + w eps^2 s^2) s, boundary: w sqrt(t)),
// the products are summed in FP32 over blocks of kFlush loop nodes and each
// block sum is added to an FP64 accumulator.
// ---------------------------------------------------------------------------

constexpr int kTile = kBlock;  // loop nodes staged per round (one per thread)
constexpr int kFlush = 16;     // FP32 block length before the FP64 accumulation

// Accumulates, for every output r of this lane, sum over loop nodes j in
// [j0, j1) of w_j * entry(P_r, X_j) with the entry kind INTERIOR.  j0, j1
// are block-uniform (contains barriers).
template <int R, bool INTERIOR>
__device__ __forceinline__ void mf32_span(const float4* __restrict__ X, const double* __restrict__ w, int64_t j0,
                                          int64_t j1, const float (&px)[R], const float (&py)[R],
                                          const float (&pz)[R], const EntryConst& c, double (&acc)[R],
                                          float4* __restrict__ lds0, float2* __restrict__ lds1) {
    for (int64_t t0 = j0; t0 < j1; t0 += kTile) {
        const int64_t j = t0 + threadIdx.x;
        float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
        float2 b = make_float2(0.f, 0.f);
        if (j < j1) {
            const float4 q = X[j];
            const double wj = w[j];
            if (INTERIOR) {
                a = make_float4(q.x, q.y, q.z, (float)(wj * c.k2));
                b = make_float2((float)(wj * c.e2x2), (float)(wj * c.e2));
            } else {
                a = make_float4(q.x, q.y, q.z, (float)wj);
            }
        }
        __syncthreads();  // the previous tile has been consumed
        lds0[threadIdx.x] = a;
        if (INTERIOR) lds1[threadIdx.x] = b;
        __syncthreads();
        const int64_t rem = j1 - t0;
        const int cnt = rem < kTile ? (int)rem : kTile;
        const int cnt_pad = (cnt + kFlush - 1) / kFlush * kFlush;  // padded nodes carry w = 0
        for (int k0 = 0; k0 < cnt_pad; k0 += kFlush) {
            float s32[R];
#pragma unroll
            for (int r = 0; r < R; ++r) s32[r] = 0.f;
#pragma unroll
            for (int k = k0; k < k0 + kFlush; ++k) {
                const float4 q = lds0[k];
                float2 qb = make_float2(0.f, 0.f);
                if (INTERIOR) qb = lds1[k];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const float dx = px[r] - q.x, dy = py[r] - q.y, dz = pz[r] - q.z;
                    const float t = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, 1.0f)));
                    if (INTERIOR) {
                        const float s = __builtin_amdgcn_rsqf(t);
                        const float inner = fmaf(qb.y, s * s, fmaf(q.w, t, qb.x));
                        s32[r] = fmaf(inner, s, s32[r]);
                    } else {
                        s32[r] = fmaf(__builtin_amdgcn_sqrtf(t), q.w, s32[r]);
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] += (double)s32[r];
        }
    }
}

// y = A x partials, FP32 entries: a block owns kBlock * R rows of one kind.
template <int R>
__global__ __launch_bounds__(kBlock) void k_mf32_rows(const float4* __restrict__ X, const double* __restrict__ x,
                                                      int64_t n, int64_t n_int, int64_t nb_int, int64_t slice_len,
                                                      EntryConst c, double* __restrict__ P, int64_t ldp,
                                                      const GkbState* __restrict__ st) {
    __shared__ float4 lds0[kTile];
    __shared__ float2 lds1[kTile];
    if (st != nullptr && st->stopped) return;
    const int64_t b = blockIdx.x;
    const bool interior = b < nb_int;
    const int64_t base = interior ? b * kBlock * R : n_int + (b - nb_int) * kBlock * R;
    const int64_t row_end = interior ? n_int : n;
    float px[R], py[R], pz[R];
    double acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t row = base + r * kBlock + threadIdx.x;
        const float4 q = X[row < row_end ? row : 0];
        px[r] = q.x;
        py[r] = q.y;
        pz[r] = q.z;
        acc[r] = 0.0;
    }
    const int64_t j0 = (int64_t)blockIdx.y * slice_len;
    const int64_t j1 = j0 + slice_len < n ? j0 + slice_len : n;
    if (interior)
        mf32_span<R, true>(X, x, j0, j1, px, py, pz, c, acc, lds0, lds1);
    else
        mf32_span<R, false>(X, x, j0, j1, px, py, pz, c, acc, lds0, lds1);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t row = base + r * kBlock + threadIdx.x;
        if (row < row_end) P[(int64_t)blockIdx.y * ldp + row] = acc[r];
    }
}

// y = A^T x partials, FP32 entries: a block owns kBlock * R columns; the loop
// runs over the slice's interior rows, then its boundary rows.
template <int R>
__global__ __launch_bounds__(kBlock) void k_mf32_cols(const float4* __restrict__ X, const double* __restrict__ x,
                                                      int64_t n, int64_t n_int, int64_t slice_len, EntryConst c,
                                                      double* __restrict__ P, int64_t ldp,
                                                      const GkbState* __restrict__ st) {
    __shared__ float4 lds0[kTile];
    __shared__ float2 lds1[kTile];
    if (st != nullptr && st->stopped) return;
    const int64_t base = (int64_t)blockIdx.x * kBlock * R;
    float px[R], py[R], pz[R];
    double acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t col = base + r * kBlock + threadIdx.x;
        const float4 q = X[col < n ? col : 0];
        px[r] = q.x;
        py[r] = q.y;
        pz[r] = q.z;
        acc[r] = 0.0;
    }
    const int64_t i0 = (int64_t)blockIdx.y * slice_len;
    const int64_t i1 = i0 + slice_len < n ? i0 + slice_len : n;
    const int64_t m1 = i1 < n_int ? i1 : n_int;
    if (i0 < m1) mf32_span<R, true>(X, x, i0, m1, px, py, pz, c, acc, lds0, lds1);
    const int64_t m0 = i0 > n_int ? i0 : n_int;
    if (m0 < i1) mf32_span<R, false>(X, x, m0, i1, px, py, pz, c, acc, lds0, lds1);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t col = base + r * kBlock + threadIdx.x;
        if (col < n) P[(int64_t)blockIdx.y * ldp + col] = acc[r];
    }
}

// ---------------------------------------------------------------------------
// Stored FP64 operator
// ---------------------------------------------------------------------------

// A[i][j], one block = RB rows x 512 columns (two columns per lane, 16-byte
// non-temporal stores); the column records stay in registers across rows.
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

// y = A x - shift z on the stored matrix: each wave streams RW rows with
// 16-byte loads, x comes from cache; one wave reduction per row.
template <int RW>
__global__ __launch_bounds__(kBlock) void k_stored_rows(const double* __restrict__ A, int64_t lda, int64_t n,
                                                        const double* __restrict__ x,
                                                        const double* __restrict__ shift_ptr, double shift_val,
                                                        const double* __restrict__ z, double* __restrict__ y,
                                                        const GkbState* __restrict__ st) {
    if (st != nullptr && st->stopped) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t row0 = ((int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave) * RW;
    if (row0 >= n) return;  // wave-uniform; no barriers in this kernel
    const double* rows[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) rows[r] = A + (row0 + r < n ? row0 + r : n - 1) * lda;
    double acc[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) acc[r] = 0.0;
    const int64_t ne = (n + 1) & ~(int64_t)1;  // x and A are zero-padded to an even length
#pragma unroll 2
    for (int64_t c = 2 * lane; c < ne; c += 2 * kWave) {
        const v2d xv = load2(x + c);
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const v2d a = load_nt(rows[r] + c);
            acc[r] = fma(a.y, xv.y, fma(a.x, xv.x, acc[r]));
        }
    }
#pragma unroll
    for (int r = 0; r < RW; ++r) acc[r] = wave_sum(acc[r]);
    if (lane == 0) {
        const double sh = (z != nullptr) ? (shift_ptr != nullptr ? *shift_ptr : shift_val) : 0.0;
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const int64_t row = row0 + r;
            if (row < n) y[row] = (z != nullptr) ? acc[r] - sh * z[row] : acc[r];
        }
    }
}

// A^T x partials on the stored matrix: a block owns 512 columns (two per
// lane) of a tile of rows_per_tile rows; x_i is wave-uniform.
__global__ __launch_bounds__(kBlock) void k_stored_cols(const double* __restrict__ A, int64_t lda, int64_t n,
                                                        const double* __restrict__ x, int64_t rows_per_tile,
                                                        double* __restrict__ P, int64_t ldp,
                                                        const GkbState* __restrict__ st) {
    if (st != nullptr && st->stopped) return;
    const int64_t c = (int64_t)blockIdx.x * (2 * kBlock) + 2 * threadIdx.x;
    if (c >= lda) return;
    const int64_t i0 = (int64_t)blockIdx.y * rows_per_tile;
    const int64_t i1 = i0 + rows_per_tile < n ? i0 + rows_per_tile : n;
    double a0 = 0.0, a1 = 0.0;
    const double* p = A + c;
#pragma unroll 8
    for (int64_t i = i0; i < i1; ++i) {
        const double xi = x[i];
        const v2d a = load_nt(p + i * lda);
        a0 = fma(a.x, xi, a0);
        a1 = fma(a.y, xi, a1);
    }
    v2d out;
    out.x = a0;
    out.y = a1;
    *reinterpret_cast<v2d*>(P + (int64_t)blockIdx.y * ldp + c) = out;
}

// ---------------------------------------------------------------------------
// Rows of A as a product sees them (entry checks).
// ---------------------------------------------------------------------------

template <typename R>
__global__ __launch_bounds__(kBlock) void k_gen_rows(const typename NodeOf<R>::type* __restrict__ X, int64_t n,
                                                     int64_t n_int, int64_t row0, EntryConst c,
                                                     double* __restrict__ out) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t i = row0 + blockIdx.y;
    if (j >= n) return;
    const auto p = X[i];
    const auto q = X[j];
    const R t = t_of(p.x, p.y, p.z, q.x, q.y, q.z);
    const R e = i < n_int ? entry_interior(t, c) : entry_boundary(t, c);
    out[(int64_t)blockIdx.y * n + j] = (double)e;
}

// ---------------------------------------------------------------------------
// Evaluation u(P_e) = sum_j coef_j phi(|P_e - X_j|), FP64, split over centres.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_eval_partial(const double4* __restrict__ X,
                                                         const double* __restrict__ coef, int64_t n,
                                                         const double4* __restrict__ E, int64_t m,
                                                         int64_t slice_len, EntryConst c,
                                                         double* __restrict__ P, int64_t ldp) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool valid = e < m;
    const double4 p = E[valid ? e : 0];
    const int64_t j0 = (int64_t)blockIdx.y * slice_len;
    const int64_t j1 = j0 + slice_len < n ? j0 + slice_len : n;
    double a0 = 0.0, a1 = 0.0;
    mf_span<double, 1>(X, coef, j0, j1, p.x, p.y, p.z, c, a0, a1);
    if (valid) P[(int64_t)blockIdx.y * ldp + e] = a0 + a1;
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------

void launch_mf_rows(int prec, const void* X, const double* x, int64_t n, int64_t n_int, int S, int64_t slice_len,
                    const EntryConst& c, double* P, int64_t ldp, const GkbState* st, hipStream_t s) {
    const int64_t rows_per_block = prec == 64 ? kBlock : (int64_t)kBlock * kMf32Rows;
    const int64_t nb_int = (n_int + rows_per_block - 1) / rows_per_block;
    const int64_t nb_bnd = (n - n_int + rows_per_block - 1) / rows_per_block;
    dim3 grid((unsigned)(nb_int + nb_bnd), (unsigned)S);
    if (prec == 64)
        k_mf_rows<double><<<grid, kBlock, 0, s>>>((const double4*)X, x, n, n_int, nb_int, slice_len, c, P, ldp, st);
    else
        k_mf32_rows<kMf32Rows><<<grid, kBlock, 0, s>>>((const float4*)X, x, n, n_int, nb_int, slice_len, c, P, ldp,
                                                       st);
}

void launch_mf_cols(int prec, const void* X, const double* x, int64_t n, int64_t n_int, int S, int64_t slice_len,
                    const EntryConst& c, double* P, int64_t ldp, const GkbState* st, hipStream_t s) {
    const int64_t cols_per_block = prec == 64 ? kBlock : (int64_t)kBlock * kMf32Rows;
    dim3 grid((unsigned)((n + cols_per_block - 1) / cols_per_block), (unsigned)S);
    if (prec == 64)
        k_mf_cols<double><<<grid, kBlock, 0, s>>>((const double4*)X, x, n, n_int, slice_len, c, P, ldp, st);
    else
        k_mf32_cols<kMf32Rows><<<grid, kBlock, 0, s>>>((const float4*)X, x, n, n_int, slice_len, c, P, ldp, st);
}

void launch_reduce_slices(const double* P, int64_t ldp, int S, int64_t n, const double* shift_ptr,
                          double shift_val, const double* z, double* y, const GkbState* st, hipStream_t s) {
    k_reduce_slices<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(P, ldp, S, n, shift_ptr, shift_val, z,
                                                                            y, st);
}

void launch_assemble(const double4* X, int64_t n, int64_t n_int, int64_t lda, const EntryConst& c, double* A,
                     hipStream_t s) {
    constexpr int RB = 64;
    dim3 grid((unsigned)((lda + 2 * kBlock - 1) / (2 * kBlock)), (unsigned)((n + RB - 1) / RB));
    k_assemble<RB><<<grid, kBlock, 0, s>>>(X, n, n_int, lda, c, A);
}

void launch_stored_rows(int rw, const double* A, int64_t lda, int64_t n, const double* x, const double* shift_ptr,
                        double shift_val, const double* z, double* y, const GkbState* st, hipStream_t s) {
    const int waves_per_block = kBlock / kWave;
    if (rw == 8) {
        const int64_t nb = (n + 8 * waves_per_block - 1) / (8 * waves_per_block);
        k_stored_rows<8><<<(unsigned)nb, kBlock, 0, s>>>(A, lda, n, x, shift_ptr, shift_val, z, y, st);
    } else if (rw == 4) {
        const int64_t nb = (n + 4 * waves_per_block - 1) / (4 * waves_per_block);
        k_stored_rows<4><<<(unsigned)nb, kBlock, 0, s>>>(A, lda, n, x, shift_ptr, shift_val, z, y, st);
    } else {
        const int64_t nb = (n + 2 * waves_per_block - 1) / (2 * waves_per_block);
        k_stored_rows<2><<<(unsigned)nb, kBlock, 0, s>>>(A, lda, n, x, shift_ptr, shift_val, z, y, st);
    }
}

void launch_stored_cols(const double* A, int64_t lda, int64_t n, const double* x, int64_t rows_per_tile, int tiles,
                        double* P, int64_t ldp, const GkbState* st, hipStream_t s) {
    dim3 grid((unsigned)((lda + 2 * kBlock - 1) / (2 * kBlock)), (unsigned)tiles);
    k_stored_cols<<<grid, kBlock, 0, s>>>(A, lda, n, x, rows_per_tile, P, ldp, st);
}

void launch_gen_rows(int prec, const void* X, int64_t n, int64_t n_int, int64_t row0, int64_t count,
                     const EntryConst& c, double* out, hipStream_t s) {
    dim3 grid((unsigned)((n + kBlock - 1) / kBlock), (unsigned)count);
    if (prec == 64)
        k_gen_rows<double><<<grid, kBlock, 0, s>>>((const double4*)X, n, n_int, row0, c, out);
    else
        k_gen_rows<float><<<grid, kBlock, 0, s>>>((const float4*)X, n, n_int, row0, c, out);
}

void launch_eval_partial(const double4* X, const double* coef, int64_t n, const double4* E, int64_t m, int S,
                         int64_t slice_len, const EntryConst& c, double* P, int64_t ldp, hipStream_t s) {
    dim3 grid((unsigned)((m + kBlock - 1) / kBlock), (unsigned)S);
    k_eval_partial<<<grid, kBlock, 0, s>>>(X, coef, n, E, m, slice_len, c, P, ldp);
}

}  // namespace mqh
