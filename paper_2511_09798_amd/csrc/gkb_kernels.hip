// gkb_kernels.hip -- vector kernels of the Golub-Kahan bidiagonalisation
// (Algorithm 1) on gfx950: norms with the breakdown test, scaling, full
// reorthogonalisation by classical Gram-Schmidt applied twice, and the lift
// coef = Z y.  All reductions are deterministic (fixed trees, fixed orders).
//
// Bases W (n x (ell+1)) and Z (n x ell) are column-major with leading
// dimension ldn, so every basis vector is contiguous and zero past n.
#include <float.h>

#include "kernels.hpp"

namespace mqh {

// ---------------------------------------------------------------------------
// State and small fills
// ---------------------------------------------------------------------------

__global__ void k_init_state(GkbState* st, int32_t ell, double* alpha, double* beta, Bz bz) {
    const int64_t z = blockIdx.y;  // batch: state z, alpha + z bz.a, beta + z bz.b
    st += z;
    if (alpha != nullptr) alpha += z * bz.a;
    if (beta != nullptr) beta += z * bz.b;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        st->stopped = 0;
        st->ell_done = ell;
        st->flag = 0;
        st->pad = 0;
        st->scale = 0.0;
        st->snap_stopped = 0;
        st->pad2 = 0;
        st->snap_scale = 0.0;
    }
    if (alpha != nullptr && i < ell) alpha[i] = 0.0;
    if (beta != nullptr && i <= ell) beta[i] = 0.0;
}

// Keep at most ell steps (a run stopped early by a breakdown keeps fewer).
__global__ void k_cap_ell(GkbState* st, int32_t ell) {
    if (threadIdx.x == 0 && st->ell_done > ell) st->ell_done = ell;
}

__global__ void k_fill(double* __restrict__ x, int64_t n, double v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

// x[z stride + i] *= a for i < n, z < gridDim.y (the interior entries of
// right-hand sides under the row scaling D = diag(A)^-1).
__global__ void k_scale(double* __restrict__ x, int64_t n, double a, int64_t stride) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[(int64_t)blockIdx.y * stride + i] *= a;
}

// ---------------------------------------------------------------------------
// Norms
// ---------------------------------------------------------------------------

// partial[b] = sum of x_i^2 over the grid-stride share of block b.
__global__ __launch_bounds__(kBlock) void k_sumsq_partial(const double* __restrict__ x, int64_t n,
                                                          double* __restrict__ partial, GkbState* __restrict__ st,
                                                          Bz bz) {
    __shared__ double lds[kBlock / kWave];
    const int64_t z = blockIdx.z;  // batch: x + z bz.a, partial + z bz.b, state z
    x += z * bz.a;
    partial += z * bz.b;
    if (st != nullptr) st += z;
    if (st != nullptr && blockIdx.x == 0 && threadIdx.x == 0) {
        // the state the normalisation that consumes these partials decides from
        st->snap_stopped = st->stopped;
        st->snap_scale = st->scale;
    }
    if (st != nullptr && st->stopped) return;  // uniform over the grid
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        s = fma(x[i], x[i], s);
    s = block_sum<kBlock>(s, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Norm of a Krylov vector from its partial sums of squares, breakdown test
// and normalisation dst = x / norm (kind 0: beta_1 = ||f||; kind 1:
// alpha_{j+1}; kind 2: beta_{j+2}, 0-based j).  The threshold is
// n * DBL_EPSILON * (running max of alpha, beta_{>=2}).  Every block sums the
// partials in the same order (thread t takes t, t + 256, ..., then the block
// reduction), so all blocks hold the same norm and take the same decision
// from the same state: the snapshot (snap_stopped, snap_scale) that the
// kernel producing the partials wrote, which no block of this launch writes;
// block 0 records the decision in stopped, scale and the scalars.  With Vg, the
// normalised vector also goes, in FP32, to column z of the sorted
// block-product operand, Vg[iperm[i]][z] (zeros for a stopped run).
__global__ __launch_bounds__(kBlock) void k_finalize_scale(const double* __restrict__ partial, int nparts, int kind,
                                                           int32_t j, int64_t n, double* __restrict__ alpha,
                                                           double* __restrict__ beta, GkbState* __restrict__ st,
                                                           const double* __restrict__ x, double* __restrict__ dst,
                                                           const int32_t* __restrict__ iperm, float* __restrict__ Vg,
                                                           Bz bz) {
    __shared__ double lds[kBlock / kWave];
    __shared__ int s_stopped;
    const int64_t z = blockIdx.y;  // batch: partial + z bz.a, alpha, beta + z bz.b, x + z bz.c, dst + z bz.d, state z
    partial += z * bz.a;
    alpha += z * bz.b;
    beta += z * bz.b;
    x += z * bz.c;
    dst += z * bz.d;
    st += z;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (threadIdx.x == 0) s_stopped = st->snap_stopped;
    __syncthreads();
    if (s_stopped) {  // block-uniform
        if (Vg != nullptr && i < n) Vg[(int64_t)iperm[i] * kBlkRhs + z] = 0.f;
        return;
    }
    double s = 0.0;
    for (int q = threadIdx.x; q < nparts; q += kBlock) s += partial[q];
    s = block_sum<kBlock>(s, lds);
    const double nrm = sqrt(s);
    bool ok;
    if (kind == 0) {
        ok = nrm > 0.0;
    } else {
        const double tau = (double)n * DBL_EPSILON * st->snap_scale;
        ok = nrm > tau;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (kind == 0) {
            beta[0] = nrm;
            if (!ok) {
                st->stopped = 1;
                st->ell_done = 0;
                st->flag = 2;
            }
        } else if (kind == 1) {
            if (!ok) {
                st->stopped = 1;
                st->ell_done = j;
                st->flag = 1;
            } else {
                alpha[j] = nrm;
            }
        } else {
            if (!ok) {
                st->stopped = 1;
                st->ell_done = j + 1;
                st->flag = 2;
                beta[j + 1] = 0.0;
            } else {
                beta[j + 1] = nrm;
            }
        }
        if (ok && kind != 0 && nrm > st->snap_scale) st->scale = nrm;
    }
    if (i >= n) return;
    if (!ok) {
        if (Vg != nullptr) Vg[(int64_t)iperm[i] * kBlkRhs + z] = 0.f;
        return;
    }
    const double d = x[i] / nrm;
    dst[i] = d;
    if (Vg != nullptr) Vg[(int64_t)iperm[i] * kBlkRhs + z] = (float)d;
}

// ---------------------------------------------------------------------------
// Classical Gram-Schmidt against m orthonormal columns V[:, 0:m]
// ---------------------------------------------------------------------------

// partial[b * m + k] = sum over the kGtRows rows of block row b of V[k][i] x_i.
// A block owns kGtRows rows and kGtCols consecutive columns (blockIdx.y).
// Rows in kGtQ passes of 512: in pass q wave w takes rows 512 q + 128 w ..
// + 127 of the block, lane l the pair 2l, 2l + 1 (one 16-byte load per
// column, 1 KB per wave load); then each column is reduced over the block in
// a fixed order.  V is zero past n up to ldn (a multiple of 64), so the pair
// i, i + 1 with i < n even stays inside the padded column.  Two columns per
// block: consecutive blocks then stream consecutive 8 KB pieces of the same
// two columns, which the HBM serves faster than eight columns' pieces at
// once (measured at n = 100000: 7.0 against 6.0 TB/s for 300 columns, 6.4
// against 4.6 for 150).
constexpr int kGtQ = 2;
constexpr int kGtRows = kGtQ * 4 * 2 * 64;  // 1024
constexpr int kGtCols = 2;

// (The reduction is a second launch: handing the partials to the last block
// of the same launch needs a device-scope release in every block, which on
// this GPU writes back the L2 of the block's XCD; measured 1.25 ms per call
// against 30 us for the two launches.)
__global__ __launch_bounds__(kBlock) void k_gemvt_partial(const double* __restrict__ V, int64_t ldn, int64_t n,
                                                          int32_t m, const double* __restrict__ x,
                                                          double* __restrict__ partial,
                                                          const GkbState* __restrict__ st, Bz bz) {
    __shared__ double lds[kBlock / kWave][kGtCols];
    const int64_t z = blockIdx.z;  // batch: V + z bz.a, x + z bz.b, partial + z bz.c, state z
    V += z * bz.a;
    x += z * bz.b;
    partial += z * bz.c;
    if (st != nullptr) st += z;
    if (st != nullptr && st->stopped) return;  // uniform over the grid
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int64_t ib = (int64_t)blockIdx.x * kGtRows + w * (2 * kWave) + 2 * lane;
    const int k0 = blockIdx.y * kGtCols;
    double x0[kGtQ], x1[kGtQ];
    bool in[kGtQ];
#pragma unroll
    for (int q = 0; q < kGtQ; ++q) {
        const int64_t i = ib + q * (kBlock * 2);
        in[q] = i < n;
        x0[q] = in[q] ? x[i] : 0.0;
        x1[q] = in[q] && i + 1 < n ? x[i + 1] : 0.0;
    }
    // rows past n read row 0 (their x is zero): no branch around the loads,
    // so all of a lane's loads are in flight together
    int64_t off[kGtQ];
#pragma unroll
    for (int q = 0; q < kGtQ; ++q) off[q] = in[q] ? ib + q * (kBlock * 2) : 0;
    // a column past m (the last group of an odd m) reads column m - 1; its
    // sum is not stored
    double acc[kGtCols];
#pragma unroll
    for (int cc = 0; cc < kGtCols; ++cc) {
        acc[cc] = 0.0;
        const double* v = V + (int64_t)(k0 + cc < m ? k0 + cc : m - 1) * ldn;
#pragma unroll
        for (int q = 0; q < kGtQ; ++q) {
            const v2d a = load2(v + off[q]);
            acc[cc] = fma(a.y, x1[q], fma(a.x, x0[q], acc[cc]));
        }
    }
#pragma unroll
    for (int cc = 0; cc < kGtCols; ++cc) {
        const double sc = wave_sum(acc[cc]);
        if (lane == 0) lds[w][cc] = sc;
    }
    __syncthreads();
    if (threadIdx.x < kGtCols && k0 + (int)threadIdx.x < m) {
        const int cc = threadIdx.x;
        partial[(int64_t)blockIdx.x * m + k0 + cc] = ((lds[0][cc] + lds[1][cc]) + lds[2][cc]) + lds[3][cc];
    }
}

// c[k] = sum_b partial[b * sb + k * sk] (k_gemvt_partial: sb = m, sk = 1;
// k_update_gemvt: sb = 1, sk = nb): one wave per column, lanes take b = lane,
// lane + 64, ... and the wave reduction combines them in a fixed order.
__global__ __launch_bounds__(kBlock) void k_gemvt_reduce(const double* __restrict__ partial, int nb, int32_t m,
                                                         int64_t sb, int64_t sk, double* __restrict__ c,
                                                         const GkbState* __restrict__ st, Bz bz) {
    const int64_t z = blockIdx.y;  // batch: partial + z bz.a, c + z bz.b, state z
    partial += z * bz.a;
    c += z * bz.b;
    if (st != nullptr) st += z;
    if (st != nullptr && st->stopped) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int k = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (k >= m) return;  // wave-uniform; no barriers
    double s = 0.0;
    for (int b = lane; b < nb; b += kWave) s += partial[(int64_t)b * sb + (int64_t)k * sk];
    s = wave_sum(s);
    if (lane == 0) c[k] = s;
}

// x_i -= sum_k V[k][i] c_k for the kUpdRows rows of block b; optionally
// partial[b] = sum over the block of the updated x_i^2.  Lane l of every wave
// owns the block's rows 2l, 2l + 1 (16-byte loads, 1 KB per wave load); wave
// w sums the columns k = w, w + 4, ... with eight loads in flight, and the
// four waves' sums are added in wave order through LDS.
constexpr int kUpdRows = 2 * kWave;

__global__ __launch_bounds__(kBlock) void k_update(const double* __restrict__ V, int64_t ldn, int64_t n, int32_t m,
                                                   const double* __restrict__ c, double* __restrict__ x,
                                                   double* __restrict__ sumsq_partial, GkbState* __restrict__ st,
                                                   Bz bz) {
    constexpr int kW = kBlock / kWave;
    __shared__ double part[kW][kUpdRows];
    __shared__ double lds[kW];
    const int64_t z = blockIdx.z;  // batch: V + z bz.a, c + z bz.b, x + z bz.c, sumsq + z bz.d, state z
    V += z * bz.a;
    c += z * bz.b;
    x += z * bz.c;
    if (sumsq_partial != nullptr) sumsq_partial += z * bz.d;
    if (st != nullptr) st += z;
    if (st != nullptr && sumsq_partial != nullptr && blockIdx.x == 0 && threadIdx.x == 0) {
        // the state the normalisation that consumes these partials decides from
        st->snap_stopped = st->stopped;
        st->snap_scale = st->scale;
    }
    if (st != nullptr && st->stopped) return;  // uniform over the grid
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int64_t i0 = (int64_t)blockIdx.x * kUpdRows + 2 * lane;  // i0 even, so i0 + 1 < ldn when i0 < n
    double s0 = 0.0, s1 = 0.0, t0 = 0.0, t1 = 0.0;
    if (i0 < n) {
        const double* v = V + i0;
        int k = w;
#pragma unroll 4
        for (; k + kW < m; k += 2 * kW) {
            const v2d a = load2(v + (int64_t)k * ldn);
            const v2d b = load2(v + (int64_t)(k + kW) * ldn);
            const double ca = c[k], cb = c[k + kW];
            s0 = fma(a.x, ca, s0);
            s1 = fma(a.y, ca, s1);
            t0 = fma(b.x, cb, t0);
            t1 = fma(b.y, cb, t1);
        }
        if (k < m) {
            const v2d a = load2(v + (int64_t)k * ldn);
            s0 = fma(a.x, c[k], s0);
            s1 = fma(a.y, c[k], s1);
        }
    }
    part[w][2 * lane] = s0 + t0;
    part[w][2 * lane + 1] = s1 + t1;
    __syncthreads();
    double xi = 0.0;
    const int64_t i = (int64_t)blockIdx.x * kUpdRows + threadIdx.x;
    if (threadIdx.x < kUpdRows && i < n) {
        const int t = threadIdx.x;
        xi = x[i] - (((part[0][t] + part[1][t]) + part[2][t]) + part[3][t]);
        x[i] = xi;
    }
    if (sumsq_partial != nullptr) {
        const double s = block_sum<kBlock>(xi * xi, lds);
        if (threadIdx.x == 0) sumsq_partial[blockIdx.x] = s;
    }
}

// The middle of classical Gram-Schmidt applied twice in one pass over V:
// x -= V c (the first pass's update), then partial[k * nb + b] = sum over the
// kFuRows rows of block b of V[k][i] x_i for the updated x (the second
// pass's projection coefficients, reduced by k_gemvt_reduce).  The block's
// rows of V[:, 0:m] come from HBM once and stay in LDS (m x kFuLd doubles of
// dynamic shared memory) between the two, so CGS2 reads the basis three
// times instead of four.  Thread t takes the row pair 2 (t % 16), + 1 and
// the columns k = t / 16, t / 16 + 16, ...; the 16 column groups' sums are
// added in group order through LDS.  A pair past n reads rows 0, 1 of the
// column, a pair that straddles n the zero padding below ldn (finite values
// either way; their x is zero), and rows past n are not written.  The grid
// has 8 ceil(nb / 8) workgroups, and workgroup w takes row block
// (w % 8) ceil(nb / 8) + w / 8: workgroups are handed to the 8 XCDs in turn,
// so each XCD takes a contiguous range of row blocks and its L2 holds whole
// lines of the column-major partial sums.
constexpr int kFuRows = 32;
constexpr int kFuLd = kFuRows + 1;             // padded LDS row of the tile
constexpr int kFuPairs = kFuRows / 2;
constexpr int kFuGroups = kBlock / kFuPairs;   // 16
static_assert(kFuGroups * kFuPairs == kBlock, "fused CGS2 tile layout");
static_assert(kFusedCgsMaxCols * kFuLd * 8 + (kFuGroups + 1) * kFuRows * 8 <= 65536, "fused CGS2 LDS within 64 KB");

__global__ __launch_bounds__(kBlock) void k_update_gemvt(const double* __restrict__ V, int64_t ldn, int64_t n,
                                                         int32_t m, const double* __restrict__ c,
                                                         double* __restrict__ x, double* __restrict__ partial,
                                                         int nb, const GkbState* __restrict__ st, Bz bz) {
    extern __shared__ double tile[];  // [m][kFuLd]
    __shared__ double part[kFuGroups][kFuRows];
    __shared__ double xs[kFuRows];
    const int64_t z = blockIdx.z;  // batch: V + z bz.a, c + z bz.b, x + z bz.c, partial + z bz.d, state z
    V += z * bz.a;
    c += z * bz.b;
    x += z * bz.c;
    partial += z * bz.d;
    if (st != nullptr) st += z;
    if (st != nullptr && st->stopped) return;  // uniform over the grid
    const int per = (nb + 7) / 8;
    const int b = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (b >= nb) return;  // uniform over the workgroup
    const int t = threadIdx.x, rp = t % kFuPairs, cg = t / kFuPairs;
    const int64_t i0 = (int64_t)b * kFuRows + 2 * rp;
    const double* v = V + (i0 < n ? i0 : 0);
    double* tr = tile + 2 * rp;
    double s0 = 0.0, s1 = 0.0;
    int k = cg;
#pragma unroll 2
    for (; k + 3 * kFuGroups < m; k += 4 * kFuGroups) {
        v2d a[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) a[u] = load2(v + (int64_t)(k + u * kFuGroups) * ldn);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int kk = k + u * kFuGroups;
            tr[kk * kFuLd] = a[u].x;
            tr[kk * kFuLd + 1] = a[u].y;
            const double ck = c[kk];
            s0 = fma(a[u].x, ck, s0);
            s1 = fma(a[u].y, ck, s1);
        }
    }
    for (; k < m; k += kFuGroups) {
        const v2d a = load2(v + (int64_t)k * ldn);
        tr[k * kFuLd] = a.x;
        tr[k * kFuLd + 1] = a.y;
        const double ck = c[k];
        s0 = fma(a.x, ck, s0);
        s1 = fma(a.y, ck, s1);
    }
    part[cg][2 * rp] = s0;
    part[cg][2 * rp + 1] = s1;
    __syncthreads();
    if (t < kFuRows) {
        double sum = 0.0;
#pragma unroll
        for (int g = 0; g < kFuGroups; ++g) sum += part[g][t];
        const int64_t i = (int64_t)b * kFuRows + t;
        double xi = 0.0;
        if (i < n) {
            xi = x[i] - sum;
            x[i] = xi;
        }
        xs[t] = xi;
    }
    __syncthreads();
    for (int kk = t; kk < m; kk += kBlock) {
        const double* r = tile + kk * kFuLd;
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < kFuRows; ++i) acc = fma(r[i], xs[i], acc);
        partial[(int64_t)kk * nb + b] = acc;
    }
}

// ---------------------------------------------------------------------------
// Lift coef = Z y (Algorithm 2 step 5 / Algorithm 4 last step)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_lift(const double* __restrict__ Z, int64_t ldz, int64_t n,
                                                 int32_t ell, const int32_t* __restrict__ ell_ptr,
                                                 const double* __restrict__ y, double* __restrict__ coef, Bz bz) {
    {
        const int64_t z = blockIdx.y;  // batch: Z + z bz.a, y + z bz.b, coef + z bz.c, ell_ptr + z bz.d
        Z += z * bz.a;
        y += z * bz.b;
        coef += z * bz.c;
        if (ell_ptr != nullptr) ell_ptr += z * bz.d;
    }
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int32_t m = ell_ptr != nullptr ? *ell_ptr : ell;
    double s0 = 0.0, s1 = 0.0;
    int k = 0;
    for (; k + 1 < m; k += 2) {
        s0 = fma(Z[(int64_t)k * ldz + i], y[k], s0);
        s1 = fma(Z[(int64_t)(k + 1) * ldz + i], y[k + 1], s1);
    }
    if (k < m) s0 = fma(Z[(int64_t)k * ldz + i], y[k], s0);
    coef[i] = s0 + s1;
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------

void launch_init_state(GkbState* st, int32_t ell, double* alpha, double* beta, hipStream_t s) {
    launch_init_state_b(st, ell, alpha, beta, 1, Bz{}, s);
}

void launch_init_state_b(GkbState* st, int32_t ell, double* alpha, double* beta, int nz, Bz bz, hipStream_t s) {
    const int nt = 256;
    k_init_state<<<dim3((ell + 1 + nt) / nt, nz), nt, 0, s>>>(st, ell, alpha, beta, bz);
}

void launch_cap_ell(GkbState* st, int32_t ell, hipStream_t s) { k_cap_ell<<<1, 64, 0, s>>>(st, ell); }

__global__ void k_fill_f32(float* __restrict__ x, int64_t n, float v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

void launch_fill_f32(float* x, int64_t n, float v, hipStream_t s) {
    if (n <= 0) return;
    k_fill_f32<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(x, n, v);
}

void launch_scale(double* x, int64_t n, double a, int nz, int64_t stride, hipStream_t s) {
    if (n <= 0 || nz <= 0) return;
    k_scale<<<dim3((unsigned)((n + kBlock - 1) / kBlock), (unsigned)nz), kBlock, 0, s>>>(x, n, a, stride);
}

void launch_fill(double* x, int64_t n, double v, hipStream_t s) {
    if (n <= 0) return;
    k_fill<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(x, n, v);
}

int sumsq_blocks(int64_t n) {
    int64_t nb = (n + kBlock - 1) / kBlock;
    return (int)(nb < 1024 ? nb : 1024);
}

void launch_sumsq_partial(const double* x, int64_t n, double* partial, int nb, GkbState* st, hipStream_t s) {
    launch_sumsq_partial_b(x, n, partial, nb, st, 1, Bz{}, s);
}

void launch_sumsq_partial_b(const double* x, int64_t n, double* partial, int nb, GkbState* st, int nz, Bz bz,
                            hipStream_t s) {
    k_sumsq_partial<<<dim3(nb, 1, nz), kBlock, 0, s>>>(x, n, partial, st, bz);
}

void launch_finalize_scale(const double* partial, int nparts, int kind, int32_t j, int64_t n, double* alpha,
                           double* beta, GkbState* st, const double* x, double* dst, hipStream_t s) {
    launch_finalize_scale_b(partial, nparts, kind, j, n, alpha, beta, st, x, dst, nullptr, nullptr, 1, Bz{}, s);
}

void launch_finalize_scale_b(const double* partial, int nparts, int kind, int32_t j, int64_t n, double* alpha,
                             double* beta, GkbState* st, const double* x, double* dst, const int32_t* iperm,
                             float* Vg, int nz, Bz bz, hipStream_t s) {
    k_finalize_scale<<<dim3((unsigned)((n + kBlock - 1) / kBlock), nz), kBlock, 0, s>>>(
        partial, nparts, kind, j, n, alpha, beta, st, x, dst, iperm, Vg, bz);
}

int gemvt_blocks(int64_t n) { return (int)((n + kGtRows - 1) / kGtRows); }

void launch_gemvt(const double* V, int64_t ldn, int64_t n, int32_t m, const double* x, double* partial, double* c,
                  const GkbState* st, hipStream_t s) {
    launch_gemvt_b(V, ldn, n, m, x, partial, c, st, 1, 0, 0, 0, 0, s);
}

void launch_gemvt_b(const double* V, int64_t ldn, int64_t n, int32_t m, const double* x, double* partial, double* c,
                    const GkbState* st, int nz, int64_t sV, int64_t sx, int64_t sp, int64_t sc, hipStream_t s) {
    const int nb = gemvt_blocks(n);
    k_gemvt_partial<<<dim3(nb, (m + kGtCols - 1) / kGtCols, nz), kBlock, 0, s>>>(V, ldn, n, m, x, partial, st,
                                                                                 Bz{sV, sx, sp, 0});
    k_gemvt_reduce<<<dim3((m + kBlock / kWave - 1) / (kBlock / kWave), nz), kBlock, 0, s>>>(
        partial, nb, m, m, 1, c, st, Bz{sp, sc, 0, 0});
}

int fused_cgs_blocks(int64_t n) { return (int)((n + kFuRows - 1) / kFuRows); }

void launch_update_gemvt_b(const double* V, int64_t ldn, int64_t n, int32_t m, double* c, double* x,
                           double* partial, const GkbState* st, int nz, int64_t sV, int64_t sc, int64_t sx,
                           int64_t sp, hipStream_t s) {
    const int nb = fused_cgs_blocks(n);
    const size_t lds = (size_t)m * kFuLd * sizeof(double);
    k_update_gemvt<<<dim3(8 * ((nb + 7) / 8), 1, nz), kBlock, lds, s>>>(V, ldn, n, m, c, x, partial, nb, st,
                                                                       Bz{sV, sc, sx, sp});
    k_gemvt_reduce<<<dim3((m + kBlock / kWave - 1) / (kBlock / kWave), nz), kBlock, 0, s>>>(
        partial, nb, m, 1, nb, c, st, Bz{sp, sc, 0, 0});
}

void launch_update_gemvt(const double* V, int64_t ldn, int64_t n, int32_t m, double* c, double* x,
                         double* partial, const GkbState* st, hipStream_t s) {
    launch_update_gemvt_b(V, ldn, n, m, c, x, partial, st, 1, 0, 0, 0, 0, s);
}

void launch_update(const double* V, int64_t ldn, int64_t n, int32_t m, const double* c, double* x,
                   double* sumsq_partial, GkbState* st, hipStream_t s) {
    launch_update_b(V, ldn, n, m, c, x, sumsq_partial, st, 1, Bz{}, s);
}

void launch_update_b(const double* V, int64_t ldn, int64_t n, int32_t m, const double* c, double* x,
                     double* sumsq_partial, GkbState* st, int nz, Bz bz, hipStream_t s) {
    k_update<<<dim3((unsigned)update_blocks(n), 1, nz), kBlock, 0, s>>>(V, ldn, n, m, c, x, sumsq_partial, st, bz);
}

int update_blocks(int64_t n) { return (int)((n + kUpdRows - 1) / kUpdRows); }

void launch_lift(const double* Z, int64_t ldz, int64_t n, int32_t ell, const int32_t* ell_ptr, const double* y,
                 double* coef, hipStream_t s, int nz, Bz bz) {
    k_lift<<<dim3((unsigned)((n + kBlock - 1) / kBlock), nz), kBlock, 0, s>>>(Z, ldz, n, ell, ell_ptr, y, coef, bz);
}

}  // namespace mqh
