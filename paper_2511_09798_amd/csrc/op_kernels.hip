// op_kernels.hip -- the matrix-free Kansa operator on gfx950: products with
// FP64 entries or FP32 entries and FP64 accumulation (single vectors and
// blocks of right-hand sides), the deterministic split-K reduction, the rows
// of A as the products generate them and the evaluation of the RBF
// expansion.  (The stored matrix is in stored_kernels.hip.)
//
// Layout: n nodes as double4/float4 records (centred, scaled by eps; the
// 4th lane is padding).  Vectors have a leading dimension ldn (multiple of
// 64, >= n) and are zero past n.
#include "kernels.hpp"

namespace mqh {

// ---------------------------------------------------------------------------
// A span of loop nodes against one output position (the evaluation of the
// RBF expansion): the loop index is wave-uniform, so the loop node's record
// and weight are scalar loads and each term costs only VALU work.  Split
// over the loop range, the partial sums go to P[slice * ldp + out] and
// k_reduce_slices adds them in slice order.
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

// y_o = sum_s P[s][i] - shift * z_o with o = perm[i] (o = i when perm is
// null; shift from *shift_ptr when given); the slices are summed in four
// interleaved groups combined in a fixed order.
__global__ __launch_bounds__(kBlock) void k_reduce_slices(const double* __restrict__ P, int64_t ldp, int S,
                                                          int64_t n, const int32_t* __restrict__ perm,
                                                          const double* __restrict__ shift_ptr, double shift_val,
                                                          const double* __restrict__ z, double* __restrict__ y,
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
    const int64_t o = perm != nullptr ? (int64_t)perm[i] : i;
    if (z != nullptr) {
        const double sh = shift_ptr != nullptr ? *shift_ptr : shift_val;
        s -= sh * z[o];
    }
    y[o] = s;
}

// ---------------------------------------------------------------------------
// FP32-evaluated matrix-free products: the squared distances on the matrix
// cores.
//
// Nodes are visited in a spatially sorted order (Morton order within each
// class, interior first) and cut into blocks of kMfmFixed "fixed" nodes, each
// with a frame centre c among its nodes.  With d = P - c (P the eps-scaled
// node, in FP32),
//     t_ij = 1 + |d_i - d_j|^2 = |d_i|^2 + sum_k a_ik b_kj,
//     a_i = (-2 d_i, 1),  b_j = (d_j, 1 + |d_j|^2),
// a K = 4 contraction per 16 x 16 tile of entries.  Each FP32 factor is split
// exactly into three bf16 parts by truncation (h = top 8 significant bits,
// m = next 8, l = the last 8), and the eight cross products that matter at
// FP32 precision (all but l*l, 2^-32 relative) are laid out along K = 32 of
// one v_mfma_f32_16x16x32_bf16: t comes out with FP32 accuracy at half the
// matrix-core time of the FP32 MFMA.  Close pairs have small |d_i|, |d_j|
// (the frame sits among the fixed nodes), so t keeps its relative accuracy
// where 1 + eps^2 r^2 is near 1.  The entries are evaluated on the VALU from
// t: by the pair products (one vector) and the block products (16 vectors)
// below.
//
// Lane layout of v_mfma_f32_16x16x32_bf16 (wave64): lane l holds A[l%16][k]
// and B[k][l%16] for k = 8(l/16) .. 8(l/16)+7, and D[4(l/16)+r][l%16],
// r = 0..3.  Lane group g = l/16 carries coordinate g (g < 3) or the
// 1 * (1 + |d_j|^2) term (g = 3).
// ---------------------------------------------------------------------------

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));


// Exact split x = h + m + l of a finite FP32 value into three bf16 values,
// returned as FP32 bit patterns with zero low halves: h keeps the top 16 bits
// of x, m those of x - h (exact), l = x - h - m (exact, at most 8 significant
// bits).
__device__ __forceinline__ void split_bf16x3(float x, unsigned& h, unsigned& m, unsigned& l) {
    h = __float_as_uint(x) & 0xFFFF0000u;
    const float r1 = x - __uint_as_float(h);
    m = __float_as_uint(r1) & 0xFFFF0000u;
    l = __float_as_uint(r1 - __uint_as_float(m));
}

// Two bf16 values in one dword: lo's high half in bits 0..15, hi's in 16..31.
__device__ __forceinline__ unsigned pack_bf16(unsigned lo, unsigned hi) {
    return __builtin_amdgcn_perm(hi, lo, 0x07060302u);
}

// Eight K slots of one coordinate: the cross products
// (h,h) (h,m) (m,h) (h,l) (l,h) (m,m) (m,l) (l,m) of a (fixed side) and b.
__device__ __forceinline__ v4u fixed_terms(float a) {
    unsigned h, m, l;
    split_bf16x3(a, h, m, l);
    v4u r;
    r[0] = pack_bf16(h, h);
    r[1] = pack_bf16(m, h);
    r[2] = pack_bf16(l, m);
    r[3] = pack_bf16(m, l);
    return r;
}
__device__ __forceinline__ v4u loop_terms(float b) {
    unsigned h, m, l;
    split_bf16x3(b, h, m, l);
    v4u r;
    r[0] = pack_bf16(h, m);
    r[1] = pack_bf16(h, l);
    r[2] = pack_bf16(h, m);
    r[3] = pack_bf16(l, m);
    return r;
}

// ---------------------------------------------------------------------------
// FP32-evaluated products over unordered pairs of nodes.
//
// The entry of A depends on t_ij = 1 + eps^2 r_ij^2 and on the kind of its
// row only, so A_ij and A_ji share t and s = t^(-1/2): for an interior row
// the entry is (kappa^2 t + 2 eps^2 + eps^2 s^2) s, for a boundary row
// t s = sqrt(t).  A product y = A x (or A^T x) therefore needs each
// unordered pair {i, j} once: y_i += A_ij x_j and y_j += A_ji x_i (A^T: the
// two entries swap).  On this GPU the rsqrt of an entry costs as much as all
// its other VALU work together and overlaps none of it, so halving the
// pairs halves the dominant cost.
//
// Work item (k, s) of the SymLayout: fixed blocks fb of super-row k one
// after another; for each, the loop blocks c >= fb of segment s in chunks
// of at most two blocks of one class (the block's own square fb == fb on its
// own, row sums only).  Per 16 x 16 tile the MFMA above gives t (frame of
// the fixed block); a lane holds 4 fixed rows x 1 loop column per tile and
// kMfmFt tiles.  Row sums stay per lane in FP32 over a chunk, then FP64;
// a tile's column sums (a lane's 8 rows in FP32) are added over pairs of
// lane groups by a swizzle and stored to LDS, and after the chunk the 8
// partials of each loop node are added in FP64 and collected in LDS over the
// item's fixed blocks.  Weights come
// from CF[q].w (w = x[perm[q]] in FP32).  Work items are launched largest
// first and write their partials at their place in (super-row, segment) order.
// ---------------------------------------------------------------------------

__device__ __forceinline__ int64_t sym_blk_start(int b, const SymLayout& L) {
    return b < L.nb_int ? (int64_t)b * kMfmFixed : L.n_int + (int64_t)(b - L.nb_int) * kMfmFixed;
}
__device__ __forceinline__ int64_t sym_blk_end(int b, const SymLayout& L) {
    const int64_t e = sym_blk_start(b, L) + kMfmFixed;
    const int64_t lim = b < L.nb_int ? L.n_int : L.n;
    return e < lim ? e : lim;
}

// NT staged tiles of 16 loop nodes against the lane's fixed rows.  RI / CI:
// the row sums / column sums take the interior formula (else the boundary
// one); SYM: column sums wanted (off the block's own square).
template <bool RI, bool CI, bool SYM, int NT>
__device__ __forceinline__ void mfs_tiles(const v4u* __restrict__ lds_b, const float* __restrict__ lds_w,
                                          const v4u (&a)[kMfmFt], const v4f (&C)[kMfmFt],
                                          const float (&xi)[kMfmFt][4], float k2, float e2x2, float e2,
                                          double (&acc)[kMfmFt][4], float* __restrict__ colw) {
    const int lane = threadIdx.x & (kWave - 1), g = lane >> 4, jj = lane & 15;
    float s32[kMfmFt][4];
#pragma unroll
    for (int f = 0; f < kMfmFt; ++f)
#pragma unroll
        for (int r = 0; r < 4; ++r) s32[f][r] = 0.f;
    v4f t[kMfmFt];
    float wl = lds_w[jj];
    {
        const v8bf bk = __builtin_bit_cast(v8bf, lds_b[jj * 4 + g]);
#pragma unroll
        for (int f = 0; f < kMfmFt; ++f)
            t[f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a[f]), bk, C[f], 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        if (u < NT) {
            v4f tn[kMfmFt];
            float wn = wl;
            if (u + 1 < NT) {
                const v8bf bn = __builtin_bit_cast(v8bf, lds_b[((u + 1) * 16 + jj) * 4 + g]);
                wn = lds_w[(u + 1) * 16 + jj];
#pragma unroll
                for (int f = 0; f < kMfmFt; ++f)
                    tn[f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a[f]), bn, C[f], 0, 0, 0);
            }
            float cp = 0.f;
#pragma unroll
            for (int f = 0; f < kMfmFt; ++f) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float tt = t[f][r];
                    if (RI && CI) {
                        const float sv = __builtin_amdgcn_rsqf(tt);
                        const float e = fmaf(e2, sv * sv, fmaf(k2, tt, e2x2)) * sv;
                        s32[f][r] = fmaf(e, wl, s32[f][r]);
                        if (SYM) cp = fmaf(e, xi[f][r], cp);
                    } else if (!RI && !CI) {
                        const float e = __builtin_amdgcn_sqrtf(tt);
                        s32[f][r] = fmaf(e, wl, s32[f][r]);
                        if (SYM) cp = fmaf(e, xi[f][r], cp);
                    } else {
                        const float sv = __builtin_amdgcn_rsqf(tt);
                        const float ei = fmaf(e2, sv * sv, fmaf(k2, tt, e2x2)) * sv;
                        const float eb = tt * sv;
                        s32[f][r] = fmaf(RI ? ei : eb, wl, s32[f][r]);
                        cp = fmaf(CI ? ei : eb, xi[f][r], cp);
                    }
                }
            }
            // keep the row and column sums at their tile: left to itself the
            // compiler sinks them to their uses after the loop and holds every
            // tile's entries live until then
#pragma unroll
            for (int f = 0; f < kMfmFt; ++f)
                asm volatile("" : "+v"(s32[f][0]), "+v"(s32[f][1]), "+v"(s32[f][2]), "+v"(s32[f][3]));
            if (SYM) {
                // lanes l and l ^ 16 hold the same loop node: add them (ds_swizzle,
                // xor 16 within each half-wave) and let the lower lane store
                const float o = __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(cp), 0x401F));
                cp += o;
                if ((lane & 16) == 0) colw[u * 16] = cp;
            }
            if (u + 1 < NT) {
#pragma unroll
                for (int f = 0; f < kMfmFt; ++f) t[f] = tn[f];
                wl = wn;
            }
        }
    }
#pragma unroll
    for (int f = 0; f < kMfmFt; ++f)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[f][r] += (double)s32[f][r];
}

template <int NT>
__device__ __forceinline__ void mfs_dispatch(bool ri, bool ci, const v4u* lds_b, const float* lds_w,
                                             const v4u (&a)[kMfmFt], const v4f (&C)[kMfmFt],
                                             const float (&xi)[kMfmFt][4], float k2, float e2x2, float e2,
                                             double (&acc)[kMfmFt][4], float* colw) {
    if (ri && ci)
        mfs_tiles<true, true, true, NT>(lds_b, lds_w, a, C, xi, k2, e2x2, e2, acc, colw);
    else if (!ri && !ci)
        mfs_tiles<false, false, true, NT>(lds_b, lds_w, a, C, xi, k2, e2x2, e2, acc, colw);
    else if (ri)
        mfs_tiles<true, false, true, NT>(lds_b, lds_w, a, C, xi, k2, e2x2, e2, acc, colw);
    else
        mfs_tiles<false, true, true, NT>(lds_b, lds_w, a, C, xi, k2, e2x2, e2, acc, colw);
}

// One work item (blockIdx.x) of the SymLayout.  TRANS: y = A^T x.
// RowP[item][(fb - kF) kMfmFixed + row], ColP[item][(c - c0) kMfmFixed + node].
template <bool TRANS>
__global__ __launch_bounds__(kBlock) void k_mfs(const float4* __restrict__ XS, const float4* __restrict__ CF,
                                                SymLayout L, const float4* __restrict__ frames, EntryConst c,
                                                double* __restrict__ RowP, double* __restrict__ ColP,
                                                const GkbState* __restrict__ st) {
    __shared__ v4u lds_b[4 * kMfmChunk];
    __shared__ float lds_w[kMfmChunk];
    __shared__ float lds_col[2 * (kBlock / kWave)][kMfmChunk];  // per (wave, lane-group pair)
    __shared__ double colacc[kSymMaxLb * kMfmFixed];
    if (st != nullptr && st->stopped) return;
    const int2 item = L.items[blockIdx.x];  // launch order: the largest items first
    const int64_t slot = (int64_t)L.item_first[item.x] + item.y;  // the item's place in the partials
    const int b0 = item.x * L.F;
    const int b1 = b0 + L.F < L.nb ? b0 + L.F : L.nb;
    const int c0 = b0 + item.y * L.Lb;
    const int c1 = c0 + L.Lb < L.nb ? c0 + L.Lb : L.nb;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), g = lane >> 4, jj = lane & 15, wv = tid / kWave;
    for (int i = tid; i < kSymMaxLb * kMfmFixed; i += kBlock) colacc[i] = 0.0;
    // the entry constants in vector registers: an FP32 instruction with a
    // scalar operand does not pair with another in one issue cycle
    float k2 = c.k2f, e2x2 = c.e2x2f, e2 = c.e2f;
    asm volatile("" : "+v"(k2), "+v"(e2x2), "+v"(e2));
    double* red = reinterpret_cast<double*>(lds_b);  // 64 rows x 17 (padded) doubles, between chunks
    for (int fb = b0; fb < b1; ++fb) {
        const int64_t fs = sym_blk_start(fb, L), fe = sym_blk_end(fb, L);
        const bool fint = fb < L.nb_int;
        const float4 fr = frames[fb];
        v4u a[kMfmFt];
        v4f C[kMfmFt];
        float xi[kMfmFt][4];
        double acc[kMfmFt][4];
#pragma unroll
        for (int f = 0; f < kMfmFt; ++f) {
            const int64_t base = fs + (int64_t)(wv * kMfmFt + f) * 16;
            const int64_t i = base + jj;
            float d[3] = {0.f, 0.f, 0.f};
            if (i < fe) {
                const float4 q = XS[i];
                d[0] = q.x - fr.x;
                d[1] = q.y - fr.y;
                d[2] = q.z - fr.z;
            }
            if (g < 3) {
                a[f] = fixed_terms(-2.0f * d[g]);
            } else {
                const unsigned one = 0x3F80u;  // bf16 1.0
                a[f][0] = one | (one << 16);
                a[f][1] = one;
                a[f][2] = 0u;
                a[f][3] = 0u;
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i2 = base + 4 * g + r;
                float d2 = 0.f, w = 0.f;
                if (i2 < fe) {
                    const float4 q = XS[i2];
                    const float ex = q.x - fr.x, ey = q.y - fr.y, ez = q.z - fr.z;
                    d2 = fmaf(ez, ez, fmaf(ey, ey, ex * ex));
                    w = CF[i2].w;
                }
                C[f][r] = d2;
                xi[f][r] = w;
                acc[f][r] = 0.0;
            }
        }
        for (int cb = c0 > fb ? c0 : fb; cb < c1;) {
            const bool diag = cb == fb;
            const bool cint = cb < L.nb_int;
            int ce = cb + 1;
            if (!diag && ce < c1 && (ce < L.nb_int) == cint && sym_blk_end(cb, L) - sym_blk_start(cb, L) == kMfmFixed)
                ce = cb + 2;
            const int64_t j0 = sym_blk_start(cb, L), j1 = sym_blk_end(ce - 1, L);
            // stage the chunk's loop nodes in the fixed block's frame: B
            // operand (4 lane groups x 8 bf16) and weight; past j1: d = 0, w = 0
            const int64_t j = j0 + tid;
            float dx = 0.f, dy = 0.f, dz = 0.f, w = 0.f;
            if (j < j1) {
                const float4 q = XS[j];
                w = CF[j].w;
                dx = q.x - fr.x;
                dy = q.y - fr.y;
                dz = q.z - fr.z;
            }
            const v4u bb0 = loop_terms(dx), bb1 = loop_terms(dy), bb2 = loop_terms(dz);
            unsigned h, m, l;
            split_bf16x3(fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, 1.0f))), h, m, l);
            v4u bb3;
            bb3[0] = pack_bf16(h, m);
            bb3[1] = l >> 16;
            bb3[2] = 0u;
            bb3[3] = 0u;
            __syncthreads();  // the previous chunk (or the row reduction) is done with LDS
            lds_b[tid * 4 + 0] = bb0;
            lds_b[tid * 4 + 1] = bb1;
            lds_b[tid * 4 + 2] = bb2;
            lds_b[tid * 4 + 3] = bb3;
            lds_w[tid] = w;
            __syncthreads();
            // row sums: formula of the rows of A the fixed nodes stand for
            // (A x: the fixed rows; A^T x: the loop rows); column sums: the other
            const bool ri = TRANS ? cint : fint, ci = TRANS ? fint : cint;
            float* colw = &lds_col[2 * wv + (g >> 1)][jj];
            if (diag) {
                if (fint)
                    mfs_tiles<true, true, false, 8>(lds_b, lds_w, a, C, xi, k2, e2x2, e2, acc, colw);
                else
                    mfs_tiles<false, false, false, 8>(lds_b, lds_w, a, C, xi, k2, e2x2, e2, acc, colw);
            } else if (ce == cb + 2) {
                mfs_dispatch<16>(ri, ci, lds_b, lds_w, a, C, xi, k2, e2x2, e2, acc, colw);
            } else {
                mfs_dispatch<8>(ri, ci, lds_b, lds_w, a, C, xi, k2, e2x2, e2, acc, colw);
            }
            if (!diag) {
                // the chunk's column sums: the 8 (wave, lane-group pair) partials of each loop node
                __syncthreads();
                if (tid < (int)(j1 - j0)) {
                    double v = 0.0;
#pragma unroll
                    for (int q = 0; q < 2 * (kBlock / kWave); ++q) v += (double)lds_col[q][tid];
                    colacc[(cb - c0) * kMfmFixed + tid] += v;
                }
            }
            cb = ce;
        }
        // the fixed block's row sums: each row's 16 lane partials in a fixed order
        double* rp = RowP + slot * L.F * kMfmFixed + (int64_t)(fb - b0) * kMfmFixed;
#pragma unroll
        for (int f = 0; f < kMfmFt; ++f) {
            __syncthreads();
#pragma unroll
            for (int r = 0; r < 4; ++r) red[(wv * 16 + 4 * g + r) * 17 + jj] = acc[f][r];
            __syncthreads();
            if (tid < 64) {
                const int node = tid;
                double sum = 0.0;
                for (int q = 0; q < 16; ++q) sum += red[node * 17 + q];
                const int row = ((node >> 4) * kMfmFt + f) * 16 + (node & 15);
                rp[row] = fs + row < fe ? sum : 0.0;
            }
        }
    }
    __syncthreads();
    double* cpo = ColP + slot * L.Lb * kMfmFixed;
    for (int i = tid; i < L.Lb * kMfmFixed; i += kBlock) cpo[i] = colacc[i];
}

// ---------------------------------------------------------------------------
// FP64 products over unordered pairs of nodes: the work items, lane layout
// and partials of k_mfs with every quantity in FP64.  A lane holds the
// coordinates and weights of 4 fixed rows (4g + r) of each of its kMfmFt
// tiles and takes loop node jj of each staged tile of 16; t = 1 + |P_i -
// P_j|^2 comes from the coordinate differences (FP64 VALU; the matrix cores
// at FP64 would save little and leave t exposed to the rank-4 form's
// cancellation), s = t^(-1/2) from the FP64 estimate and one third-order step,
// the entry as in the single-entry FP64 products.  Row sums stay per lane in
// FP64 and are reduced over the 16 lanes of a row at the end of the fixed
// block; column sums are added over the lane's 8 rows, over lane groups g by
// a swizzle and LDS, and collected per item as in k_mfs.  XS64: sorted
// coordinates, the weight x[perm[q]] in .w (written by k_gather_w64).
// ---------------------------------------------------------------------------

__device__ __forceinline__ double swizzle_xor16(double v) {
    const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), 0x401F);
    const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), 0x401F);
    return __hiloint2double(hi, lo);
}

template <bool RI, bool CI, bool SYM, int NT>
__device__ __forceinline__ void mfs64_tiles(const double4* __restrict__ lds_p, const double (&px)[kMfmFt][4],
                                            const double (&py)[kMfmFt][4], const double (&pz)[kMfmFt][4],
                                            const double (&xi)[kMfmFt][4], double k2, double e2x2, double e2,
                                            double (&acc)[kMfmFt][4], double* __restrict__ colw) {
    const int lane = threadIdx.x & (kWave - 1), jj = lane & 15;
    for (int u = 0; u < NT; ++u) {
        const double4 q = lds_p[u * 16 + jj];
        double cp = 0.0;
#pragma unroll
        for (int f = 0; f < kMfmFt; ++f) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const double dx = px[f][r] - q.x, dy = py[f][r] - q.y, dz = pz[f][r] - q.z;
                const double t = fma(dz, dz, fma(dy, dy, fma(dx, dx, 1.0)));
                const double sv = rsqrt_f64(t);
                if (RI && CI) {
                    const double e = fma(e2, sv * sv, fma(k2, t, e2x2)) * sv;
                    acc[f][r] = fma(e, q.w, acc[f][r]);
                    if (SYM) cp = fma(e, xi[f][r], cp);
                } else if (!RI && !CI) {
                    const double e = t * sv;
                    acc[f][r] = fma(e, q.w, acc[f][r]);
                    if (SYM) cp = fma(e, xi[f][r], cp);
                } else {
                    const double ei = fma(e2, sv * sv, fma(k2, t, e2x2)) * sv;
                    const double eb = t * sv;
                    acc[f][r] = fma(RI ? ei : eb, q.w, acc[f][r]);
                    cp = fma(CI ? ei : eb, xi[f][r], cp);
                }
            }
        }
        // keep the row sums at their tile (left to itself the compiler sinks
        // them past the loop and holds every tile's entries live)
#pragma unroll
        for (int f = 0; f < kMfmFt; ++f)
            asm volatile("" : "+v"(acc[f][0]), "+v"(acc[f][1]), "+v"(acc[f][2]), "+v"(acc[f][3]));
        if (SYM) {
            // lanes l and l ^ 16 hold the same loop node: add them and let the lower lane store
            cp += swizzle_xor16(cp);
            if ((lane & 16) == 0) colw[u * 16] = cp;
        }
    }
}

template <int NT>
__device__ __forceinline__ void mfs64_dispatch(bool ri, bool ci, const double4* lds_p, const double (&px)[kMfmFt][4],
                                               const double (&py)[kMfmFt][4], const double (&pz)[kMfmFt][4],
                                               const double (&xi)[kMfmFt][4], double k2, double e2x2, double e2,
                                               double (&acc)[kMfmFt][4], double* colw) {
    if (ri && ci)
        mfs64_tiles<true, true, true, NT>(lds_p, px, py, pz, xi, k2, e2x2, e2, acc, colw);
    else if (!ri && !ci)
        mfs64_tiles<false, false, true, NT>(lds_p, px, py, pz, xi, k2, e2x2, e2, acc, colw);
    else if (ri)
        mfs64_tiles<true, false, true, NT>(lds_p, px, py, pz, xi, k2, e2x2, e2, acc, colw);
    else
        mfs64_tiles<false, true, true, NT>(lds_p, px, py, pz, xi, k2, e2x2, e2, acc, colw);
}

template <bool TRANS>
__global__ __launch_bounds__(kBlock) void k_mfs64(const double4* __restrict__ XS64, SymLayout L, EntryConst c,
                                                  double* __restrict__ RowP, double* __restrict__ ColP,
                                                  const GkbState* __restrict__ st) {
    __shared__ double4 lds_p[kMfmChunk];
    __shared__ double lds_col[2 * (kBlock / kWave)][kMfmChunk];  // per (wave, lane-group pair)
    __shared__ double colacc[kSymMaxLb * kMfmFixed];
    double* red = &lds_col[0][0];  // 64 rows x 17 (padded), between chunks (four workgroups fit a CU's LDS)
    if (st != nullptr && st->stopped) return;
    const int2 item = L.items[blockIdx.x];
    const int64_t slot = (int64_t)L.item_first[item.x] + item.y;
    const int b0 = item.x * L.F;
    const int b1 = b0 + L.F < L.nb ? b0 + L.F : L.nb;
    const int c0 = b0 + item.y * L.Lb;
    const int c1 = c0 + L.Lb < L.nb ? c0 + L.Lb : L.nb;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), g = lane >> 4, jj = lane & 15, wv = tid / kWave;
    for (int i = tid; i < kSymMaxLb * kMfmFixed; i += kBlock) colacc[i] = 0.0;
    const double k2 = c.k2, e2x2 = c.e2x2, e2 = c.e2;
    for (int fb = b0; fb < b1; ++fb) {
        const int64_t fs = sym_blk_start(fb, L), fe = sym_blk_end(fb, L);
        const bool fint = fb < L.nb_int;
        double px[kMfmFt][4], py[kMfmFt][4], pz[kMfmFt][4], xi[kMfmFt][4], acc[kMfmFt][4];
#pragma unroll
        for (int f = 0; f < kMfmFt; ++f) {
            const int64_t base = fs + (int64_t)(wv * kMfmFt + f) * 16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i2 = base + 4 * g + r;
                const double4 q = XS64[i2 < fe ? i2 : fs];
                const bool in = i2 < fe;
                px[f][r] = q.x;
                py[f][r] = q.y;
                pz[f][r] = q.z;
                xi[f][r] = in ? q.w : 0.0;
                acc[f][r] = 0.0;
            }
        }
        for (int cb = c0 > fb ? c0 : fb; cb < c1;) {
            const bool diag = cb == fb;
            const bool cint = cb < L.nb_int;
            int ce = cb + 1;
            if (!diag && ce < c1 && (ce < L.nb_int) == cint && sym_blk_end(cb, L) - sym_blk_start(cb, L) == kMfmFixed)
                ce = cb + 2;
            const int64_t j0 = sym_blk_start(cb, L), j1 = sym_blk_end(ce - 1, L);
            // stage the chunk's loop nodes (coordinates and weight); past j1 the
            // first node with weight 0 (its column sums are not collected)
            const int64_t j = j0 + tid;
            double4 q = XS64[j < j1 ? j : j0];
            if (!(j < j1)) q.w = 0.0;
            __syncthreads();  // the previous chunk (or the row reduction) is done with LDS
            lds_p[tid] = q;
            __syncthreads();
            const bool ri = TRANS ? cint : fint, ci = TRANS ? fint : cint;
            double* colw = &lds_col[2 * wv + (g >> 1)][jj];
            if (diag) {
                if (fint)
                    mfs64_tiles<true, true, false, 8>(lds_p, px, py, pz, xi, k2, e2x2, e2, acc, colw);
                else
                    mfs64_tiles<false, false, false, 8>(lds_p, px, py, pz, xi, k2, e2x2, e2, acc, colw);
            } else if (ce == cb + 2) {
                mfs64_dispatch<16>(ri, ci, lds_p, px, py, pz, xi, k2, e2x2, e2, acc, colw);
            } else {
                mfs64_dispatch<8>(ri, ci, lds_p, px, py, pz, xi, k2, e2x2, e2, acc, colw);
            }
            if (!diag) {
                // the chunk's column sums: the 8 (wave, lane-group pair) partials of each loop node
                __syncthreads();
                if (tid < (int)(j1 - j0)) {
                    double v = 0.0;
#pragma unroll
                    for (int qq = 0; qq < 2 * (kBlock / kWave); ++qq) v += lds_col[qq][tid];
                    colacc[(cb - c0) * kMfmFixed + tid] += v;
                }
            }
            cb = ce;
        }
        // the fixed block's row sums: each row's 16 lane partials in a fixed order
        double* rp = RowP + slot * L.F * kMfmFixed + (int64_t)(fb - b0) * kMfmFixed;
#pragma unroll
        for (int f = 0; f < kMfmFt; ++f) {
            __syncthreads();
#pragma unroll
            for (int r = 0; r < 4; ++r) red[(wv * 16 + 4 * g + r) * 17 + jj] = acc[f][r];
            __syncthreads();
            if (tid < 64) {
                const int node = tid;
                double sum = 0.0;
                for (int qq = 0; qq < 16; ++qq) sum += red[node * 17 + qq];
                const int row = ((node >> 4) * kMfmFt + f) * 16 + (node & 15);
                rp[row] = fs + row < fe ? sum : 0.0;
            }
        }
    }
    __syncthreads();
    double* cpo = ColP + slot * L.Lb * kMfmFixed;
    for (int i = tid; i < L.Lb * kMfmFixed; i += kBlock) cpo[i] = colacc[i];
}

// XS64[q].w = x[perm[q]]: the weights of a FP64 pair product in the sorted order.
__global__ __launch_bounds__(kBlock) void k_gather_w64(const double* __restrict__ x, const int32_t* __restrict__ perm,
                                                       int64_t n, double4* __restrict__ XS64,
                                                       const GkbState* __restrict__ st) {
    if (st != nullptr && st->stopped) return;
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= n) return;
    XS64[q].w = x[perm[q]];
}

// y_o = (row partials of the items of q's super-row + column partials of
// the items whose segment holds q's block) - shift z_o, o = perm[q]; the
// partials are added in item order, four running sums combined at the end.
__global__ __launch_bounds__(kBlock) void k_mfs_reduce(SymLayout L, const double* __restrict__ RowP,
                                                       const double* __restrict__ ColP,
                                                       const int32_t* __restrict__ perm,
                                                       const double* __restrict__ shift_ptr, double shift_val,
                                                       const double* __restrict__ z, double* __restrict__ y,
                                                       const GkbState* __restrict__ st) {
    if (st != nullptr && st->stopped) return;
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= L.n) return;
    const int beta = q < L.n_int ? (int)(q / kMfmFixed) : L.nb_int + (int)((q - L.n_int) / kMfmFixed);
    const int64_t off = q - sym_blk_start(beta, L);
    const int k = beta / L.F;
    const int64_t rs = (int64_t)L.F * kMfmFixed, cs = (int64_t)L.Lb * kMfmFixed;
    const int64_t roff = (int64_t)(beta - k * L.F) * kMfmFixed + off;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    const int i0 = L.item_first[k], i1 = L.item_first[k + 1];
    int it = i0;
    for (; it + 3 < i1; it += 4) {
        a0 += RowP[(int64_t)it * rs + roff];
        a1 += RowP[(int64_t)(it + 1) * rs + roff];
        a2 += RowP[(int64_t)(it + 2) * rs + roff];
        a3 += RowP[(int64_t)(it + 3) * rs + roff];
    }
    for (; it < i1; ++it) a0 += RowP[(int64_t)it * rs + roff];
    double b0 = 0.0, b1 = 0.0, b2 = 0.0, b3 = 0.0;
    auto col = [&](int kk) {
        const int sg = (beta - kk * L.F) / L.Lb;
        const int cst = kk * L.F + sg * L.Lb;
        return ColP[(int64_t)(L.item_first[kk] + sg) * cs + (int64_t)(beta - cst) * kMfmFixed + off];
    };
    int kk = 0;
    for (; kk + 3 <= k; kk += 4) {
        b0 += col(kk);
        b1 += col(kk + 1);
        b2 += col(kk + 2);
        b3 += col(kk + 3);
    }
    for (; kk <= k; ++kk) b0 += col(kk);
    double s = ((a0 + a1) + (a2 + a3)) + ((b0 + b1) + (b2 + b3));
    const int64_t o = perm[q];
    if (z != nullptr) {
        const double sh = shift_ptr != nullptr ? *shift_ptr : shift_val;
        s -= sh * z[o];
    }
    y[o] = s;
}

// CF[q] = (w kappa^2, 2 w eps^2, w eps^2, w) with w = x[perm[q]]: the
// weight-folded entry coefficients of the sorted nodes for one product.
__global__ __launch_bounds__(kBlock) void k_gather_coef(const double* __restrict__ x,
                                                        const int32_t* __restrict__ perm, int64_t n, EntryConst c,
                                                        float4* __restrict__ CF, const GkbState* __restrict__ st) {
    if (st != nullptr && st->stopped) return;
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= n) return;
    const double w = x[perm[q]];
    CF[q] = make_float4((float)(w * c.k2), (float)(w * c.e2x2), (float)(w * c.e2), (float)w);
}

// ---------------------------------------------------------------------------
// Block products for kBlkRhs right-hand sides at once (lockstep Golub-Kahan
// runs sharing each pass over A): P[slice][k][q] = sum over the slice's loop
// nodes j of A(q, j) v_k[j] (rows) or A(j, q) v_k[j] (columns), in sorted
// node order.
//
// Per 16 x 16 tile the squared distances come from the same bf16x3 MFMA as
// in the pair products with the operands swapped (A = loop nodes, B = fixed
// nodes), so a lane holds t for 4 loop nodes j = 4g + r and one fixed node.
// The contraction E (16 fixed x 16 loop) V (16 loop x 16 rhs) runs on the
// matrix cores in FP16 with both operands split in two: the entries, scaled
// by 2^se, as e = e_h + e_l (e_h = fp16(e) to nearest, e_l = fp16(e - e_h)),
// the right-hand sides, each column scaled by its own power of two, as v =
// v_h + v_l alike, and E V ~ E_h V_h + E_l V_h + E_h V_l: three
// v_mfma_f32_16x16x16_f16 (a lane group's 4 K slots are its 4 loop nodes).  e_h + e_l keeps e to 2^-22
// relative (the FP32 entries carry an error of that order from their rsqrt
// already), and the dropped E_l V_l is below 2^-22 |e v|.  Products of two
// fp16 values are exact in FP32; sums are FP32 over one 256-node chunk,
// FP64 across chunks and slices, and the scales are taken out exactly in
// FP64.  On this GPU the FP32 matrix instructions do not overlap VALU work
// while the FP16 ones largely do: four v_mfma_f32_16x16x4_f32 per tile
// (128 cycles, exposed) become three FP16 ones (24 cycles, mostly hidden)
// and 8 VALU instructions for the split of 4 entries.
// ---------------------------------------------------------------------------

typedef _Float16 v2h __attribute__((ext_vector_type(2)));
typedef _Float16 v4h __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));
typedef unsigned int v2u __attribute__((ext_vector_type(2)));

constexpr float kBlkRange = 16384.0f;  // scaled entries and right-hand sides stay below this (fp16 max 65504)

// Two FP32 values as fp16 pairs: H = (fp16(a), fp16(b)) rounded to nearest,
// L = the same of the remainders a - H.lo, b - H.hi (exact in FP32).
__device__ __forceinline__ void split_f16x2(float a, float b, unsigned& H, unsigned& L) {
    const v2h h = __builtin_convertvector((v2f){a, b}, v2h);
    const v2h l = __builtin_convertvector((v2f){a - (float)h[0], b - (float)h[1]}, v2h);
    H = __builtin_bit_cast(unsigned, h);
    L = __builtin_bit_cast(unsigned, l);
}

// Entries of the lane's 4 loop nodes x FT fixed nodes from their squared
// distances, scaled by 2^se, split into (H01, H23, L01, L23).  MIX = 1: the
// interior formula, 0: the boundary one, 2: by the loop node's class
// (node jb + r interior when below n_int; the chunk of a column product that
// straddles the classes).
template <int MIX, int FT>
__device__ __forceinline__ void block_split(const v4f (&t)[FT], const BlockEntry& c, int64_t jb, int64_t n_int,
                                            unsigned (&h)[FT][4]) {
#pragma unroll
    for (int f = 0; f < FT; ++f) {
        float e[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float tt = t[f][r];
            if (MIX == 1) {
                const float sv = __builtin_amdgcn_rsqf(tt);
                e[r] = fmaf(c.e2, sv * sv, fmaf(c.k2, tt, c.e2x2)) * sv;
            } else if (MIX == 0) {
                e[r] = __builtin_amdgcn_sqrtf(tt) * c.bsc;
            } else {
                const float sv = __builtin_amdgcn_rsqf(tt);
                const float ei = fmaf(c.e2, sv * sv, fmaf(c.k2, tt, c.e2x2)) * sv;
                const float eb = tt * sv * c.bsc;
                e[r] = jb + r < n_int ? ei : eb;
            }
        }
        split_f16x2(e[0], e[1], h[f][0], h[f][2]);
        split_f16x2(e[2], e[3], h[f][1], h[f][3]);
    }
}

// Squared distances of tile u (16 staged loop nodes) to the lane's fixed nodes.
template <int FT>
__device__ __forceinline__ void block_tdist(const v4u* __restrict__ lds_a, int u, int jj, int g, const v4u (&bf)[FT],
                                            const v4f (&Cf)[FT], v4f (&t)[FT]) {
    const v8bf ak = __builtin_bit_cast(v8bf, lds_a[(u * 16 + jj) * 4 + g]);
#pragma unroll
    for (int f = 0; f < FT; ++f)
        t[f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ak, __builtin_bit_cast(v8bf, bf[f]), Cf[f], 0, 0, 0);
}

// The 16 staged tiles of one chunk (first loop node t0) against the lane's
// fixed tiles, as a three-stage pipeline, fully unrolled: the squared
// distances of tile u + 2, the entries and their split of tile u + 1 and
// the contraction of tile u are in flight together.
template <int MIX, int FT>
__device__ __forceinline__ void mfh_chunk(const v4u* __restrict__ lds_a, const uint4* __restrict__ lds_v, int64_t t0,
                                          int64_t n_int, const BlockEntry& c, const v4u (&bf)[FT],
                                          const v4f (&Cf)[FT], double (&acc)[FT][4]) {
    const int lane = threadIdx.x & (kWave - 1), g = lane >> 4, jj = lane & 15;
    constexpr int kTiles = kMfmChunk / 16;
    // one instruction shape on each accumulator: a chain feeding its own
    // result back as C is the case the matrix cores forward without waiting
    // (a 16x16x16 reading the fresh result of a 16x16x32 as C is not)
    v4f d2[FT];
#pragma unroll
    for (int f = 0; f < FT; ++f) d2[f] = v4f{0.f, 0.f, 0.f, 0.f};
    v4f tc[FT], tn[FT];
    unsigned hc[FT][4];
    block_tdist<FT>(lds_a, 0, jj, g, bf, Cf, tc);
    block_tdist<FT>(lds_a, 1, jj, g, bf, Cf, tn);
    block_split<MIX, FT>(tc, c, t0 + 4 * g, n_int, hc);
#pragma unroll
    for (int u = 0; u < kTiles; ++u) {
        // the lane group's 4 loop nodes, split, for right-hand side jj
        const uint4 bv = lds_v[(u * 4 + g) * kBlkRhs + jj];
        v4f tnn[FT];
        if (u + 2 < kTiles) block_tdist<FT>(lds_a, u + 2, jj, g, bf, Cf, tnn);
        unsigned hn[FT][4];
        if (u + 1 < kTiles) block_split<MIX, FT>(tn, c, t0 + (u + 1) * 16 + 4 * g, n_int, hn);
        // the lane group's 4 loop nodes in the K slots: e_h v_h, e_l v_h, e_h v_l
        const v2u vhi = {bv.x, bv.y}, vlo = {bv.z, bv.w};
#pragma unroll
        for (int f = 0; f < FT; ++f) {
            const v2u ehi = {hc[f][0], hc[f][1]}, elo = {hc[f][2], hc[f][3]};
            d2[f] = __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(v4h, ehi), __builtin_bit_cast(v4h, vhi),
                                                          d2[f], 0, 0, 0);
            d2[f] = __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(v4h, elo), __builtin_bit_cast(v4h, vhi),
                                                          d2[f], 0, 0, 0);
            d2[f] = __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(v4h, ehi), __builtin_bit_cast(v4h, vlo),
                                                          d2[f], 0, 0, 0);
        }
        if (u + 1 < kTiles) {
#pragma unroll
            for (int f = 0; f < FT; ++f) {
#pragma unroll
                for (int q = 0; q < 4; ++q) hc[f][q] = hn[f][q];
                tn[f] = tnn[f];
            }
        }
    }
#pragma unroll
    for (int f = 0; f < FT; ++f)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[f][r] += (double)d2[f][r];
}

// One slice [j0, j1) of loop nodes (block-uniform; contains barriers; j0 a
// multiple of kMfmChunk).  ROWS: the fixed nodes' class (fint) picks the
// formula; columns: each chunk's loop nodes do.
template <bool ROWS, int FT>
__device__ __forceinline__ void mfh_span(const float4* __restrict__ XS, const uint4* __restrict__ Vh, int64_t j0,
                                         int64_t j1, int64_t n_int, bool fint, const float4& fr, const BlockEntry& c,
                                         const v4u (&bf)[FT], const v4f (&Cf)[FT], double (&acc)[FT][4],
                                         v4u* __restrict__ lds_a, uint4* __restrict__ lds_v) {
    for (int64_t t0 = j0; t0 < j1; t0 += kMfmChunk) {
        const int64_t j = t0 + threadIdx.x;
        float dx = 0.f, dy = 0.f, dz = 0.f;
        if (j < j1) {
            const float4 q = XS[j];
            dx = q.x - fr.x;
            dy = q.y - fr.y;
            dz = q.z - fr.z;
        }
        const v4u a0 = loop_terms(dx), a1 = loop_terms(dy), a2 = loop_terms(dz);
        unsigned h, m, l;
        split_bf16x3(fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, 1.0f))), h, m, l);
        v4u a3;
        a3[0] = pack_bf16(h, m);
        a3[1] = l >> 16;
        a3[2] = 0u;
        a3[3] = 0u;
        // the chunk's split right-hand sides: kMfmChunk / 4 quads x kBlkRhs
        // (a quad past j1 lies past n, where Vh holds zeros, or in the next
        // slice, which starts at a multiple of kMfmChunk: none is read)
        uint4 vq[4];
#pragma unroll
        for (int m4 = 0; m4 < 4; ++m4) {
            const int i = threadIdx.x + m4 * kBlock;
            const int64_t node = t0 + 4 * (i / kBlkRhs);
            vq[m4] = node < j1 ? Vh[((t0 >> 2) + i / kBlkRhs) * kBlkRhs + (i % kBlkRhs)] : make_uint4(0u, 0u, 0u, 0u);
        }
        __syncthreads();  // the previous chunk has been consumed
        lds_a[threadIdx.x * 4 + 0] = a0;
        lds_a[threadIdx.x * 4 + 1] = a1;
        lds_a[threadIdx.x * 4 + 2] = a2;
        lds_a[threadIdx.x * 4 + 3] = a3;
#pragma unroll
        for (int m4 = 0; m4 < 4; ++m4) lds_v[threadIdx.x + m4 * kBlock] = vq[m4];
        __syncthreads();
        const int64_t cend = t0 + kMfmChunk < j1 ? t0 + kMfmChunk : j1;
        if (ROWS ? fint : cend <= n_int)
            mfh_chunk<1, FT>(lds_a, lds_v, t0, n_int, c, bf, Cf, acc);
        else if (ROWS || t0 >= n_int)
            mfh_chunk<0, FT>(lds_a, lds_v, t0, n_int, c, bf, Cf, acc);
        else
            mfh_chunk<2, FT>(lds_a, lds_v, t0, n_int, c, bf, Cf, acc);
    }
}

template <bool ROWS, int FT>
__global__ __launch_bounds__(kBlock) void k_mfh_block(const float4* __restrict__ XS, const uint4* __restrict__ Vh,
                                                      const float* __restrict__ vsc, int64_t n, int64_t n_int,
                                                      int64_t nb_int, int64_t slice_len,
                                                      const float4* __restrict__ frames, BlockEntry c,
                                                      double* __restrict__ P, int64_t ldp) {
    __shared__ v4u lds_a[4 * kMfmChunk];
    __shared__ uint4 lds_v[(kMfmChunk / 4) * kBlkRhs];
    // blocks of kFix = 64 FT fixed nodes per class; the frame is that of the
    // kMfmFixed-node block holding the first of them
    constexpr int kFix = (kBlock / kWave) * FT * 16;
    const int64_t b = blockIdx.x;
    const bool fint = b < nb_int;
    const int64_t fb0 = fint ? b * kFix : n_int + (b - nb_int) * kFix;
    const int64_t fend = fint ? n_int : n;
    const int64_t fb1 = fb0 + kFix < fend ? fb0 + kFix : fend;
    const int64_t nbf_int = (n_int + kMfmFixed - 1) / kMfmFixed;
    const float4 fr = frames[fint ? (b * kFix) / kMfmFixed : nbf_int + ((b - nb_int) * kFix) / kMfmFixed];
    const int lane = threadIdx.x & (kWave - 1), g = lane >> 4, jj = lane & 15, wv = threadIdx.x / kWave;
    v4u bf[FT];
    v4f Cf[FT];
    double acc[FT][4];
#pragma unroll
    for (int f = 0; f < FT; ++f) {
        const int64_t i = fb0 + (int64_t)(wv * FT + f) * 16 + jj;
        float d[3] = {0.f, 0.f, 0.f};
        if (i < fb1) {
            const float4 q = XS[i];
            d[0] = q.x - fr.x;
            d[1] = q.y - fr.y;
            d[2] = q.z - fr.z;
        }
        if (g < 3) {
            bf[f] = fixed_terms(-2.0f * d[g]);
        } else {
            const unsigned one = 0x3F80u;  // bf16 1.0
            bf[f][0] = one | (one << 16);
            bf[f][1] = one;
            bf[f][2] = 0u;
            bf[f][3] = 0u;
        }
        const float d2 = fmaf(d[2], d[2], fmaf(d[1], d[1], d[0] * d[0]));
        Cf[f] = v4f{d2, d2, d2, d2};
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[f][r] = 0.0;
    }
    const int64_t j0 = (int64_t)blockIdx.y * slice_len;
    const int64_t j1 = j0 + slice_len < n ? j0 + slice_len : n;
    // the entry constants in vector registers: an FP32 instruction with a
    // scalar operand does not pair with another in one issue cycle
    BlockEntry cv = c;
    asm volatile("" : "+v"(cv.k2), "+v"(cv.e2x2), "+v"(cv.e2), "+v"(cv.bsc));
    mfh_span<ROWS, FT>(XS, Vh, j0, j1, n_int, fint, fr, cv, bf, Cf, acc, lds_a, lds_v);
    // the scales out: 2^-se of the entries and the column's own
    const double un = c.unscale / (double)vsc[jj];
#pragma unroll
    for (int f = 0; f < FT; ++f) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t i = fb0 + (int64_t)(wv * FT + f) * 16 + 4 * g + r;
            if (i < fb1) P[((int64_t)blockIdx.y * kBlkRhs + jj) * ldp + i] = acc[f][r] * un;
        }
    }
}

// Vh[q][k] = the split of the scaled values vsc[k] Vg[4q + r][k], r = 0..3
// (zeros past n): (H01, H23, L01, L23), fp16 pairs as in split_f16x2.
// Values beyond the scaled range are clamped to it (NaN stays NaN); the
// block products only receive such values from steps whose results are
// discarded (after a breakdown), the unit-norm operands of the Golub-Kahan
// runs stay within it by construction.
__global__ __launch_bounds__(kBlock) void k_split_block(const float* __restrict__ Vg, int64_t n,
                                                        const float* __restrict__ vsc, uint4* __restrict__ Vh) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t nq = (n + 3) / 4;
    if (e >= nq * kBlkRhs) return;
    const int64_t q = e / kBlkRhs;
    const int k = (int)(e % kBlkRhs);
    const float sc = vsc[k];
    float v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t j = 4 * q + r;
        float x = j < n ? Vg[j * kBlkRhs + k] * sc : 0.f;
        if (__builtin_isfinite(x) && fabsf(x) > kBlkRange) x = copysignf(kBlkRange, x);
        v[r] = x;
    }
    uint4 o;
    split_f16x2(v[0], v[1], o.x, o.z);
    split_f16x2(v[2], v[3], o.y, o.w);
    Vh[e] = o;
}

// vsc[k] = 2^(14 - e_k) with max_j |Vg[j][k]| < 2^e_k (1 for a zero column):
// column k scaled below kBlkRange.  One workgroup per column.
__global__ __launch_bounds__(kBlock) void k_block_vscale(const float* __restrict__ Vg, int64_t n,
                                                         float* __restrict__ vsc) {
    __shared__ float red[kBlock / kWave];
    const int k = blockIdx.x;
    float m = 0.f;
    for (int64_t j = threadIdx.x; j < n; j += kBlock) m = fmaxf(m, fabsf(Vg[j * kBlkRhs + k]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, kWave));
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        float mm = 0.f;
        for (int w = 0; w < kBlock / kWave; ++w) mm = fmaxf(mm, red[w]);
        float s = 1.f;
        if (mm > 0.f) {
            int ex;
            (void)frexpf(mm, &ex);
            int p = 14 - ex;
            p = p > 126 ? 126 : (p < -126 ? -126 : p);
            s = ldexpf(1.f, p);
        }
        vsc[k] = s;
    }
}

// Vg[q][k] = x_k[perm[q]] in FP32 for k < s (zero for s <= k < kBlkRhs and
// for stopped runs); x_k = X + k * ldx.
__global__ __launch_bounds__(kBlock) void k_gather_block(const double* __restrict__ X, int64_t ldx, int s,
                                                         const int32_t* __restrict__ perm, int64_t n,
                                                         const GkbState* __restrict__ st, float* __restrict__ Vg) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= n * kBlkRhs) return;
    const int64_t q = e / kBlkRhs;
    const int k = (int)(e % kBlkRhs);
    const bool live = k < s && (st == nullptr || !st[k].stopped);
    Vg[e] = live ? (float)X[k * ldx + perm[q]] : 0.f;
}

// Vg[e] = a fixed pseudo-random value in [-0.5, 0.5) (an operand for timing
// runs: finite, with the spread of real data).
__global__ __launch_bounds__(kBlock) void k_fill_hash(float* __restrict__ Vg, int64_t count) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= count) return;
    uint32_t h = (uint32_t)e * 0x9E3779B1u;
    h ^= h >> 15;
    h *= 0x85EBCA77u;
    h ^= h >> 13;
    Vg[e] = (float)(h >> 8) * (1.0f / 16777216.0f) - 0.5f;
}

// y_k[perm[i]] = sum_slices P[slice][k][i] - shift_k z_k[perm[i]] for right-hand
// side k = blockIdx.y (shift_k = shift[k * sstride], z_k = z + k * ldz,
// y_k = y + k * ldy); skipped when state k has stopped.
__global__ __launch_bounds__(kBlock) void k_reduce_block(const double* __restrict__ P, int64_t ldp, int S, int64_t n,
                                                         const int32_t* __restrict__ perm,
                                                         const double* __restrict__ shift, int64_t sstride,
                                                         const double* __restrict__ z, int64_t ldz,
                                                         double* __restrict__ y, int64_t ldy,
                                                         const GkbState* __restrict__ st) {
    const int k = blockIdx.y;
    if (st != nullptr && st[k].stopped) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double a0 = 0.0, a1 = 0.0;
    int sl = 0;
    for (; sl + 1 < S; sl += 2) {
        a0 += P[((int64_t)sl * kBlkRhs + k) * ldp + i];
        a1 += P[((int64_t)(sl + 1) * kBlkRhs + k) * ldp + i];
    }
    if (sl < S) a0 += P[((int64_t)sl * kBlkRhs + k) * ldp + i];
    double v = a0 + a1;
    const int64_t o = perm[i];
    if (z != nullptr) v -= shift[k * sstride] * z[k * ldz + o];
    y[k * ldy + o] = v;
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

int64_t mfm_blocks(int64_t n, int64_t n_int) {
    return (n_int + kMfmFixed - 1) / kMfmFixed + (n - n_int + kMfmFixed - 1) / kMfmFixed;
}

void launch_gather_coef(const double* x, const int32_t* perm, int64_t n, const EntryConst& c, float4* CF,
                        const GkbState* st, hipStream_t s) {
    k_gather_coef<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(x, perm, n, c, CF, st);
}

void launch_mfs_product(int trans, const float4* XS, const float4* frames, const float4* CF, const SymLayout& L,
                        const EntryConst& c, double* RowP, double* ColP, const GkbState* st, hipStream_t s) {
    if (L.nitems <= 0) return;
    if (trans)
        k_mfs<true><<<(unsigned)L.nitems, kBlock, 0, s>>>(XS, CF, L, frames, c, RowP, ColP, st);
    else
        k_mfs<false><<<(unsigned)L.nitems, kBlock, 0, s>>>(XS, CF, L, frames, c, RowP, ColP, st);
}

void launch_gather_w64(const double* x, const int32_t* perm, int64_t n, double4* XS64, const GkbState* st,
                       hipStream_t s) {
    k_gather_w64<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(x, perm, n, XS64, st);
}

void launch_mfs64_product(int trans, const double4* XS64, const SymLayout& L, const EntryConst& c, double* RowP,
                          double* ColP, const GkbState* st, hipStream_t s) {
    if (L.nitems <= 0) return;
    if (trans)
        k_mfs64<true><<<(unsigned)L.nitems, kBlock, 0, s>>>(XS64, L, c, RowP, ColP, st);
    else
        k_mfs64<false><<<(unsigned)L.nitems, kBlock, 0, s>>>(XS64, L, c, RowP, ColP, st);
}

void launch_mfs_reduce(const SymLayout& L, const double* RowP, const double* ColP, const int32_t* perm,
                       const double* shift_ptr, double shift_val, const double* z, double* y, const GkbState* st,
                       hipStream_t s) {
    if (L.n <= 0) return;
    k_mfs_reduce<<<(unsigned)((L.n + kBlock - 1) / kBlock), kBlock, 0, s>>>(L, RowP, ColP, perm, shift_ptr, shift_val,
                                                                          z, y, st);
}

int64_t mfh_block_blocks(int64_t n, int64_t n_int, int ft) {
    const int64_t fix = (kBlock / kWave) * ft * 16;
    return (n_int + fix - 1) / fix + (n - n_int + fix - 1) / fix;
}

BlockEntry block_entry(const EntryConst& c, double tmax) {
    // every term of the interior entry (kappa^2 t + 2 eps^2 + eps^2 s^2) s is
    // positive and at most kappa^2 sqrt(tmax), 2 eps^2, eps^2 (s <= 1); the
    // boundary entry sqrt(t) is at most sqrt(tmax)
    const double st = sqrt(tmax > 1.0 ? tmax : 1.0);
    double bound = fabs((double)c.k2f) * st + fabs((double)c.e2x2f) + fabs((double)c.e2f);
    if (st > bound) bound = st;
    int ex = 0;
    (void)frexp(bound, &ex);  // bound < 2^ex
    int se = 14 - ex;
    se = se > 60 ? 60 : (se < -60 ? -60 : se);
    BlockEntry b{};
    b.k2 = ldexpf(c.k2f, se);
    b.e2x2 = ldexpf(c.e2x2f, se);
    b.e2 = ldexpf(c.e2f, se);
    b.bsc = ldexpf(1.0f, se);
    b.unscale = ldexp(1.0, -se);
    return b;
}

void launch_mfh_block(int trans, int ft, const float4* XS, const float4* frames, const uint4* Vh, const float* vsc,
                      int64_t n, int64_t n_int, int S, int64_t slice_len, const BlockEntry& c, double* P,
                      int64_t ldp, hipStream_t s) {
    const int64_t fix = (kBlock / kWave) * ft * 16;
    const int64_t nb_int = (n_int + fix - 1) / fix;
    dim3 grid((unsigned)mfh_block_blocks(n, n_int, ft), (unsigned)S);
    if (ft == 1) {
        if (trans)
            k_mfh_block<false, 1><<<grid, kBlock, 0, s>>>(XS, Vh, vsc, n, n_int, nb_int, slice_len, frames, c, P, ldp);
        else
            k_mfh_block<true, 1><<<grid, kBlock, 0, s>>>(XS, Vh, vsc, n, n_int, nb_int, slice_len, frames, c, P, ldp);
    } else {
        if (trans)
            k_mfh_block<false, 2><<<grid, kBlock, 0, s>>>(XS, Vh, vsc, n, n_int, nb_int, slice_len, frames, c, P, ldp);
        else
            k_mfh_block<true, 2><<<grid, kBlock, 0, s>>>(XS, Vh, vsc, n, n_int, nb_int, slice_len, frames, c, P, ldp);
    }
}

void launch_split_block(const float* Vg, int64_t n, const float* vsc, uint4* Vh, hipStream_t s) {
    const int64_t cnt = (n + 3) / 4 * kBlkRhs;
    if (cnt <= 0) return;
    k_split_block<<<(unsigned)((cnt + kBlock - 1) / kBlock), kBlock, 0, s>>>(Vg, n, vsc, Vh);
}

void launch_block_vscale(const float* Vg, int64_t n, float* vsc, hipStream_t s) {
    k_block_vscale<<<kBlkRhs, kBlock, 0, s>>>(Vg, n, vsc);
}

void launch_fill_hash(float* Vg, int64_t count, hipStream_t s) {
    if (count <= 0) return;
    k_fill_hash<<<(unsigned)((count + kBlock - 1) / kBlock), kBlock, 0, s>>>(Vg, count);
}

void launch_gather_block(const double* X, int64_t ldx, int nrhs, const int32_t* perm, int64_t n,
                         const GkbState* st, float* Vg, hipStream_t s) {
    k_gather_block<<<(unsigned)((n * kBlkRhs + kBlock - 1) / kBlock), kBlock, 0, s>>>(X, ldx, nrhs, perm, n, st, Vg);
}

void launch_reduce_block(const double* P, int64_t ldp, int S, int64_t n, int nrhs, const int32_t* perm,
                         const double* shift, int64_t sstride, const double* z, int64_t ldz, double* y, int64_t ldy,
                         const GkbState* st, hipStream_t s) {
    k_reduce_block<<<dim3((unsigned)((n + kBlock - 1) / kBlock), nrhs), kBlock, 0, s>>>(P, ldp, S, n, perm, shift,
                                                                                       sstride, z, ldz, y, ldy, st);
}

void launch_reduce_slices(const double* P, int64_t ldp, int S, int64_t n, const int32_t* perm,
                          const double* shift_ptr, double shift_val, const double* z, double* y,
                          const GkbState* st, hipStream_t s) {
    k_reduce_slices<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(P, ldp, S, n, perm, shift_ptr,
                                                                            shift_val, z, y, st);
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
