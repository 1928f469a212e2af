// kernels.hpp -- host-side launchers of the gfx950 kernels (one stream each;
// every launch is asynchronous).  Shapes and layouts are documented at the
// kernels.
#pragma once

#include "common.hpp"

namespace mqh {

constexpr int kMaxEll = 1024;   // largest projected problem (Golub-Kahan steps)
constexpr int kMaxGrid = 4096;  // largest lambda grid
constexpr int kMfmFt = 2;       // 16-node fixed tiles per wave in the FP32-evaluated products
constexpr int kMfmFixed = (kBlock / kWave) * kMfmFt * 16;  // fixed nodes per block (128)
constexpr int kMfmChunk = kBlock;  // loop nodes staged in LDS per round (one per thread)
constexpr int kBlkRhs = 16;        // right-hand sides of a block product (lockstep Golub-Kahan runs)
constexpr int kMaxSlices = 64;     // largest split of a product's sum over nodes
constexpr int kFsBlock = 32;       // rows per block of the full SVD's one-sided block Jacobi
constexpr int kFsMaxChunks = 64;   // row chunks of the full solutions' G^T q
constexpr int kFsUpdTiles = 8;     // 64-column tiles per workgroup of the full SVD's row update

// Learned predictor network: 24 inputs, three tanh layers of width 128, 2 outputs.
constexpr int kMlpIn = 24;
constexpr int kMlpWidth = 128;
constexpr int kMlpOut = 2;
constexpr int kMlpLayers = 4;
constexpr int kMlpProbe = 10;  // Golub-Kahan steps read by the features (alpha_1..10, beta_2..11)
constexpr int64_t kMlpParams = (int64_t)kMlpIn * kMlpWidth + kMlpWidth + 2 * ((int64_t)kMlpWidth * kMlpWidth + kMlpWidth) +
                               (int64_t)kMlpWidth * kMlpOut + kMlpOut;

// Stored matrix in kTile x kTile tiles, the symmetric interior-interior and
// boundary-boundary blocks stored once (upper tiles); layout at the stored
// operator in op_kernels.hip.  Work items of a product: (R, first position,
// tile count, 0), at most kTileChunk tiles of one tile row each, rows in order.
constexpr int kTile = 128;
constexpr int64_t kTileElems = (int64_t)kTile * kTile;
constexpr int kTileChunk = 16;
struct PackedLayout {
    int64_t n, n_int;
    int32_t nti, nt;            // interior tile rows, all tile rows
    int32_t nitems, pad;        // work items of a product
    const int64_t* tile_base;   // nt + 1 entries: first stored tile of each tile row
    const int4* items;          // nitems work items
    const int32_t* item_first;  // nt + 1 entries: first item of each tile row
};

// FP32-evaluated products over unordered node pairs (each pair's t and
// rsqrt once, feeding y_i and y_j): nodes in the sorted order cut into
// blocks of kMfmFixed per class (interior blocks 0 .. nb_int-1, boundary
// blocks nb_int .. nb-1).  Work item (k, s): fixed blocks [kF, kF + F) (a
// super-row) against loop blocks [kF + s Lb, kF + (s+1) Lb) (a segment),
// only pairs of blocks b <= c (b == c: the block's own square, row sums
// only).  Each item writes F x kMfmFixed row partials and Lb x kMfmFixed
// column partials; a node's output adds the row partials of its super-row's
// items and the column partials of the items whose segment holds it.
constexpr int kSymMaxF = 8;    // fixed blocks per super-row (at most)
constexpr int kSymMaxLb = 14;  // loop blocks per segment (at most; the LDS of four workgroups per CU)
struct SymLayout {
    int64_t n, n_int;
    int32_t nb_int, nb;         // blocks of kMfmFixed nodes per class, all blocks
    int32_t F, Lb;              // fixed blocks per super-row, loop blocks per segment
    int32_t nsr, nitems;        // super-rows, work items
    const int2* items;          // (super-row, segment) of every item, in launch order (largest first)
    const int32_t* item_first;  // nsr + 1 entries: first item of each super-row
};

// Result of the parameter choice, device-resident.
struct ParamOut {
    double lambda;
    double crit;
    double rho;
    double eta;
    int32_t k;
    uint32_t flags;  // 2 = GCV minimum at a grid end, 4 = L-curve corner next to a grid end
};

// operator (op_kernels.hip)
int64_t mfm_blocks(int64_t n, int64_t n_int);
void launch_gather_coef(const double* x, const int32_t* perm, int64_t n, const EntryConst& c, float4* CF,
                        const GkbState* st, hipStream_t s);
void launch_mfs_product(int trans, const float4* XS, const float4* frames, const float4* CF, const SymLayout& L,
                        const EntryConst& c, double* RowP, double* ColP, const GkbState* st, hipStream_t s);
// FP64 products over unordered node pairs (same work items and partials as
// the FP32 form; XS64 sorted coordinates, weights written into .w by the gather)
void launch_gather_w64(const double* x, const int32_t* perm, int64_t n, double4* XS64, const GkbState* st,
                       hipStream_t s);
void launch_mfs64_product(int trans, const double4* XS64, const SymLayout& L, const EntryConst& c, double* RowP,
                          double* ColP, const GkbState* st, hipStream_t s);
void launch_mfs_reduce(const SymLayout& L, const double* RowP, const double* ColP, const int32_t* perm,
                       const double* shift_ptr, double shift_val, const double* z, double* y, const GkbState* st,
                       hipStream_t s);
// Block products over blocks of 64 ft fixed nodes (ft = 1 or 2: fixed tiles of
// 16 per wave); mfh_block_blocks gives the grid's block count.  Vh: the
// right-hand sides split for the FP16 matrix cores by launch_split_block
// (vsc: the power-of-two scale of each column, launch_block_vscale or 2^14
// for columns of at most unit size); block_entry: the entry constants scaled
// by 2^se so that no entry of a problem whose squared distances stay below
// tmax exceeds 2^14, and 2^-se.
struct BlockEntry {
    float k2, e2x2, e2, bsc;  // interior constants times 2^se, 2^se for the boundary entries
    double unscale;           // 2^-se
};
BlockEntry block_entry(const EntryConst& c, double tmax);
int64_t mfh_block_blocks(int64_t n, int64_t n_int, int ft);
void launch_mfh_block(int trans, int ft, const float4* XS, const float4* frames, const uint4* Vh, const float* vsc,
                      int64_t n, int64_t n_int, int S, int64_t slice_len, const BlockEntry& c, double* P,
                      int64_t ldp, hipStream_t s);
void launch_split_block(const float* Vg, int64_t n, const float* vsc, uint4* Vh, hipStream_t s);
void launch_block_vscale(const float* Vg, int64_t n, float* vsc, hipStream_t s);
void launch_fill_hash(float* Vg, int64_t count, hipStream_t s);
void launch_gather_block(const double* X, int64_t ldx, int nrhs, const int32_t* perm, int64_t n,
                         const GkbState* st, float* Vg, hipStream_t s);
void launch_reduce_block(const double* P, int64_t ldp, int S, int64_t n, int nrhs, const int32_t* perm,
                         const double* shift, int64_t sstride, const double* z, int64_t ldz, double* y, int64_t ldy,
                         const GkbState* st, hipStream_t s);
void launch_reduce_slices(const double* P, int64_t ldp, int S, int64_t n, const int32_t* perm,
                          const double* shift_ptr, double shift_val, const double* z, double* y,
                          const GkbState* st, hipStream_t s);
// dense row-major A (lda >= n, zero columns past n): the full SVD's work matrix
void launch_assemble(const double4* X, int64_t n, int64_t n_int, int64_t lda, const EntryConst& c, double* A,
                     hipStream_t s);
// stored tiled matrix: assembly (grid max_row_tiles x nt), product partials
// (PR: nitems x kTile, PC: stored tiles x kTile) and their reduction into
// y = op(A) x - shift z, rows of A
void launch_assemble_packed(const double4* X, const PackedLayout& L, int32_t max_row_tiles, const EntryConst& c,
                            double* A, hipStream_t s);
void launch_packed_product(int trans, const double* A, const PackedLayout& L, const double* x, double* PR, double* PC,
                           const GkbState* st, hipStream_t s);
void launch_packed_reduce(int trans, const PackedLayout& L, const double* PR, const double* PC,
                          const double* shift_ptr, double shift_val, const double* z, double* y, const GkbState* st,
                          hipStream_t s);
void launch_packed_rows(const double* A, const PackedLayout& L, int64_t row0, int64_t count, double* out,
                        hipStream_t s);
void launch_gen_rows(int prec, const void* X, int64_t n, int64_t n_int, int64_t row0, int64_t count,
                     const EntryConst& c, double* out, hipStream_t s);
void launch_eval_partial(const double4* X, const double* coef, int64_t n, const double4* E, int64_t m, int S,
                         int64_t slice_len, const EntryConst& c, double* P, int64_t ldp, hipStream_t s);

// predictor network (mlp_kernels.hip)
int64_t mlp_param_offset(int layer);
void launch_mlp_forward(const float* params, const float* x, int B, float* y, float* hidden, hipStream_t s);
void launch_mlp_backward(const float* params, const float* x, const float* hidden, const float* dy, int B,
                         float* grad, float* work, hipStream_t s);
void launch_mse(const float* y, const float* t, const float* w, int B, float* loss, float* dy, hipStream_t s);
void launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                 int32_t t, hipStream_t s);
void launch_mlp_features(const double* alpha, const double* beta, double kappa, double eps, double n, double h,
                         const float* mean, const float* stdv, float* x, hipStream_t s);

// Golub-Kahan vectors (gkb_kernels.hip)
void launch_cap_ell(GkbState* st, int32_t ell, hipStream_t s);
void launch_init_state(GkbState* st, int32_t ell, double* alpha, double* beta, hipStream_t s);
void launch_fill(double* x, int64_t n, double v, hipStream_t s);
// x[z stride + i] *= a for i < n, z < nz
void launch_scale(double* x, int64_t n, double a, int nz, int64_t stride, hipStream_t s);
int sumsq_blocks(int64_t n);
void launch_sumsq_partial(const double* x, int64_t n, double* partial, int nb, GkbState* st, hipStream_t s);
// norm of x from partial sums of squares, breakdown test, dst = x / norm
void launch_finalize_scale(const double* partial, int nparts, int kind, int32_t j, int64_t n, double* alpha,
                           double* beta, GkbState* st, const double* x, double* dst, hipStream_t s);
int gemvt_blocks(int64_t n);
// c = V^T x through block partials (gemvt_blocks(n) x m); x -= V c
void launch_gemvt(const double* V, int64_t ldn, int64_t n, int32_t m, const double* x, double* partial, double* c,
                  const GkbState* st, hipStream_t s);
int update_blocks(int64_t n);
void launch_update(const double* V, int64_t ldn, int64_t n, int32_t m, const double* c, double* x,
                   double* sumsq_partial, GkbState* st, hipStream_t s);
// x -= V c, then c = V^T x for the updated x, reading V once (partials:
// fused_cgs_blocks(n) x m); for m <= kFusedCgsMaxCols (the LDS tile within 64 KB)
constexpr int kFusedCgsMaxCols = 224;
int fused_cgs_blocks(int64_t n);
void launch_update_gemvt(const double* V, int64_t ldn, int64_t n, int32_t m, double* c, double* x,
                         double* partial, const GkbState* st, hipStream_t s);
// partial buffers of the reorthogonalisation for n rows and up to cols columns
inline int64_t cgs_partial_doubles(int64_t n, int64_t cols) {
    const int64_t b = fused_cgs_blocks(n) > gemvt_blocks(n) ? fused_cgs_blocks(n) : gemvt_blocks(n);
    return b * cols;
}
void launch_lift(const double* Z, int64_t ldz, int64_t n, int32_t ell, const int32_t* ell_ptr, const double* y,
                 double* coef, hipStream_t s, int nz = 1, Bz bz = Bz{});
// batched forms: nz slices, strides per slice as stated at the kernels
void launch_init_state_b(GkbState* st, int32_t ell, double* alpha, double* beta, int nz, Bz bz, hipStream_t s);
void launch_sumsq_partial_b(const double* x, int64_t n, double* partial, int nb, GkbState* st, int nz, Bz bz,
                            hipStream_t s);
// iperm / Vg: also write the normalised vectors into the sorted FP32
// block-product operand (both NULL: not)
void launch_finalize_scale_b(const double* partial, int nparts, int kind, int32_t j, int64_t n, double* alpha,
                             double* beta, GkbState* st, const double* x, double* dst, const int32_t* iperm,
                             float* Vg, int nz, Bz bz, hipStream_t s);
void launch_gemvt_b(const double* V, int64_t ldn, int64_t n, int32_t m, const double* x, double* partial, double* c,
                    const GkbState* st, int nz, int64_t sV, int64_t sx, int64_t sp, int64_t sc, hipStream_t s);
void launch_update_b(const double* V, int64_t ldn, int64_t n, int32_t m, const double* c, double* x,
                     double* sumsq_partial, GkbState* st, int nz, Bz bz, hipStream_t s);
void launch_update_gemvt_b(const double* V, int64_t ldn, int64_t n, int32_t m, double* c, double* x,
                           double* partial, const GkbState* st, int nz, int64_t sV, int64_t sc, int64_t sx,
                           int64_t sp, hipStream_t s);
void launch_fill_f32(float* x, int64_t n, float v, hipStream_t s);

// projected SVD (svd_kernels.hip; the QR iteration in proj_kernels.hip).
// The workspace of a problem holds svd_ws_doubles(l) doubles (l = the
// allocation's step count, also V's ld); problem z of a batch uses
// ws + z * pb.ws.  mode 0: multisection and twisted factorisations, the QR
// iteration for problems that fail the acceptance test; 1: the QR iteration
// only; 2: the fast path only.  status per problem: 0 fast path, 1 QR
// iteration converged, -1 QR iteration at its limit, 2 fast path rejected
// (mode 2 only).
constexpr int kSvdTiles = 1024;  // 32 x 32 tiles of 32: l up to kMaxEll
static_assert(kMaxEll <= 32 * 32, "Gram tile maxima sized for l <= 1024");
// Workspace of one problem (svd_ws_doubles(L) doubles; L = the allocation's l):
struct SvdWs {
    double* U;      // L x L, column j = u_j, ld L (the fallback's rotation matrix)
    double* E;      // L x L, V^T V - I, ld L
    double* d;      // L: diagonal of B
    double* e;      // L: superdiagonal of B (L - 1 used)
    double* g;      // L: beta_1 e_1 after the left rotations
    double* lam;    // L: s_j^2
    double* h;      // L: u_j^T g
    double* res;    // L: residual of triple j over its bound
    double* tmax;   // 2 * kSvdTiles: tile maxima of |V^T V - I| and |U^T U - I|
    double* misc;   // [0] eigenvalue bound, [1] pivot floor
    int32_t* flag;  // [0] setup or values unresolved, [1] fallback needed
};

__device__ __forceinline__ SvdWs svd_ws(double* base, int32_t L) {
    const int64_t LL = (int64_t)L * L;
    SvdWs w;
    w.U = base;
    w.E = base + LL;
    w.d = base + 2 * LL;
    w.e = w.d + L;
    w.g = w.e + L;
    w.lam = w.g + L;
    w.h = w.lam + L;
    w.res = w.h + L;
    w.tmax = w.res + L;
    w.misc = w.tmax + 2 * kSvdTiles;
    w.flag = reinterpret_cast<int32_t*>(w.misc + 8);
    return w;
}
constexpr size_t svd_ws_doubles(int32_t l) {
    return 2 * (size_t)l * (size_t)l + 6 * (size_t)l + 2 * (size_t)kSvdTiles + 16;
}
void launch_bidiag_svd(const double* alpha, const double* beta, int32_t l, const int32_t* l_ptr, double* ws,
                       double* sv, double* ftil, double* V, int64_t ldv, int32_t* status, int mode, hipStream_t s,
                       int nz = 1, ProjBatch pb = ProjBatch{});
void launch_bidiag_qr(const double* alpha, const double* beta, int32_t l, const int32_t* l_ptr, double* ws,
                      double* sv, double* ftil, double* V, int64_t ldv, int32_t* status, bool flagged_only,
                      hipStream_t s, int nz, ProjBatch pb);
// The multisection path without its setup, for one problem whose workspace
// already holds B (d, e), g, the bounds and the flags: values, vectors, Gram
// matrices, acceptance test (status 0 or 2) and the correction of V.
void launch_msvd_core(int32_t l, double* ws, double* sv, double* ftil, double* V, int64_t ldv, int32_t* status,
                      hipStream_t s);

// Projected problem of the block Golub-Kahan path by a band reduction of C^T
// (band_kernels.hip, band.hpp).  Sizes: N = ell s columns of C, Mc = N + s
// rows; the chase holds C^T in LDS (band_fits), T = steps of its schedule.
constexpr int kBandLdsDoubles = 20160;  // N band::width(s) at most: 157.5 KiB of LDS
constexpr int kBandDataDoubles = 7200;  // (N + s)(s + 1) at most
constexpr int kBandMaxN = kMaxEll;
constexpr int kBandMaxSteps = 4096;
bool band_fits(int N, int s);
int band_ntasks(int N, int s, int* nsteps);  // reflectors per side; *nsteps = T
void launch_band_chase(const double* C, int64_t ldc, int N, int s, int T, double* RR, double* LL, int32_t* toff,
                       double* d, double* e, hipStream_t st);
void launch_band_data(const double* E1, int N, int s, const double* RR, const int32_t* toff, int T, const double* d,
                      const double* e, double* ws, double* G, double* fn2, hipStream_t st);
void launch_band_mm(int mode, const double* A, int64_t lda, int N, int s, const double* X, const double* X2,
                    const double* sv, const ParamOut* po, double* out, hipStream_t st);
void launch_band_solve(const double* Yh, int N, int s, const double* LL, const int32_t* toff, int T, double* Y,
                       hipStream_t st);

// projected problem (proj_kernels.hip)
void launch_param_choice(const double* sv, const double* ft, int32_t l, const int32_t* l_ptr, int32_t method,
                         int32_t rule, int32_t J, double lambda_fixed, int32_t k_fixed, double omega, double* curve,
                         ParamOut* out, hipStream_t s, int nz = 1, ProjBatch pb = ProjBatch{});
void launch_lsqr(const double* alpha, const double* beta, int32_t l, const int32_t* l_ptr, int64_t n, int32_t rule,
                 int32_t k_fixed, double* rho, double* eta, ParamOut* out, double* y, int32_t l_max, hipStream_t s, int nz = 1, ProjBatch pb = ProjBatch{});
void launch_proj_solution(const double* sv, const double* ft, const double* V, int64_t ldv, int32_t l,
                          const int32_t* l_ptr, int32_t method, double lambda, int32_t k, const ParamOut* po,
                          double* y, int32_t l_max, hipStream_t s, int nz = 1, ProjBatch pb = ProjBatch{});

// Full SVD (full_kernels.hip)
void launch_fs_setf(double* G, int64_t ldg, int64_t n, const double* f, hipStream_t s);
// pair_ok (per schedule slot) and blk_stamp (per block): the bookkeeping that
// lets a round leave out pairs whose rows have not changed since they were
// last found orthogonal (same != 0: the row order is that of the previous
// sweep); slot0 = round x pairs, g = the global round.
void launch_fs_gram(const double* G, int64_t ldg, int64_t ncol, const int32_t* rowidx, const int2* pairs, int npairs,
                    int S, int64_t chunk, double* Pg, const int32_t* pair_ok, const int32_t* blk_stamp, int64_t slot0,
                    int same, hipStream_t s);
void launch_fs_eig(const double* Pg, int S, int npairs, double tol, double inv_f, int max_inner, double* Pout,
                   int32_t* flag, double* off, const int2* pairs, int32_t* pair_ok, int32_t* blk_stamp, int64_t slot0,
                   int32_t g, int same, hipStream_t s);
void launch_fs_update(double* G, int64_t ldg, int64_t ncol, const int32_t* rowidx, const int2* pairs, int npairs,
                      const double* Pin, const int32_t* flag, hipStream_t s);
// out[0] = max off, out[1] = number of entries above tol
void launch_fs_maxoff(const double* off, int64_t count, double tol, double* out, hipStream_t s);
void launch_fs_norms(const double* G, int64_t ldg, int64_t rows, int64_t n, double* sig, double* fh, hipStream_t s);
void launch_fs_rank(const double* sig, const double* fh, int64_t n, int32_t* rank, double* sv, double* fs,
                    int32_t* order, hipStream_t s);
// Parameter choice for nz data columns at once (one workgroup each): column
// z's sorted data at fs + z vs, ||f_z||^2 at fnorm2v[z] (device), its tail
// buffer at tail + z (n + 1), its choice at out + z.
void launch_full_param(const double* sv, const double* fs, int64_t n, int64_t rcap, const double* fnorm2v,
                       int64_t vs, int32_t method, int32_t rule, int32_t J, double lambda_fixed, int32_t k_fixed,
                       double* tail, ParamOut* out, int nz, hipStream_t s);
// Solutions: preconditioned conjugate gradients on (G G^T + lambda^2 I) y = f^
// (Tikhonov) or G_k G_k^T y = f^_k (TSVD), x = G^T y, for nz data columns at
// once: vectors of column z at + z vs, its scalars at pc + 4 z ([0] q^T B q,
// [2], [3] r^T D^-1 r of alternate iterations), its choice at po + z.  part:
// nz x fs_gemvt_chunks(n) x n doubles.
int fs_gemvt_chunks(int64_t n);
void launch_fs_gemvt(const double* G, int64_t ldg, int64_t n, const double* q, int64_t vs, double* part, double* x,
                     int nz, hipStream_t s);
void launch_fs_pcg_start(const double* sig, const double* fh, const int32_t* rank, int64_t n, int32_t method,
                         int64_t rcap, const ParamOut* po, int64_t vs, double* y, double* r, double* q, double* t,
                         double* pc, int slot, int nz, hipStream_t s);
void launch_fs_pcg_iter(const double* G, int64_t ldg, int64_t n, const double* sig, const int32_t* rank,
                        int32_t method, int64_t rcap, const ParamOut* po, int64_t vs, double* pc, int cur, int nxt,
                        double* y, double* r, const double* q, double* w, double* t, double* part, double* x, int nz,
                        hipStream_t s);
// ||A x - f|| = ||G x - f^|| and ||x|| of the returned solutions into po[z].rho, po[z].eta.
void launch_fs_solution_norms(const double* G, int64_t ldg, int64_t n, const double* x, const double* fh, int64_t vs,
                              double* t, double* w, double* pc, ParamOut* po, int nz, hipStream_t s);
void launch_fs_pcg_dir(const double* sig, const int32_t* rank, int64_t n, int32_t method, int64_t rcap,
                       const ParamOut* po, int64_t vs, const double* pc, int cur, int nxt, const double* r, double* q,
                       int nz, hipStream_t s);
// out[z vs + i] = G[i][col0 + z] for i < rows, z < nz (data columns of the work matrix)
void launch_fs_col(const double* G, int64_t ldg, int64_t rows, int64_t col0, int64_t vs, double* out, int nz,
                   hipStream_t s);
// fs[z vs + rank[i]] = fh[z vs + i]: data columns in descending singular-value order
void launch_fs_gather(const int32_t* rank, const double* fh, int64_t n, int64_t vs, double* fs, int nz, hipStream_t s);

// Block Golub-Kahan (block_kernels.hip): c = V^T P through split-K partials
// (part: blk_chunks(n, m) x m x 16, c: m x 16, row col = c + 16 col), P -= V c
// (sub = 1) or P = V c (sub = 0; V may be P), one pass of (shifted) Cholesky
// QR on a 16 x 16 Gram matrix.
int blk_chunks(int64_t n, int32_t m, int64_t* chunk);
void launch_blk_gemvt(const double* V, int64_t ldv, int64_t n, int32_t m, const double* P, int64_t ldp, int32_t s,
                      double* part, double* c, hipStream_t st);
void launch_blk_update(const double* V, int64_t ldv, int64_t n, int32_t m, const double* c, int64_t cs, int64_t ks,
                       double* P, int64_t ldp, int32_t s, int32_t sub, hipStream_t st);
void launch_blk_chol(const double* G, int32_t s, int64_t n, int32_t shifted, double* Rinv, double* Racc,
                     int32_t* status, hipStream_t st);
void launch_blk_eye(double* Racc, int32_t* status, hipStream_t st);
// Device state of a block Golub-Kahan run: the breakdown test of every QR
// without a host round trip.
struct BlkState {
    int32_t stopped, ell_done, flag, invalid;
    double scale;
};
void launch_blk_check(const double* Racc, const int32_t* status, int32_t s, int32_t kind, int32_t j, double tau,
                      BlkState* bs, double* C, int64_t ldc, double* E1, double* mat, hipStream_t st);
// G (zero) <- [C | (E1; 0)]: the Jacobi route's work matrix from the device copies of C and E1
void launch_blk_fill_g(const double* C, int64_t ldc, int64_t m, int64_t ls, const double* E1, int32_t s, double* G,
                       int64_t ldg, hipStream_t st);

// Measurement helpers (peak_kernels.hip): peak_blocks() workgroups of kBlock
// threads; the copy moves count doubles (count even, x and y 16-byte aligned).
int peak_blocks();
void launch_peak_copy(const double* x, double* y, int64_t count, hipStream_t s);
void launch_peak_read(const double* x, int64_t count, double* out, hipStream_t s);
void launch_peak_fma32(float* out, int iters, hipStream_t s);
void launch_peak_fma64(double* out, int iters, hipStream_t s);
void launch_peak_mfma64(double* out, int iters, hipStream_t s);
void launch_peak_rsq(float* out, int iters, int mix, hipStream_t s);
void launch_peak_mfma_bf16(float* out, int iters, hipStream_t s);
double peak_fma_ops(int iters);
double peak_mfma_flops(int iters);
double peak_mfma_bf16_flops(int iters);

}  // namespace mqh
