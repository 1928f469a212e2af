/*
 * mqhelm.h -- C ABI of the MI355X (gfx950) GKB / Ine-TSVD / HKT solver for
 * multiquadric-RBF Kansa collocation of the 3-D Helmholtz problem.
 *
 * Paper: M. El Guide, K. Jbilou, K. Lachhab, D. Ouazar, "Efficient
 * Krylov-Regularization Solvers for Multiquadric RBF Discretizations of the
 * 3D Helmholtz Equation" (arXiv 2511.09798).
 *
 * Problem (Section 2.1):  Lap u + kappa^2 u = f in Omega, u = g on its boundary.
 * Unknowns: coefficients c of u(X) = sum_j c_j phi(|X - X_j|) with the
 * multiquadric phi(r) = sqrt(1 + eps^2 r^2) (eq. (3)) centred at the nodes.
 * Kansa matrix A (N x N, eqs. (8), (10), (11)):
 *   interior rows i < N_I :  A_ij = Lap phi(r_ij) + kappa^2 phi(r_ij),
 *                            Lap phi(r) = eps^2 (3 + 2 eps^2 r^2) / (1 + eps^2 r^2)^{3/2};
 *   boundary rows i >= N_I:  A_ij = phi(r_ij)   (Dirichlet data);
 * right-hand side f = [f_I; g_B].
 *
 * Conventions shared by every call
 * --------------------------------
 * - Node arrays are row-major n x 3 float64 (x, y, z interleaved).  The node
 *   (= centre = coefficient) order is [interior; boundary].
 * - All other arrays are contiguous float64 (int32 where stated).
 * - Pointers are host pointers unless the call's flags carry
 *   MQH_FLAG_DEVICE_PTRS, in which case every array argument of that call is
 *   a device pointer on the problem's device (e.g. a torch tensor's data_ptr()).
 * - The caller owns every array it passes.  Inputs are read during the call
 *   (host inputs are copied); outputs are written before the call returns
 *   (device outputs: written in stream order on the call's stream; the call
 *   synchronises that stream before returning).
 * - Return value: MQH_OK (0); a negative error (outputs untouched, any
 *   *info still filled); or a positive warning (outputs valid).  No C++
 *   exception or abort crosses this interface.  mqh_last_error() returns a
 *   thread-local message for the last failure.
 * - A problem handle is used by one host thread at a time; calls on one
 *   handle are serialised on its stream.
 */
#ifndef MQHELM_H
#define MQHELM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MQH_VERSION 10700 /* 1.7.0 */

/* ---- status codes ---- */
#define MQH_OK 0
#define MQH_EINVAL (-1)   /* bad argument: NaN/Inf input, n <= 0, eps <= 0, ell < 1, ell > n or > MQH_MAX_ELL, ... */
#define MQH_ENOMEM (-2)   /* device allocation failed (e.g. the stored matrix does not fit), or it would take
                             the library past the cap set by the environment variable MQH_DEVICE_MEM_CAP
                             (bytes; read at every allocation; unset or empty: no cap) */
#define MQH_EDEVICE (-3)  /* a HIP runtime call or kernel launch failed */
#define MQH_WBREAKDOWN 1  /* Golub-Kahan stopped early (ell_done < ell); outputs valid for ell_done steps */
#define MQH_WEDGE 2       /* chosen lambda sits at an end of the search grid */
#define MQH_WNOCONV 3     /* full SVD: the Jacobi sweeps stopped at their limit (results of the last sweep),
                             or the full solution's iteration at its cap (MQH_INFO_SOLVE_NOCONV) */

/* ---- operator modes (how A enters the products) ---- */
#define MQH_OP_STORED_FP64 0   /* A assembled once in HBM, FP64 products.  Stored in 128 x 128 tiles;
                                  the interior-interior and boundary-boundary blocks of A are symmetric
                                  (their entries depend on |X_i - X_j| only) and are stored once, so A
                                  takes about 8 (N^2 - (N_I^2 + N_B^2) / 2) bytes (53 GB instead of 80 GB
                                  at N = 100 000, N_I = 80 000) */
#define MQH_OP_MATFREE_FP64 1  /* entries regenerated inside every product, FP64 throughout */
#define MQH_OP_MATFREE_FP32 2  /* entries evaluated in FP32 (the squared distances on the matrix
                                  cores, FP32-accurate), accumulated in FP64 */

/* ---- methods and parameter-choice rules ---- */
#define MQH_METHOD_INE_TSVD 0 /* Algorithm 2 */
#define MQH_METHOD_HKT 1      /* Algorithm 4 */
#define MQH_METHOD_LSQR 2     /* LSQR iterate with early stopping (Section 3.4), see mqh_lsqr */
#define MQH_RULE_GCV 0        /* eq. (30) (HKT) / projected TSVD-GCV (Ine-TSVD) / Krylov GCV (LSQR) */
#define MQH_RULE_LCURVE 1     /* maximum curvature of (log rho, log eta) on the grid / discrete (LSQR) */
#define MQH_RULE_FIXED 2      /* lambda = lambda_fixed (HKT) / k = k_trunc (Ine-TSVD, LSQR) */
#define MQH_RULE_WGCV 3       /* weighted GCV, trace term scaled by gcv_weight (HKT, Ine-TSVD) */

/* ---- call flags ---- */
#define MQH_FLAG_DEVICE_PTRS 1u     /* array arguments are device pointers */
#define MQH_FLAG_TIME_PRODUCTS 2u   /* mqh_solve: time every product kernel with HIP events on the problem's stream */
#define MQH_FLAG_FIXED_SHAPES 4u    /* mqh_problem_create: launch shapes of the block products from the size
                                       alone instead of timing the candidates on first use (results then
                                       do not depend on timing noise; see mqh_gkb_multi) */
#define MQH_FLAG_GRAPH 8u           /* mqh_solve_multi / mqh_solve_sweep: run each group's Golub-Kahan loop
                                       as a captured HIP graph, kept with the problem and replayed while
                                       the group size, ell, reorth and row scaling stay the same (ignored
                                       with MQH_FLAG_TIME_PRODUCTS) */
#define MQH_FLAG_ROW_SCALE 16u      /* mqh_apply, mqh_apply_multi, mqh_matrix_rows, mqh_gkb, mqh_gkb_multi:
                                       the operator is D A with D = diag(A)^-1 (see mqh_solve_opts.row_scale);
                                       mqh_gkb / mqh_gkb_multi also scale f to D f */

#define MQH_FLAG_PROJ_QR 32u         /* mqh_proj_svd: the implicit QR iteration only (the fast path's fallback) */
#define MQH_FLAG_PROJ_NO_FALLBACK 64u /* mqh_proj_svd: the fast path only; MQH_EDEVICE if it fails its acceptance
                                        test (for tests of the fast path) */
#define MQH_FLAG_BLOCK_JACOBI 128u    /* mqh_solve_block: the projected problem through the one-sided Jacobi full
                                        SVD only (the band path's fallback) */

/* ---- info flags ---- */
#define MQH_INFO_BREAKDOWN 1u
#define MQH_INFO_GCV_AT_EDGE 2u
#define MQH_INFO_LCURVE_AT_EDGE 4u
#define MQH_INFO_SOLVE_NOCONV 8u  /* full solve: the conjugate gradients stopped at their cap above their tolerance */
#define MQH_INFO_SVD_QR 16u       /* the projected SVD failed the fast path's acceptance test and was computed by
                                     the implicit QR iteration (same outputs to rounding, about 100 times slower) */
#define MQH_INFO_BLOCK_JACOBI 32u /* mqh_solve_block: the projected problem went through the Jacobi full SVD
                                     (too large for the band reduction, its SVD failed the acceptance test, or
                                     MQH_FLAG_BLOCK_JACOBI) */

/* Largest number of Golub-Kahan steps a solve accepts (projected problem size). */
#define MQH_MAX_ELL 1024
#define MQH_FULL_MAX_N 32768  /* largest n of the full-SVD reference path (8.6 GB work matrix) */
#define MQH_FULL_CG_MAX 1024  /* conjugate-gradient iterations of a full solution at most */
#define MQH_BLOCK_MAX_DIM 4096  /* (ell + 1) nrhs at most for the block Golub-Kahan calls */
#define MQH_BLOCK_RHS 16 /* right-hand sides run in lockstep per group (mqh_gkb_multi, mqh_solve_multi) */

/* ---- learned predictor network: 24 inputs, three tanh layers of width 128, 2 outputs ---- */
#define MQH_MLP_IN 24
#define MQH_MLP_WIDTH 128
#define MQH_MLP_OUT 2
#define MQH_MLP_PROBE 10      /* Golub-Kahan steps read by the features */
#define MQH_MLP_NPARAMS 36482 /* 24*128+128 + 2*(128*128+128) + 128*2+2 */

typedef struct mqh_problem mqh_problem;

/* Options of a solve (Algorithms 2 and 4; Section 3). */
typedef struct {
    int32_t ell;          /* Golub-Kahan steps, 1 <= ell <= min(n, MQH_MAX_ELL) */
    int32_t reorth;       /* 1: full reorthogonalisation (classical Gram-Schmidt twice); 0: none */
    int32_t method;       /* MQH_METHOD_* */
    int32_t rule;         /* MQH_RULE_* */
    int32_t k_trunc;      /* Ine-TSVD / LSQR with MQH_RULE_FIXED: rank / iteration k (1..ell) */
    int32_t n_grid;       /* lambda grid size J (>= 3; 0 -> 200) */
    double lambda_fixed;  /* HKT with MQH_RULE_FIXED: lambda >= 0 */
    uint32_t flags;       /* MQH_FLAG_* for this call */
    int32_t row_scale;    /* 0: the paper's system A c = f (eq. (11)).  1: the rows scaled by
                             D = diag(A)^-1 (interior rows divided by 3 eps^2 + kappa^2, the value
                             of L phi at r = 0; boundary rows by 1), i.e. the method runs on
                             (D A) c = D f (not in the paper: an opt-in equilibration of the two
                             row classes).  Every Golub-Kahan scalar, Ritz value, residual norm
                             and GCV value then refers to the scaled system; the coefficients are
                             its regularised solution.  mqh_solve, mqh_solve_multi and
                             mqh_solve_sweep; the block, full-SVD and learned solves take 0 only.
                             A stored matrix is kept assembled for the scaling of the last call
                             that used it: a call with the other scaling assembles it again. */
    double gcv_weight;    /* MQH_RULE_WGCV: weight omega in (0, 1] of the trace term (1 -> plain GCV) */
} mqh_solve_opts;

/* Outcome of a solve. */
typedef struct {
    int32_t ell_done;      /* Golub-Kahan steps kept (< ell after a breakdown) */
    int32_t k_chosen;      /* Ine-TSVD rank / LSQR stopping index (0 for HKT) */
    double lambda_chosen;  /* HKT lambda (0 for Ine-TSVD) */
    double crit;           /* GCV value at the choice, or curvature for the L-curve rule */
    double resid_norm;     /* projected residual norm rho_l at the choice (eq. (28); LSQR: rho_k) */
    double sol_norm;       /* projected solution norm eta_l = ||y|| (eq. (29); LSQR: eta_k) */
    uint32_t flags;        /* MQH_INFO_* */
    int32_t reserved;
    double t_ms[8];        /* [0] data upload, [1] Golub-Kahan loop, [2] projected SVD,
                              [3] parameter choice + projected solution, [4] lift,
                              [5] total (upload to results on host),
                              [6] summed time of the ell A^T-product kernels,
                              [7] summed time of the ell A-product kernels
                              ([6],[7] only with MQH_FLAG_TIME_PRODUCTS; the split-K
                              reduction that follows a product is not included) */
} mqh_solve_info;

/* Learned predictor of the regularisation parameter and the stopping index
 * (used by mqh_solve_learned).  The network reads the standardised features
 *   (log alpha_1..alpha_10, log beta_2..beta_11, log kappa, log eps, log n, log h)
 * and predicts, after de-standardisation (out = y * out_std + out_mean),
 *   out[0] = log(lambda / alpha_1)   out[1] = ell_stop / ell. */
typedef struct {
    const float* params;          /* MQH_MLP_NPARAMS device floats, layer by layer: W (out x in, row-major), b */
    float in_mean[MQH_MLP_IN];    /* feature standardisation: (x - in_mean) / in_std */
    float in_std[MQH_MLP_IN];
    float out_mean[MQH_MLP_OUT];
    float out_std[MQH_MLP_OUT];
    double h;                     /* fill distance of the node set, (domain volume / n)^(1/3) */
    int32_t ell_step;             /* the predicted stop index is rounded up to a multiple of this (>= 1) */
    int32_t reserved;
    double judge_ratio;           /* 0: GCV only reports; >= 1: also veto lambda_net when
                                     GCV(lambda_net) > judge_ratio * min GCV */
} mqh_predictor;

/* What the learned solve did. */
typedef struct {
    int32_t ell_pred;             /* Golub-Kahan steps run (predicted stop index) */
    int32_t used_net_lambda;      /* 1: the network's lambda, 0: the GCV fallback */
    double lambda_net;            /* alpha_1 exp(out[0]) */
    double lambda_gcv;            /* the GCV choice at ell_pred (the judge) */
    double gcv_net;               /* GCV_l(lambda_net) */
    double gcv_min;               /* GCV_l(lambda_gcv) */
    double out[MQH_MLP_OUT];      /* de-standardised network outputs */
} mqh_learned_info;

int mqh_version(void);
const char* mqh_status_str(int status);
const char* mqh_last_error(void);

/*
 * Create a problem: copies the nodes to the device and, for
 * MQH_OP_STORED_FP64, assembles A there (eqs. (8), (10)).
 *   x_int    n_int x 3 interior nodes (may be NULL when n_int == 0)
 *   x_bnd    n_bnd x 3 boundary nodes (may be NULL when n_bnd == 0)
 *   kappa    wavenumber (finite); eps > 0 shape parameter (eq. (3))
 *   op_mode  MQH_OP_*
 *   stream   hipStream_t to run on, or NULL for a stream the library creates
 *   flags    MQH_FLAG_DEVICE_PTRS if x_int / x_bnd are device pointers,
 *            MQH_FLAG_FIXED_SHAPES (see there)
 * Errors: MQH_EINVAL (n_int < 0, n_bnd < 0, n = 0, non-finite input,
 * eps <= 0, unknown mode), MQH_ENOMEM (stored matrix or buffers do not fit),
 * MQH_EDEVICE.  On error *out is set to NULL.
 */
int mqh_problem_create(const double* x_int, int64_t n_int, const double* x_bnd, int64_t n_bnd, double kappa,
                       double eps, int32_t op_mode, void* stream, uint32_t flags, mqh_problem** out);

/* Free every device buffer of the problem (NULL is accepted). */
int mqh_problem_destroy(mqh_problem* p);

/* Problem size n = n_int + n_bnd, or -1 for NULL. */
int64_t mqh_problem_size(const mqh_problem* p);

/* Bytes of device memory the library holds at this moment, over all problems
 * and devices (what MQH_DEVICE_MEM_CAP is compared with). */
int64_t mqh_device_bytes(void);

/*
 * One product of the Golub-Kahan recurrence (Algorithm 1, steps 3 and 5):
 *   trans = 0:  y = A x - shift * z
 *   trans = 1:  y = A^T x - shift * z
 * x, z, y have length n; z may be NULL (then the shift is ignored).  y must
 * not alias x.  The product runs in the problem's operator mode.
 */
int mqh_apply(mqh_problem* p, int32_t trans, const double* x, double shift, const double* z, double* y,
              uint32_t flags);

/*
 * Rows [row0, row0 + count) of A as the problem's operator mode sees them
 * (the stored matrix, or entries generated the way the matrix-free products
 * generate them; in MQH_OP_MATFREE_FP32 the entries by the direct FP32
 * formula, which the products reproduce up to a few FP32 roundings), written
 * row-major count x n to out.  For checks of the entry generator (eq. (8)).
 */
int mqh_matrix_rows(mqh_problem* p, int64_t row0, int64_t count, double* out, uint32_t flags);

/*
 * Golub-Kahan bidiagonalisation (Algorithm 1) started from f (length n),
 * ell steps, with full reorthogonalisation (classical Gram-Schmidt twice,
 * applied before each norm) when reorth = 1.
 * Outputs (any may be NULL):
 *   W      n x (ell+1) column-major (column k = w_{k+1}), leading dimension n
 *   Z      n x ell column-major (column k = z_{k+1})
 *   alpha  ell values alpha_1..alpha_ell
 *   beta   ell+1 values beta_1 = ||f|| .. beta_{ell+1}
 *   ell_done  host int32: steps kept.  A step stops when alpha_j or
 *             beta_{j+1} <= n * DBL_EPSILON * max(alpha_i, beta_{i+1} so far);
 *             an alpha breakdown keeps j-1 steps, a beta breakdown keeps j
 *             steps with beta_{j+1} = 0.  Entries past ell_done are zero.
 * Returns MQH_WBREAKDOWN when ell_done < ell or beta_{ell+1} = 0 was forced.
 */
int mqh_gkb(mqh_problem* p, const double* f, int32_t ell, int32_t reorth, double* W, double* Z, double* alpha,
            double* beta, int32_t* ell_done, uint32_t flags);

/*
 * SVD of the (ell+1) x ell lower bidiagonal C_ell with diagonal
 * alpha_1..alpha_ell and subdiagonal beta_2..beta_{ell+1} (Algorithm 2
 * step 2, Algorithm 4 step 2), computed on the device:
 *   sv    ell singular values, descending
 *   ftil  ell+1 projected data f~ = U~^T (beta_1 e_1) (f~_{ell+1} is the
 *         least-squares residual of min ||C y - beta_1 e_1||)
 *   V     ell x ell column-major right singular vectors (column i = v~_i),
 *         may be NULL
 * alpha (ell) and beta (ell+1, beta[0] = beta_1) are inputs.  Signs of
 * singular vectors are arbitrary (f~_i and v~_i flip together).
 * Method: Givens rotations take C_ell to an upper bidiagonal B; each
 * singular value by multisection on the inertia of B^T B - x I (differential
 * qd form, high relative accuracy), each pair of vectors by twisted
 * factorisations of B^T B - s^2 I and B B^T - s^2 I, then a symmetric
 * orthogonalisation.  An acceptance test (Gram matrices within 1e-9 of I,
 * residuals ||B v - s u||, ||B^T u - s v|| within 1e-9 s) guards the result;
 * a problem that fails it (tight clusters, exactly singular B) is computed
 * again by the implicit QR iteration with the zero-shift sweeps of Demmel and
 * Kahan.  flags: MQH_FLAG_DEVICE_PTRS, MQH_FLAG_PROJ_QR, MQH_FLAG_PROJ_NO_FALLBACK.
 * stream: hipStream_t or NULL (default stream).  1 <= ell <= MQH_MAX_ELL.
 * Errors: MQH_EINVAL (arguments, non-finite host input, both PROJ flags),
 * MQH_EDEVICE (QR iteration at its limit; fast path rejected under
 * MQH_FLAG_PROJ_NO_FALLBACK).
 */
int mqh_proj_svd(const double* alpha, const double* beta, int32_t ell, double* sv, double* ftil, double* V,
                 void* stream, uint32_t flags);

/*
 * mqh_proj_svd without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same computation and outputs as mqh_proj_svd
 * (bit for bit); every array is a device pointer on the current device and
 * stream runs on that device (NULL: the default stream).  V may be NULL.
 * The workspace (the left vectors, a Gram matrix and the bidiagonal's
 * bookkeeping for ell = MQH_NOALLOC_MAX_ELL, V when V is NULL, a status
 * word) is a fixed array of MQH_NOALLOC_SCRATCH_BYTES in the library's
 * device memory, one per GPU, held until the process ends; hence
 * 1 <= ell <= MQH_NOALLOC_MAX_ELL (MQH_EINVAL beyond).  All calls on one GPU
 * share that array: calls that overlap in time on one GPU (other streams or
 * host threads) race and must be serialised by the caller.  The call
 * synchronises the stream to read the status word (MQH_EDEVICE if the QR
 * iteration did not converge).  No hipMalloc, hipFree or allocating library
 * routine is called.
 */
#define MQH_NOALLOC_MAX_ELL 512
#define MQH_NOALLOC_SCRATCH_BYTES 6332800 /* 8 (3 * 512 * 512 + 6 * 512 + 2 * 1024 + 48): about 6 MiB */
int mqh_proj_svd_noalloc(const double* alpha, const double* beta, int32_t ell, double* sv, double* ftil, double* V,
                         void* stream);

/*
 * Parameter choice on the projected problem (Section 3.2-3.3), on the device.
 *   method HKT:      rule GCV    -> lambda* = argmin GCV_l (eq. (30)) on a
 *                                   log grid of n_grid points over
 *                                   [max(s_l, 16 eps_mach s_1), s_1], then
 *                                   golden-section refinement of log lambda
 *                                   in the bracketing cells;
 *                    rule WGCV   -> the same with the weighted GCV
 *                                   rho_l^2 / ((l+1) - w sum_i phi_i)^2,
 *                                   w = gcv_weight in (0, 1];
 *                    rule LCURVE -> grid point of maximum signed curvature
 *                                   of (log rho_l, log eta_l), end points excluded;
 *                    rule FIXED  -> lambda_fixed.
 *   method INE_TSVD: rule FIXED  -> k = k_trunc; otherwise k* = argmin over
 *                                   k = 1..max(1, ell/2) of
 *                                   (sum_{i>k} f~_i^2 + f~_{l+1}^2)/((l+1)-w k)^2
 *                                   (w = gcv_weight for WGCV, else 1).
 * Inputs sv (ell, descending), ftil (ell+1).  Outputs (host scalars; NULL
 * allowed): lambda, k, crit (GCV value / curvature at the choice),
 * info_flags (MQH_INFO_*); curve (n_grid values of the criterion on the
 * grid, pointer kind per flags, NULL allowed).
 * Returns MQH_WEDGE when the choice is at a grid end.
 */
int mqh_param_choice(const double* sv, const double* ftil, int32_t ell, int32_t method, int32_t rule,
                     int32_t n_grid, double lambda_fixed, int32_t k_trunc, double gcv_weight, double* lambda,
                     int32_t* k, double* crit, uint32_t* info_flags, double* curve, void* stream, uint32_t flags);

/*
 * LSQR iterates on the projected problem and their stopping index
 * (Section 3.4), on the device.  The k-th LSQR iterate is Z_k y_k with
 * y_k = argmin ||C_k y - beta_1 e_1|| (C_k the leading (k+1) x k block of
 * C_ell); rho_k = ||C_k y_k - beta_1 e_1|| = ||A Z_k y_k - f|| and
 * eta_k = ||y_k|| = ||Z_k y_k|| (eq. (26), orthonormal bases).
 *   rule GCV    -> k* = argmin rho_k^2 / (n - k)^2 over k = 1..min(ell, n-1)
 *                  (the k-th iterate's influence matrix is a rank-k
 *                  projector), ties to the smaller k;
 *   rule LCURVE -> corner of the discrete L-curve p_k = (log rho_k,
 *                  log eta_k): maximum signed Menger curvature of
 *                  (p_{k+1}, p_k, p_{k-1}) over k = 2..ell-1, ties to the
 *                  smaller k; MQH_INFO_LCURVE_AT_EDGE (and MQH_WEDGE) when
 *                  the corner is k = 2 or ell-1 or no triple qualifies
 *                  (then k* = ell);
 *   rule FIXED  -> k* = k_trunc (1..ell).
 * Inputs alpha (ell), beta (ell+1, beta[0] = beta_1), n = rows of A.
 * Outputs: k, crit (GCV value / curvature at k*; host scalars, NULL
 * allowed), info_flags, y (ell entries: y_k* then zeros), rho and eta
 * (ell entries each, NULL allowed).  1 <= ell <= MQH_MAX_ELL, n > ell - 1.
 */
int mqh_lsqr(const double* alpha, const double* beta, int32_t ell, int64_t n, int32_t rule, int32_t k_trunc,
             int32_t* k, double* crit, uint32_t* info_flags, double* y, double* rho, double* eta, void* stream,
             uint32_t flags);

/*
 * Projected solution (Algorithm 2 step 5 / Algorithm 4 step 8 in SVD form):
 *   HKT:      y = sum_i s_i / (s_i^2 + lambda^2) f~_i v~_i
 *   Ine-TSVD: y = sum_{i<=k} f~_i / s_i v~_i
 * sv (ell), ftil (ell+1), V (ell x ell column-major) in; y (ell) out.
 */
int mqh_proj_solution(const double* sv, const double* ftil, const double* V, int32_t ell, int32_t method,
                      double lambda, int32_t k, double* y, void* stream, uint32_t flags);

/*
 * Lift coef = Z y (Algorithm 2 step 5, Algorithm 4 last step): Z is
 * n x ell column-major with leading dimension n, y has ell entries,
 * coef n entries.
 */
int mqh_lift(const double* Z, int64_t n, int32_t ell, const double* y, double* coef, void* stream,
             uint32_t flags);

/*
 * Whole solve (Algorithm 2 or 4, or LSQR with early stopping, Section 3.4):
 * f = [f_int (n_int); g_bnd (n_bnd)] -> Golub-Kahan (ell steps) -> projected
 * SVD -> parameter choice -> projected solution -> coef = Z y (n).  For
 * MQH_METHOD_LSQR the SVD runs only when ritz_sv is requested and the
 * projected steps are those of mqh_lsqr.  Optional outputs (NULL allowed): gkb_alpha
 * (ell), gkb_beta (ell+1), ritz_sv (ell); entries past info->ell_done are 0.
 * info may be NULL.  opts->flags decides the pointer kind of every array.
 * Returns MQH_OK, MQH_WBREAKDOWN, MQH_WEDGE (edge and breakdown: breakdown
 * wins) or an error.
 */
int mqh_solve(mqh_problem* p, const double* f_int, const double* g_bnd, const mqh_solve_opts* opts, double* coef,
              double* gkb_alpha, double* gkb_beta, double* ritz_sv, mqh_solve_info* info);

/*
 * Several right-hand sides on the same A (Algorithm 1, one independent run
 * per right-hand side; Algorithm 4 for the solve).  The runs go in groups of
 * MQH_BLOCK_RHS in lockstep: step j of every run of a group is enqueued
 * together, so one pass over A serves the whole group.  In
 * MQH_OP_MATFREE_FP32 a group of two or more shares a block product: the
 * FP32-evaluated entries of a tile multiply all the group's vectors on the
 * matrix cores as FP16 products of operands split in two parts each (the
 * entries scaled by a power of two per problem, each vector by its own;
 * 2^-22 relative per part, products exact in FP32, FP32 sums over 256
 * nodes, FP64 across chunks and slices); a group of one, and the FP64
 * forms, run one product per run, bit-identical to mqh_gkb / mqh_solve.
 * The tile shape and slice count of the block products (the split of the
 * sum over nodes, so the order of the FP64 additions) are picked on the
 * first block product of a problem by timing a few candidates, unless the
 * problem was created with MQH_FLAG_FIXED_SHAPES;
 * results are bit-reproducible for a given problem handle either way.  Everything else (norms,
 * reorthogonalisation, scalars, breakdown tests, projected SVD, parameter
 * choice, lift) is per run in FP64 as in the single-run calls.
 *
 * mqh_apply_multi: Y_k = op(A) X_k - shifts[k] Z_k for k < nrhs, the
 * products of Algorithm 1 (steps 3 and 5) for a group; X_k at X + k * ldx,
 * Z_k at Zs + k * ldz (Zs NULL: no shift term), Y_k at Y + k * ldy, all
 * leading dimensions >= n; shifts is a host array of nrhs values (NULL:
 * zeros); Y must not alias X or Zs.
 *
 * F: nrhs right-hand sides [f_int; g_bnd] of length n, column k at
 *    F + k * ldf (ldf >= n).
 * mqh_gkb_multi outputs (any may be NULL), run k's block after those of
 * runs 0..k-1, each laid out as in mqh_gkb:
 *   W (ell+1) n doubles per run, Z ell n, alpha ell, beta ell+1, ell_done 1.
 * mqh_solve_multi: opts as in mqh_solve (MQH_FLAG_TIME_PRODUCTS sums the
 * product kernels of each group: t_ms[6], t_ms[7] report the group's
 * totals, as do the other t_ms); coef column k at coef + k * ldc
 * (ldc >= n); info: nrhs records (NULL allowed).
 * Returns MQH_WBREAKDOWN if any run broke down, else MQH_WEDGE if any
 * choice sits at the edge of its range, else MQH_OK; errors as mqh_solve.
 * Workspace: per group 2 (ell+1) n doubles of bases per run (grown on
 * demand, kept with the problem).
 */
int mqh_apply_multi(mqh_problem* p, int32_t trans, const double* X, int64_t ldx, int32_t nrhs, const double* shifts,
                    const double* Zs, int64_t ldz, double* Y, int64_t ldy, uint32_t flags);
int mqh_gkb_multi(mqh_problem* p, const double* F, int64_t ldf, int32_t nrhs, int32_t ell, int32_t reorth, double* W,
                  double* Z, double* alpha, double* beta, int32_t* ell_done, uint32_t flags);
int mqh_solve_multi(mqh_problem* p, const double* F, int64_t ldf, int32_t nrhs, const mqh_solve_opts* opts,
                    double* coef, int64_t ldc, mqh_solve_info* info);

/*
 * A sweep of independent problems (a frequency sweep: one problem per
 * wavenumber), each solved as by mqh_solve_multi with the same opts.
 * `workers` host threads take the items in order and run them side by
 * side, each problem on its own stream, so that the kernels of one problem
 * overlap those of another (problems created with stream = NULL each own a
 * stream; problems sharing a stream run one after the other).  A problem
 * may appear once.  Per item: status receives mqh_solve_multi's return
 * value; F, coef, info as there (opts->flags applies to every item).
 * Returns the first error met (mqh_last_error has its message; items not
 * yet started keep MQH_EINVAL), else MQH_WBREAKDOWN if any item broke
 * down, else MQH_WEDGE if any choice sits at an edge, else MQH_OK.
 * Items must not be touched while the call runs.
 */
typedef struct {
    mqh_problem* p;
    const double* F;        /* nrhs right-hand sides, leading dimension ldf */
    int64_t ldf;
    int32_t nrhs;
    int32_t status;         /* out */
    double* coef;           /* out: nrhs coefficient vectors, leading dimension ldc */
    int64_t ldc;
    mqh_solve_info* info;   /* out: nrhs records, or NULL */
} mqh_sweep_item;

int mqh_solve_sweep(mqh_sweep_item* items, int32_t count, const mqh_solve_opts* opts, int32_t workers);

/*
 * Block Golub-Kahan: nrhs <= MQH_BLOCK_RHS right-hand sides that share one
 * Krylov space (Algorithm 1 with the n x nrhs block F in place of f; the
 * paper has one right-hand side per problem).  The recurrence:
 *   W_1 E_1 = F,
 *   Z_j D_j^T = A^T W_j - Z_{j-1} E_j^T,   W_{j+1} E_{j+1} = A Z_j - W_j D_j,
 * each right side reorthogonalised against every earlier block of its basis
 * (classical Gram-Schmidt twice) and factored by a QR with a non-negative
 * diagonal in R (shifted Cholesky QR applied three times, on the FP64
 * matrix cores).  A Z_ell = W_{ell+1} C with C the lower block bidiagonal
 * (ell + 1) nrhs x ell nrhs matrix of the D_j (lower triangular, diagonal
 * blocks) and E_{j+1} (upper triangular, below them).  A QR whose R has a
 * diagonal entry at most n eps times the largest diagonal entry of the D
 * and E blocks so far (E_1 left out) is a breakdown: at a D block ell_done =
 * j - 1 (flag 1), at an E block ell_done = j with E_{j+1} = 0 (flag 2).
 * The products use the problem's operator (FP32-evaluated block products
 * on the matrix cores for MQH_OP_MATFREE_FP32 and nrhs >= 2).
 *
 * F: n x nrhs, leading dimension ldf >= n.  Needs ell >= 1, ell nrhs <= n
 * and (ell + 1) nrhs <= MQH_BLOCK_MAX_DIM.  The sources must be linearly
 * independent to working precision: zero or repeated sources (a pivot of
 * the QR of F that is not positive, or a diagonal entry of E_1 at most
 * n DBL_EPSILON times its largest) are MQH_EINVAL, since W_1 would carry a
 * direction of rounding noise.  Host or device pointers
 * (MQH_FLAG_DEVICE_PTRS in flags / opts->flags).  The workspace (the bases,
 * (2 ell + 1) nrhs n doubles, and the projected problem's) stays on the
 * problem between calls and is reused by calls of the same nrhs and ell;
 * mqh_problem_destroy frees it.
 *
 * mqh_gkb_block: C ((ell + 1) nrhs x ell nrhs, row-major; blocks past
 *   ell_done are zero), E1 (nrhs x nrhs row-major, NULL allowed), W
 *   (n x (ell + 1) nrhs column-major, leading dimension n, NULL allowed),
 *   Z (n x ell nrhs, NULL allowed).  Returns MQH_WBREAKDOWN after a
 *   breakdown.
 * mqh_solve_block: for each source k the Tikhonov solution on the shared
 *   space, y_k = argmin ||C y - (E_1 e_k; 0)||^2 + lambda_k^2 ||y||^2 and
 *   coef_k = Z y_k (column k of coef, leading dimension ldc >= n).
 *   opts->method must be MQH_METHOD_HKT; opts->ell is the number of block
 *   steps; opts->rule MQH_RULE_GCV (per source, the full-problem GCV of
 *   eq. (25) on the (ell + 1) nrhs projected rows, s_perp = what the
 *   retained components leave of ||E_1 e_k||^2, on the grid of
 *   mqh_param_choice; for nrhs = 1 this is the projected GCV of eq. (30))
 *   or MQH_RULE_FIXED (lambda_fixed for every source).  The projected
 *   problem is solved through the SVD of C: C^T (upper banded, bandwidth
 *   nrhs) is reduced to a bidiagonal by Householder bulge chasing in one
 *   workgroup's LDS (ell_done nrhs (3 nrhs + 1) <= 19 600 and ell_done nrhs
 *   <= 1024: for 16 sources up to 25 block steps), whose SVD the
 *   multisection path of mqh_proj_svd computes, the data and solutions
 *   going through the reflectors.  Larger problems, a failed acceptance
 *   test of that SVD, or MQH_FLAG_BLOCK_JACOBI in opts->flags take the
 *   full-SVD path on [C | 0] (square) instead (MQH_INFO_BLOCK_JACOBI).  sv
 *   (ell_done nrhs, NULL allowed): singular values of C, descending.  info:
 *   nrhs records (NULL allowed): ell_done, lambda_chosen, crit (GCV at the
 *   choice), resid_norm = ||A coef_k - f_k|| and sol_norm = ||coef_k|| (from
 *   the projected problem; equal by the block relations), flags
 *   (MQH_INFO_BREAKDOWN, MQH_INFO_GCV_AT_EDGE, MQH_INFO_SOLVE_NOCONV), t_ms
 *   [0] upload, [1] block recurrence, [2] projected problem (SVD, choices,
 *   solutions), [3] lift and download, [5] total, [6] Jacobi sweeps of the
 *   projected SVD, [7] conjugate-gradient iterations of this source (both 0
 *   on the band path).
 *   Returns MQH_WBREAKDOWN, else MQH_WNOCONV, else MQH_WEDGE (any source),
 *   else MQH_OK.
 */
int mqh_gkb_block(mqh_problem* p, const double* F, int64_t ldf, int32_t nrhs, int32_t ell, double* C, double* E1,
                  double* W, double* Z, int32_t* ell_done, int32_t* flag, uint32_t flags);
int mqh_solve_block(mqh_problem* p, const double* F, int64_t ldf, int32_t nrhs, const mqh_solve_opts* opts,
                    double* coef, int64_t ldc, double* sv, mqh_solve_info* info);

/*
 * Reference path: the full SVD of A and the classical regularised solutions
 * built on it, for n <= MQH_FULL_MAX_N (every call assembles A in FP64 into
 * its own n x (n + 1) work matrix, 8 n^2 bytes, freed on return).
 *
 * The SVD is one-sided block Jacobi on the rows of [A | f]: row rotations Q
 * (each sweep orders the rows by decreasing norm and pairs 32-row blocks in
 * a round-robin order; per pair the rotation of one cyclic Jacobi sweep,
 * two on matrices of at most 10 blocks, on the 64 x 64 Gram matrix of their
 * rows) until, in a whole sweep, every pair
 * of rows has the component of the smaller along the larger at most
 * 16 sqrt(n) DBL_EPSILON ||A||_F, or the largest such component stays below
 * twice that (the rounding floor of the measure) without falling by a
 * quarter for three sweeps (singular values to a small multiple of that
 * absolute level).  Then
 * A = Q^T Sigma Ubar^T: sigma_i are the row norms of Q A, U^T f = Q f is the
 * rotated f column, and the solutions are combinations of the rows of Q A
 * (U and V are never formed).
 *
 * mqh_full_svd: sv (n, descending); fhat (n, NULL allowed) = U^T f in the
 *   same order (f NULL: fhat = 0); sweeps (host, NULL allowed) = Jacobi
 *   sweeps run; off (host, NULL allowed) = the last sweep's largest
 *   off-diagonal measure.  MQH_WNOCONV if 100 sweeps did not bring it below
 *   32 sqrt(n) DBL_EPSILON.
 * mqh_full_solve: Algorithm 3 (Tikh-Reg: opts->method = MQH_METHOD_HKT,
 *   the Tikhonov filter, eq. (17)) or the TSVD solution of eq. (14)
 *   (opts->method = MQH_METHOD_INE_TSVD, the TSVD filter on the full SVD);
 *   opts->rule MQH_RULE_GCV (eq. (25): N in the denominator; lambda on
 *   opts->n_grid log-spaced points on [max(sigma_r, 16 eps sigma_1), sigma_1]
 *   with golden-section refinement; TSVD rank k over 1 .. min(r, n - 1),
 *   ties to the smaller k) or MQH_RULE_FIXED (lambda_fixed / k_trunc);
 *   opts->ell and reorth are ignored.  coef (n) out; sv (n, NULL allowed)
 *   out; info: ell_done = Jacobi sweeps, k_chosen, lambda_chosen, crit =
 *   GCV at the choice, resid_norm = ||A coef - f|| and sol_norm = ||coef||
 *   of the returned coef (computed from it, not from the filter formula),
 *   flags (MQH_INFO_GCV_AT_EDGE), t_ms [0] assembly, [1] Jacobi sweeps,
 *   [2] singular values and order, [3] parameter choice, [4] solution,
 *   [5] total, [6] the last sweep's largest off-diagonal measure, [7] the
 *   conjugate-gradient iterations of the solution (at most MQH_FULL_CG_MAX; at the cap
 *   above the tolerance MQH_INFO_SOLVE_NOCONV is set and MQH_WNOCONV
 *   returned: this happens when lambda lies below the accuracy of the SVD,
 *   as GCV chooses on exact data, where the Tikhonov solution is not
 *   determined by the data).  The solution is
 *   x = G^T y, G = Q A the rotated rows, with (G G^T + lambda^2 I) y = Q f
 *   (Tikhonov) or G_k G_k^T y = (Q f)_k on the k rows of the largest sigma
 *   (TSVD), solved by conjugate gradients preconditioned with the diagonal:
 *   exact for any orthogonal Q, whether or not the rows are orthogonal.
 */
int mqh_full_svd(mqh_problem* p, const double* f, double* sv, double* fhat, int32_t* sweeps, double* off,
                 uint32_t flags);
int mqh_full_solve(mqh_problem* p, const double* f_int, const double* g_bnd, const mqh_solve_opts* opts, double* coef,
                   double* sv, mqh_solve_info* info);

/*
 * The predictor network's kernels (FP32; every array is a device pointer and
 * flags must contain MQH_FLAG_DEVICE_PTRS).  Batches are row-major.
 *   mqh_mlp_forward:  y (batch x 2) from x (batch x 24); hidden receives the
 *                     tanh outputs, 3 blocks of batch x 128 (kept for backward).
 *   mqh_mlp_backward: grad (MQH_MLP_NPARAMS) of a loss from dy = dL/dy
 *                     (batch x 2), x and hidden; work: 2 x batch x 128 floats.
 *   mqh_mlp_loss:     loss = sum_b sum_k w_k (y - t)^2 / batch (one float,
 *                     NULL allowed) and dy = dloss/dy (NULL allowed); w has 2 entries.
 *   mqh_mlp_adam:     one Adam step (bias-corrected moments, step >= 1) on n parameters.
 * Reductions run in a fixed order (deterministic).
 */
int mqh_mlp_forward(const float* params, const float* x, int32_t batch, float* y, float* hidden, void* stream,
                    uint32_t flags);
int mqh_mlp_backward(const float* params, const float* x, const float* hidden, const float* dy, int32_t batch,
                     float* grad, float* work, void* stream, uint32_t flags);
int mqh_mlp_loss(const float* y, const float* t, const float* w, int32_t batch, float* loss, float* dy, void* stream,
                 uint32_t flags);
int mqh_mlp_adam(float* params, const float* grad, float* m, float* v, int64_t n, float lr, float beta1, float beta2,
                 float eps, int32_t step, void* stream, uint32_t flags);

/*
 * HKT with a learned stopping index and regularisation parameter, GCV as
 * judge and fallback (Algorithm 4 with an early stop).  Runs MQH_MLP_PROBE
 * Golub-Kahan steps, evaluates the predictor on the device, continues to
 * ell_pred = the predicted stop index (rounded up to a multiple of
 * pred->ell_step, within [MQH_MLP_PROBE, opts->ell]), computes the projected
 * SVD and the GCV choice lambda_gcv at ell_pred (the judge: linfo reports
 * lambda_gcv, GCV(lambda_net) and min GCV), and solves with the network's
 * lambda_net = alpha_1 exp(out[0]) unless it falls back to lambda_gcv:
 * lambda_net not finite or positive, more than a factor 10 outside GCV's
 * search range [max(s_l, 16 eps_mach s_1), s_1], or (judge_ratio >= 1)
 * GCV(lambda_net) > judge_ratio * GCV(lambda_gcv).
 * opts: method HKT, rule GCV, ell >= MQH_MLP_PROBE; kappa > 0; row_scale 0
 * or 1 (1: the whole run on D A and D f as in mqh_solve, so the features come
 * from the scaled process: use a predictor trained on such runs).
 * coef (n) out; info and linfo may be NULL.
 */
int mqh_solve_learned(mqh_problem* p, const double* f_int, const double* g_bnd, const mqh_solve_opts* opts,
                      const mqh_predictor* pred, double* coef, mqh_solve_info* info, mqh_learned_info* linfo);

/*
 * Evaluate u(X_e) = sum_j coef_j phi(|X_e - X_j|) at m points
 * (eq. (18)), FP64: coef (n), x_eval (m x 3) in, u (m) out.
 */
int mqh_eval(mqh_problem* p, const double* coef, const double* x_eval, int64_t m, double* u, uint32_t flags);

#ifdef __cplusplus
}
#endif

#endif /* MQHELM_H */
