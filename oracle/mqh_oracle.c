/*
 * mqh_oracle.c -- plain, slow, obviously-correct FP64 CPU reference.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path links,
 * loads or calls this file; only the tests, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no code, header or constant
 * with the HIP implementation.
 *
 * What it computes (paper: Efficient Krylov-Regularization Solvers for
 * Multiquadric RBF Discretizations of the 3D Helmholtz Equation):
 *   - the multiquadric kernel phi(r) = sqrt(1 + eps^2 r^2)            (eq. (3))
 *   - its 3-D Laplacian and the Helmholtz-applied kernel
 *       L phi = Lap(phi) + kappa^2 phi                               (eqs. (7), (8))
 *   - the Kansa matrix A = [H; R]: interior rows L phi, Dirichlet
 *     boundary rows phi, centres = nodes                              (eqs. (10), (11))
 *   - products A v and A^T u, stored or entry-by-entry, optionally with the
 *     rows scaled by D = diag(A)^{-1} (an opt-in equilibration, not in the paper)
 *   - Golub-Kahan bidiagonalisation with full reorthogonalisation     (Algorithm 1)
 *   - one-sided Jacobi SVD of a small dense matrix (projected SVD)    (Algorithm 2 step 2, Algorithm 4 step 2)
 *   - the lift alpha = Z y and evaluation u(X) = sum_j alpha_j phi   (Algorithm 2 step 5, eq. (18))
 *
 * Everything is double precision; sqrt and division are IEEE correctly
 * rounded.  Loops are written in the order of the definitions; OpenMP only
 * distributes independent output elements (each output element is summed
 * in one fixed order by one thread, so results do not depend on the thread
 * count).
 *
 * Node layout: X is n x 3 row-major (x,y,z interleaved), rows ordered
 * [interior (n_int); boundary (n - n_int)].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Kernel and matrix entries                                            */
/* ------------------------------------------------------------------ */

/* phi(r; eps) = sqrt(1 + eps^2 r^2)  (eq. (3)). */
double orc_phi(double r, double eps) { return sqrt(1.0 + eps * eps * r * r); }

/* 3-D Laplacian of the radial function phi(|x - c|).  For a radial f(r) in
 * three dimensions Lap f = f'' + (2/r) f'.  With t = 1 + eps^2 r^2:
 *   f'  = eps^2 r / sqrt(t)
 *   f'' = eps^2 / sqrt(t) - eps^4 r^2 / t^(3/2) = eps^2 / t^(3/2)
 * so Lap f = eps^2/t^(3/2) + 2 eps^2/sqrt(t) = eps^2 (3 + 2 eps^2 r^2) / t^(3/2).
 * The paper does not print this expression (it only names Lap(phi) in eq. (7)). */
double orc_lap_phi(double r, double eps) {
    double e2 = eps * eps;
    double t = 1.0 + e2 * r * r;
    return e2 * (3.0 + 2.0 * e2 * r * r) / (t * sqrt(t));
}

/* Helmholtz-applied kernel L phi = Lap(phi) + kappa^2 phi  (eq. (8)). */
double orc_lphi(double r, double kappa, double eps) {
    return orc_lap_phi(r, eps) + kappa * kappa * orc_phi(r, eps);
}

static double dist3(const double* a, const double* b) {
    double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return sqrt(dx * dx + dy * dy + dz * dz);
}

/* A_ij: interior rows (i < n_int) are L phi(|X_i - X_j|); boundary rows are
 * phi(|X_i - X_j|) (Dirichlet, u = g; eq. (10)). */
double orc_entry(const double* X, int64_t n_int, int64_t i, int64_t j, double kappa, double eps) {
    double r = dist3(X + 3 * i, X + 3 * j);
    return (i < n_int) ? orc_lphi(r, kappa, eps) : orc_phi(r, eps);
}

/* Dense row-major n x n assembly of A. */
void orc_assemble(const double* X, int64_t n, int64_t n_int, double kappa, double eps, double* A) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j)
            A[i * n + j] = orc_entry(X, n_int, i, j, kappa, eps);
}

/* Interpolation matrix B_ij = phi(|X_i - X_j|)  (eq. (5)), m x n with
 * rows at points P (m x 3) and columns at centres X (n x 3). */
void orc_interp_matrix(const double* P, int64_t m, const double* X, int64_t n, double eps, double* B) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j)
            B[i * n + j] = orc_phi(dist3(P + 3 * i, X + 3 * j), eps);
}

/* ------------------------------------------------------------------ */
/* Operator: y = A x  or  y = A^T x, stored (A != NULL) or entry-wise    */
/* ------------------------------------------------------------------ */

typedef struct {
    const double* A; /* row-major n x n, or NULL for entry-by-entry evaluation */
    const double* X; /* nodes n x 3 */
    int64_t n, n_int;
    double kappa, eps;
    const double* d; /* row scale of the entry-by-entry operator (NULL: none); see orc_row_scale */
} orc_op;

/* Entry of the operator: A_ij, or d_i A_ij under row scaling. */
static double op_entry(const orc_op* op, int64_t i, int64_t j) {
    double a = orc_entry(op->X, op->n_int, i, j, op->kappa, op->eps);
    return op->d ? op->d[i] * a : a;
}

static void op_apply(const orc_op* op, int trans, const double* x, double* y) {
    const int64_t n = op->n;
    if (!trans) {
        /* y_i = sum_j A_ij x_j, j ascending */
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double s = 0.0;
            if (op->A) {
                const double* row = op->A + i * n;
                for (int64_t j = 0; j < n; ++j) s += row[j] * x[j];
            } else {
                for (int64_t j = 0; j < n; ++j)
                    s += op_entry(op, i, j) * x[j];
            }
            y[i] = s;
        }
    } else {
        /* y_j = sum_i A_ij x_i, i ascending.  Columns are processed in
         * blocks of 512 so that a stored row segment (4 KB) is read
         * contiguously; every y_j is still one sum in ascending i, so the
         * block width changes no result. */
        enum { BS = 512 };
        const int64_t nb = (n + BS - 1) / BS;
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t b = 0; b < nb; ++b) {
            int64_t j0 = b * BS, j1 = j0 + BS < n ? j0 + BS : n;
            double acc[BS];
            for (int64_t j = j0; j < j1; ++j) acc[j - j0] = 0.0;
            for (int64_t i = 0; i < n; ++i) {
                double xi = x[i];
                if (op->A) {
                    const double* row = op->A + i * n;
                    for (int64_t j = j0; j < j1; ++j) acc[j - j0] += row[j] * xi;
                } else {
                    for (int64_t j = j0; j < j1; ++j)
                        acc[j - j0] += op_entry(op, i, j) * xi;
                }
            }
            for (int64_t j = j0; j < j1; ++j) y[j] = acc[j - j0];
        }
    }
}

/*
 * Row scaling of the stacked system A c = f (eq. (11)) by D = diag(A)^{-1}:
 * d_i = 1 / A_ii.  Not in the paper: an opt-in equilibration of the two row
 * classes (interior rows carry L phi, of size about 3 eps^2 + kappa^2 at
 * r = 0, boundary rows phi, of size 1 there).  The scaled problem is
 * (D A) c = D f, with the same solution c when A is nonsingular.
 */
void orc_row_scale(const double* X, int64_t n, int64_t n_int, double kappa, double eps, double* d) {
    for (int64_t i = 0; i < n; ++i) d[i] = 1.0 / orc_entry(X, n_int, i, i, kappa, eps);
}

/* Public product: A == NULL selects entry-by-entry evaluation; d (NULL
 * allowed) scales the rows of the entry-by-entry operator (a stored A is
 * passed already scaled). */
void orc_apply_rs(const double* A, const double* X, int64_t n, int64_t n_int, double kappa, double eps,
                  const double* d, int trans, const double* x, double* y) {
    orc_op op = {A, X, n, n_int, kappa, eps, A ? NULL : d};
    op_apply(&op, trans, x, y);
}

void orc_apply(const double* A, const double* X, int64_t n, int64_t n_int, double kappa, double eps,
               int trans, const double* x, double* y) {
    orc_apply_rs(A, X, n, n_int, kappa, eps, NULL, trans, x, y);
}

/* Sampled rows (trans = 0) or columns (trans = 1) of the product, entry by
 * entry: out[k] = (A x)_{idx[k]} or (A^T x)_{idx[k]}.  Used to check single
 * outputs at sizes where a full product is too slow on the CPU. */
void orc_apply_sampled_rs(const double* X, int64_t n, int64_t n_int, double kappa, double eps, const double* d,
                          int trans, const double* x, const int64_t* idx, int64_t cnt, double* out) {
    orc_op op = {NULL, X, n, n_int, kappa, eps, d};
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < cnt; ++k) {
        int64_t o = idx[k];
        double s = 0.0;
        for (int64_t l = 0; l < n; ++l) {
            double a = trans ? op_entry(&op, l, o) : op_entry(&op, o, l);
            s += a * x[l];
        }
        out[k] = s;
    }
}

void orc_apply_sampled(const double* X, int64_t n, int64_t n_int, double kappa, double eps, int trans,
                       const double* x, const int64_t* idx, int64_t cnt, double* out) {
    orc_apply_sampled_rs(X, n, n_int, kappa, eps, NULL, trans, x, idx, cnt, out);
}

/* ------------------------------------------------------------------ */
/* Golub-Kahan bidiagonalisation with full reorthogonalisation (Alg. 1) */
/* ------------------------------------------------------------------ */

static double dot(const double* a, const double* b, int64_t n) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* Classical Gram-Schmidt of v against the m orthonormal columns of V
 * (column-major, leading dimension n), done twice ("twice is enough").
 * c_k = V_k^T v for all k first, then v -= sum_k c_k V_k. */
static void cgs2(const double* V, int64_t n, int64_t m, double* v, double* c) {
    for (int pass = 0; pass < 2; ++pass) {
        if (m == 0) return;
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < m; ++k) c[k] = dot(V + k * n, v, n);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double s = 0.0;
            for (int64_t k = 0; k < m; ++k) s += V[k * n + i] * c[k];
            v[i] -= s;
        }
    }
}

static double norm2(const double* v, int64_t n) { return sqrt(dot(v, v, n)); }

/*
 * Runs ell steps of Algorithm 1 on A (stored, or entry-wise when A == NULL).
 *
 *   beta_1 = ||f||, w_1 = f / beta_1, z_0 = 0
 *   for j = 1..ell:
 *     r = A^T w_j - beta_j z_{j-1};  reorthogonalise r against z_1..z_{j-1}
 *     alpha_j = ||r||;  z_j = r / alpha_j
 *     p = A z_j - alpha_j w_j;       reorthogonalise p against w_1..w_j
 *     beta_{j+1} = ||p||;  w_{j+1} = p / beta_{j+1}
 *
 * The paper lists reorthogonalisation after both updates and calls it
 * optional; here it is full (against every earlier vector) and applied to r
 * and p before their norms are taken, which is the same as reorthogonalising
 * z_j and w_{j+1} and renormalising.
 *
 * Breakdown (the paper only says the process stops when some alpha_j or
 * beta_{j+1} vanishes): alpha_j or beta_{j+1} <= tau with
 * tau = n * DBL_EPSILON * max(alpha_i, beta_{i+1} so far) (beta_1 = ||f|| is
 * not an operator scale and is left out).  On an alpha
 * breakdown the run keeps ell_eff = j-1 steps; on a beta breakdown it keeps
 * ell_eff = j and sets beta_{j+1} = 0 (w_{j+1} = 0).
 *
 * Outputs: W (n x (ell+1), column-major), Z (n x ell), alpha[ell],
 * beta[ell+1] (beta[0] = beta_1 = ||f||).  Returns ell_eff; *flag is set to
 * 1 on an alpha breakdown and 2 on a beta breakdown, else 0.
 * If reorth == 0 no reorthogonalisation is done (plain Algorithm 1).
 * d (NULL allowed): the run is on the row-scaled operator D A of an
 * entry-by-entry A (a stored A is passed already scaled); f is passed
 * scaled by the caller.
 */
int64_t orc_gkb_rs(const double* A, const double* X, int64_t n, int64_t n_int, double kappa, double eps,
                   const double* d, const double* f, int64_t ell, int reorth, double* W, double* Z, double* alpha,
                   double* beta, int* flag) {
    orc_op op = {A, X, n, n_int, kappa, eps, A ? NULL : d};
    double* r = (double*)malloc(sizeof(double) * n);
    double* c = (double*)malloc(sizeof(double) * (ell + 2));
    *flag = 0;
    memset(W, 0, sizeof(double) * n * (ell + 1));
    memset(Z, 0, sizeof(double) * n * ell);
    for (int64_t j = 0; j < ell; ++j) alpha[j] = 0.0;
    for (int64_t j = 0; j <= ell; ++j) beta[j] = 0.0;

    double b1 = norm2(f, n);
    beta[0] = b1;
    if (!(b1 > 0.0)) { free(r); free(c); *flag = 2; return 0; }
    for (int64_t i = 0; i < n; ++i) W[i] = f[i] / b1;
    double scale = 0.0; /* running max of alpha_j, beta_{j+1} (operator scale; beta_1 = ||f|| is data) */
    int64_t ell_eff = ell;

    for (int64_t j = 0; j < ell; ++j) {
        /* paper step j+1:  r = A^T w_{j+1} - beta_{j+1} z_j */
        op_apply(&op, 1, W + j * n, r);
        if (j > 0)
            for (int64_t i = 0; i < n; ++i) r[i] -= beta[j] * Z[(j - 1) * n + i];
        if (reorth) cgs2(Z, n, j, r, c);
        double a = norm2(r, n);
        double tau = (double)n * DBL_EPSILON * scale;
        if (!(a > tau)) { *flag = 1; ell_eff = j; break; }
        alpha[j] = a;
        if (a > scale) scale = a;
        for (int64_t i = 0; i < n; ++i) Z[j * n + i] = r[i] / a;

        /* p = A z_{j+1} - alpha_{j+1} w_{j+1} */
        op_apply(&op, 0, Z + j * n, r);
        for (int64_t i = 0; i < n; ++i) r[i] -= a * W[j * n + i];
        if (reorth) cgs2(W, n, j + 1, r, c);
        double b = norm2(r, n);
        tau = (double)n * DBL_EPSILON * scale;
        if (!(b > tau)) { *flag = 2; beta[j + 1] = 0.0; ell_eff = j + 1; break; }
        beta[j + 1] = b;
        if (b > scale) scale = b;
        for (int64_t i = 0; i < n; ++i) W[(j + 1) * n + i] = r[i] / b;
    }
    free(r);
    free(c);
    return ell_eff;
}

/* Algorithm 1 on the unscaled operator (d = NULL). */
int64_t orc_gkb(const double* A, const double* X, int64_t n, int64_t n_int, double kappa, double eps,
                const double* f, int64_t ell, int reorth, double* W, double* Z, double* alpha, double* beta,
                int* flag) {
    return orc_gkb_rs(A, X, n, n_int, kappa, eps, NULL, f, ell, reorth, W, Z, alpha, beta, flag);
}

/* ------------------------------------------------------------------ */
/* One-sided (Hestenes) Jacobi SVD of a dense m x n matrix, m >= n        */
/* ------------------------------------------------------------------ */

/*
 * M is m x n column-major (overwritten).  On return sv[n] holds the
 * singular values in descending order, U (m x n, column-major) the left
 * singular vectors and V (n x n, column-major) the right ones, so that
 * M = U diag(sv) V^T.  Cyclic-by-rows ordering with Rutishauser's rotation;
 * a pair is rotated while |g_p . g_q| > tol * ||g_p|| ||g_q|| with
 * tol = m * DBL_EPSILON, and sweeps repeat until none is rotated.
 * Columns whose norm is exactly zero get u = 0.
 * Returns the number of sweeps, or -1 if it did not converge in 100.
 */
int orc_jacobi_svd(double* M, int64_t m, int64_t n, double* sv, double* U, double* V) {
    for (int64_t i = 0; i < n * n; ++i) V[i] = 0.0;
    for (int64_t i = 0; i < n; ++i) V[i * n + i] = 1.0;
    const double tol = (double)m * DBL_EPSILON;
    int sweeps = 0;
    int rotated = 1;
    while (rotated) {
        if (sweeps >= 100) return -1;
        rotated = 0;
        ++sweeps;
        for (int64_t p = 0; p < n - 1; ++p) {
            for (int64_t q = p + 1; q < n; ++q) {
                double* gp = M + p * m;
                double* gq = M + q * m;
                double a = dot(gp, gp, m), b = dot(gq, gq, m), c = dot(gp, gq, m);
                if (c == 0.0 || fabs(c) <= tol * sqrt(a) * sqrt(b)) continue;
                rotated = 1;
                double zeta = (b - a) / (2.0 * c);
                double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double cs = 1.0 / sqrt(1.0 + t * t);
                double sn = cs * t;
                for (int64_t i = 0; i < m; ++i) {
                    double x = gp[i], y = gq[i];
                    gp[i] = cs * x - sn * y;
                    gq[i] = sn * x + cs * y;
                }
                double* vp = V + p * n;
                double* vq = V + q * n;
                for (int64_t i = 0; i < n; ++i) {
                    double x = vp[i], y = vq[i];
                    vp[i] = cs * x - sn * y;
                    vq[i] = sn * x + cs * y;
                }
            }
        }
    }
    /* singular values = column norms; sort descending (selection sort on an index) */
    int64_t* ord = (int64_t*)malloc(sizeof(int64_t) * n);
    double* nrm = (double*)malloc(sizeof(double) * n);
    for (int64_t k = 0; k < n; ++k) { ord[k] = k; nrm[k] = norm2(M + k * m, m); }
    for (int64_t a = 0; a < n; ++a) {
        int64_t best = a;
        for (int64_t b = a + 1; b < n; ++b)
            if (nrm[ord[b]] > nrm[ord[best]]) best = b;
        int64_t t = ord[a]; ord[a] = ord[best]; ord[best] = t;
    }
    double* Vs = (double*)malloc(sizeof(double) * n * n);
    memcpy(Vs, V, sizeof(double) * n * n);
    for (int64_t k = 0; k < n; ++k) {
        int64_t s = ord[k];
        sv[k] = nrm[s];
        for (int64_t i = 0; i < m; ++i) U[k * m + i] = nrm[s] > 0.0 ? M[s * m + i] / nrm[s] : 0.0;
        for (int64_t i = 0; i < n; ++i) V[k * n + i] = Vs[s * n + i];
    }
    free(Vs);
    free(nrm);
    free(ord);
    return sweeps;
}

/* ------------------------------------------------------------------ */
/* Projected SVD of the (ell+1) x ell lower bidiagonal C_ell             */
/* ------------------------------------------------------------------ */

/*
 * C_ell has diagonal alpha_1..alpha_ell and subdiagonal beta_2..beta_{ell+1}
 * (Algorithm 1, last step).  Its SVD C = U~ S~ V~^T is computed with the
 * dense Jacobi routine above.  The thin SVD gives the first ell columns of
 * U~; the last column is the unit null vector of C^T, n_1 = 1,
 * n_{j+1} = -alpha_j n_j / beta_{j+1}, normalised.  The projected data are
 * f~ = U~^T (beta_1 e_1), i.e. f~_i = beta_1 U~_{1,i}, i = 1..ell+1
 * (eqs. (28), (29) need f~_{ell+1}).
 *
 * alpha[ell], beta[ell+1] with beta[0] = beta_1.  Outputs: sv[ell]
 * (descending), ftil[ell+1], V (ell x ell column-major, column i = v~_i).
 * Returns the Jacobi sweep count or -1.
 */
int orc_proj_svd(const double* alpha, const double* beta, int64_t ell, double* sv, double* ftil, double* V) {
    int64_t m = ell + 1;
    double* C = (double*)calloc((size_t)(m * ell), sizeof(double));
    double* U = (double*)malloc(sizeof(double) * m * ell);
    for (int64_t j = 0; j < ell; ++j) {
        C[j * m + j] = alpha[j];        /* diagonal alpha_{j+1} */
        C[j * m + j + 1] = beta[j + 1]; /* subdiagonal beta_{j+2} */
    }
    int sw = orc_jacobi_svd(C, m, ell, sv, U, V);
    for (int64_t i = 0; i < ell; ++i) ftil[i] = beta[0] * U[i * m + 0];
    /* Unit null vector n of C^T (C^T n = 0 reads alpha_j n_j + beta_{j+1} n_{j+1} = 0):
     * n_1 = 1, n_{j+1} = -alpha_j n_j / beta_{j+1}, rescaled whenever an entry
     * grows past 1e150 so that nothing overflows.  If beta_{ell+1} = 0 the
     * last row of C is zero and the null vector is e_{ell+1}. */
    if (beta[ell] == 0.0) {
        ftil[ell] = 0.0;
    } else {
        double* nv = (double*)malloc(sizeof(double) * m);
        nv[0] = 1.0;
        for (int64_t j = 0; j < ell; ++j) {
            nv[j + 1] = -alpha[j] * nv[j] / beta[j + 1];
            if (fabs(nv[j + 1]) > 1e150)
                for (int64_t k = 0; k <= j + 1; ++k) nv[k] *= 1e-150;
        }
        double s2 = 0.0;
        for (int64_t k = 0; k < m; ++k) s2 += nv[k] * nv[k];
        ftil[ell] = beta[0] * nv[0] / sqrt(s2);
        free(nv);
    }
    free(C);
    free(U);
    return sw;
}

/* ------------------------------------------------------------------ */
/* Lift and evaluation                                                  */
/* ------------------------------------------------------------------ */

/* alpha = Z y, Z n x ell column-major (Algorithm 2 step 5, Algorithm 4 last step). */
void orc_lift(const double* Z, int64_t n, int64_t ell, const double* y, double* coef) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t k = 0; k < ell; ++k) s += Z[k * n + i] * y[k];
        coef[i] = s;
    }
}

/* u(P_e) = sum_j coef_j phi(|P_e - X_j|)  (eq. (18)). */
void orc_eval(const double* X, int64_t n, double eps, const double* coef, const double* P, int64_t m,
              double* u) {
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; ++e) {
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j) s += coef[j] * orc_phi(dist3(P + 3 * e, X + 3 * j), eps);
        u[e] = s;
    }
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
