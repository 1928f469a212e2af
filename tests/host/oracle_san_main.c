/* Drives every entry point of the oracle (oracle/mqh_oracle.c) on small
 * seeded inputs, for a build with AddressSanitizer and UndefinedBehavior-
 * Sanitizer: any out-of-bounds access, leak or undefined operation in the
 * oracle's C code ends the run with a report and a non-zero status.
 * Prints one line per exercised routine. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

double orc_phi(double r, double eps);
double orc_lap_phi(double r, double eps);
double orc_lphi(double r, double kappa, double eps);
double orc_entry(const double* X, int64_t n_int, int64_t i, int64_t j, double kappa, double eps);
void orc_assemble(const double* X, int64_t n, int64_t n_int, double kappa, double eps, double* A);
void orc_interp_matrix(const double* P, int64_t m, const double* X, int64_t n, double eps, double* B);
void orc_row_scale(const double* X, int64_t n, int64_t n_int, double kappa, double eps, double* d);
void orc_apply_rs(const double* A, const double* X, int64_t n, int64_t n_int, double kappa, double eps,
                  const double* d, int trans, const double* x, double* y);
void orc_apply_sampled_rs(const double* X, int64_t n, int64_t n_int, double kappa, double eps, const double* d,
                          int trans, const double* x, const int64_t* idx, int64_t cnt, double* out);
int64_t orc_gkb_rs(const double* A, const double* X, int64_t n, int64_t n_int, double kappa, double eps,
                   const double* d, const double* f, int64_t ell, int reorth, double* W, double* Z, double* alpha,
                   double* beta, int* flag);
int orc_jacobi_svd(double* M, int64_t m, int64_t n, double* sv, double* U, double* V);
int orc_proj_svd(const double* alpha, const double* beta, int64_t ell, double* s, double* ftil, double* V);
void orc_lift(const double* Z, int64_t n, int64_t ell, const double* y, double* out);
void orc_eval(const double* X, int64_t n, double eps, const double* coef, const double* P, int64_t m, double* u);

static uint64_t rng_state = 88172645463325252ull;
static double urand(void) { /* xorshift64, uniform in [0, 1) */
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

static double* vec(int64_t n) {
    double* v = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) v[i] = urand() - 0.5;
    return v;
}

static int run(int64_t n, int64_t n_int, int64_t ell) {
    const double kappa = 3.0, eps = 2.5;
    double* X = vec(3 * n);
    double* A = (double*)malloc(sizeof(double) * (size_t)(n * n));
    double* f = vec(n);
    double* x = vec(n);
    double* y = vec(n);
    double* d = vec(n);
    orc_assemble(X, n, n_int, kappa, eps, A);
    orc_row_scale(X, n, n_int, kappa, eps, d);
    double diag_err = 0.0;
    for (int64_t i = 0; i < n; ++i) diag_err = fmax(diag_err, fabs(d[i] * A[i * n + i] - 1.0));
    for (int trans = 0; trans < 2; ++trans) {
        orc_apply_rs(A, X, n, n_int, kappa, eps, NULL, trans, x, y);
        orc_apply_rs(NULL, X, n, n_int, kappa, eps, d, trans, x, y);
        int64_t idx[3] = {0, n / 2, n - 1};
        double out[3];
        orc_apply_sampled_rs(X, n, n_int, kappa, eps, d, trans, x, idx, 3, out);
    }
    double* W = (double*)malloc(sizeof(double) * (size_t)(n * (ell + 1)));
    double* Z = (double*)malloc(sizeof(double) * (size_t)(n * ell));
    double* al = (double*)malloc(sizeof(double) * (size_t)ell);
    double* be = (double*)malloc(sizeof(double) * (size_t)(ell + 1));
    int flag = 0;
    int64_t le = 0;
    for (int reorth = 0; reorth < 2; ++reorth) {
        le = orc_gkb_rs(A, X, n, n_int, kappa, eps, NULL, f, ell, reorth, W, Z, al, be, &flag);
        le = orc_gkb_rs(NULL, X, n, n_int, kappa, eps, d, f, ell, reorth, W, Z, al, be, &flag);
    }
    double* s = (double*)malloc(sizeof(double) * (size_t)(le > 0 ? le : 1));
    double* ft = (double*)malloc(sizeof(double) * (size_t)(le + 1));
    double* V = (double*)malloc(sizeof(double) * (size_t)(le > 0 ? le * le : 1));
    int sw = le > 0 ? orc_proj_svd(al, be, le, s, ft, V) : 0;
    double* yv = vec(le);
    double* coef = (double*)malloc(sizeof(double) * (size_t)n);
    orc_lift(Z, n, le, yv, coef);
    const int64_t m = 17;
    double* P = vec(3 * m);
    double* u = (double*)malloc(sizeof(double) * (size_t)m);
    double* B = (double*)malloc(sizeof(double) * (size_t)(m * n));
    orc_eval(X, n, eps, coef, P, m, u);
    orc_interp_matrix(P, m, X, n, eps, B);
    /* dense Jacobi SVD of A (n x n, column-major copy) */
    double* M = (double*)malloc(sizeof(double) * (size_t)(n * n));
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) M[j * n + i] = A[i * n + j];
    double* sv = (double*)malloc(sizeof(double) * (size_t)n);
    double* U = (double*)malloc(sizeof(double) * (size_t)(n * n));
    double* VV = (double*)malloc(sizeof(double) * (size_t)(n * n));
    int swa = orc_jacobi_svd(M, n, n, sv, U, VV);
    printf("n %lld n_int %lld ell %lld: steps kept %lld flag %d, projected sweeps %d, full sweeps %d, "
           "|d A_ii - 1| %.1e, phi %.3f lphi %.3f\n",
           (long long)n, (long long)n_int, (long long)ell, (long long)le, flag, sw, swa, diag_err,
           orc_phi(0.5, eps), orc_lphi(0.5, kappa, eps) + 0.0 * orc_lap_phi(0.5, eps));
    free(X); free(A); free(f); free(x); free(y); free(d); free(W); free(Z); free(al); free(be);
    free(s); free(ft); free(V); free(yv); free(coef); free(P); free(u); free(B); free(M); free(sv);
    free(U); free(VV);
    return (sw < 0 || swa < 0) ? 1 : 0;
}

int main(void) {
    int bad = 0;
    bad |= run(40, 25, 12);   /* interior and boundary rows */
    bad |= run(33, 0, 8);     /* boundary rows only */
    bad |= run(31, 31, 6);    /* interior rows only */
    bad |= run(12, 8, 12);    /* ell = n: full Krylov space, breakdown path */
    bad |= run(1, 1, 1);      /* one node */
    return bad;
}
