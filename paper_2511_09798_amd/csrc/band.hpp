// band.hpp -- reduction of the projected matrix of the block Golub-Kahan
// process to a scalar bidiagonal by Householder bulge chasing (host and
// device), the first step of its SVD (the projected problem of Algorithm 4
// with a block of right-hand sides).
//
// The block recurrence gives C, (l + 1) s x l s, lower block bidiagonal with
// lower triangular diagonal blocks and upper triangular blocks below them:
// C[i][c] != 0 only for 0 <= i - c <= s.  Its transpose M = C^T (N = l s
// rows, Mc = N + s columns) is upper banded with bandwidth b = s.  Two-sided
// Householder reflectors take M to an upper bidiagonal N x (N + 1) matrix
// Bt (d on the diagonal, e above it), M = Q Bt P^T; then C = P Bt^T Q^T, with
// Bt^T the (N + 1) x N lower bidiagonal of the scalar process (alpha = d,
// beta_{j+1} = e_j), whose SVD the multisection path computes.  The data of
// the projected problem go through P^T, the solutions through Q.
//
// Sweep i (0 <= i < min(N, Mc - 1)) cleans row i beyond its superdiagonal.
// Its task t works on the columns [c0, c1], c0 = i + 1 + t b,
// c1 = min(c0 + b - 1, Mc - 1):
//  * a right reflector on those columns, applied to the rows r0 .. r1 =
//    min(c1, N - 1), zeroes M[r0][c0 + 1 .. c1] (r0 = i for t = 0, else
//    c0 - b: the row the previous task's left reflector filled);
//  * a left reflector on the rows c0 .. r1, applied to the columns c0 ..
//    min(c1 + b, Mc - 1), zeroes M[c0 + 1 .. r1][c0]; it fills row c0 past
//    its band, which task t + 1 cleans.
// Each task annihilates one row and one column of its bulge; the rest of the
// fill stays within b - 1 below and 2 b - 1 above the diagonal and is taken
// by later sweeps (the classical one-column-per-sweep bulge chase of the
// successive band reduction, here for a rectangular band).  Task (i, t)
// touches rows and columns within [c0 - b, c0 + 2b - 1], so task t' of
// sweep i + 1 only depends on tasks t <= t' + 2 of sweep i: with sweep i
// starting at step kLag i, the tasks of one step are disjoint, and running
// the steps in order gives the same result, bit for bit, as running the
// sweeps one after another.
#pragma once

#include <math.h>
#include <stdint.h>

#ifdef __HIPCC__
#define MQH_HD __host__ __device__
#define MQH_UNROLL _Pragma("unroll")
#else
#define MQH_HD
#define MQH_UNROLL
#endif

namespace mqh {
namespace band {

constexpr int kMaxB = 16;  // bandwidth (sources of a block) at most
constexpr int kLag = 3;    // sweep i + 1 runs task t at the step where sweep i runs task t + kLag

// Number of tasks of sweep i (see above): t with c0 = i + 1 + t b <= Mc - 2
// (a right reflector on at least two columns) and r0 <= N - 1.
MQH_HD inline int ntasks(int i, int N, int Mc, int b) {
    if (b < 2 || Mc - 3 - i < 0) return 0;
    const int t1 = (Mc - 3 - i) / b;
    const int t2 = N - 2 - i >= 0 ? (N - 2 - i) / b + 1 : 0;
    return (t1 < t2 ? t1 : t2) + 1;
}

MQH_HD inline int nsweeps(int N, int Mc) { return N < Mc - 1 ? N : Mc - 1; }

// Columns of task (i, t) and the row its right reflector cleans.
MQH_HD inline void task_cols(int i, int t, int b, int Mc, int& r0, int& c0, int& c1) {
    c0 = i + 1 + t * b;
    c1 = c0 + b - 1 < Mc - 1 ? c0 + b - 1 : Mc - 1;
    r0 = t == 0 ? i : c0 - b;
}

// Steps of the pipelined schedule: the last step runs the last task of some
// sweep, 1 + max_i (kLag i + ntasks(i) - 1) (0 without tasks).
MQH_HD inline int nsteps(int N, int Mc, int b) {
    int last = -1;
    const int ns = nsweeps(N, Mc);
    for (int i = 0; i < ns; ++i) {
        const int nt = ntasks(i, N, Mc, b);
        if (nt > 0 && kLag * i + nt - 1 > last) last = kLag * i + nt - 1;
    }
    return last + 1;
}

// The tasks of step T are those of the sweeps i = ihi, ihi - 1, .., ihi -
// cnt + 1 (ihi = min(nsweeps - 1, T / kLag)), task t = T - kLag i of each:
// T - kLag i - ntasks(i) falls strictly as i grows, so the sweeps with a task
// at step T are the top of that range.  Returns cnt; rank q of the step is
// sweep ihi - q.
MQH_HD inline int step_top(int T, int N, int Mc) {
    const int ns = nsweeps(N, Mc);
    return T / kLag < ns - 1 ? T / kLag : ns - 1;
}
MQH_HD inline int step_tasks(int T, int N, int Mc, int b, int& ihi) {
    ihi = step_top(T, N, Mc);
    int cnt = 0;
    for (int i = ihi; i >= 0 && T - kLag * i < ntasks(i, N, Mc, b); --i) ++cnt;
    return cnt;
}

// Band storage: row r at B + r * W, column c at offset c - r + b - 1, with W
// >= 3 b + 1 chosen so that W - 1, the distance from (r, c) to (r + 1, c), is
// odd: the lanes of a wave that read one column of consecutive rows then
// fall in different LDS banks.
MQH_HD inline int width(int b) { return 3 * b + 2 + (b & 1); }
MQH_HD inline int64_t at(int r, int c, int b) { return (int64_t)r * width(b) + (c - r) + (b - 1); }

// Householder reflector H = I - tau v v^T with v_0 = 1 and H x = beta e_0,
// for x_0 .. x_{n-1} read at x[k * xs] (n <= kMaxB).  v_1 .. v_{n-1} go to
// v[1 ..] (v[0] = 1, v[k] = 0 for k >= n); when x_1 .. x_{n-1} are all zero,
// tau = 0 and beta = x_0.  The norm is taken on x scaled by its largest
// entry.  The loops run over kMaxB with the entries past n zero, so that on
// the device v stays in registers.
MQH_HD inline double reflector(const double* x, int64_t xs, int n, double (&v)[kMaxB], double* beta) {
    double xv[kMaxB];
    MQH_UNROLL
    for (int k = 0; k < kMaxB; ++k) xv[k] = k < n ? x[k * xs] : 0.0;
    double amax = fabs(xv[0]), tmax = 0.0;
    MQH_UNROLL
    for (int k = 1; k < kMaxB; ++k) {
        const double a = fabs(xv[k]);
        amax = a > amax ? a : amax;
        tmax = a > tmax ? a : tmax;
    }
    const double x0 = xv[0];
    if (!(tmax > 0.0)) {
        MQH_UNROLL
        for (int k = 0; k < kMaxB; ++k) v[k] = k == 0 ? 1.0 : 0.0;
        *beta = x0;
        return 0.0;
    }
    const double inv = 1.0 / amax;
    double ss = 0.0;
    MQH_UNROLL
    for (int k = 0; k < kMaxB; ++k) {
        const double y = xv[k] * inv;
        ss = fma(y, y, ss);
    }
    const double nrm = amax * sqrt(ss);
    const double bt = x0 >= 0.0 ? -nrm : nrm;
    const double sc = 1.0 / (x0 - bt);
    MQH_UNROLL
    for (int k = 0; k < kMaxB; ++k) v[k] = k == 0 ? 1.0 : xv[k] * sc;
    *beta = bt;
    return (bt - x0) / bt;
}

// y <- H y on the n entries y[k * ys]: y -= tau v (v^T y).
MQH_HD inline void apply(const double (&v)[kMaxB], double tau, int n, double* y, int64_t ys) {
    double yv[kMaxB];
    MQH_UNROLL
    for (int k = 0; k < kMaxB; ++k) yv[k] = k < n ? y[k * ys] : 0.0;
    double w = 0.0;
    MQH_UNROLL
    for (int k = 0; k < kMaxB; ++k) w = fma(v[k], yv[k], w);
    const double tw = tau * w;
    MQH_UNROLL
    for (int k = 0; k < kMaxB; ++k)
        if (k < n) y[k * ys] = fma(-tw, v[k], yv[k]);
}

// One Givens step of the lower-to-upper reduction of Bt^T ((N + 1) x N lower
// bidiagonal, alpha on the diagonal, beta below): with a the current
// diagonal entry of column j and bj = beta_{j+1}, the rotation of rows j and
// j + 1 that zeroes beta_{j+1}; it returns the new diagonal entry r >= 0 and
// (c, s) (c = 1, s = 0 when both are zero).
MQH_HD inline double givens(double a, double bj, double* c, double* s) {
    const double r = hypot(a, bj);
    if (r == 0.0) {
        *c = 1.0;
        *s = 0.0;
        return 0.0;
    }
    *c = a / r;
    *s = bj / r;
    return r;
}

}  // namespace band
}  // namespace mqh
