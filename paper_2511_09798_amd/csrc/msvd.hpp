// msvd.hpp -- scalar recurrences of the projected SVD by multisection and
// twisted factorisations (the fast path of Algorithm 2 step 2 and
// Algorithm 4 step 2; the implicit QR iteration of bidiag_svd.hpp is the
// fallback).  Usable on the host and on the device.
//
// After the left rotations that reduce C_l to an upper bidiagonal B (d on
// the diagonal, e above it), the squared singular values of B are the
// eigenvalues of
//     B^T B = L D L^T,  D_i = d_i^2,  L_i = e_i / d_i   (so L_i^2 D_i = e_i^2,
//                                                          D_i L_i = d_i e_i),
// and of B B^T, which is the same form on the reversed sequences
// (d_{n-1}, .., d_0), (e_{n-2}, .., e_0).  A bidiagonal determines its
// singular values to high relative accuracy, and so do these factored forms;
// the differential qd transforms below work on them without forming B^T B:
//  * negcount: the stationary transform L D L^T - x I = L+ D+ L+^T; the
//    number of negative D+_i is the number of eigenvalues below x
//    (Sylvester's law of inertia), which drives the bisection of the values;
//  * stationary + progressive_twist: the top-down (L+ D+ L+^T) and bottom-up
//    (U- D- U-^T) factorisations of L D L^T - lambda I at an eigenvalue
//    lambda; gamma_k = s_k + p_k + lambda is the pivot of the factorisation
//    twisted at k, and the k of least |gamma_k| gives the eigenvector by one
//    step of inverse iteration (twisted_solve) with z_k = 1.
// Pivots below pivmin in magnitude are replaced by -pivmin (a perturbation
// of x within the rounding of the data), so no recurrence divides by zero;
// in the count a quotient that comes out NaN is taken as 1.
#pragma once

#include <math.h>
#include <stdint.h>

#ifdef __HIPCC__
#define MQH_HD __host__ __device__
#else
#define MQH_HD
#endif

namespace mqh {
namespace msvd {

// Number of eigenvalues of L D L^T below x, from d2 = d^2 (n) and e2 = e^2
// (n - 1).  Elements are read at d2[i * ds], e2[i * es] (ds, es = +1 or -1 on
// suitably placed pointers give the reversed sequences).
MQH_HD inline int negcount(const double* d2, int ds, const double* e2, int es, int n, double x, double pivmin) {
    double s = -x;
    int neg = 0;
    for (int i = 0; i < n - 1; ++i) {
        double dp = s + d2[i * ds];
        dp = fabs(dp) < pivmin ? -pivmin : dp;
        neg += dp < 0.0 ? 1 : 0;
        double t = s / dp;
        t = t == t ? t : 1.0;
        s = t * e2[i * es] - x;
    }
    double dp = s + d2[(n - 1) * ds];
    dp = fabs(dp) < pivmin ? -pivmin : dp;
    return neg + (dp < 0.0 ? 1 : 0);
}

// Top-down transform at lambda: s_0 = -lambda; for i < n - 1,
// D+_i = s_i + d_i^2, L+_i = d_i e_i / D+_i, s_{i+1} = e_i^2 s_i / D+_i - lambda.
// Writes s[0..n-1] and lp[0..n-2].
MQH_HD inline void stationary(const double* d, int ds, const double* e, int es, int n, double lam, double pivmin,
                              double* lp, double* s) {
    double si = -lam;
    for (int i = 0; i < n - 1; ++i) {
        const double di = d[i * ds], ei = e[i * es];
        s[i] = si;
        double dp = si + di * di;
        dp = fabs(dp) < pivmin ? -pivmin : dp;
        const double r = 1.0 / dp;
        lp[i] = (di * ei) * r;
        si = (ei * ei) * (si * r) - lam;
    }
    s[n - 1] = si;
}

// Bottom-up transform at lambda: p_{n-1} = d_{n-1}^2 - lambda; for
// i = n-2 .. 0, D-_{i+1} = e_i^2 + p_{i+1}, U-_i = d_i e_i / D-_{i+1},
// p_i = p_{i+1} d_i^2 / D-_{i+1} - lambda; with gamma_k = s_k + p_k + lambda
// on the way.  Returns the twist index r = argmin |gamma_k| (the smallest k
// on ties) and its gamma; U-_i replaces s_i in su (s_i is read first).
MQH_HD inline int progressive_twist(const double* d, int ds, const double* e, int es, int n, double lam,
                                    double pivmin, double* su, double* gamma_r) {
    double p = d[(n - 1) * ds] * d[(n - 1) * ds] - lam;
    double gbest = su[n - 1] + p + lam;
    int r = n - 1;
    for (int i = n - 2; i >= 0; --i) {
        const double di = d[i * ds], ei = e[i * es];
        double dm = ei * ei + p;
        dm = fabs(dm) < pivmin ? -pivmin : dm;
        const double q = 1.0 / dm;
        const double um = (di * ei) * q;
        p = p * (di * di) * q - lam;
        const double g = su[i] + p + lam;
        if (fabs(g) <= fabs(gbest)) {  // ties to the smaller index
            gbest = g;
            r = i;
        }
        su[i] = um;
    }
    *gamma_r = gbest;
    return r;
}

// One direction of the twisted solve from z_r = 1: dir < 0 gives
// z_i = -L+_i z_{i+1} for i = r-1 .. 0, dir > 0 gives z_{i+1} = -U-_i z_i for
// i = r .. n-2.  z shares storage with lp (lp_i is read before z_i is
// written, and the two directions touch disjoint entries); z_r itself is
// set by the caller.
MQH_HD inline void twisted_solve(double* lp_z, const double* um, int n, int r, int dir) {
    double z = 1.0;
    if (dir < 0) {
        for (int i = r - 1; i >= 0; --i) {
            z = -lp_z[i] * z;
            lp_z[i] = z;
        }
    } else {
        for (int i = r; i < n - 1; ++i) {
            z = -um[i] * z;
            lp_z[i + 1] = z;
        }
    }
}

// d x + e y - s w for one row of B v - s u (or B^T u - s v) with the
// rounding error of e y added back (two-product by fma): near a singular
// triple d x + e y nearly cancels against s w, and without the correction
// the rounding of the products, eps (|d x| + |e y|), would swamp a residual
// that is small relative to a tiny s.
MQH_HD inline double resid_row(double d, double x, double e, double y, double s, double w) {
    const double p = e * y;
    const double pe = fma(e, y, -p);
    const double q = fma(d, x, p);
    return fma(-s, w, q) + pe;
}

// Multisection points: P points strictly inside (lo, hi), equally spaced in
// log2 while the bracket spans more than a factor of two (from
// max(lo, hi 2^-1000) when lo = 0), equally spaced otherwise.
MQH_HD inline double section_point(double lo, double hi, int t, int P) {
    const double f = (double)(t + 1) / (double)(P + 1);
    if (lo == 0.0 || hi > 2.0 * lo) {
        const double a = log2(lo > hi * 0x1p-1000 ? lo : hi * 0x1p-1000);
        const double b = log2(hi);
        return exp2(a + (b - a) * f);
    }
    return lo + (hi - lo) * f;
}

// Upper bound of the eigenvalues of B^T B: the square of max_i (|d_i| + |e_i|, |d_i| + |e_{i-1}|),
// which bounds ||B||_2 by the geometric mean of the 1- and infinity-norms.
MQH_HD inline double eig_bound(const double* d, const double* e, int n) {
    double m = 0.0;
    for (int i = 0; i < n; ++i) {
        const double a = fabs(d[i]);
        const double r = a + (i < n - 1 ? fabs(e[i]) : 0.0);
        const double c = a + (i > 0 ? fabs(e[i - 1]) : 0.0);
        m = r > m ? r : m;
        m = c > m ? c : m;
    }
    return m * m * (1.0 + 64.0 * 2.220446049250313e-16);
}

// Thresholds of the fast path's acceptance test: the Gram matrices of the
// computed right and left vectors within kOrthTol of I, and for every
// triple max(||B v - s u||, ||B^T u - s v||) <= resid_bound(s, s_1, n).  The
// absolute term is the floor that rounding the vectors to double already
// puts under any residual (about eps sqrt(n) s_1), with a wide margin.
constexpr double kOrthTol = 1e-9;
constexpr double kResTol = 1e-9;
MQH_HD inline double resid_bound(double s, double s1, int n) {
    return kResTol * s + 64.0 * (double)n * 2.220446049250313e-16 * s1;
}
constexpr int kSections = 256;  // multisection points per round

}  // namespace msvd
}  // namespace mqh
