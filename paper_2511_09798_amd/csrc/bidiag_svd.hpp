// bidiag_svd.hpp -- scalar core of the projected SVD (Algorithm 2 step 2,
// Algorithm 4 step 2): the SVD of the (l+1) x l lower bidiagonal C_l with
// diagonal alpha_1..alpha_l and subdiagonal beta_2..beta_{l+1}, together with
// f~ = U~^T (beta_1 e_1).
//
// Method (implicit QR on the bidiagonal, Golub-Kahan with the zero-shift
// variant of Demmel and Kahan for relative accuracy):
//  1. Left Givens rotations reduce C to an upper bidiagonal B (l x l) plus a
//     zero row, and carry beta_1 e_1 along: g (l entries) and the residual
//     phibar = f~_{l+1} (up to sign) of min ||C y - beta_1 e_1||.
//  2. Implicit QR sweeps on B, chasing the bulge from top to bottom, with a
//     shift from the trailing 2 x 2 block or with zero shift when a shift
//     would cost relative accuracy.  Left rotations are applied to g at once
//     (so g ends as U_B^T g = f~_{1:l}); right rotations are recorded per
//     sweep (c, s for columns k, k+1) and applied to V by the caller.
//  3. Deflation by the relative test |e_k| <= tol * mu_k with the forward
//     recurrence mu_{k+1} = |d_{k+1}| mu_k / (mu_k + |e_k|).
// The functions are plain scalar code usable on the host and on the device.
#pragma once

#include <math.h>
#include <stdint.h>

#ifdef __HIPCC__
#define MQH_HD __host__ __device__
#else
#define MQH_HD
#endif

namespace mqh {
namespace bsvd {

constexpr double kEps = 2.220446049250313e-16;  // DBL_EPSILON
constexpr double kTol = 16.0 * kEps;            // relative deflation tolerance
constexpr double kTiny = 2.2250738585072014e-308;

// 1/sqrt(q) to about one ulp: on the device the hardware estimate refined by
// two Newton steps, on the host the library square root.
MQH_HD inline double inv_sqrt(double q) {
#ifdef __HIP_DEVICE_COMPILE__
    double y = __builtin_amdgcn_rsq(q);
    double h = q * y;
    double r = fma(-h, y, 1.0);
    y = fma(0.5 * y, r, y);
    h = q * y;
    r = fma(-h, y, 1.0);
    return fma(0.5 * y, r, y);
#else
    return 1.0 / sqrt(q);
#endif
}

// Givens rotation: c = f / r, s = g / r, r = sqrt(f^2 + g^2) >= 0, so that
// [c s; -s c] [f; g] = [r; 0].  The squares are formed directly when they
// neither overflow nor underflow, otherwise after scaling by max(|f|, |g|).
MQH_HD inline void make_rot(double f, double g, double& c, double& s, double& r) {
    if (g == 0.0) {
        c = f < 0.0 ? -1.0 : 1.0;
        s = 0.0;
        r = fabs(f);
        return;
    }
    if (f == 0.0) {
        c = 0.0;
        s = g < 0.0 ? -1.0 : 1.0;
        r = fabs(g);
        return;
    }
    const double q = fma(f, f, g * g);
    if (q > 1e-290 && q < 1e290) {
        const double inv = inv_sqrt(q);
        r = q * inv;
        c = f * inv;
        s = g * inv;
        return;
    }
    const double af = fabs(f), ag = fabs(g);
    const double mx = af > ag ? af : ag;
    const double mn = af > ag ? ag : af;
    const double t = mn / mx;
    r = mx * sqrt(1.0 + t * t);
    c = f / r;
    s = g / r;
}

// Step 1: C (lower bidiagonal, (l+1) x l) -> upper bidiagonal B (d, e) and
// g = first l entries of Q^T (beta_1 e_1); returns the last entry (the
// least-squares residual, signed).
MQH_HD inline double reduce_lower(const double* alpha, const double* beta, int l, double* d, double* e, double* g) {
    double rhobar = alpha[0];
    double phibar = beta[0];
    for (int i = 0; i < l; ++i) {
        double c, s, rho;
        make_rot(rhobar, beta[i + 1], c, s, rho);
        d[i] = rho;
        g[i] = c * phibar;
        phibar = -s * phibar;
        if (i + 1 < l) {
            e[i] = s * alpha[i + 1];
            rhobar = c * alpha[i + 1];
        }
    }
    return phibar;
}

// Smallest singular value of the 2 x 2 upper triangular [f h; 0 k]:
// s_max s_min = |f k| and s_max = (sqrt((|f|+|k|)^2 + h^2) + sqrt((|f|-|k|)^2 + h^2)) / 2.
MQH_HD inline double smin2(double f, double h, double k) {
    const double af = fabs(f), ah = fabs(h), ak = fabs(k);
    double sc = af > ah ? af : ah;
    sc = sc > ak ? sc : ak;
    if (sc == 0.0) return 0.0;
    const double a = af / sc, b = ah / sc, cc = ak / sc;
    const double smax = 0.5 * (sqrt((a + cc) * (a + cc) + b * b) + sqrt((a - cc) * (a - cc) + b * b));
    if (smax == 0.0) return 0.0;
    return sc * ((a * cc) / smax);
}

// One bulge-chasing sweep with shift mu on rows/columns ll..m (upper
// bidiagonal d, e).  Records right rotations in rc/rs[0 .. m-ll-1] and
// applies left rotations to g.  The running entries are carried in
// registers; each array element is read once and written once.
MQH_HD inline void sweep_shifted(double* d, double* e, double* g, int ll, int m, double mu, double* rc, double* rs) {
    double dk = d[ll], ek = e[ll], gk = g[ll];
    double f = (fabs(dk) - mu) * ((dk < 0.0 ? -1.0 : 1.0) + mu / dk);
    double gg = ek;
    for (int k = ll; k < m; ++k) {
        double dk1 = d[k + 1];
        double ek1 = k + 1 < m ? e[k + 1] : 0.0;
        const double gk1 = g[k + 1];
        double c, s, r;
        make_rot(f, gg, c, s, r);  // right rotation, columns k, k+1
        if (k > ll) e[k - 1] = r;
        f = c * dk + s * ek;
        ek = c * ek - s * dk;
        gg = s * dk1;
        dk1 = c * dk1;
        rc[k - ll] = c;
        rs[k - ll] = s;
        make_rot(f, gg, c, s, r);  // left rotation, rows k, k+1
        d[k] = r;
        f = c * ek + s * dk1;
        dk1 = c * dk1 - s * ek;
        if (k + 1 < m) {
            gg = s * ek1;
            ek1 = c * ek1;
        }
        g[k] = c * gk + s * gk1;
        gk = -s * gk + c * gk1;
        dk = dk1;
        ek = ek1;
    }
    e[m - 1] = f;
    d[m] = dk;
    g[m] = gk;
}

// Zero-shift sweep (Demmel-Kahan): the shifted sweep with mu = 0, written
// so that no cancellation occurs and tiny singular values keep their
// relative accuracy.
MQH_HD inline void sweep_zero(double* d, double* e, double* g, int ll, int m, double* rc, double* rs) {
    double cs = 1.0, sn = 0.0, oldcs = 1.0, oldsn = 0.0, r;
    double dk = d[ll], gk = g[ll];
    for (int k = ll; k < m; ++k) {
        const double ek = e[k];
        const double dk1 = d[k + 1];
        const double gk1 = g[k + 1];
        make_rot(dk * cs, ek, cs, sn, r);
        if (k > ll) e[k - 1] = oldsn * r;
        double dnew;
        make_rot(oldcs * r, dk1 * sn, oldcs, oldsn, dnew);
        d[k] = dnew;
        rc[k - ll] = cs;
        rs[k - ll] = sn;
        g[k] = oldcs * gk + oldsn * gk1;
        gk = -oldsn * gk + oldcs * gk1;
        dk = dk1;
    }
    const double h = dk * cs;
    d[m] = h * oldcs;
    e[m - 1] = h * oldsn;
    g[m] = gk;
}

// Driver state between sweeps.
struct Driver {
    int n;       // matrix size l
    int m;       // bottom index of the part not yet converged
    long iters;  // inner rotation steps so far
    long maxit;  // limit on inner steps (6 n^2)
    int status;  // 0 running, 1 converged, -1 no convergence
};

MQH_HD inline void driver_init(Driver& dv, int n) {
    dv.n = n;
    dv.m = n - 1;
    dv.iters = 0;
    dv.maxit = 6L * n * n + 64;
    dv.status = n <= 1 ? 1 : 0;
}

// Advances to the next sweep and performs it.  Returns 1 after a sweep on
// rows ll..m (*ll_out, *m_out set; the rotations in rc/rs must then be
// applied to V), 0 when converged, -1 on failure.
MQH_HD inline int driver_step(Driver& dv, double* d, double* e, double* g, double* rc, double* rs, int* ll_out,
                              int* m_out) {
    for (;;) {
        if (dv.status != 0) return dv.status > 0 ? 0 : -1;
        const int m = dv.m;
        if (m <= 0) {
            dv.status = 1;
            return 0;
        }
        // bottom deflation
        if (fabs(e[m - 1]) <= kTol * fabs(d[m]) || fabs(e[m - 1]) <= kTiny) {
            e[m - 1] = 0.0;
            dv.m = m - 1;
            continue;
        }
        // top of the unreduced block
        int ll = m - 1;
        while (ll > 0 && e[ll - 1] != 0.0) --ll;
        // one pass over the block: relative test with the forward recurrence
        // mu_{k+1} = |d_{k+1}| mu_k / (mu_k + |e_k|), smallest mu (an estimate of
        // the smallest singular value), largest entry, exactly zero diagonal
        double mu = fabs(d[ll]);
        double sminl = mu, smax = mu;
        bool split = false, zero = d[ll] == 0.0;
        for (int k = ll; k < m; ++k) {
            const double aek = fabs(e[k]);
            if (aek <= kTol * mu) {
                e[k] = 0.0;
                split = true;
                break;
            }
            const double adk1 = fabs(d[k + 1]);
            mu = adk1 * (mu / (mu + aek));
            sminl = mu < sminl ? mu : sminl;
            smax = aek > smax ? aek : smax;
            smax = adk1 > smax ? adk1 : smax;
            zero = zero || adk1 == 0.0;
        }
        if (split) continue;
        // an exactly zero diagonal entry: perturb within rounding of the block norm
        if (zero)
            for (int k = ll; k <= m; ++k)
                if (d[k] == 0.0) d[k] = kEps * kEps * smax;
        if (dv.iters > dv.maxit) {
            dv.status = -1;
            return -1;
        }
        // shift
        double shift = 0.0;
        if ((double)dv.n * kTol * (sminl / smax) > kEps) {
            shift = smin2(d[m - 1], e[m - 1], d[m]);
            const double sll = fabs(d[ll]);
            if (sll > 0.0 && (shift / sll) * (shift / sll) < kEps) shift = 0.0;
        }
        if (shift == 0.0)
            sweep_zero(d, e, g, ll, m, rc, rs);
        else
            sweep_shifted(d, e, g, ll, m, shift, rc, rs);
        dv.iters += m - ll;
        *ll_out = ll;
        *m_out = m;
        return 1;
    }
}

// Applies the recorded right rotations of one sweep to one row of V,
// V[row, ll..m], with V column-major (V[k * ldv + row]).  Entries are
// loaded eight at a time ahead of the rotation chain.
MQH_HD inline void apply_row(double* V, int64_t ldv, int row, int ll, int m, const double* rc, const double* rs) {
    double x = V[(int64_t)ll * ldv + row];
    for (int k0 = ll; k0 < m; k0 += 8) {
        const int cnt = m - k0 < 8 ? m - k0 : 8;
        double y[8];
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (q < cnt) y[q] = V[(int64_t)(k0 + 1 + q) * ldv + row];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            if (q < cnt) {
                const double c = rc[k0 - ll + q], s = rs[k0 - ll + q];
                V[(int64_t)(k0 + q) * ldv + row] = c * x + s * y[q];
                x = -s * x + c * y[q];
            }
        }
    }
    V[(int64_t)m * ldv + row] = x;
}

}  // namespace bsvd
}  // namespace mqh
