// proj_kernels.hip -- the projected problem on the device (one workgroup
// each): SVD of C_l (Algorithm 2 step 2, Algorithm 4 step 2), parameter
// choice by GCV (optionally weighted) / L-curve / projected TSVD-GCV
// (Section 3.2-3.3), the projected solution y (Algorithm 2 step 5,
// Algorithm 4 step 8, SVD form), and the LSQR iterates with their stopping
// index (Section 3.4).
#include <float.h>

#include "bidiag_svd.hpp"
#include "kernels.hpp"

namespace mqh {

constexpr int kProjThreads = 256;

// ---------------------------------------------------------------------------
// SVD of C_l by the implicit QR iteration (the fallback of the fast path in
// svd_kernels.hip).  Lane 0 of wave 0 runs the scalar bulge chase; the other
// four waves apply the right rotations of the previous sweep to their rows
// of the work matrix Vw (the workspace's U, column-major, ld = L) at the same
// time, through two rotation buffers.  Outputs: sv (descending), ftil (l+1),
// V (ld = ldv).  l is taken from *l_ptr when given (steps kept by the
// Golub-Kahan run).  With flagged_only the kernel returns at once unless the
// fast path flagged the problem.  status[0] = 1 on convergence, -1 if the
// iteration limit was hit.
// ---------------------------------------------------------------------------
constexpr int kSvdThreads = kProjThreads + kWave;  // one chain wave + four applier waves

__global__ __launch_bounds__(kSvdThreads) void k_bidiag_svd(const double* __restrict__ alpha,
                                                            const double* __restrict__ beta, int32_t L,
                                                            const int32_t* __restrict__ l_ptr,
                                                            double* __restrict__ ws, double* __restrict__ sv,
                                                            double* __restrict__ ftil, double* __restrict__ V,
                                                            int64_t ldv, int32_t* __restrict__ status,
                                                            int32_t flagged_only, ProjBatch pb) {
    const int64_t z = blockIdx.x;  // batch: problem z
    const SvdWs wsz = svd_ws(ws + z * pb.ws, L);
    if (flagged_only && wsz.flag[1] == 0) return;
    double* __restrict__ Vw = wsz.U;
    const int64_t ldw = L;
    alpha += z * pb.vec;
    beta += z * pb.vec;
    if (l_ptr != nullptr) l_ptr += z * pb.lstr;
    sv += z * pb.vec;
    ftil += z * pb.vec;
    V += z * pb.mat;
    if (status != nullptr) status += z;
    __shared__ double d[kMaxEll], e[kMaxEll], g[kMaxEll];
    __shared__ double rc[2][kMaxEll], rs[2][kMaxEll];
    __shared__ int rank[kMaxEll];
    __shared__ int s_ll[2], s_m[2], s_res[2];
    const int tid = threadIdx.x;
    const int l = l_ptr != nullptr ? *l_ptr : L;
    if (l <= 0) {
        if (tid == 0) {
            if (status) status[0] = 1;
            ftil[0] = beta[0];
        }
        return;
    }
    for (int64_t idx = tid; idx < (int64_t)l * l; idx += kSvdThreads) {
        const int64_t col = idx / l, row = idx % l;
        Vw[col * ldw + row] = (col == row) ? 1.0 : 0.0;
    }
    bsvd::Driver dv;
    if (tid == 0) {
        for (int i = 0; i < l; ++i) e[i] = 0.0;
        ftil[l] = bsvd::reduce_lower(alpha, beta, l, d, e, g);
        bsvd::driver_init(dv, l);
        int ll = 0, m = 0;
        s_res[0] = bsvd::driver_step(dv, d, e, g, rc[0], rs[0], &ll, &m);
        s_ll[0] = ll;
        s_m[0] = m;
    }
    __syncthreads();
    int b = 0;
    for (;;) {
        if (s_res[b] != 1) break;  // block-uniform
        if (tid >= kWave) {
            const int ll = s_ll[b], m = s_m[b];
            for (int row = tid - kWave; row < l; row += kSvdThreads - kWave)
                bsvd::apply_row(Vw, ldw, row, ll, m, rc[b], rs[b]);
        } else if (tid == 0) {
            int ll = 0, m = 0;
            s_res[1 - b] = bsvd::driver_step(dv, d, e, g, rc[1 - b], rs[1 - b], &ll, &m);
            s_ll[1 - b] = ll;
            s_m[1 - b] = m;
        }
        __syncthreads();
        b = 1 - b;
    }
    if (tid == 0 && status != nullptr) status[0] = s_res[b] == 0 ? 1 : -1;
    // order descending: rank of |d_i| among all (ties by index), one i per thread
    for (int i = tid; i < l; i += kSvdThreads) {
        const double si = fabs(d[i]);
        int rk = 0;
        for (int j = 0; j < l; ++j) {
            const double sj = fabs(d[j]);
            rk += (sj > si || (sj == si && j < i)) ? 1 : 0;
        }
        rank[i] = rk;
    }
    __syncthreads();
    for (int i = tid; i < l; i += kSvdThreads) {
        sv[rank[i]] = fabs(d[i]);
        ftil[rank[i]] = g[i];
    }
    for (int64_t idx = tid; idx < (int64_t)l * l; idx += kSvdThreads) {
        const int64_t i = idx / l, row = idx % l;
        const double sg = d[i] < 0.0 ? -1.0 : 1.0;
        V[(int64_t)rank[i] * ldv + row] = sg * Vw[i * ldw + row];
    }
}

// ---------------------------------------------------------------------------
// Parameter choice
// ---------------------------------------------------------------------------

// GCV numerator and trace sum for one lambda, evaluated by one thread.
__device__ inline void gcv_terms(const double* sv, const double* ft, int l, double lam, double& num, double& tr) {
    const double l2 = lam * lam;
    double a = 0.0, t = 0.0;
    for (int i = 0; i < l; ++i) {
        const double s2 = sv[i] * sv[i];
        const double den = s2 + l2;
        const double psi = l2 / den;
        const double x = psi * ft[i];
        a = fma(x, x, a);
        t += s2 / den;
    }
    num = fma(ft[l], ft[l], a);
    tr = t;
}

// rho_l^2 / ((l+1) - omega sum_i phi_i)^2: eq. (30) for omega = 1, the
// weighted GCV otherwise.
__device__ inline double gcv_value(const double* sv, const double* ft, int l, double lam, double omega) {
    double num, tr;
    gcv_terms(sv, ft, l, lam, num, tr);
    const double den = (double)(l + 1) - omega * tr;
    return num / (den * den);
}

// Signed curvature of (log rho, log eta) in t = log lambda (analytic derivatives,
// d phi_i / dt = -2 phi_i psi_i).
__device__ inline double lcurve_kappa(const double* sv, const double* ft, int l, double lam) {
    const double l2 = lam * lam;
    double R = ft[l] * ft[l], R1 = 0.0, R2 = 0.0, E = 0.0, E1 = 0.0, E2 = 0.0;
    for (int i = 0; i < l; ++i) {
        const double s2 = sv[i] * sv[i];
        const double den = s2 + l2;
        const double ph = s2 / den, ps = l2 / den;
        const double f2 = ft[i] * ft[i];
        const double g2 = f2 / s2;
        R += ps * ps * f2;
        R1 += 4.0 * ph * ps * ps * f2;
        R2 += 8.0 * f2 * ph * ps * ps * (2.0 * ph - ps);
        E += ph * ph * g2;
        E1 += -4.0 * ph * ph * ps * g2;
        E2 += 8.0 * g2 * ph * ph * ps * (2.0 * ps - ph);
    }
    const double x1 = R1 / (2.0 * R), x2 = (R2 * R - R1 * R1) / (2.0 * R * R);
    const double y1 = E1 / (2.0 * E), y2 = (E2 * E - E1 * E1) / (2.0 * E * E);
    const double q = x1 * x1 + y1 * y1;
    return (x1 * y2 - x2 * y1) / (q * sqrt(q));
}

// Block-parallel (weighted) GCV for the refinement loop.
__device__ inline double gcv_block(const double* sv, const double* ft, int l, double lam, double omega, double* lds) {
    const double l2 = lam * lam;
    double a = 0.0, t = 0.0;
    for (int i = threadIdx.x; i < l; i += kProjThreads) {
        const double s2 = sv[i] * sv[i];
        const double den = s2 + l2;
        const double x = (l2 / den) * ft[i];
        a = fma(x, x, a);
        t += s2 / den;
    }
    a = block_sum<kProjThreads>(a, lds);
    t = block_sum<kProjThreads>(t, lds);
    const double num = fma(ft[l], ft[l], a);
    const double den = (double)(l + 1) - omega * t;
    return num / (den * den);
}

__global__ __launch_bounds__(kProjThreads) void k_param_choice(const double* __restrict__ sv,
                                                               const double* __restrict__ ft, int32_t l_arg,
                                                               const int32_t* __restrict__ l_ptr, int32_t method,
                                                               int32_t rule, int32_t J, double lambda_fixed,
                                                               int32_t k_fixed, double omega_arg,
                                                               double* __restrict__ curve,
                                                               ParamOut* __restrict__ out, ProjBatch pb) {
    {
        const int64_t z = blockIdx.x;  // batch: problem z
        sv += z * pb.vec;
        ft += z * pb.vec;
        if (l_ptr != nullptr) l_ptr += z * pb.lstr;
        if (curve != nullptr) curve += z * pb.curve;
        out += z;
    }
    __shared__ double vals[kMaxGrid];
    __shared__ double lds[kProjThreads / kWave];
    __shared__ double s_lo, s_hi;
    const int tid = threadIdx.x;
    const int l = l_ptr != nullptr ? *l_ptr : l_arg;
    // rule 3: weighted GCV (rule 0 with the trace term scaled by omega)
    const double omega = rule == 3 ? omega_arg : 1.0;
    if (rule == 3) rule = 0;
    if (l <= 0) {
        if (tid == 0) {
            out->lambda = 0.0;
            out->k = 0;
            out->crit = 0.0;
            out->flags = 0;
            out->rho = ft[0] >= 0.0 ? ft[0] : -ft[0];
            out->eta = 0.0;
        }
        return;
    }
    if (method == 0) {  // Ine-TSVD
        if (tid == 0) {
            int k;
            const int kmax = l / 2 > 1 ? l / 2 : 1;
            // suffix sums r_k = sum_{i >= k} ft_i^2 over 0-based i in [k, l]
            double best = 0.0;
            int bestk = 1;
            if (rule == 2) {
                k = k_fixed < 1 ? 1 : (k_fixed > l ? l : k_fixed);
            } else {
                double tail = ft[l] * ft[l];
                for (int i = l - 1; i >= kmax; --i) tail = fma(ft[i], ft[i], tail);
                // tail now = sum_{i >= kmax} ; walk k downwards to 1
                double den = (double)(l + 1) - omega * (double)kmax;
                double gk = tail / (den * den);
                best = gk;
                bestk = kmax;
                for (int kk = kmax - 1; kk >= 1; --kk) {
                    tail = fma(ft[kk], ft[kk], tail);
                    den = (double)(l + 1) - omega * (double)kk;
                    gk = tail / (den * den);
                    if (gk <= best) {  // ties -> smaller k
                        best = gk;
                        bestk = kk;
                    }
                }
                k = bestk;
            }
            double res = ft[l] * ft[l], nrm = 0.0;
            for (int i = k; i < l; ++i) res = fma(ft[i], ft[i], res);
            for (int i = 0; i < k; ++i) {
                const double q = ft[i] / sv[i];
                nrm = fma(q, q, nrm);
            }
            const double den = (double)(l + 1) - omega * (double)k;
            out->lambda = 0.0;
            out->k = k;
            out->crit = res / (den * den);
            out->flags = 0;
            out->rho = sqrt(res);
            out->eta = sqrt(nrm);
        }
        return;
    }
    // HKT: lambda
    double lam = lambda_fixed, crit = 0.0;
    uint32_t flags = 0;
    if (rule != 2) {
        if (tid == 0) {
            const double hi = sv[0];
            double lo = sv[l - 1] > 16.0 * DBL_EPSILON * hi ? sv[l - 1] : 16.0 * DBL_EPSILON * hi;
            if (!(lo < hi)) lo = 16.0 * DBL_EPSILON * hi;
            s_lo = log(lo);
            s_hi = log(hi);
        }
        __syncthreads();
        const double t0 = s_lo, t1 = s_hi;
        const double step = (t1 - t0) / (double)(J - 1);
        for (int j = tid; j < J; j += kProjThreads) {
            const double lj = j == J - 1 ? exp(t1) : exp(t0 + step * (double)j);
            const double v = rule == 0 ? gcv_value(sv, ft, l, lj, omega) : lcurve_kappa(sv, ft, l, lj);
            vals[j] = v;
            if (curve != nullptr) curve[j] = v;
        }
        __syncthreads();
        __shared__ int s_k;
        if (tid == 0) {
            int kb;
            if (rule == 0) {  // argmin, ties -> larger lambda
                kb = 0;
                for (int j = 1; j < J; ++j)
                    if (vals[j] <= vals[kb]) kb = j;
                if (kb == 0 || kb == J - 1) flags |= 2u;
            } else {  // argmax over inner points, ties -> larger lambda
                kb = 1;
                for (int j = 2; j < J - 1; ++j)
                    if (vals[j] >= vals[kb]) kb = j;
                if (kb == 1 || kb == J - 2) flags |= 4u;
            }
            s_k = kb;
        }
        __syncthreads();
        const int kb = s_k;
        const double tk = kb == J - 1 ? t1 : t0 + step * (double)kb;
        lam = exp(tk);
        crit = vals[kb];
        if (rule == 0 && kb > 0 && kb < J - 1) {
            // golden-section search of log(lambda) on the two cells around the grid minimum
            const double gr = 0.6180339887498949;  // (sqrt(5) - 1) / 2
            double a = t0 + step * (double)(kb - 1);
            double b = kb + 1 == J - 1 ? t1 : t0 + step * (double)(kb + 1);
            double c = b - gr * (b - a), dd = a + gr * (b - a);
            double fc = gcv_block(sv, ft, l, exp(c), omega, lds), fd = gcv_block(sv, ft, l, exp(dd), omega, lds);
            int it = 0;
            while (fabs(b - a) > 1e-10 && it < 200) {
                if (fc < fd) {
                    b = dd;
                    dd = c;
                    fd = fc;
                    c = b - gr * (b - a);
                    fc = gcv_block(sv, ft, l, exp(c), omega, lds);
                } else {
                    a = c;
                    c = dd;
                    fc = fd;
                    dd = a + gr * (b - a);
                    fd = gcv_block(sv, ft, l, exp(dd), omega, lds);
                }
                ++it;
            }
            const double lr = exp(0.5 * (a + b));
            const double gv = gcv_block(sv, ft, l, lr, omega, lds);
            if (!(gv > crit)) {
                lam = lr;
                crit = gv;
            }
        }
    }
    // rho, eta at the chosen lambda
    {
        const double l2 = lam * lam;
        double r = 0.0, e = 0.0;
        for (int i = tid; i < l; i += kProjThreads) {
            const double s2 = sv[i] * sv[i];
            const double den = s2 + l2;
            const double x = (l2 / den) * ft[i];
            const double q = (sv[i] / den) * ft[i];
            r = fma(x, x, r);
            e = fma(q, q, e);
        }
        r = block_sum<kProjThreads>(r, lds);
        e = block_sum<kProjThreads>(e, lds);
        if (tid == 0) {
            out->lambda = lam;
            out->k = 0;
            out->crit = rule == 2 ? gcv_value(sv, ft, l, lam, 1.0) : crit;
            out->flags = flags;
            out->rho = sqrt(fma(ft[l], ft[l], r));
            out->eta = sqrt(e);
        }
    }
}

// y_r = sum_i V[i][r] w_i with w_i = s_i/(s_i^2+lambda^2) f~_i (HKT) or
// f~_i/s_i for i < k (Ine-TSVD); lambda and k from *po when given.
__global__ __launch_bounds__(kBlock) void k_proj_solution(const double* __restrict__ sv,
                                                          const double* __restrict__ ft,
                                                          const double* __restrict__ V, int64_t ldv, int32_t l_arg,
                                                          const int32_t* __restrict__ l_ptr, int32_t method,
                                                          double lambda, int32_t k, const ParamOut* __restrict__ po,
                                                          double* __restrict__ y, ProjBatch pb) {
    {
        const int64_t z = blockIdx.y;  // batch: problem z
        sv += z * pb.vec;
        ft += z * pb.vec;
        V += z * pb.mat;
        if (l_ptr != nullptr) l_ptr += z * pb.lstr;
        if (po != nullptr) po += z;
        y += z * pb.vec;
    }
    const int l = l_ptr != nullptr ? *l_ptr : l_arg;
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= l) return;
    const double lam = po != nullptr ? po->lambda : lambda;
    const int kk = po != nullptr ? po->k : k;
    const double l2 = lam * lam;
    double s = 0.0;
    if (method == 1) {
        for (int i = 0; i < l; ++i) {
            const double w = sv[i] / (sv[i] * sv[i] + l2) * ft[i];
            s = fma(V[(int64_t)i * ldv + r], w, s);
        }
    } else {
        for (int i = 0; i < kk && i < l; ++i) s = fma(V[(int64_t)i * ldv + r], ft[i] / sv[i], s);
    }
    y[r] = s;
}

// ---------------------------------------------------------------------------
// LSQR iterates on the projected problem (Section 3.4).  The k-th LSQR
// iterate is Z_k y_k with y_k = argmin ||C_k y - beta_1 e_1||.  Left Givens
// rotations reduce C_l to upper bidiagonal R (d, e) column by column while
// carrying beta_1 e_1 (g); after k rotations the leading k x k block of R and
// g_{1:k} are those of C_k, and the carried remainder is the residual
// rho_k = ||C_k y_k - beta_1 e_1||.  eta_k = ||y_k|| by back substitution,
// one k per thread.  Stopping index: rule 0 minimises rho_k^2 / (n - k)^2
// over k <= min(l, n - 1) (the influence matrix of the k-th iterate is a
// rank-k projector), ties to the smaller k; rule 1 takes the corner of the
// discrete L-curve p_k = (log rho_k, log eta_k): the largest signed Menger
// curvature of (p_{k+1}, p_k, p_{k-1}) over k = 2..l-1 (triples with a side
// below 1e-12 of the extent of the points skipped; ties to the smaller k;
// k = l with the edge flag when none qualifies); rule 2 takes k = k_fixed.
// Outputs: y (l_max entries, y_k then zeros), out (k, crit, rho, eta,
// flags), and rho / eta for every k when given.
// ---------------------------------------------------------------------------

__device__ inline double menger(double ax, double ay, double bx, double by, double cx, double cy) {
    const double ux = bx - ax, uy = by - ay, vx = cx - bx, vy = cy - by, wx = cx - ax, wy = cy - ay;
    const double la = sqrt(ux * ux + uy * uy), lb = sqrt(vx * vx + vy * vy), lc = sqrt(wx * wx + wy * wy);
    return 2.0 * (ux * vy - uy * vx) / (la * lb * lc);
}

__global__ __launch_bounds__(kProjThreads) void k_lsqr(const double* __restrict__ alpha,
                                                       const double* __restrict__ beta, int32_t l_arg,
                                                       const int32_t* __restrict__ l_ptr, int64_t n, int32_t rule,
                                                       int32_t k_fixed, double* __restrict__ rho_out,
                                                       double* __restrict__ eta_out, ParamOut* __restrict__ out,
                                                       double* __restrict__ y, int32_t l_max, ProjBatch pb) {
    {
        const int64_t z = blockIdx.x;  // batch: problem z
        alpha += z * pb.vec;
        beta += z * pb.vec;
        if (l_ptr != nullptr) l_ptr += z * pb.lstr;
        if (rho_out != nullptr) rho_out += z * pb.vec;
        if (eta_out != nullptr) eta_out += z * pb.vec;
        out += z;
        y += z * pb.vec;
    }
    __shared__ double d[kMaxEll], e[kMaxEll], g[kMaxEll], rho[kMaxEll], eta[kMaxEll];
    __shared__ int s_k;
    const int tid = threadIdx.x;
    const int l = l_ptr != nullptr ? *l_ptr : l_arg;
    for (int i = tid; i < l_max; i += kProjThreads) y[i] = 0.0;
    if (l <= 0) {
        if (tid == 0) {
            out->lambda = 0.0;
            out->k = 0;
            out->crit = 0.0;
            out->flags = 0;
            out->rho = fabs(beta[0]);
            out->eta = 0.0;
        }
        return;
    }
    if (tid == 0) {
        double rhobar = alpha[0], phibar = beta[0];
        for (int i = 0; i < l; ++i) {
            double c, s, r;
            bsvd::make_rot(rhobar, beta[i + 1], c, s, r);
            d[i] = r;
            g[i] = c * phibar;
            phibar = -s * phibar;
            rho[i] = fabs(phibar);
            if (i + 1 < l) {
                e[i] = s * alpha[i + 1];
                rhobar = c * alpha[i + 1];
            }
        }
    }
    __syncthreads();
    for (int k = tid + 1; k <= l; k += kProjThreads) {
        double yi = g[k - 1] / d[k - 1];
        double ss = yi * yi;
        for (int i = k - 2; i >= 0; --i) {
            yi = (g[i] - e[i] * yi) / d[i];
            ss = fma(yi, yi, ss);
        }
        eta[k - 1] = sqrt(ss);
    }
    __syncthreads();
    for (int i = tid; i < l; i += kProjThreads) {
        if (rho_out) rho_out[i] = rho[i];
        if (eta_out) eta_out[i] = eta[i];
    }
    if (tid == 0) {
        int k = l;
        double crit = 0.0;
        uint32_t flags = 0;
        if (rule == 2) {
            k = k_fixed < 1 ? 1 : (k_fixed > l ? l : k_fixed);
            const double nk = (double)(n - k);
            crit = n > k ? rho[k - 1] * rho[k - 1] / (nk * nk) : 0.0;
        } else if (rule == 0) {
            const int kmax = (int64_t)l < n - 1 ? l : (int)(n - 1);
            k = 1;
            crit = 0.0;
            if (kmax >= 1) {
                for (int kk = 1; kk <= kmax; ++kk) {
                    const double nk = (double)(n - kk);
                    const double gk = rho[kk - 1] * rho[kk - 1] / (nk * nk);
                    if (kk == 1 || gk < crit) {
                        crit = gk;
                        k = kk;
                    }
                }
            }
        } else {
            // discrete L-curve corner
            k = l;
            crit = 0.0;
            flags = 4u;
            if (l >= 3) {
                double xlo = 0.0, xhi = 0.0, ylo = 0.0, yhi = 0.0;
                for (int i = 0; i < l; ++i) {
                    const double x = log(rho[i] > DBL_MIN ? rho[i] : DBL_MIN);
                    const double yy = log(eta[i] > DBL_MIN ? eta[i] : DBL_MIN);
                    xlo = i == 0 || x < xlo ? x : xlo;
                    xhi = i == 0 || x > xhi ? x : xhi;
                    ylo = i == 0 || yy < ylo ? yy : ylo;
                    yhi = i == 0 || yy > yhi ? yy : yhi;
                }
                const double ext = xhi - xlo > yhi - ylo ? xhi - xlo : yhi - ylo;
                const double tol = 1e-12 * ext;
                bool found = false;
                for (int kk = 2; kk < l; ++kk) {  // p_{kk+1}, p_kk, p_{kk-1} at 0-based kk, kk-1, kk-2
                    const double ax = log(rho[kk] > DBL_MIN ? rho[kk] : DBL_MIN);
                    const double ay = log(eta[kk] > DBL_MIN ? eta[kk] : DBL_MIN);
                    const double bx = log(rho[kk - 1] > DBL_MIN ? rho[kk - 1] : DBL_MIN);
                    const double by = log(eta[kk - 1] > DBL_MIN ? eta[kk - 1] : DBL_MIN);
                    const double cx = log(rho[kk - 2] > DBL_MIN ? rho[kk - 2] : DBL_MIN);
                    const double cy = log(eta[kk - 2] > DBL_MIN ? eta[kk - 2] : DBL_MIN);
                    const double lab = sqrt((bx - ax) * (bx - ax) + (by - ay) * (by - ay));
                    const double lbc = sqrt((cx - bx) * (cx - bx) + (cy - by) * (cy - by));
                    const double lac = sqrt((cx - ax) * (cx - ax) + (cy - ay) * (cy - ay));
                    if (!(lab > tol && lbc > tol && lac > tol)) continue;
                    const double kap = menger(ax, ay, bx, by, cx, cy);
                    if (!found || kap > crit) {
                        found = true;
                        crit = kap;
                        k = kk;
                    }
                }
                if (found) flags = (k == 2 || k == l - 1) ? 4u : 0u;
            }
        }
        s_k = k;
        out->lambda = 0.0;
        out->k = k;
        out->crit = crit;
        out->flags = flags;
        out->rho = rho[k - 1];
        out->eta = eta[k - 1];
    }
    __syncthreads();
    if (tid == 0) {
        const int k = s_k;
        double yi = g[k - 1] / d[k - 1];
        y[k - 1] = yi;
        for (int i = k - 2; i >= 0; --i) {
            yi = (g[i] - e[i] * yi) / d[i];
            y[i] = yi;
        }
    }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------

void launch_bidiag_qr(const double* alpha, const double* beta, int32_t l, const int32_t* l_ptr, double* ws,
                      double* sv, double* ftil, double* V, int64_t ldv, int32_t* status, bool flagged_only,
                      hipStream_t s, int nz, ProjBatch pb) {
    k_bidiag_svd<<<nz, kSvdThreads, 0, s>>>(alpha, beta, l, l_ptr, ws, sv, ftil, V, ldv, status,
                                            flagged_only ? 1 : 0, pb);
}

void launch_param_choice(const double* sv, const double* ft, int32_t l, const int32_t* l_ptr, int32_t method,
                         int32_t rule, int32_t J, double lambda_fixed, int32_t k_fixed, double omega, double* curve,
                         ParamOut* out, hipStream_t s, int nz, ProjBatch pb) {
    k_param_choice<<<nz, kProjThreads, 0, s>>>(sv, ft, l, l_ptr, method, rule, J, lambda_fixed, k_fixed, omega, curve,
                                               out, pb);
}

void launch_lsqr(const double* alpha, const double* beta, int32_t l, const int32_t* l_ptr, int64_t n, int32_t rule,
                 int32_t k_fixed, double* rho, double* eta, ParamOut* out, double* y, int32_t l_max, hipStream_t s,
                 int nz, ProjBatch pb) {
    k_lsqr<<<nz, kProjThreads, 0, s>>>(alpha, beta, l, l_ptr, n, rule, k_fixed, rho, eta, out, y, l_max, pb);
}

void launch_proj_solution(const double* sv, const double* ft, const double* V, int64_t ldv, int32_t l,
                          const int32_t* l_ptr, int32_t method, double lambda, int32_t k, const ParamOut* po,
                          double* y, int32_t l_max, hipStream_t s, int nz, ProjBatch pb) {
    k_proj_solution<<<dim3((l_max + kBlock - 1) / kBlock, nz), kBlock, 0, s>>>(sv, ft, V, ldv, l, l_ptr, method,
                                                                               lambda, k, po, y, pb);
}

}  // namespace mqh
