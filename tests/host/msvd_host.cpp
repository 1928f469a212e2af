// Host build of the fast projected SVD (paper_2511_09798_amd/csrc/msvd.hpp
// with the left rotations of bidiag_svd.hpp), for CPU tests of its logic.
// The steps are those of the device kernels in svd_kernels.hip, run one
// after another: setup, multisection of every value, twisted vectors,
// Gram matrices, acceptance test, symmetric correction.
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "../../paper_2511_09798_amd/csrc/bidiag_svd.hpp"
#include "../../paper_2511_09798_amd/csrc/msvd.hpp"

using namespace mqh;

// Returns 0 (accepted), 2 (rejected by the acceptance test); rounds[0] = the
// largest number of multisection rounds, orth[0..1] = max |V^T V - I| and
// max |U^T U - I| before the correction, orth[2] = the largest residual over its bound.
extern "C" int msvd_host(const double* alpha, const double* beta, int l, double* sv, double* ftil, double* V,
                         int* rounds, double* orth) {
    std::vector<double> d(l), e(l, 0.0), g(l), lam(l), U((size_t)l * l), h(l), res(l);
    ftil[l] = bsvd::reduce_lower(alpha, beta, l, d.data(), e.data(), g.data());
    double emax = 0.0;
    bool bad = false;
    for (int i = 0; i < l; ++i) {
        emax = e[i] * e[i] > emax ? e[i] * e[i] : emax;
        bad = bad || !(d[i] > 0.0) || !isfinite(d[i]) || !isfinite(e[i]);
    }
    const double bound = msvd::eig_bound(d.data(), e.data(), l);
    const double pivmin = DBL_MIN * (emax > 1.0 ? emax : 1.0);
    std::vector<double> d2(l), e2(l);
    for (int i = 0; i < l; ++i) {
        d2[i] = d[i] * d[i];
        e2[i] = e[i] * e[i];
    }
    const int P = msvd::kSections;
    std::vector<double> xs(P);
    std::vector<int> cs(P);
    rounds[0] = 0;
    for (int j = 0; j < l; ++j) {
        const int k = l - 1 - j;
        double lo = 0.0, hi = bound;
        int round = 0;
        for (; round < 64; ++round) {
            if (hi - lo <= 2.0 * DBL_EPSILON * hi) break;
            int ts = -1;
            for (int t = 0; t < P; ++t) {
                xs[t] = msvd::section_point(lo, hi, t, P);
                cs[t] = msvd::negcount(d2.data(), 1, e2.data(), 1, l, xs[t], pivmin);
                if (cs[t] <= k) ts = t;
            }
            const double nlo = ts >= 0 ? xs[ts] : lo;
            const double nhi = ts + 1 < P ? xs[ts + 1] : hi;
            if (nlo == lo && nhi == hi) break;
            lo = nlo;
            hi = nhi;
        }
        rounds[0] = round > rounds[0] ? round : rounds[0];
        lam[j] = lo + 0.5 * (hi - lo);
        sv[j] = sqrt(lam[j]);
        bad = bad || !(lo > 0.0);
    }
    std::vector<double> A0(l), B0(l), A1(l), B1(l);
    for (int j = 0; j < l; ++j) {
        double* A[2] = {A0.data(), A1.data()};
        double* Bv[2] = {B0.data(), B1.data()};
        int r[2];
        for (int side = 0; side < 2; ++side) {
            const double* dp = side ? d.data() + (l - 1) : d.data();
            const double* ep = (side && l >= 2) ? e.data() + (l - 2) : e.data();
            const int st = side ? -1 : 1;
            msvd::stationary(dp, st, ep, st, l, lam[j], pivmin, A[side], Bv[side]);
            double gr;
            r[side] = msvd::progressive_twist(dp, st, ep, st, l, lam[j], pivmin, Bv[side], &gr);
        }
        for (int side = 0; side < 2; ++side) {
            msvd::twisted_solve(A[side], Bv[side], l, r[side], -1);
            msvd::twisted_solve(A[side], Bv[side], l, r[side], 1);
            A[side][r[side]] = 1.0;
        }
        double nv = 0.0, nu = 0.0;
        for (int i = 0; i < l; ++i) {
            nv += A0[i] * A0[i];
            nu += A1[i] * A1[i];
        }
        const double iv = 1.0 / sqrt(nv), iu = 1.0 / sqrt(nu);
        double t = 0.0;
        for (int i = 0; i < l; ++i) t += A1[l - 1 - i] * (d[i] * A0[i] + (i + 1 < l ? e[i] * A0[i + 1] : 0.0));
        const double su = t < 0.0 ? -iu : iu;
        double r1 = 0.0, r2 = 0.0, hg = 0.0;
        for (int i = 0; i < l; ++i) {
            const double vk = A0[i] * iv, vk1 = i + 1 < l ? A0[i + 1] * iv : 0.0;
            const double uk = A1[l - 1 - i] * su, ukm = i > 0 ? A1[l - i] * su : 0.0;
            const double ra = msvd::resid_row(d[i], vk, i + 1 < l ? e[i] : 0.0, vk1, sv[j], uk);
            const double rb = msvd::resid_row(d[i], uk, i > 0 ? e[i - 1] : 0.0, ukm, sv[j], vk);
            hg += uk * g[i];
            r1 += ra * ra;
            r2 += rb * rb;
        }
        for (int i = 0; i < l; ++i) {
            V[(size_t)j * l + i] = A0[i] * iv;
            U[(size_t)j * l + i] = A1[l - 1 - i] * su;
        }
        h[j] = hg;
        const double rr = sqrt(r1 > r2 ? r1 : r2) / msvd::resid_bound(sv[j], sv[0], l);
        res[j] = rr == rr ? rr : INFINITY;
    }
    std::vector<double> E((size_t)l * l);
    double mo[2] = {0.0, 0.0}, mr = 0.0;
    for (int which = 0; which < 2; ++which) {
        const double* M = which ? U.data() : V;
        for (int i = 0; i < l; ++i)
            for (int jj = 0; jj < l; ++jj) {
                double a = 0.0;
                for (int k = 0; k < l; ++k) a += M[(size_t)i * l + k] * M[(size_t)jj * l + k];
                a -= i == jj ? 1.0 : 0.0;
                if (!which) E[(size_t)i * l + jj] = a;
                const double aa = a == a ? fabs(a) : INFINITY;
                mo[which] = aa > mo[which] ? aa : mo[which];
            }
    }
    for (int i = 0; i < l; ++i) mr = res[i] > mr ? res[i] : mr;
    orth[0] = mo[0];
    orth[1] = mo[1];
    orth[2] = mr;
    if (bad || mo[0] > msvd::kOrthTol || mo[1] > msvd::kOrthTol || mr > 1.0) return 2;
    std::vector<double> Vn((size_t)l * l), w(l);
    for (int r = 0; r < l; ++r)
        for (int jj = 0; jj < l; ++jj) {
            double a = 0.0;
            for (int i = 0; i < l; ++i) a += V[(size_t)i * l + r] * E[(size_t)i * l + jj];
            Vn[(size_t)jj * l + r] = V[(size_t)jj * l + r] - 0.5 * a;
        }
    memcpy(V, Vn.data(), sizeof(double) * (size_t)l * l);
    for (int r = 0; r < l; ++r) {
        double a = 0.0;
        for (int jj = 0; jj < l; ++jj) a += U[(size_t)jj * l + r] * h[jj];
        w[r] = a;
    }
    for (int jj = 0; jj < l; ++jj) {
        double a = 0.0;
        for (int r = 0; r < l; ++r) a += U[(size_t)jj * l + r] * w[r];
        ftil[jj] = 1.5 * h[jj] - 0.5 * a;
    }
    return 0;
}
