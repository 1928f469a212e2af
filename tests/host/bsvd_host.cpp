// Host build of the projected-SVD core used by the device kernel
// (paper_2511_09798_amd/csrc/bidiag_svd.hpp), for CPU tests of its logic.
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "../../paper_2511_09798_amd/csrc/bidiag_svd.hpp"

using namespace mqh::bsvd;

// Same sequence as the device kernel: reduce, sweep until converged
// (applying each sweep's right rotations to every row of V), then take
// absolute values, flip V columns of negative d and order descending.
extern "C" int bsvd_host(const double* alpha, const double* beta, int l, double* sv, double* ftil, double* V,
                         long* iters) {
    double* d = (double*)malloc(sizeof(double) * l);
    double* e = (double*)calloc(l > 1 ? l - 1 : 1, sizeof(double));
    double* g = (double*)malloc(sizeof(double) * l);
    double* rc = (double*)malloc(sizeof(double) * l);
    double* rs = (double*)malloc(sizeof(double) * l);
    double* W = (double*)calloc((size_t)l * l, sizeof(double));
    for (int i = 0; i < l; ++i) W[(int64_t)i * l + i] = 1.0;
    ftil[l] = reduce_lower(alpha, beta, l, d, e, g);
    Driver dv;
    driver_init(dv, l);
    int ll = 0, m = 0, st;
    while ((st = driver_step(dv, d, e, g, rc, rs, &ll, &m)) == 1)
        for (int r = 0; r < l; ++r) apply_row(W, l, r, ll, m, rc, rs);
    *iters = dv.iters;
    if (st == 0) {
        for (int i = 0; i < l; ++i) {
            double si = fabs(d[i]);
            int rk = 0;
            for (int j = 0; j < l; ++j) {
                double sj = fabs(d[j]);
                if (sj > si || (sj == si && j < i)) ++rk;
            }
            double sg = d[i] < 0.0 ? -1.0 : 1.0;
            sv[rk] = si;
            ftil[rk] = g[i];
            for (int r = 0; r < l; ++r) V[(int64_t)rk * l + r] = sg * W[(int64_t)i * l + r];
        }
    }
    free(d); free(e); free(g); free(rc); free(rs); free(W);
    return st;
}
