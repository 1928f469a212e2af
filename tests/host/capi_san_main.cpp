// Drives the C ABI (include/mqhelm.h) through a build of the library whose
// host code carries AddressSanitizer and UndefinedBehaviorSanitizer: the
// argument checks (no device needed), then, when a GPU is present, every
// entry point on small seeded problems in all three operator modes.  Any
// sanitizer report ends the run with a non-zero status.  Prints one line per
// exercised group of calls and "done" at the end.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <vector>

#include "mqhelm.h"

static uint64_t g_rng = 88172645463325252ull;
static double urand() {
    g_rng ^= g_rng << 13;
    g_rng ^= g_rng >> 7;
    g_rng ^= g_rng << 17;
    return (double)(g_rng >> 11) * (1.0 / 9007199254740992.0);
}

#define EXPECT(cond)                                                      \
    do {                                                                  \
        if (!(cond)) {                                                    \
            printf("FAILED %s at line %d: %s\n", #cond, __LINE__, mqh_last_error()); \
            return 1;                                                     \
        }                                                                 \
    } while (0)

static int argument_checks() {
    std::vector<double> x(30, 0.5), a(8, 1.0), b(9, 1.0), out(9);
    mqh_problem* p = nullptr;
    EXPECT(mqh_problem_create(nullptr, 0, nullptr, 0, 1.0, 1.0, 0, nullptr, 0, &p) == MQH_EINVAL && p == nullptr);
    EXPECT(mqh_problem_create(x.data(), 5, x.data(), 5, 1.0, -1.0, 0, nullptr, 0, &p) == MQH_EINVAL);
    EXPECT(mqh_problem_create(x.data(), 5, nullptr, 0, 1.0, 1.0, 9, nullptr, 0, &p) == MQH_EINVAL);
    EXPECT(mqh_apply(nullptr, 0, x.data(), 0.0, nullptr, x.data(), 0) == MQH_EINVAL);
    EXPECT(mqh_proj_svd(a.data(), b.data(), 0, out.data(), out.data(), nullptr, nullptr, 0) == MQH_EINVAL);
    EXPECT(mqh_proj_svd_noalloc(a.data(), b.data(), MQH_NOALLOC_MAX_ELL + 1, out.data(), out.data(), nullptr,
                                nullptr) == MQH_EINVAL);
    double lam = 0.0;
    EXPECT(mqh_param_choice(a.data(), b.data(), 8, MQH_METHOD_HKT, MQH_RULE_GCV, 2, 0.0, 0, 1.0, &lam, nullptr,
                            nullptr, nullptr, nullptr, nullptr, 0) == MQH_EINVAL);
    EXPECT(mqh_problem_destroy(nullptr) == MQH_OK && mqh_problem_size(nullptr) == -1);
    EXPECT(mqh_status_str(12345) != nullptr);
    printf("argument checks\n");
    return 0;
}

static int one_mode(int mode) {
    const int64_t n_int = 150, n_bnd = 90, n = n_int + n_bnd;
    const int32_t ell = 20;
    std::vector<double> xi(3 * n_int), xb(3 * n_bnd), f(n), g(n_bnd), coef(n), y(n), W((ell + 1) * n), Z(ell * n);
    for (auto& v : xi) v = urand();
    for (auto& v : xb) v = urand();
    for (auto& v : f) v = urand() - 0.5;
    for (auto& v : g) v = urand() - 0.5;
    mqh_problem* p = nullptr;
    EXPECT(mqh_problem_create(xi.data(), n_int, xb.data(), n_bnd, 3.0, 2.0, mode, nullptr, MQH_FLAG_FIXED_SHAPES,
                              &p) == MQH_OK);
    for (int t = 0; t < 2; ++t)
        for (uint32_t rs = 0; rs <= MQH_FLAG_ROW_SCALE; rs += MQH_FLAG_ROW_SCALE)
            EXPECT(mqh_apply(p, t, f.data(), 0.5, f.data(), y.data(), rs) == MQH_OK);
    std::vector<double> rows(3 * n);
    EXPECT(mqh_matrix_rows(p, n - 3, 3, rows.data(), 0) == MQH_OK);
    std::vector<double> al(ell), be(ell + 1), sv(ell);
    int32_t done = 0;
    EXPECT(mqh_gkb(p, f.data(), ell, 1, W.data(), Z.data(), al.data(), be.data(), &done, 0) >= 0);
    mqh_solve_opts o = {};
    o.ell = ell;
    o.reorth = 1;
    o.gcv_weight = 1.0;
    mqh_solve_info info;
    const int32_t methods[][2] = {{MQH_METHOD_HKT, MQH_RULE_GCV}, {MQH_METHOD_HKT, MQH_RULE_LCURVE},
                                  {MQH_METHOD_INE_TSVD, MQH_RULE_GCV}, {MQH_METHOD_LSQR, MQH_RULE_GCV},
                                  {MQH_METHOD_LSQR, MQH_RULE_LCURVE}};
    for (auto& mr : methods)
        for (int rs = 0; rs < 2; ++rs) {
            o.method = mr[0];
            o.rule = mr[1];
            o.row_scale = rs;
            EXPECT(mqh_solve(p, f.data(), f.data() + n_int, &o, coef.data(), al.data(), be.data(), sv.data(),
                             &info) >= 0);
        }
    o.method = MQH_METHOD_HKT;
    o.rule = MQH_RULE_FIXED;
    o.lambda_fixed = 1e-3;
    o.row_scale = 0;
    EXPECT(mqh_solve(p, f.data(), f.data() + n_int, &o, coef.data(), nullptr, nullptr, nullptr, nullptr) >= 0);
    std::vector<double> ue(40), xe(3 * 40);
    for (auto& v : xe) v = urand();
    EXPECT(mqh_eval(p, coef.data(), xe.data(), 40, ue.data(), 0) == MQH_OK);
    // several right-hand sides: lockstep runs, a sweep of one, the block process
    const int nr = 3;
    std::vector<double> F(nr * n), C(nr * n), Cb((ell + 1) * nr * ell * nr), E1(nr * nr);
    for (auto& v : F) v = urand() - 0.5;
    std::vector<mqh_solve_info> infos(nr);
    o.rule = MQH_RULE_GCV;
    EXPECT(mqh_solve_multi(p, F.data(), n, nr, &o, C.data(), n, infos.data()) >= 0);
    std::vector<double> Wm(nr * (ell + 1) * n), Zm(nr * ell * n), am(nr * ell), bm(nr * (ell + 1));
    std::vector<int32_t> dm(nr);
    EXPECT(mqh_gkb_multi(p, F.data(), n, nr, ell, 1, Wm.data(), Zm.data(), am.data(), bm.data(), dm.data(), 0) >= 0);
    mqh_sweep_item item = {p, F.data(), n, nr, 0, C.data(), n, infos.data()};
    EXPECT(mqh_solve_sweep(&item, 1, &o, 1) >= 0);
    const int32_t lb = 4;
    std::vector<double> Cbk((lb + 1) * nr * lb * nr);
    int32_t bd = 0, bf = 0;
    EXPECT(mqh_gkb_block(p, F.data(), n, nr, lb, Cbk.data(), E1.data(), nullptr, nullptr, &bd, &bf, 0) >= 0);
    o.ell = lb;
    std::vector<double> svb(lb * nr);
    EXPECT(mqh_solve_block(p, F.data(), n, nr, &o, C.data(), n, svb.data(), infos.data()) >= 0);
    o.ell = ell;
    if (mode == MQH_OP_STORED_FP64) {
        std::vector<double> svf(n), fh(n);
        int32_t sweeps = 0;
        double off = 0.0;
        EXPECT(mqh_full_svd(p, f.data(), svf.data(), fh.data(), &sweeps, &off, 0) >= 0);
        EXPECT(mqh_full_solve(p, f.data(), f.data() + n_int, &o, coef.data(), svf.data(), &info) >= 0);
    }
    EXPECT(mqh_problem_destroy(p) == MQH_OK);
    printf("operator mode %d: products, rows, Golub-Kahan, solves, evaluation, multi, sweep, block%s\n", mode,
           mode == MQH_OP_STORED_FP64 ? ", full SVD" : "");
    return 0;
}

static int projected() {
    const int32_t ell = 30;
    std::vector<double> a(ell), b(ell + 1), sv(ell), ft(ell + 1), V(ell * ell), y(ell), rho(ell), eta(ell);
    for (int i = 0; i < ell; ++i) a[i] = exp(-0.3 * i) * (1.0 + 0.1 * urand());
    for (int i = 0; i <= ell; ++i) b[i] = exp(-0.3 * i) * (0.5 + 0.1 * urand());
    EXPECT(mqh_proj_svd(a.data(), b.data(), ell, sv.data(), ft.data(), V.data(), nullptr, 0) == MQH_OK);
    double lam = 0.0, crit = 0.0;
    int32_t k = 0;
    uint32_t fl = 0;
    std::vector<double> curve(200);
    EXPECT(mqh_param_choice(sv.data(), ft.data(), ell, MQH_METHOD_HKT, MQH_RULE_GCV, 0, 0.0, 0, 1.0, &lam, &k, &crit,
                            &fl, curve.data(), nullptr, 0) >= 0);
    EXPECT(mqh_proj_solution(sv.data(), ft.data(), V.data(), ell, MQH_METHOD_HKT, lam, 0, y.data(), nullptr, 0) ==
           MQH_OK);
    EXPECT(mqh_lsqr(a.data(), b.data(), ell, 1000, MQH_RULE_GCV, 0, &k, &crit, &fl, y.data(), rho.data(), eta.data(),
                    nullptr, 0) >= 0);
    const int64_t n = 100;
    std::vector<double> Z(ell * n, 0.01), c(n);
    EXPECT(mqh_lift(Z.data(), n, ell, y.data(), c.data(), nullptr, 0) == MQH_OK);
    double *da = nullptr, *db = nullptr, *dsv = nullptr, *dft = nullptr;
    EXPECT(hipMalloc(&da, ell * 8) == hipSuccess && hipMalloc(&db, (ell + 1) * 8) == hipSuccess &&
           hipMalloc(&dsv, ell * 8) == hipSuccess && hipMalloc(&dft, (ell + 1) * 8) == hipSuccess);
    EXPECT(hipMemcpy(da, a.data(), ell * 8, hipMemcpyHostToDevice) == hipSuccess);
    EXPECT(hipMemcpy(db, b.data(), (ell + 1) * 8, hipMemcpyHostToDevice) == hipSuccess);
    EXPECT(mqh_proj_svd_noalloc(da, db, ell, dsv, dft, nullptr, nullptr) == MQH_OK);
    (void)hipFree(da);
    (void)hipFree(db);
    (void)hipFree(dsv);
    (void)hipFree(dft);
    printf("projected problem: SVD, parameter choice, solution, LSQR, lift, allocation-free SVD\n");
    return 0;
}

int main() {
    if (argument_checks()) return 1;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        printf("no GPU: argument checks only\ndone\n");
        return 0;
    }
    for (int mode = 0; mode <= 2; ++mode)
        if (one_mode(mode)) return 1;
    if (projected()) return 1;
    EXPECT(mqh_device_bytes() == 0);  // every problem released its memory
    printf("done\n");
    return 0;
}
