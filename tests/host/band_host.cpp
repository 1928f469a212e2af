// Host build of the band reduction of the block projected matrix
// (paper_2511_09798_amd/csrc/band.hpp), for CPU tests of its logic: the
// bulge chase in the pipelined step order of the device kernels or sweep by
// sweep, the data through the right reflectors and the lower-to-upper
// rotations, and the solutions through the left reflectors in reverse.
// Reflectors are stored by their place in the step order (step-major, rank
// q = sweep ihi - q within a step), as on the device.
#include <stdint.h>
#include <string.h>

#include <vector>

#include "../../paper_2511_09798_amd/csrc/band.hpp"

using namespace mqh;

namespace {

// toff[T] = tasks before step T (nsteps + 1 entries)
void step_offsets(int N, int Mc, int b, std::vector<int>& toff) {
    const int T = band::nsteps(N, Mc, b);
    toff.assign((size_t)T + 1, 0);
    for (int s = 0; s < T; ++s) {
        int ihi;
        toff[(size_t)s + 1] = toff[(size_t)s] + band::step_tasks(s, N, Mc, b, ihi);
    }
}

void run_task(double* B, int N, int Mc, int b, int i, int t, double* rr, double* ll) {
    int r0, c0, c1;
    band::task_cols(i, t, b, Mc, r0, c0, c1);
    const int nj = c1 - c0 + 1, r1 = c1 < N - 1 ? c1 : N - 1;
    double v[band::kMaxB], beta;
    const double tau = band::reflector(B + band::at(r0, c0, b), 1, nj, v, &beta);
    for (int k = 0; k < b; ++k) rr[k] = k < nj ? v[k] : 0.0;
    rr[b] = tau;
    if (tau != 0.0) {
        for (int r = r0 + 1; r <= r1; ++r) band::apply(v, tau, nj, B + band::at(r, c0, b), 1);
        B[band::at(r0, c0, b)] = beta;
        for (int k = 1; k < nj; ++k) B[band::at(r0, c0 + k, b)] = 0.0;
    }
    const int ni = r1 - c0 + 1;
    for (int k = 0; k <= b; ++k) ll[k] = 0.0;
    ll[0] = 1.0;
    if (ni >= 2) {
        const int64_t cs = band::width(b) - 1;  // from (r, c) to (r + 1, c)
        const double tau2 = band::reflector(B + band::at(c0, c0, b), cs, ni, v, &beta);
        for (int k = 0; k < ni; ++k) ll[k] = v[k];
        ll[b] = tau2;
        if (tau2 != 0.0) {
            const int ce = c1 + b < Mc - 1 ? c1 + b : Mc - 1;
            for (int c = c0 + 1; c <= ce; ++c) {
                // column c of rows c0 .. r1; entries outside a row's band are zero and stay zero
                double y[band::kMaxB];
                for (int k = 0; k < ni; ++k) {
                    const int r = c0 + k;
                    y[k] = (c - r >= -(b - 1) && c - r <= 2 * b - 1) ? B[band::at(r, c, b)] : 0.0;
                }
                band::apply(v, tau2, ni, y, 1);
                for (int k = 0; k < ni; ++k) {
                    const int r = c0 + k;
                    if (c - r >= -(b - 1) && c - r <= 2 * b - 1) B[band::at(r, c, b)] = y[k];
                }
            }
            B[band::at(c0, c0, b)] = beta;
            for (int k = 1; k < ni; ++k) B[band::at(c0 + k, c0, b)] = 0.0;
        }
    }
}

}  // namespace

extern "C" {

int band_nsteps(int N, int Mc, int b) { return band::nsteps(N, Mc, b); }

int band_ntasks_total(int N, int Mc, int b) {
    std::vector<int> toff;
    step_offsets(N, Mc, b, toff);
    return toff.back();
}

// C: Mc x N row-major (leading dimension ldc).  pipelined = 1: the step
// order; 0: sweep after sweep.  d, e (N): the bidiagonal of M = C^T; RR, LL
// (tasks x (b + 1)): v_0 .. v_{b-1}, tau per task; toff (nsteps + 1).
int band_reduce(const double* C, int64_t ldc, int N, int Mc, int b, int pipelined, double* d, double* e,
                double* RR, double* LL, int* toff_out) {
    if (b < 1 || b > band::kMaxB || N < 1 || Mc < N + 1) return -1;
    const int W = band::width(b);
    std::vector<double> B((size_t)N * W, 0.0);
    for (int r = 0; r < N; ++r)
        for (int c = r; c <= r + b && c < Mc; ++c) B[(size_t)band::at(r, c, b)] = C[(int64_t)c * ldc + r];
    std::vector<int> toff;
    step_offsets(N, Mc, b, toff);
    const int T = (int)toff.size() - 1;
    auto slot = [&](int i, int t) {
        int ihi;
        band::step_tasks(band::kLag * i + t, N, Mc, b, ihi);
        return toff[(size_t)(band::kLag * i + t)] + (ihi - i);
    };
    if (pipelined) {
        for (int s = 0; s < T; ++s) {
            int ihi;
            const int cnt = band::step_tasks(s, N, Mc, b, ihi);
            for (int q = 0; q < cnt; ++q) {
                const int i = ihi - q, t = s - band::kLag * i;
                const int k = toff[(size_t)s] + q;
                run_task(B.data(), N, Mc, b, i, t, RR + (int64_t)k * (b + 1), LL + (int64_t)k * (b + 1));
            }
        }
    } else {
        for (int i = 0; i < band::nsweeps(N, Mc); ++i)
            for (int t = 0; t < band::ntasks(i, N, Mc, b); ++t) {
                const int k = slot(i, t);
                run_task(B.data(), N, Mc, b, i, t, RR + (int64_t)k * (b + 1), LL + (int64_t)k * (b + 1));
            }
    }
    for (int i = 0; i < N; ++i) {
        d[i] = B[(size_t)band::at(i, i, b)];
        e[i] = B[(size_t)band::at(i, i + 1, b)];
    }
    for (int s = 0; s <= T; ++s) toff_out[s] = toff[(size_t)s];
    return T;
}

// X (Mc x ns row-major) through the right reflectors in step order, then the
// rotations taking Bt^T (alpha = d, beta_{j+1} = e_j) to the upper
// bidiagonal (du, eu); X's first N + 1 rows rotated alike.
void band_data(double* X, int ns, int N, int Mc, int b, const double* RR, const int* toff, int T, const double* d,
               const double* e, double* du, double* eu) {
    for (int s = 0; s < T; ++s) {
        int ihi;
        const int cnt = band::step_tasks(s, N, Mc, b, ihi);
        for (int q = 0; q < cnt; ++q) {
            const int i = ihi - q, t = s - band::kLag * i;
            int r0, c0, c1;
            band::task_cols(i, t, b, Mc, r0, c0, c1);
            const double* rr = RR + (int64_t)(toff[s] + q) * (b + 1);
            if (rr[b] == 0.0) continue;
            double v[band::kMaxB];
            for (int k = 0; k < band::kMaxB; ++k) v[k] = k < b ? rr[k] : 0.0;
            for (int k = 0; k < ns; ++k) band::apply(v, rr[b], c1 - c0 + 1, X + (int64_t)c0 * ns + k, ns);
        }
    }
    double a = d[0];
    for (int j = 0; j < N; ++j) {
        double c, sn;
        du[j] = band::givens(a, e[j], &c, &sn);
        const double an = j + 1 < N ? d[j + 1] : 0.0;
        eu[j] = sn * an;
        a = c * an;
        for (int k = 0; k < ns; ++k) {
            const double g0 = X[(int64_t)j * ns + k], g1 = X[(int64_t)(j + 1) * ns + k];
            X[(int64_t)j * ns + k] = c * g0 + sn * g1;
            X[(int64_t)(j + 1) * ns + k] = -sn * g0 + c * g1;
        }
    }
}

// Y (N x ns row-major) through the left reflectors, last step first.
void band_solution(double* Y, int ns, int N, int Mc, int b, const double* LL, const int* toff, int T) {
    for (int s = T - 1; s >= 0; --s) {
        int ihi;
        const int cnt = band::step_tasks(s, N, Mc, b, ihi);
        for (int q = 0; q < cnt; ++q) {
            const int i = ihi - q, t = s - band::kLag * i;
            int r0, c0, c1;
            band::task_cols(i, t, b, Mc, r0, c0, c1);
            const double* ll = LL + (int64_t)(toff[s] + q) * (b + 1);
            if (ll[b] == 0.0) continue;
            const int r1 = c1 < N - 1 ? c1 : N - 1;
            double v[band::kMaxB];
            for (int k = 0; k < band::kMaxB; ++k) v[k] = k < b ? ll[k] : 0.0;
            for (int k = 0; k < ns; ++k) band::apply(v, ll[b], r1 - c0 + 1, Y + (int64_t)c0 * ns + k, ns);
        }
    }
}

}  // extern "C"
