// mlp_kernels.hip -- the learned predictor's network on gfx950, FP32: a
// 24-128-128-128-2 multilayer perceptron with tanh hidden layers, its
// back-propagation, the weighted mean squared error and Adam.  Parameters are
// flat, layer by layer: W_l (out x in, row-major) then b_l.  Batches are
// row-major (sample-major).  All reductions run in a fixed order, so
// training is deterministic.
#include <math.h>

#include "kernels.hpp"

namespace mqh {

constexpr int kMlpSizes[kMlpLayers + 1] = {kMlpIn, kMlpWidth, kMlpWidth, kMlpWidth, kMlpOut};

// ---------------------------------------------------------------------------
// FP32 GEMM, C (M x N) = op(A) op(B), 64 x 64 tiles, K in chunks of 16,
// 256 threads with a 4 x 4 block of C each.
//   op(A)(m, k) = TA ? A[k * lda + m] : A[m * lda + k]
//   op(B)(k, n) = TB ? B[n * ldb + k] : B[k * ldb + n]
// Epilogues: 0 plain; 1 tanh(acc + bias[n]); 2 acc + bias[n];
// 3 acc * (1 - H[m][n]^2) (the tanh derivative from the layer's output H).
// ---------------------------------------------------------------------------
constexpr int kGT = 64, kGK = 16;

template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void k_gemm32(int M, int N, int K, const float* __restrict__ A, int lda,
                                                const float* __restrict__ B, int ldb, float* __restrict__ C, int ldc,
                                                const float* __restrict__ bias, const float* __restrict__ H,
                                                int ldh) {
    __shared__ float As[kGK][kGT + 4];
    __shared__ float Bs[kGK][kGT + 4];
    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;
    const int m0 = blockIdx.y * kGT, n0 = blockIdx.x * kGT;
    float acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.f;
    for (int k0 = 0; k0 < K; k0 += kGK) {
        // 64 x 16 of op(A) and 16 x 64 of op(B): four elements per thread each
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + q * 256;
            const int kk = e & 15, mm = e >> 4;  // A tile: As[kk][mm]
            const int m = m0 + mm, k = k0 + kk;
            float va = 0.f;
            if (m < M && k < K) va = TA ? A[(int64_t)k * lda + m] : A[(int64_t)m * lda + k];
            As[kk][mm] = va;
            const int nn = e & 63, kb = e >> 6;  // B tile: Bs[kb][nn]
            const int n = n0 + nn, k2 = k0 + kb;
            float vb = 0.f;
            if (n < N && k2 < K) vb = TB ? B[(int64_t)n * ldb + k2] : B[(int64_t)k2 * ldb + n];
            Bs[kb][nn] = vb;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kGK; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int m = m0 + ty * 4 + i;
        if (m >= M) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int n = n0 + tx * 4 + j;
            if (n >= N) continue;
            float v = acc[i][j];
            if (EPI == 1) v = tanhf(v + bias[n]);
            if (EPI == 2) v = v + bias[n];
            if (EPI == 3) {
                const float h = H[(int64_t)m * ldh + n];
                v = v * (1.f - h * h);
            }
            C[(int64_t)m * ldc + n] = v;
        }
    }
}

template <bool TA, bool TB, int EPI>
void gemm32(int M, int N, int K, const float* A, int lda, const float* B, int ldb, float* C, int ldc,
            const float* bias, const float* H, int ldh, hipStream_t s) {
    dim3 grid((unsigned)((N + kGT - 1) / kGT), (unsigned)((M + kGT - 1) / kGT));
    k_gemm32<TA, TB, EPI><<<grid, 256, 0, s>>>(M, N, K, A, lda, B, ldb, C, ldc, bias, H, ldh);
}

// db[n] = sum over the batch of dZ[b][n], one thread per column, in order.
__global__ __launch_bounds__(kBlock) void k_colsum(const float* __restrict__ dZ, int B, int N,
                                                   float* __restrict__ db) {
    const int n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
    for (int b = 0; b < B; ++b) s += dZ[(int64_t)b * N + n];
    db[n] = s;
}

// Weighted MSE: dY = 2 w_k (Y - T) / B and loss = sum w_k (Y - T)^2 / B
// (one block; the per-thread partial sums are combined in a fixed order).
__global__ __launch_bounds__(kBlock) void k_mse(const float* __restrict__ Y, const float* __restrict__ T,
                                                const float* __restrict__ w, int B, int K, float* __restrict__ loss,
                                                float* __restrict__ dY) {
    __shared__ double lds[kBlock / kWave];
    double s = 0.0;
    const float inv = 1.0f / (float)B;
    for (int e = threadIdx.x; e < B * K; e += kBlock) {
        const int k = e % K;
        const float r = Y[e] - T[e];
        if (dY) dY[e] = 2.f * w[k] * r * inv;
        s += (double)w[k] * (double)r * (double)r;
    }
    s = block_sum<kBlock>(s, lds);
    if (threadIdx.x == 0 && loss) *loss = (float)(s / (double)B);
}

// Adam (bias-corrected): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// p -= lr (m c1) / (sqrt(v c2) + eps) with c1 = 1/(1-b1^t), c2 = 1/(1-b2^t).
__global__ __launch_bounds__(kBlock) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                                 float* __restrict__ m, float* __restrict__ v, int64_t n, float lr,
                                                 float b1, float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = fmaf(b1, m[i], (1.f - b1) * gi);
    const float vi = fmaf(b2, v[i], (1.f - b2) * gi * gi);
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// Standardised predictor input from the first Golub-Kahan scalars:
// x = ((log alpha_1..alpha_p, log beta_2..beta_{p+1}, log kappa, log eps,
// log n, log h) - mean) / std, p = kMlpProbe (one thread).
__global__ void k_mlp_features(const double* __restrict__ alpha, const double* __restrict__ beta, double kappa,
                               double eps, double n, double h, const float* __restrict__ mean,
                               const float* __restrict__ stdv, float* __restrict__ x) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double raw[kMlpIn];
    for (int j = 0; j < kMlpProbe; ++j) {
        raw[j] = log(alpha[j]);
        raw[kMlpProbe + j] = log(beta[j + 1]);
    }
    raw[2 * kMlpProbe + 0] = log(kappa);
    raw[2 * kMlpProbe + 1] = log(eps);
    raw[2 * kMlpProbe + 2] = log(n);
    raw[2 * kMlpProbe + 3] = log(h);
    for (int i = 0; i < kMlpIn; ++i) x[i] = (float)((raw[i] - (double)mean[i]) / (double)stdv[i]);
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------

int64_t mlp_param_offset(int layer) {
    int64_t off = 0;
    for (int l = 0; l < layer; ++l) off += (int64_t)kMlpSizes[l + 1] * kMlpSizes[l] + kMlpSizes[l + 1];
    return off;
}

// hidden: batch x (kMlpLayers - 1) x kMlpWidth, layer-major blocks of
// batch x kMlpWidth (the tanh outputs, kept for the backward pass).
void launch_mlp_forward(const float* params, const float* x, int B, float* y, float* hidden, hipStream_t s) {
    const float* in = x;
    int in_dim = kMlpIn;
    for (int l = 0; l < kMlpLayers; ++l) {
        const int out_dim = kMlpSizes[l + 1];
        const float* W = params + mlp_param_offset(l);
        const float* b = W + (int64_t)out_dim * in_dim;
        if (l < kMlpLayers - 1) {
            float* h = hidden + (int64_t)l * B * kMlpWidth;
            gemm32<false, true, 1>(B, out_dim, in_dim, in, in_dim, W, in_dim, h, out_dim, b, nullptr, 0, s);
            in = h;
        } else {
            gemm32<false, true, 2>(B, out_dim, in_dim, in, in_dim, W, in_dim, y, out_dim, b, nullptr, 0, s);
        }
        in_dim = out_dim;
    }
}

// work: 2 x batch x kMlpWidth floats (dZ of the current and next layer).
void launch_mlp_backward(const float* params, const float* x, const float* hidden, const float* dy, int B,
                         float* grad, float* work, hipStream_t s) {
    const float* dz = dy;  // dL/dz of the output layer
    float* bufs[2] = {work, work + (int64_t)B * kMlpWidth};
    for (int l = kMlpLayers - 1; l >= 0; --l) {
        const int out_dim = kMlpSizes[l + 1], in_dim = kMlpSizes[l];
        const float* W = params + mlp_param_offset(l);
        float* gW = grad + mlp_param_offset(l);
        float* gb = gW + (int64_t)out_dim * in_dim;
        const float* hin = l == 0 ? x : hidden + (int64_t)(l - 1) * B * kMlpWidth;
        // dW = dz^T h_in (out x in), db = column sums of dz
        gemm32<true, false, 0>(out_dim, in_dim, B, dz, out_dim, hin, in_dim, gW, in_dim, nullptr, nullptr, 0, s);
        k_colsum<<<(unsigned)((out_dim + kBlock - 1) / kBlock), kBlock, 0, s>>>(dz, B, out_dim, gb);
        if (l > 0) {
            // dz_{l-1} = (dz W) * (1 - h_in^2)
            float* nd = bufs[l & 1];
            gemm32<false, false, 3>(B, in_dim, out_dim, dz, out_dim, W, in_dim, nd, in_dim, nullptr, hin, in_dim, s);
            dz = nd;
        }
    }
}

void launch_mse(const float* y, const float* t, const float* w, int B, float* loss, float* dy, hipStream_t s) {
    k_mse<<<1, kBlock, 0, s>>>(y, t, w, B, kMlpOut, loss, dy);
}

void launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                 int32_t t, hipStream_t s) {
    const float c1 = (float)(1.0 / (1.0 - pow((double)b1, (double)t)));
    const float c2 = (float)(1.0 / (1.0 - pow((double)b2, (double)t)));
    k_adam<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(p, g, m, v, n, lr, b1, b2, eps, c1, c2);
}

void launch_mlp_features(const double* alpha, const double* beta, double kappa, double eps, double n, double h,
                         const float* mean, const float* stdv, float* x, hipStream_t s) {
    k_mlp_features<<<1, 64, 0, s>>>(alpha, beta, kappa, eps, n, h, mean, stdv, x);
}

}  // namespace mqh
