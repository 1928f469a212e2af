// peak_kernels.hip -- measurement helpers (libmqhpeak), not part of the solver: the rates
// the rooflines are checked against on the GPU at hand.  A device-to-device
// copy and a read-only stream (HBM), FP32 and FP64 FMA chains as the VALU issues them in this build
// (unpacked: every HIP source here is compiled without packed FP32), an
// FP64 matrix-core chain (v_mfma_f64_16x16x4f64), and the issue rates of the
// FP32 product's instructions (v_rsq_f32 alone and mixed with FMAs, the bf16
// matrix-core instruction).

#include "common.hpp"
#include "kernels.hpp"

namespace mqh {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int kPeakChains = 16;  // independent FMA chains per lane
constexpr int kPeakCopyUnroll = 4;  // independent 16-byte loads in flight per lane (copy)
constexpr int kPeakReadUnroll = 8;  // the same for the read-only stream
constexpr int kPeakMfma = 4;    // independent matrix-core accumulators per wave

// Grid-stride copy, kPeakCopyUnroll loads issued before their stores; the
// loads of one step are kBlock apart, so a wave reads 1 KiB runs.
__global__ __launch_bounds__(kBlock) void k_peak_copy(const double2* __restrict__ x, double2* __restrict__ y,
                                                      int64_t n2) {
    const int64_t step = (int64_t)gridDim.x * kBlock * kPeakCopyUnroll;
    int64_t i = (int64_t)blockIdx.x * kBlock * kPeakCopyUnroll + threadIdx.x;
    for (; i + (kPeakCopyUnroll - 1) * kBlock < n2; i += step) {
        double2 v[kPeakCopyUnroll];
#pragma unroll
        for (int u = 0; u < kPeakCopyUnroll; ++u) v[u] = x[i + u * kBlock];
#pragma unroll
        for (int u = 0; u < kPeakCopyUnroll; ++u) y[i + u * kBlock] = v[u];
    }
    for (int u = 0; u < kPeakCopyUnroll; ++u)
        if (i + u * kBlock < n2) y[i + u * kBlock] = x[i + u * kBlock];
}

// Grid-stride read of x (kPeakReadUnroll loads in flight per lane), summed
// per lane and stored once per thread so the loads are not dead code.
__global__ __launch_bounds__(kBlock) void k_peak_read(const double2* __restrict__ x, int64_t n2,
                                                      double* __restrict__ out) {
    const int64_t step = (int64_t)gridDim.x * kBlock * kPeakReadUnroll;
    int64_t i = (int64_t)blockIdx.x * kBlock * kPeakReadUnroll + threadIdx.x;
    double s = 0.0;
    for (; i + (kPeakReadUnroll - 1) * kBlock < n2; i += step) {
        double2 v[kPeakReadUnroll];
#pragma unroll
        for (int u = 0; u < kPeakReadUnroll; ++u) v[u] = x[i + u * kBlock];
#pragma unroll
        for (int u = 0; u < kPeakReadUnroll; ++u) s += v[u].x + v[u].y;
    }
    for (int u = 0; u < kPeakReadUnroll; ++u)
        if (i + u * kBlock < n2) s += x[i + u * kBlock].x + x[i + u * kBlock].y;
    out[(int64_t)blockIdx.x * kBlock + threadIdx.x] = s;
}

// kPeakChains chains v <- v a + b of iters steps each (a < 1: values stay
// near b / (1 - a)); the sum is stored so nothing is dead code.  a and b vary
// per lane so that they live in vector registers: gfx950 pairs two FP32
// instructions in one issue cycle only when neither reads a scalar register.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_peak_fma(T* __restrict__ out, int iters, T a0, T b0) {
    const T jitter = (T)1 + (T)(threadIdx.x & 7) * (T)1e-7;
    const T a = a0 * jitter, b = b0 * jitter;
    T v[kPeakChains];
#pragma unroll
    for (int k = 0; k < kPeakChains; ++k) v[k] = (T)(threadIdx.x + k) * (T)1e-3;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < kPeakChains; ++k) v[k] = fma(v[k], a, b);
    }
    T s = 0;
#pragma unroll
    for (int k = 0; k < kPeakChains; ++k) s += v[k];
    out[(int64_t)blockIdx.x * kBlock + threadIdx.x] = s;
}

// kPeakChains chains v <- rsq(v) + b (one v_rsq_f32 and one add per step;
// b > 1 keeps v in [b, b + 1]).  With mix, four independent FMAs on other
// chains follow each rsq: the instruction mix of the FP32 product's
// interior entry, which shows whether the transcendental unit's work
// overlaps ordinary VALU instructions.
__global__ __launch_bounds__(kBlock) void k_peak_rsq(float* __restrict__ out, int iters, float b0, int mix) {
    const float b = b0 * (1.f + (float)(threadIdx.x & 7) * 1e-7f);
    const float a = 0.999f * (1.f + (float)(threadIdx.x & 3) * 1e-7f);
    float v[kPeakChains], w[kPeakChains];
#pragma unroll
    for (int k = 0; k < kPeakChains; ++k) {
        v[k] = b + (float)k * 1e-3f;
        w[k] = (float)(threadIdx.x + k) * 1e-3f;
    }
    if (mix) {
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int k = 0; k < kPeakChains; ++k) {
                v[k] = __builtin_amdgcn_rsqf(v[k]) + b;
                w[k] = fmaf(fmaf(fmaf(fmaf(w[k], a, b), a, b), a, b), a, b);
            }
        }
    } else {
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int k = 0; k < kPeakChains; ++k) v[k] = __builtin_amdgcn_rsqf(v[k]) + b;
        }
    }
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < kPeakChains; ++k) s += v[k] + w[k];
    out[(int64_t)blockIdx.x * kBlock + threadIdx.x] = s;
}

// kPeakMfma accumulators, iters steps of v_mfma_f32_16x16x32_bf16 each (the
// instruction that forms t in the FP32 product).
__global__ __launch_bounds__(kBlock) void k_peak_mfma_bf16(float* __restrict__ out, int iters) {
    v8bf a, bb;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        a[i] = (__bf16)(1e-3f * (float)((threadIdx.x + i) & 63));
        bb[i] = (__bf16)(0.5f - 1e-3f * (float)i);
    }
    v4f acc[kPeakMfma];
#pragma unroll
    for (int q = 0; q < kPeakMfma; ++q) acc[q] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int q = 0; q < kPeakMfma; ++q) acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bb, acc[q], 0, 0, 0);
    }
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < kPeakMfma; ++q) s += acc[q][0] + acc[q][1] + acc[q][2] + acc[q][3];
    out[(int64_t)blockIdx.x * kBlock + threadIdx.x] = s;
}

// kPeakMfma accumulators, iters matrix-core steps each.
__global__ __launch_bounds__(kBlock) void k_peak_mfma64(double* __restrict__ out, int iters) {
    const double a = 1e-3 * (double)(threadIdx.x & (kWave - 1)), b = 0.5;
    v4d acc[kPeakMfma];
#pragma unroll
    for (int q = 0; q < kPeakMfma; ++q) acc[q] = v4d{0.0, 0.0, 0.0, 0.0};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int q = 0; q < kPeakMfma; ++q) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[q], 0, 0, 0);
    }
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kPeakMfma; ++q) s += acc[q][0] + acc[q][1] + acc[q][2] + acc[q][3];
    out[(int64_t)blockIdx.x * kBlock + threadIdx.x] = s;
}

}  // namespace

int peak_blocks() { return 256 * 8; }  // 8 workgroups of 4 waves per CU

void launch_peak_copy(const double* x, double* y, int64_t count, hipStream_t s) {
    k_peak_copy<<<(unsigned)peak_blocks(), kBlock, 0, s>>>(reinterpret_cast<const double2*>(x),
                                                           reinterpret_cast<double2*>(y), count / 2);
}

void launch_peak_read(const double* x, int64_t count, double* out, hipStream_t s) {
    k_peak_read<<<(unsigned)peak_blocks(), kBlock, 0, s>>>(reinterpret_cast<const double2*>(x), count / 2, out);
}

void launch_peak_fma32(float* out, int iters, hipStream_t s) {
    k_peak_fma<float><<<(unsigned)peak_blocks(), kBlock, 0, s>>>(out, iters, 0.999f, 1e-3f);
}

void launch_peak_fma64(double* out, int iters, hipStream_t s) {
    k_peak_fma<double><<<(unsigned)peak_blocks(), kBlock, 0, s>>>(out, iters, 0.999, 1e-3);
}

void launch_peak_mfma64(double* out, int iters, hipStream_t s) {
    k_peak_mfma64<<<(unsigned)peak_blocks(), kBlock, 0, s>>>(out, iters);
}

void launch_peak_rsq(float* out, int iters, int mix, hipStream_t s) {
    k_peak_rsq<<<(unsigned)peak_blocks(), kBlock, 0, s>>>(out, iters, 1.5f, mix);
}

void launch_peak_mfma_bf16(float* out, int iters, hipStream_t s) {
    k_peak_mfma_bf16<<<(unsigned)peak_blocks(), kBlock, 0, s>>>(out, iters);
}

// Work per launch: FMA lane operations (fma kinds) or flops (matrix cores).
double peak_fma_ops(int iters) { return (double)peak_blocks() * kBlock * kPeakChains * (double)iters; }
double peak_mfma_flops(int iters) {
    return (double)peak_blocks() * (kBlock / kWave) * kPeakMfma * (double)iters * (2.0 * 16 * 16 * 4);
}
double peak_mfma_bf16_flops(int iters) {
    return (double)peak_blocks() * (kBlock / kWave) * kPeakMfma * (double)iters * (2.0 * 16 * 16 * 32);
}

}  // namespace mqh
