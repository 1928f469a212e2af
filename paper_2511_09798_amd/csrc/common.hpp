// common.hpp -- device helpers shared by the gfx950 kernels of the MQ-RBF
// Golub-Kahan solver: launch constants, deterministic wave/block reductions,
// the Golub-Kahan device state and the multiquadric entry generators.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mqh {

constexpr int kBlock = 256;  // threads per workgroup for the streaming kernels
constexpr int kWave = 64;    // CDNA wavefront

// Device-resident state of one Golub-Kahan run.  Every kernel of the loop
// reads `stopped` first and returns at once after a breakdown, so the host
// can enqueue all ell steps without synchronising.
struct GkbState {
    int32_t stopped;   // 1 after a breakdown
    int32_t ell_done;  // steps kept (initialised to ell)
    int32_t flag;      // 0, 1 = alpha breakdown, 2 = beta breakdown
    int32_t pad;
    double scale;      // running max of alpha_j, beta_{j+1}: the operator scale
    // copies of stopped and scale taken by the kernel that produces a norm's
    // partial sums; the normalisation kernel decides from these while its
    // block 0 updates stopped and scale
    int32_t snap_stopped;
    int32_t pad2;
    double snap_scale;
};

// Per-batch-slice strides of a kernel's pointer arguments (in elements):
// slice z of a batched launch uses pointer + z * stride; which argument
// takes which stride is stated at each kernel.  Zero strides with one slice
// are the unbatched call.
struct Bz {
    int64_t a = 0, b = 0, c = 0, d = 0;
};

// Per-problem strides (in elements) of a batched launch of the projected-
// problem kernels, one workgroup (row of workgroups) per problem z:
// vec for alpha, beta, sv, ftil, y, rho, eta; mat for Vw and V; lstr for
// the step-count pointer (int32 elements); curve for the criterion curve;
// ParamOut and the status word advance by one per problem; ws for the
// projected SVD's workspace (svd_ws_doubles of the allocation's l).
struct ProjBatch {
    int64_t vec = 0, mat = 0, lstr = 0, curve = 0, ws = 0;
};

// Native 2 x FP64 vector for 16-byte (non-temporal) loads and stores.
typedef double v2d __attribute__((ext_vector_type(2)));

__device__ __forceinline__ v2d load_nt(const double* p) {
    return __builtin_nontemporal_load(reinterpret_cast<const v2d*>(p));
}
__device__ __forceinline__ void store_nt(double* p, v2d v) {
    __builtin_nontemporal_store(v, reinterpret_cast<v2d*>(p));
}
__device__ __forceinline__ v2d load2(const double* p) { return *reinterpret_cast<const v2d*>(p); }

// ---------------------------------------------------------------------------
// Deterministic reductions (fixed butterfly / fixed order, no atomics)
// ---------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Sum over a whole block of NT threads; every thread gets the total.
// `lds` must hold NT/64 doubles.  Contains barriers: call from all threads.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* lds) {
    v = wave_sum(v);
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) lds[w] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NT / kWave; ++i) s += lds[i];
    __syncthreads();
    return s;
}

// ---------------------------------------------------------------------------
// Multiquadric entries.  Nodes are stored centred on their bounding box and
// pre-multiplied by eps, so for two stored nodes P, Q
//     t = 1 + |P - Q|^2 = 1 + eps^2 r^2 .
// With s = t^{-1/2}:
//   boundary row (Dirichlet, eq. (3)):     phi      = sqrt(t)          = t s
//   interior row (eq. (8)):         L phi    = eps^2 (2t+1) t^{-3/2} + kappa^2 t^{1/2}
//                                                  = (kappa^2 t + 2 eps^2 + eps^2 s^2) s
// (the Laplacian of phi in 3-D is eps^2 (3 + 2 eps^2 r^2) / t^{3/2}, and
//  3 + 2 eps^2 r^2 = 2t + 1; all three terms are positive, so the form has
//  no cancellation).
// ---------------------------------------------------------------------------

struct EntryConst {
    double k2;    // kappa^2
    double e2;    // eps^2
    double e2x2;  // 2 eps^2
    float k2f, e2f, e2x2f, padf;
};

// 1/sqrt(t) for t >= 1 in FP64: the hardware estimate s (relative error
// below 2^-24 over t in [1, 1e6], measured) refined by one third-order step.
// With r = 1 - t s^2, 1/sqrt(t) = s (1 - r)^(-1/2) = s (1 + r/2 + 3 r^2/8 +
// 5 r^3/16 + ...); the dropped terms are below 2^-70 relative, so the result
// is within the final rounding (measured: the same largest error, 0.62 ulp,
// as two Newton steps, in five instructions instead of eight).
__device__ __forceinline__ double rsqrt_f64(double t) {
    const double s = __builtin_amdgcn_rsq(t);
    const double h = t * s;
    const double r = fma(-h, s, 1.0);
    const double p = fma(0.375, r, 0.5);
    return fma(s * r, p, s);
}

__device__ __forceinline__ double t_of(double px, double py, double pz, double qx, double qy, double qz) {
    const double dx = px - qx, dy = py - qy, dz = pz - qz;
    return fma(dz, dz, fma(dy, dy, fma(dx, dx, 1.0)));
}

__device__ __forceinline__ float t_of(float px, float py, float pz, float qx, float qy, float qz) {
    const float dx = px - qx, dy = py - qy, dz = pz - qz;
    return fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, 1.0f)));
}

__device__ __forceinline__ double entry_interior(double t, const EntryConst& c) {
    const double s = rsqrt_f64(t);
    return fma(c.e2, s * s, fma(c.k2, t, c.e2x2)) * s;
}

__device__ __forceinline__ double entry_boundary(double t, const EntryConst&) { return t * rsqrt_f64(t); }

// FP32 evaluation: one v_rsq_f32 / v_sqrt_f32 per entry (1 ulp), the rest in FP32.
__device__ __forceinline__ float entry_interior(float t, const EntryConst& c) {
    const float s = __builtin_amdgcn_rsqf(t);
    return fmaf(c.e2f, s * s, fmaf(c.k2f, t, c.e2x2f)) * s;
}

__device__ __forceinline__ float entry_boundary(float t, const EntryConst&) { return __builtin_amdgcn_sqrtf(t); }

// Node record types per evaluation precision.
template <typename R>
struct NodeOf;
template <>
struct NodeOf<double> {
    using type = double4;
};
template <>
struct NodeOf<float> {
    using type = float4;
};

}  // namespace mqh
