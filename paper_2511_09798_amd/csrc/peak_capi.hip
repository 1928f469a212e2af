// peak_capi.hip -- C ABI of the measurement library (include/mqh_peak.h): the
// reference kernels of peak_kernels.hip, timed with HIP events.
#include <string>

#include "kernels.hpp"
#include "mqh_peak.h"

using namespace mqh;

namespace {

thread_local std::string g_peak_error;

int peak_fail(int code, const std::string& msg) {
    g_peak_error = msg;
    return code;
}

int peak_hip(hipError_t e, const char* what) {
    return peak_fail(e == hipErrorOutOfMemory ? -2 : -3, std::string(what) + ": " + hipGetErrorString(e));
}

#define PKCHK(expr)                                        \
    do {                                                   \
        hipError_t _e = (expr);                            \
        if (_e != hipSuccess) return peak_hip(_e, #expr);  \
    } while (0)

}  // namespace

extern "C" {

const char* mqh_peak_last_error(void) { return g_peak_error.c_str(); }

int mqh_peak_probe(int32_t kind, int64_t size, int32_t reps, double* rate, void* stream) {
    if (rate == nullptr) return peak_fail(-1, "NULL rate");
    *rate = 0.0;
    if (kind < MQH_PEAK_COPY || kind > MQH_PEAK_MFMA_BF16) return peak_fail(-1, "unknown probe kind");
    if (reps < 1 || reps > 1000) return peak_fail(-1, "reps must be in [1, 1000]");
    const bool stream_kind = kind == MQH_PEAK_COPY || kind == MQH_PEAK_READ;
    if (stream_kind && (size < 16 || size > ((int64_t)64 << 30)))
        return peak_fail(-1, "copy / read size must be in [16 B, 64 GiB]");
    if (!stream_kind && (size < 1 || size > (1 << 20))) return peak_fail(-1, "iterations must be in [1, 2^20]");
    hipStream_t s = (hipStream_t)stream;
    struct Cleanup {
        hipStream_t own = nullptr;
        double* a = nullptr;
        double* b = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        ~Cleanup() {
            if (a) (void)hipFree(a);
            if (b) (void)hipFree(b);
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
            if (own) (void)hipStreamDestroy(own);
        }
    } c;
    if (s == nullptr) {
        PKCHK(hipStreamCreateWithFlags(&c.own, hipStreamNonBlocking));
        s = c.own;
    }
    const int64_t count = stream_kind ? (size / 16) * 2 : (int64_t)peak_blocks() * kBlock;
    PKCHK(hipMalloc((void**)&c.a, (size_t)count * sizeof(double)));
    if (stream_kind) {
        // b: the copy's destination, or the read's per-thread sums
        const int64_t nb = kind == MQH_PEAK_COPY ? count : (int64_t)peak_blocks() * kBlock;
        PKCHK(hipMalloc((void**)&c.b, (size_t)nb * sizeof(double)));
        PKCHK(hipMemsetAsync(c.a, 0, (size_t)count * sizeof(double), s));
    }
    PKCHK(hipEventCreate(&c.e0));
    PKCHK(hipEventCreate(&c.e1));
    const int iters = (int)size;
    auto launch = [&]() {
        switch (kind) {
            case MQH_PEAK_COPY: launch_peak_copy(c.a, c.b, count, s); break;
            case MQH_PEAK_READ: launch_peak_read(c.a, count, c.b, s); break;
            case MQH_PEAK_FMA_F32: launch_peak_fma32(reinterpret_cast<float*>(c.a), iters, s); break;
            case MQH_PEAK_FMA_F64: launch_peak_fma64(c.a, iters, s); break;
            case MQH_PEAK_RSQ_F32: launch_peak_rsq(reinterpret_cast<float*>(c.a), iters, 0, s); break;
            case MQH_PEAK_RSQ_FMA_F32: launch_peak_rsq(reinterpret_cast<float*>(c.a), iters, 1, s); break;
            case MQH_PEAK_MFMA_BF16: launch_peak_mfma_bf16(reinterpret_cast<float*>(c.a), iters, s); break;
            default: launch_peak_mfma64(c.a, iters, s); break;
        }
    };
    launch();  // warm-up
    PKCHK(hipGetLastError());
    PKCHK(hipEventRecord(c.e0, s));
    for (int r = 0; r < reps; ++r) launch();
    PKCHK(hipGetLastError());
    PKCHK(hipEventRecord(c.e1, s));
    PKCHK(hipEventSynchronize(c.e1));
    float ms = 0.f;
    PKCHK(hipEventElapsedTime(&ms, c.e0, c.e1));
    if (!(ms > 0.f)) return peak_fail(-3, "peak probe: no elapsed time");
    const double sec = (double)ms * 1e-3 / reps;
    double work = 0.0;
    switch (kind) {
        case MQH_PEAK_COPY: work = 2.0 * (double)count * sizeof(double); break;
        case MQH_PEAK_READ: work = (double)count * sizeof(double); break;
        case MQH_PEAK_FMA_F32:
        case MQH_PEAK_FMA_F64: work = 2.0 * peak_fma_ops(iters); break;
        case MQH_PEAK_RSQ_F32:
        case MQH_PEAK_RSQ_FMA_F32: work = peak_fma_ops(iters); break;
        case MQH_PEAK_MFMA_BF16: work = peak_mfma_bf16_flops(iters); break;
        default: work = peak_mfma_flops(iters); break;
    }
    *rate = work / sec;
    return 0;
}

}  // extern "C"
