/*
 * mqh_peak.h -- C ABI of libmqhpeak, the measurement helper that sits beside
 * the solver library (libmqhelm) and is not part of the method: the rate of
 * a reference kernel on the current device, against which the rooflines'
 * published peaks are checked (MI355X: HBM 8 TB/s, FP32 and FP64 vector 157.3
 * and 78.6 TFLOP/s, FP64 matrix 78.6 TFLOP/s).
 *
 *   MQH_PEAK_COPY:     device-to-device copy of size bytes (rounded down to
 *                      16 B); rate = bytes read + written per second.
 *   MQH_PEAK_FMA_F32:  chains of FP32 FMA (unpacked, as every kernel of the
 *                      solver is built; operands in vector registers, so
 *                      the SIMD may issue two at once), size iterations;
 *                      rate = flop/s (2 per FMA).
 *   MQH_PEAK_FMA_F64:  the same in FP64.
 *   MQH_PEAK_MFMA_F64: chains of v_mfma_f64_16x16x4f64, size iterations;
 *                      rate = flop/s.
 *   MQH_PEAK_READ:     read-only stream of size bytes (eight 16-byte loads
 *                      in flight per lane, summed per thread); rate = bytes
 *                      read per second.
 *   MQH_PEAK_RSQ_F32:  chains of v_rsq_f32 (each followed by one add), size
 *                      iterations; rate = rsq lane operations per second.
 *   MQH_PEAK_RSQ_FMA_F32: the same with four independent FP32 FMAs after
 *                      each rsq (the FP32 product's interior instruction
 *                      mix); rate = groups (rsq + add + 4 FMA) per second.
 *   MQH_PEAK_MFMA_BF16: chains of v_mfma_f32_16x16x32_bf16, size
 *                      iterations; rate = flop/s.
 * One warm-up launch, then reps timed launches (HIP events) on stream (NULL:
 * a stream of its own).  The call allocates and frees its buffers (2 x size
 * bytes for the copy).  Returns 0, or -1 (invalid argument: an unknown kind,
 * reps outside [1, 1000], a copy or read outside [16 B, 64 GiB], iterations
 * outside [1, 2^20], rate NULL), -2 (out of device memory) or -3 (device
 * error); mqh_peak_last_error() has a thread-local message.
 */
#ifndef MQH_PEAK_H
#define MQH_PEAK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MQH_PEAK_COPY 0
#define MQH_PEAK_FMA_F32 1
#define MQH_PEAK_FMA_F64 2
#define MQH_PEAK_MFMA_F64 3
#define MQH_PEAK_READ 4
#define MQH_PEAK_RSQ_F32 5
#define MQH_PEAK_RSQ_FMA_F32 6
#define MQH_PEAK_MFMA_BF16 7

int mqh_peak_probe(int32_t kind, int64_t size, int32_t reps, double* rate, void* stream);
const char* mqh_peak_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MQH_PEAK_H */
