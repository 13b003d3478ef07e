/*
 * inrf_peaks.h -- measurement kernels of the benchmark (libinrf_peaks.so):
 * the ceilings the render path's kernels are compared with, measured on the
 * device they run on rather than taken from a datasheet.  Not part of the
 * render path; nothing in libinrf.so calls them.
 *
 * Conventions as in inrf.h: status 0 = success, negative = error (message in
 * inrf_peaks_last_error()); arguments are validated before anything is
 * enqueued; device pointers are caller-owned; calls enqueue on `stream` (a
 * hipStream_t, NULL = the null stream), never allocate and never
 * synchronise.  The caller times a call with events recorded on the same
 * stream before and after it.
 */
#ifndef INRF_PEAKS_H
#define INRF_PEAKS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

const char* inrf_peaks_last_error(void);

/* Streaming read of device memory: reads `bytes` bytes at `buf` (device,
 * 16-byte aligned, bytes a positive multiple of 16), `reps` times over, with
 * 16-byte loads spread over a grid of 8 workgroups of 256 threads per
 * compute unit, and writes one XOR of what each workgroup read to
 * sink[workgroup] (device uint32, at least inrf_peak_read_sink_size()
 * entries) so that no load can be dropped.  HBM read bandwidth =
 * reps * bytes / elapsed time when the buffer is much larger than the caches
 * (e.g. 4 GiB). */
int32_t inrf_peak_read_sink_size(void);
int32_t inrf_peak_hbm_read(const void* buf, int64_t bytes, int32_t reps, uint32_t* sink, void* stream);

/* Matrix-core peak: every wave of a grid of `waves_per_simd` waves per SIMD
 * (4 SIMDs per compute unit) runs `iters` rounds of four independent
 * 16x16 matrix instructions of the given precision (0 = FP32
 * v_mfma_f32_16x16x4f32, 2,048 FLOP each; 1 = FP16 and 2 = BF16
 * v_mfma_f32_16x16x32, 16,384 FLOP each), the same instructions the
 * network uses, and writes one float per wave to sink (device, at least
 * inrf_peak_mfma_waves(waves_per_simd) entries).  FLOP of the call =
 * waves * iters * 4 * (FLOP per instruction). */
int64_t inrf_peak_mfma_waves(int32_t waves_per_simd);
int32_t inrf_peak_mfma(int32_t precision, int32_t waves_per_simd, int64_t iters, float* sink, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* INRF_PEAKS_H */
