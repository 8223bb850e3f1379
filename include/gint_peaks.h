/* gint_peaks.h — achievable peak rates of the units the grid-integration
 * kernels use, measured on the current device (MI355X, gfx950).
 *
 * These are the measured denominators reported beside the datasheet peaks
 * when a kernel's fraction of its roofline is stated: each rate is the
 * throughput of a kernel that does nothing but that instruction, in
 * independent chains on every SIMD of every CU.
 */
#ifndef GINT_PEAKS_H
#define GINT_PEAKS_H

#ifdef __cplusplus
extern "C" {
#endif

/* tflops: host double[4], receives TFLOP/s of
 *   [0] FP64 MFMA v_mfma_f64_16x16x4f64 (2048 flops per instruction),
 *   [1] FP16 MFMA v_mfma_f32_16x16x32_f16 (16384 flops per instruction, FP32 accumulate),
 *   [2] FP32 vector FMA, [3] FP64 vector FMA (2 flops per lane).
 * stream: hipStream_t (NULL = default).  Synchronous: allocates a small
 * device buffer, times one launch of each kernel with HIP events after a
 * warm-up launch, and frees the buffer.  Returns 0, or a negative code
 * (-1 NULL argument, -3 allocation failed, -4 HIP runtime error). */
int gint_peaks_measure(double *tflops, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* GINT_PEAKS_H */
