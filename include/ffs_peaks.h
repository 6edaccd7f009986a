/* Device peaks the roofline divides by, measured rather than taken from a data
 * sheet. No passage of the paper defines these: they check the denominators of
 * the decoder's roofline (int32 vector issue rate) and of the surrogate's (bf16
 * matrix-core rate) on the GPU at hand.
 *
 * Both entry points launch one kernel on `stream` (a hipStream_t, NULL = the
 * null stream), time it with HIP events recorded on that stream, synchronise
 * the stop event and write the elapsed milliseconds to *ms_out (host memory).
 * `sink` is a caller-owned device buffer of at least `blocks` words that the
 * kernels may write (it keeps their work from being removed; its contents are
 * meaningless). Work per launch:
 *   ffs_peak_valu_int32: blocks x 256 threads x iters x 64 int32 adds
 *                        (lane-ops; divide by the time for lane-ops/s);
 *   ffs_peak_mfma_bf16:  blocks x 4 waves x iters x 4 instructions of
 *                        v_mfma_f32_32x32x16_bf16, 32 x 32 x 16 x 2 FLOP each.
 * Returns 0, FFS_E_INVAL (-1) for blocks < 1, iters < 1 or a null pointer, or
 * FFS_E_DEVICE (-4) when a launch or event call fails. */
#ifndef FFS_PEAKS_H
#define FFS_PEAKS_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

int ffs_peak_valu_int32(int32_t blocks, int32_t iters, uint32_t *sink, float *ms_out, void *stream);
int ffs_peak_mfma_bf16(int32_t blocks, int32_t iters, float *sink, float *ms_out, void *stream);

#ifdef __cplusplus
}
#endif
#endif
