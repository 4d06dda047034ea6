/* les_debug.h -- instrumentation entry points of liblesmi.so.
 *
 * Not part of the method: these are for the benchmark (per-launch timing of
 * the stage kernel, a plain copy for the achievable stream bandwidth) and
 * for the tests (switching the RK step to the one-thread-per-node reference
 * kernel to cross-check the fused kernel).
 * Same conventions as les.h: status codes, never abort. */
#ifndef LES_DEBUG_H
#define LES_DEBUG_H

#include "les.h"

#ifdef __cplusplus
extern "C" {
#endif

/* on != 0: les_rk_step runs its stages through the reference kernel
 * (k_stage_ref) instead of the fused tiled kernel; on == 0: fused (default).
 * LES_ERR_ARG for a null context. */
int les_debug_use_reference(les_ctx *ctx, int on);

/* on != 0: record a HIP event pair around every stage-kernel launch on the
 * context's stream (and reset the totals); on == 0: stop recording. */
int les_debug_stage_timing(les_ctx *ctx, int on);

/* Summed elapsed milliseconds (*total_ms, host) and launch count
 * (*launches, host) of the stage launches recorded since timing was switched
 * on or last read; synchronises with the recorded events, then resets the
 * totals.  LES_ERR_ARG for a null argument. */
int les_debug_stage_time(les_ctx *ctx, double *total_ms, long long *launches);

/* Plain device-to-device copy of nbytes from src to dst (device pointers,
 * both 16-byte aligned, nbytes a positive multiple of 16), enqueued on
 * hip_stream (NULL: the default stream); the benchmark times it as the
 * achievable stream bandwidth.  LES_ERR_ARG for bad arguments, LES_ERR_HIP
 * when the launch fails.  Needs no context. */
int les_debug_stream_copy(const void *src, void *dst, long long nbytes, void *hip_stream);

/* Dynamic SGS closure (sgs = 2): evaluates the per-column coefficients of Q
 * (its ghost layers filled in place) and copies them to out (device,
 * 2 (nj+4)(ni+4) doubles: C, then D_T, per padded column (j+2)(ni+4)+(i+2)).
 * LES_ERR_STATE for a context without the dynamic closure. */
int les_debug_dynamic_coefficients(les_ctx *ctx, double *Q, double *out);

#ifdef __cplusplus
}
#endif

#endif /* LES_DEBUG_H */
