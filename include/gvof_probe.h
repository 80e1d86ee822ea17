/* gvof_probe.h -- measurement probes of the chip, separate from the method's
 * library (libgvof_probe.so).
 *
 * The FP64 clipping kernels are bound by the vector FP64 units.  This probe
 * measures what those units deliver on a plain loop of fused multiply-adds,
 * so a kernel's achieved FLOP rate can be read against a measured ceiling as
 * well as against the published one.  The caller times the launch (an event
 * pair on the same stream).
 */
#ifndef GVOF_PROBE_H
#define GVOF_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Launches `blocks` blocks of 256 threads on `stream` (a hipStream_t; NULL is
 * the null stream).  Thread t starts eight FP64 accumulators at
 * x_k = k + (t mod 7), k = 0..7, and runs `iters` rounds of x_k = fma(x_k, a, b)
 * on all eight (independent chains: 16 FLOPs per round), then writes
 * out[t] = ((x_0 + x_1) + (x_2 + x_3)) + ((x_4 + x_5) + (x_6 + x_7)).
 * Work: blocks * 256 * iters * 16 FP64 FLOPs.  With a = b = 1 every step is
 * exact, so out[t] = 28 + 8 (t mod 7) + 8 iters.
 *
 * out: device array of blocks * 256 doubles, caller-owned, written.
 * Returns 0; -1 when out is NULL, blocks < 1 or iters < 0; -4 when the
 * launch fails.  Asynchronous: the result is ready once the stream reaches it. */
int gvof_probe_fp64_fma(double* out, int32_t blocks, int32_t iters, double a, double b, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* GVOF_PROBE_H */
