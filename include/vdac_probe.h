/* Streaming-bandwidth reference for the stage kernels' roofline.
 *
 * Not part of the method: a plain kernel that streams whole FP64 planes through HBM, so that a
 * stage kernel's bytes per second can be set beside what a kernel with no stencil, no
 * arithmetic to speak of and one element per lane reaches on the same device.  It is built
 * into libvdac.so and used by the benchmark only.
 */
#ifndef VDAC_PROBE_H
#define VDAC_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Launches one pass of the plane stream on `hip_stream` (NULL: the default stream) and returns
 * without waiting.  For every i < n the kernel reads in[k * n + i] for k < n_in, and writes their
 * sum to out[k * n + i] for k < n_out (n_out = 0: reads only).  Supported (n_in, n_out):
 * (1, 0) read only, (1, 1) copy, (11, 4) the FP64 stage's plane mix (Q^{s-1}, Q^0 and three
 * planes of level n in, Q^s out).  `blocks`
 * 256-thread workgroups stride over i (blocks = 0: one element per lane, up to 2^24
 * workgroups).
 *
 * in, out: device pointers to n_in * n and max(n_out, 1) * n doubles, caller-owned (with
 * n_out = 0, out[i] is written only where the sum is NaN).  Returns 0, 1 (VDAC_E_INVALID: an
 * unsupported pair, n = 0, blocks outside [0, 2^24] or a NULL pointer) or 3 (VDAC_E_DEVICE: the
 * launch failed); last_error() names the reason. */
int vdac_stream_probe(int32_t n_in, int32_t n_out, uint64_t n, int32_t blocks, const double *in,
                      double *out, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif
