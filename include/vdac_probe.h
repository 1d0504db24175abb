/* Streaming-bandwidth references for the stage kernels' roofline.
 *
 * Not part of the method: plain kernels that stream whole FP64 planes through HBM, so that a
 * stage kernel's bytes per second can be set beside what a kernel with no stencil and no
 * arithmetic to speak of reaches on the same device: one element per lane in plane order, and
 * the stage kernel's own row-marching pattern.  They are built into libvdac.so and used by the
 * benchmark only.
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

/* One pass of the same plane mix in the row-marching stage kernel's access pattern, for a tank of
 * nx * ny cells (at most 2^29) walked in chunks of `chunk` rows, launched on `hip_stream` without
 * waiting: 64-column strips (60 written, 2 halo columns on each side) whose waves read input rows
 * j0-2 .. j1+1 of planes 0-3 and source rows j0-1 .. j1 of planes 4-10 of `in` (11 planes of
 * nx * ny doubles) and write rows j0 .. j1-1 of the 4 planes of `out`, 4 waves per workgroup in
 * the kernel's XCD-aware order.  It bounds what the stage kernel's memory pattern can reach with
 * no arithmetic.  Returns 0, 1 (VDAC_E_INVALID: a size out of range or a NULL pointer) or 3
 * (VDAC_E_DEVICE: the launch failed); it does not set last_error(). */
int vdac_march_probe(int32_t nx, int32_t ny, int32_t chunk, const double *in, double *out,
                     void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif
