// Plane-stream kernel: the bandwidth reference that the stage kernels' bytes per second are set
// beside.  One element per lane per pass over i, every plane's access coalesced, the planes'
// loads of one element issued together (compile-time plane counts), no stencil and no
// arithmetic beyond one add per plane.
#include <hip/hip_runtime.h>

#include "vdac_internal.h"

namespace vdac {
namespace {

template <int NI, int NO>
__global__ void __launch_bounds__(256) stream_planes(const double *__restrict__ in,
                                                     double *__restrict__ out, size_t n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double v[NI];
#pragma unroll
        for (int k = 0; k < NI; ++k) v[k] = in[k * n + i];
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < NI; ++k) acc += v[k];
        if constexpr (NO == 0) {
            // reads only: a store that the data (finite values) never triggers keeps them alive
            if (acc != acc) out[i] = acc;
        } else {
#pragma unroll
            for (int k = 0; k < NO; ++k) out[k * n + i] = acc;
        }
    }
}

}  // namespace

int launch_stream_probe(int n_in, int n_out, size_t n, int blocks, const double *in, double *out,
                        void *stream_)
{
    const hipStream_t stream = (hipStream_t)stream_;
    // one element per lane unless that needs more than 2^24 workgroups (the loop strides on)
    const size_t wgs = (n + 255) / 256;
    const unsigned grid = blocks > 0 ? (unsigned)blocks : (unsigned)(wgs < (1u << 24) ? wgs : (1u << 24));
    if (n_in == 1 && n_out == 0)
        hipLaunchKernelGGL((stream_planes<1, 0>), dim3(grid), dim3(256), 0, stream, in, out, n);
    else if (n_in == 1 && n_out == 1)
        hipLaunchKernelGGL((stream_planes<1, 1>), dim3(grid), dim3(256), 0, stream, in, out, n);
    else if (n_in == 11 && n_out == 4)
        hipLaunchKernelGGL((stream_planes<11, 4>), dim3(grid), dim3(256), 0, stream, in, out, n);
    else
        return (int)hipErrorInvalidValue;
    return (int)hipGetLastError();
}

}  // namespace vdac
