// serve_kernels.hip -- device-side staging of the serving loop: copies the
// LLRs of a batch of transport blocks from the caller's device buffers into
// the server's resident slots, one work group per block.
#include <hip/hip_runtime.h>

#include "tdec_internal.h"

namespace tdec {

__global__ void __launch_bounds__(256) gather_kernel(GatherArgs g)
{
    const GatherItem it = g.it[blockIdx.x];
    int16_t *dst = g.dst_base + (int64_t)it.dst_blk * 128;  // 256-byte units
    const int16_t *src = it.src;
    const int64_t n = it.n;
    const int tid = threadIdx.x, nthr = blockDim.x;
    if ((((uintptr_t)src) & 15) == 0) {
        // 8 elements per 16-byte load; the destination is 256-byte aligned
        const int64_t n8 = n >> 3;
        const uint4 *s4 = (const uint4 *)src;
        uint4 *d4 = (uint4 *)dst;
        for (int64_t i = tid; i < n8; i += nthr) d4[i] = s4[i];
        for (int64_t i = (n8 << 3) + tid; i < n; i += nthr) dst[i] = src[i];
    } else {
        for (int64_t i = tid; i < n; i += nthr) dst[i] = src[i];
    }
}

int launch_gather(const GatherArgs &g, void *stream)
{
    if (g.n <= 0) return 0;
    hipLaunchKernelGGL(gather_kernel, dim3(g.n), dim3(256), 0, (hipStream_t)stream, g);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace tdec
