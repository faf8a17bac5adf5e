// rm_kernels.hip -- rate matching of the turbo code (TS 36.212 5.1.4.1):
// the receiver adds the soft values of one transmission into a block's
// [3][K+4] soft buffer (HARQ combining, int8 or int16 inputs), the
// transmitter picks the bits a redundancy version sends.  Both walk the
// circular buffer through a host-built table: rank r of a non-<NULL> entry
// -> its index in the [3][K+4] array.
#include <hip/hip_runtime.h>

#include "tdec_internal.h"

namespace tdec {

// One work group per code block.  A transmission longer than the buffer's
// non-<NULL> entries revisits positions; it is added in chunks of one pass,
// a barrier apart, so that saturating sums are taken in transmission order.
template <typename T>
__global__ void __launch_bounds__(256) derate_kernel(const RmItem *items, const T *e,
                                                     int16_t *soft, const uint16_t *tab,
                                                     int combine)
{
    const RmItem it = items[blockIdx.x];
    const int tid = threadIdx.x, nthr = blockDim.x;
    int16_t *s = soft + it.soft_off;
    const T *src = e + it.e_off;
    const uint16_t *t = tab + it.tab_off;
    if (!combine) {
        const int n = 3 * (it.K + 4);
        for (int i = tid; i < n; i += nthr) s[i] = 0;
        __syncthreads();
    }
    for (int64_t c0 = 0; c0 < it.E; c0 += it.n_valid) {
        const int64_t c1 = min((int64_t)it.E, c0 + it.n_valid);
        for (int64_t k = c0 + tid; k < c1; k += nthr) {
            int64_t r = it.r0 + k;
            r %= it.n_valid;
            const int d = t[r];
            const int v = (int)s[d] + (int)src[k];
            s[d] = (int16_t)max(-32767, min(32767, v));
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) rate_match_kernel(const RmItem *items, const uint8_t *coded,
                                                         uint8_t *e, const uint16_t *tab)
{
    const RmItem it = items[blockIdx.x];
    const uint8_t *d = coded + it.soft_off;
    uint8_t *dst = e + it.e_off;
    const uint16_t *t = tab + it.tab_off;
    for (int64_t k = threadIdx.x; k < it.E; k += blockDim.x)
        dst[k] = d[t[(it.r0 + k) % it.n_valid]];
}

int launch_derate(const RmItem *items, int n, const void *e, int e_bytes, int16_t *soft,
                  const uint16_t *tab, int combine, void *stream)
{
    if (n <= 0) return 0;
    if (e_bytes == 1)
        hipLaunchKernelGGL(derate_kernel<int8_t>, dim3(n), dim3(256), 0, (hipStream_t)stream,
                           items, (const int8_t *)e, soft, tab, combine);
    else
        hipLaunchKernelGGL(derate_kernel<int16_t>, dim3(n), dim3(256), 0, (hipStream_t)stream,
                           items, (const int16_t *)e, soft, tab, combine);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_rate_match(const RmItem *items, int n, const uint8_t *coded, uint8_t *e,
                      const uint16_t *tab, void *stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(rate_match_kernel, dim3(n), dim3(256), 0, (hipStream_t)stream, items,
                       coded, e, tab);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace tdec
