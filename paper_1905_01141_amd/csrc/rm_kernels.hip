// rm_kernels.hip -- rate matching of the turbo code (TS 36.212 5.1.4.1):
// the receiver adds the soft values of one transmission into a block's
// [3][K+4] soft buffer (HARQ combining, int8 or int16 inputs), the
// transmitter picks the bits a redundancy version sends.  Both walk the
// circular buffer through a host-built table: rank r of a non-<NULL> entry
// -> its index in the [3][K+4] array.
#include <hip/hip_runtime.h>

#include "tdec_internal.h"

namespace tdec {

// Threads per block: the LDS buffer allows four blocks per CU, and 512
// threads each keep 32 waves of loads in flight there.
constexpr int kRmThreads = 512;

// One work group per code block; the block's [3][K+4] buffer is staged in
// LDS (read, or cleared for a first transmission, and written back once), so
// the scattered read-modify-writes of the table walk stay on chip.  The walk
// wraps its rank incrementally: one pass covers each non-<NULL> entry once.
// A transmission longer than the buffer's non-<NULL> entries revisits
// positions; it is added in chunks of one pass, a barrier apart, so that
// saturating sums are taken in transmission order.  Within one pass every
// position occurs once, so each thread issues the table and soft-value loads
// of eight values before their eight read-modify-writes.  The buffer moves as
// 8-byte words (n = 3 (K + 4) is a multiple of 4), four loads in flight.
template <typename T>
__global__ void __launch_bounds__(kRmThreads) derate_kernel(const RmItem *items, const T *e,
                                                            int16_t *soft, const uint16_t *tab,
                                                            int combine)
{
    extern __shared__ __align__(16) int16_t sb[];
    const RmItem it = items[blockIdx.x];
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int n = 3 * (it.K + 4);  // even
    int16_t *s = soft + it.soft_off;
    const T *src = e + it.e_off;
    const uint16_t *t = tab + it.tab_off;
    const bool wide = (((uintptr_t)s) & 7) == 0;
    if (wide) {
        uint2 *sw = (uint2 *)sb;
        const uint2 *gw = (const uint2 *)s;
        const int nq = n / 4;
        for (int i0 = tid; i0 < nq; i0 += 4 * nthr) {
            uint2 v[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int i = i0 + m * nthr;
                v[m] = (combine && i < nq) ? gw[i] : make_uint2(0u, 0u);
            }
#pragma unroll
            for (int m = 0; m < 4; ++m)
                if (i0 + m * nthr < nq) sw[i0 + m * nthr] = v[m];
        }
    } else {
        for (int i = tid; i < n; i += nthr) sb[i] = combine ? s[i] : (int16_t)0;
    }
    __syncthreads();
    const int nv = it.n_valid;
    for (int64_t c0 = 0; c0 < it.E; c0 += nv) {
        const int len = (int)min((int64_t)nv, (int64_t)it.E - c0);
        for (int i0 = tid; i0 < len; i0 += 8 * nthr) {
            int d[8], v[8];
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const int i = i0 + m * nthr;
                int r = it.r0 + min(i, len - 1);  // r0 < nv and i < nv
                if (r >= nv) r -= nv;
                d[m] = t[r];
                v[m] = i < len ? (int)src[c0 + i] : 0;
            }
#pragma unroll
            for (int m = 0; m < 8; ++m)
                if (i0 + m * nthr < len) {
                    const int x = (int)sb[d[m]] + v[m];
                    sb[d[m]] = (int16_t)max(-32767, min(32767, x));
                }
        }
        __syncthreads();
    }
    if (wide) {
        uint2 *gw = (uint2 *)s;
        const uint2 *sw = (const uint2 *)sb;
        for (int i = tid; i < n / 4; i += nthr) gw[i] = sw[i];
    } else {
        for (int i = tid; i < n; i += nthr) s[i] = sb[i];
    }
}

// One work group per code block: the block's coded bits are staged in LDS
// (4-byte words, four loads in flight per thread), then the transmission
// reads them in circular-buffer order, the table loads of eight values issued
// before their LDS reads and stores.
__global__ void __launch_bounds__(kRmThreads) rate_match_kernel(const RmItem *items,
                                                                const uint8_t *coded, uint8_t *e,
                                                                const uint16_t *tab)
{
    extern __shared__ __align__(16) uint8_t cbits[];
    const RmItem it = items[blockIdx.x];
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int n = 3 * (it.K + 4);  // a multiple of 4
    const uint8_t *d = coded + it.soft_off;
    uint8_t *dst = e + it.e_off;
    const uint16_t *t = tab + it.tab_off;
    if ((((uintptr_t)d) & 3) == 0) {
        const uint32_t *gw = (const uint32_t *)d;
        uint32_t *sw = (uint32_t *)cbits;
        const int nq = n / 4;
        for (int i0 = tid; i0 < nq; i0 += 4 * nthr) {
            uint32_t v[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int i = i0 + m * nthr;
                v[m] = i < nq ? gw[i] : 0u;
            }
#pragma unroll
            for (int m = 0; m < 4; ++m)
                if (i0 + m * nthr < nq) sw[i0 + m * nthr] = v[m];
        }
    } else {
        for (int i = tid; i < n; i += nthr) cbits[i] = d[i];
    }
    __syncthreads();
    const int nv = it.n_valid;
    for (int64_t c0 = 0; c0 < it.E; c0 += nv) {
        const int len = (int)min((int64_t)nv, (int64_t)it.E - c0);
        for (int i0 = tid; i0 < len; i0 += 8 * nthr) {
            int d[8];
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                int r = it.r0 + min(i0 + m * nthr, len - 1);  // r0 < nv and i < nv
                if (r >= nv) r -= nv;
                d[m] = t[r];
            }
#pragma unroll
            for (int m = 0; m < 8; ++m)
                if (i0 + m * nthr < len) dst[c0 + i0 + m * nthr] = cbits[d[m]];
        }
    }
}

int launch_derate(const RmItem *items, int n, int max_k, const void *e, int e_bytes,
                  int16_t *soft, const uint16_t *tab, int combine, void *stream)
{
    if (n <= 0) return 0;
    if (max_k < 40 || max_k > kKmax) return -1;
    const size_t lds = (size_t)3 * (max_k + 4) * sizeof(int16_t);
    if (e_bytes == 1)
        hipLaunchKernelGGL(derate_kernel<int8_t>, dim3(n), dim3(kRmThreads), lds, (hipStream_t)stream,
                           items, (const int8_t *)e, soft, tab, combine);
    else
        hipLaunchKernelGGL(derate_kernel<int16_t>, dim3(n), dim3(kRmThreads), lds, (hipStream_t)stream,
                           items, (const int16_t *)e, soft, tab, combine);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_rate_match(const RmItem *items, int n, int max_k, const uint8_t *coded, uint8_t *e,
                      const uint16_t *tab, void *stream)
{
    if (n <= 0) return 0;
    if (max_k < 40 || max_k > kKmax) return -1;
    const size_t lds = (size_t)3 * (max_k + 4);
    hipLaunchKernelGGL(rate_match_kernel, dim3(n), dim3(kRmThreads), lds, (hipStream_t)stream, items,
                       coded, e, tab);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace tdec
