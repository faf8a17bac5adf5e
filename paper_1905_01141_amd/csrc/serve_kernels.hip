// serve_kernels.hip -- device-side staging of the serving loop: copies the
// LLRs of a batch of transport blocks from the caller's device buffers into
// the server's resident slots.  Each block is cut into chunks of kChunk
// elements and every chunk gets a work group of its own (grid x = chunk,
// grid y = block), so a 75376-bit block is spread over 30 work groups instead
// of being copied by one.
#include <hip/hip_runtime.h>

#include "tdec_internal.h"

namespace tdec {

namespace {
constexpr int kThreads = 256;
constexpr int kChunk = 8192;  // int16 elements per work group (16 KB)
}  // namespace

__global__ void __launch_bounds__(kThreads) gather_kernel(GatherArgs g)
{
    const GatherItem it = g.it[blockIdx.y];
    const int64_t c0 = (int64_t)blockIdx.x * kChunk;
    if (c0 >= (int64_t)it.n) return;
    const int m = (int)min((int64_t)kChunk, (int64_t)it.n - c0);  // elements of this chunk
    // dst_base is 256-byte aligned and c0 a multiple of 8192 elements, so dst
    // is 256-byte aligned; src is only 2-byte aligned in general
    int16_t *dst = g.dst_base + (int64_t)it.dst_blk * 128 + c0;
    const int16_t *src = it.src + c0;
    const int tid = threadIdx.x;
    const uintptr_t a = (uintptr_t)src;
    if ((a & 15) == 0) {
        const int m8 = m >> 3;  // 16-byte vectors, at most 1024
        const uint4 *s4 = (const uint4 *)src;
        uint4 *d4 = (uint4 *)dst;
        uint4 v[kChunk / 8 / kThreads];
#pragma unroll
        for (int u = 0; u < kChunk / 8 / kThreads; ++u) {
            const int i = tid + u * kThreads;
            if (i < m8) v[u] = s4[i];
        }
#pragma unroll
        for (int u = 0; u < kChunk / 8 / kThreads; ++u) {
            const int i = tid + u * kThreads;
            if (i < m8) d4[i] = v[u];
        }
        for (int i = (m8 << 3) + tid; i < m; i += kThreads) dst[i] = src[i];
        return;
    }
    // dword j of dst holds elements 2j and 2j+1
    const int m2 = m >> 1;
    uint32_t *d2 = (uint32_t *)dst;
    constexpr int kPer = kChunk / 2 / kThreads;  // 16 dwords per thread
    uint32_t v[kPer];
    if ((a & 3) == 0) {
        const uint32_t *s2 = (const uint32_t *)src;
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int j = tid + u * kThreads;
            if (j < m2) v[u] = s2[j];
        }
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int j = tid + u * kThreads;
            if (j < m2) d2[j] = v[u];
        }
        if (tid == 0 && (m & 1)) dst[m - 1] = src[m - 1];
        return;
    }
    // src = 4-byte boundary + 2: aligned word w[i] (i >= 1) starts at element
    // 2i - 1 and holds elements 2i - 1 (low half) and 2i (high half), so dst
    // dword j = high(w[j]) | low(w[j+1]) << 16.  Dwords 1 .. m2 - 2 read words
    // 1 .. m2 - 1, which lie inside the chunk; dword 0, the last dword and an
    // odd tail are copied element by element.
    const uint32_t *w = (const uint32_t *)(a - 2);
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int j = tid + u * kThreads;
        if (j >= 1 && j <= m2 - 2) v[u] = (w[j] >> 16) | (w[j + 1] << 16);
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int j = tid + u * kThreads;
        if (j >= 1 && j <= m2 - 2) d2[j] = v[u];
    }
    if (tid < 2 && tid < m) dst[tid] = src[tid];
    for (int i = max(2, 2 * (m2 - 1)) + tid; i < m; i += kThreads) dst[i] = src[i];
}

int launch_gather(const GatherArgs &g, void *stream)
{
    if (g.n <= 0) return 0;
    if (g.n > kGatherMax) return -1;
    uint32_t nmax = 0;
    for (int i = 0; i < g.n; ++i) nmax = g.it[i].n > nmax ? g.it[i].n : nmax;
    if (nmax == 0) return 0;
    const unsigned chunks = (unsigned)((nmax + kChunk - 1) / kChunk);
    hipLaunchKernelGGL(gather_kernel, dim3(chunks, g.n), dim3(kThreads), 0, (hipStream_t)stream, g);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace tdec
