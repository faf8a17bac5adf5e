// probe_kernels.hip -- measured device ceilings (include/tdec_probe.h): the
// packed int16 VALU rate with the decoder's add-compare-select instructions,
// HBM streaming read and copy bandwidth, and launch overheads.
#include <hip/hip_runtime.h>

#include "tdec.h"
#include "tdec_probe.h"

namespace {

typedef short p16 __attribute__((ext_vector_type(2)));

constexpr int kProbeThreads = 256;
constexpr int kChains = 8;  // independent chains per lane: one wave issues back to back

// Eight chains of (saturating packed add, packed maximum) per lane: the two
// instructions of the decoder's recursions.  The result is stored so that
// nothing is dropped.
__global__ void __launch_bounds__(kProbeThreads) valu_probe_kernel(uint32_t *out, int iters,
                                                                   uint32_t seed)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    p16 a[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k)
        a[k] = __builtin_bit_cast(p16, seed ^ (t * 0x9E3779B9u + 0x01000193u * (uint32_t)k));
    const p16 b = __builtin_bit_cast(p16, seed * 3u + 1u);
    const p16 c = __builtin_bit_cast(p16, seed * 5u + 7u);
#pragma unroll 4
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) {
            a[k] = __builtin_elementwise_add_sat(a[k], b);
            a[k] = __builtin_elementwise_max(a[k], c);
        }
    }
    uint32_t x = 0;
#pragma unroll
    for (int k = 0; k < kChains; ++k) x ^= __builtin_bit_cast(uint32_t, a[k]);
    out[t] = x;
}

// 16-byte loads, four per thread in flight, folded into one word per thread.
__global__ void __launch_bounds__(kProbeThreads) read_probe_kernel(const uint4 *src, size_t n,
                                                                   uint32_t *out)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t acc = 0;
    size_t i = t;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const uint4 v0 = src[i], v1 = src[i + stride], v2 = src[i + 2 * stride],
                    v3 = src[i + 3 * stride];
        acc ^= v0.x ^ v0.y ^ v0.z ^ v0.w ^ v1.x ^ v1.y ^ v1.z ^ v1.w;
        acc ^= v2.x ^ v2.y ^ v2.z ^ v2.w ^ v3.x ^ v3.y ^ v3.z ^ v3.w;
    }
    for (; i < n; i += stride) {
        const uint4 v = src[i];
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    out[t] = acc;
}

__global__ void __launch_bounds__(kProbeThreads) copy_probe_kernel(const uint4 *src, uint4 *dst,
                                                                   size_t n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const uint4 v0 = src[i], v1 = src[i + stride], v2 = src[i + 2 * stride],
                    v3 = src[i + 3 * stride];
        dst[i] = v0;
        dst[i + stride] = v1;
        dst[i + 2 * stride] = v2;
        dst[i + 3 * stride] = v3;
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

__global__ void empty_kernel() {}

// Event pair on a private stream; every HIP error maps to TDEC_EDEVICE.
struct Probe {
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bool ok = true;
    explicit Probe(int device)
    {
        ok = hipSetDevice(device) == hipSuccess &&
             hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess &&
             hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
    }
    ~Probe()
    {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (st) (void)hipStreamDestroy(st);
    }
    // milliseconds between the two events, after the stream has finished
    bool elapsed(float *ms)
    {
        return hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(ms, e0, e1) == hipSuccess;
    }
};

int num_cus(int device)
{
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        return 0;
    return n;
}

}  // namespace

extern "C" int tdec_probe_valu_int16(int device, int32_t iters, double *tops)
{
    if (!tops || iters < 1 || iters > 1000000) return TDEC_EINVAL;
    Probe p(device);
    if (!p.ok) return TDEC_EDEVICE;
    const int cus = num_cus(device);
    if (cus < 1) return TDEC_EDEVICE;
    const int grid = 8 * cus;
    uint32_t *out = nullptr;
    if (hipMalloc(&out, (size_t)grid * kProbeThreads * sizeof(uint32_t)) != hipSuccess)
        return TDEC_ENOMEM;
    // one short launch to load the code, then the timed one
    hipLaunchKernelGGL(valu_probe_kernel, dim3(grid), dim3(kProbeThreads), 0, p.st, out, 16, 1u);
    bool ok = hipGetLastError() == hipSuccess && hipEventRecord(p.e0, p.st) == hipSuccess;
    hipLaunchKernelGGL(valu_probe_kernel, dim3(grid), dim3(kProbeThreads), 0, p.st, out, iters, 2u);
    ok = ok && hipGetLastError() == hipSuccess && hipEventRecord(p.e1, p.st) == hipSuccess;
    float ms = 0.f;
    ok = ok && p.elapsed(&ms) && ms > 0.f;
    (void)hipFree(out);
    if (!ok) return TDEC_EDEVICE;
    const double ops = (double)grid * kProbeThreads * iters * kChains * 2 /* instructions */ *
                       2 /* int16 halves */;
    *tops = ops / (ms * 1e-3) / 1e12;
    return TDEC_OK;
}

extern "C" int tdec_probe_hbm(int device, size_t bytes, double *read_gbs, double *copy_gbs)
{
    if (!read_gbs || !copy_gbs || bytes < ((size_t)16 << 20) || bytes > ((size_t)16 << 30) ||
        bytes % 16)
        return TDEC_EINVAL;
    Probe p(device);
    if (!p.ok) return TDEC_EDEVICE;
    const int cus = num_cus(device);
    if (cus < 1) return TDEC_EDEVICE;
    const int grid = 8 * cus;
    const size_t n = bytes / 16;
    uint4 *a = nullptr, *b = nullptr;
    uint32_t *out = nullptr;
    if (hipMalloc(&a, bytes) != hipSuccess || hipMalloc(&b, bytes) != hipSuccess ||
        hipMalloc(&out, (size_t)grid * kProbeThreads * sizeof(uint32_t)) != hipSuccess) {
        (void)hipFree(a);
        (void)hipFree(b);
        (void)hipFree(out);
        return TDEC_ENOMEM;
    }
    bool ok = hipMemsetAsync(a, 1, bytes, p.st) == hipSuccess;
    float ms_r = 0.f, ms_c = 0.f;
    // warm up each kernel once, then time it
    hipLaunchKernelGGL(read_probe_kernel, dim3(grid), dim3(kProbeThreads), 0, p.st, a, n, out);
    ok = ok && hipGetLastError() == hipSuccess && hipEventRecord(p.e0, p.st) == hipSuccess;
    hipLaunchKernelGGL(read_probe_kernel, dim3(grid), dim3(kProbeThreads), 0, p.st, a, n, out);
    ok = ok && hipGetLastError() == hipSuccess && hipEventRecord(p.e1, p.st) == hipSuccess &&
         p.elapsed(&ms_r);
    hipLaunchKernelGGL(copy_probe_kernel, dim3(grid), dim3(kProbeThreads), 0, p.st, a, b, n);
    ok = ok && hipGetLastError() == hipSuccess && hipEventRecord(p.e0, p.st) == hipSuccess;
    hipLaunchKernelGGL(copy_probe_kernel, dim3(grid), dim3(kProbeThreads), 0, p.st, a, b, n);
    ok = ok && hipGetLastError() == hipSuccess && hipEventRecord(p.e1, p.st) == hipSuccess &&
         p.elapsed(&ms_c);
    (void)hipFree(a);
    (void)hipFree(b);
    (void)hipFree(out);
    if (!ok || ms_r <= 0.f || ms_c <= 0.f) return TDEC_EDEVICE;
    *read_gbs = (double)bytes / (ms_r * 1e-3) / 1e9;
    *copy_gbs = 2.0 * (double)bytes / (ms_c * 1e-3) / 1e9;
    return TDEC_OK;
}

extern "C" int tdec_probe_launch(int device, int32_t n, double *us_launch, double *us_graph_node)
{
    if (!us_launch || !us_graph_node || n < 1 || n > 100000) return TDEC_EINVAL;
    Probe p(device);
    if (!p.ok) return TDEC_EDEVICE;
    hipLaunchKernelGGL(empty_kernel, dim3(1), dim3(64), 0, p.st);
    bool ok = hipGetLastError() == hipSuccess && hipStreamSynchronize(p.st) == hipSuccess &&
              hipEventRecord(p.e0, p.st) == hipSuccess;
    for (int i = 0; i < n && ok; ++i) {
        hipLaunchKernelGGL(empty_kernel, dim3(1), dim3(64), 0, p.st);
        ok = hipGetLastError() == hipSuccess;
    }
    float ms_l = 0.f, ms_g = 0.f;
    ok = ok && hipEventRecord(p.e1, p.st) == hipSuccess && p.elapsed(&ms_l);
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    ok = ok && hipStreamBeginCapture(p.st, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
        for (int i = 0; i < n; ++i) hipLaunchKernelGGL(empty_kernel, dim3(1), dim3(64), 0, p.st);
        ok = hipStreamEndCapture(p.st, &g) == hipSuccess && g != nullptr;
    }
    ok = ok && hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) == hipSuccess;
    ok = ok && hipGraphLaunch(ge, p.st) == hipSuccess && hipStreamSynchronize(p.st) == hipSuccess;
    ok = ok && hipEventRecord(p.e0, p.st) == hipSuccess && hipGraphLaunch(ge, p.st) == hipSuccess &&
         hipEventRecord(p.e1, p.st) == hipSuccess && p.elapsed(&ms_g);
    if (ge) (void)hipGraphExecDestroy(ge);
    if (g) (void)hipGraphDestroy(g);
    if (!ok) return TDEC_EDEVICE;
    *us_launch = ms_l * 1e3 / n;
    *us_graph_node = ms_g * 1e3 / n;
    return TDEC_OK;
}
