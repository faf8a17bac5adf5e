// enc_kernels.hip -- gfx950 kernels of the LTE turbo encoder.
//
// The paper's encoding function (Sec. IV-B, Fig. 3): a transport block is
// conditioned (CRC24A) and segmented into code blocks; each block b is
// encoded by two RSC encoders, the second one fed through the interleaver,
// giving (b, b', b'') at rate 1/3.  Constants per TS 36.212 5.1.3.2: RSC
// g0 = 1 + D^2 + D^3 (feedback), g1 = 1 + D + D^3 (parity), QPP
// interleaver, 3-step termination of each encoder.
//
// One work group per code block: the block's input bits are staged in LDS,
// the block CRC is computed by per-thread LFSR chunks combined with
// x^n mod g, then two lanes run the two (inherently serial) shift registers
// while the others copy the systematic stream.
#include <hip/hip_runtime.h>

#include "tdec_internal.h"

namespace tdec {

__device__ static uint32_t enc_mulmod(uint32_t a, uint32_t b, uint32_t poly)
{
    uint32_t r = 0;
    for (int i = 23; i >= 0; --i) {
        const uint32_t top = (r >> 23) & 1u;
        r = ((r << 1) & 0xFFFFFFu) ^ (top ? poly : 0u);
        if ((b >> i) & 1u) r ^= a;
    }
    return r;
}

__device__ static uint32_t enc_xpow(uint64_t n, uint32_t poly)
{
    uint32_t res = 1, base = 2;
    while (n) {
        if (n & 1) res = enc_mulmod(res, base, poly);
        base = enc_mulmod(base, base, poly);
        n >>= 1;
    }
    return res;
}

__device__ static inline uint32_t src_bit(const uint8_t *src, int64_t b)
{
    return (src[b >> 3] >> (7 - (b & 7))) & 1u;
}

// CRC (remainder of M(x) x^24 mod g) of bits c[0..n-1] held one per byte,
// computed by the whole work group; result valid in every thread.
__device__ static uint32_t block_crc(const uint8_t *c, int n, uint32_t poly, uint32_t *acc)
{
    const int tid = threadIdx.x, nthr = blockDim.x;
    if (tid == 0) *acc = 0;
    __syncthreads();
    const int chunk = (n + nthr - 1) / nthr;
    const int b0 = tid * chunk, b1 = min(n, b0 + chunk);
    if (b0 < b1) {
        uint32_t r = 0;
        for (int b = b0; b < b1; ++b) {
            const uint32_t top = ((r >> 23) ^ c[b]) & 1u;
            r = ((r << 1) & 0xFFFFFFu) ^ (top ? poly : 0u);
        }
        if (r && n - b1 > 0) r = enc_mulmod(r, enc_xpow((uint64_t)(n - b1), poly), poly);
        if (r) atomicXor(acc, r);
    }
    __syncthreads();
    return *acc;
}

__global__ void __launch_bounds__(64) turbo_encode_kernel(const EncCb *cbs, const uint8_t *src,
                                                          uint8_t *out)
{
    __shared__ uint8_t c[kKmax];
    __shared__ uint8_t z[2][kKmax];
    __shared__ uint8_t tl[2][6];
    __shared__ uint32_t acc;
    const EncCb cb = cbs[blockIdx.x];
    const int K = cb.K, F = cb.F, L = cb.crc ? 24 : 0;
    const int tid = threadIdx.x, nthr = blockDim.x;
    for (int k = tid; k < K; k += nthr) {
        uint8_t v = 0;
        if (k >= F && k < K - L) v = (uint8_t)src_bit(src, cb.src_bit + (k - F));
        c[k] = v;
    }
    __syncthreads();
    if (L) {
        const uint32_t p = block_crc(c, K - L, cb.crc == 1 ? kPoly24A : kPoly24B, &acc);
        if (tid < 24) c[K - 24 + tid] = (uint8_t)((p >> (23 - tid)) & 1u);
        __syncthreads();
    }
    if (tid < 2) {
        // shift register (a_{k-1}, a_{k-2}, a_{k-3})
        uint32_t a1 = 0, a2 = 0, a3 = 0;
        uint32_t pi = 0, g = (uint32_t)((cb.f1 + cb.f2) % K);
        const uint32_t f2x2 = (uint32_t)((2 * cb.f2) % K);
        for (int k = 0; k < K; ++k) {
            uint32_t u;
            if (tid == 0) {
                u = c[k];
            } else {
                u = c[pi];  // c'_k = c_{pi(k)}
                pi += g;
                if (pi >= (uint32_t)K) pi -= K;
                g += f2x2;
                if (g >= (uint32_t)K) g -= K;
            }
            const uint32_t a = u ^ a2 ^ a3;
            z[tid][k] = (uint8_t)(a ^ a1 ^ a3);
            a3 = a2;
            a2 = a1;
            a1 = a;
        }
        for (int j = 0; j < 3; ++j) {  // termination: input = feedback, a = 0
            const uint32_t u = a2 ^ a3;
            tl[tid][2 * j] = (uint8_t)u;
            tl[tid][2 * j + 1] = (uint8_t)(a1 ^ a3);
            a3 = a2;
            a2 = a1;
            a1 = 0;
        }
    }
    __syncthreads();
    uint8_t *d = out + cb.out_off;
    const int N = K + 4;
    for (int k = tid; k < K; k += nthr) {
        d[k] = c[k];
        d[N + k] = z[0][k];
        d[2 * N + k] = z[1][k];
    }
    if (tid < 12) {
        // x z x z x z of each encoder, read round robin into d0, d1, d2
        const int e = tid / 6, q = tid % 6;
        d[(q % 3) * N + K + 2 * e + q / 3] = tl[e][q];
    }
}

int launch_encode(const EncCb *cbs, int n_cb, const uint8_t *src, uint8_t *out,
                  const uint32_t *crc_tab, void *stream)
{
    (void)crc_tab;
    if (n_cb <= 0) return 0;
    hipLaunchKernelGGL(turbo_encode_kernel, dim3(n_cb), dim3(64), 0, (hipStream_t)stream, cbs, src,
                       out);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Transport block conditioning: out = payload (tbs bits) followed by its
// CRC24A, packed MSB first.
__global__ void __launch_bounds__(256) tb_crc_attach_kernel(const uint8_t *payload, int32_t tbs,
                                                            uint8_t *out)
{
    __shared__ uint32_t acc;
    const int tid = threadIdx.x, nthr = blockDim.x;
    if (tid == 0) acc = 0;
    __syncthreads();
    const int chunk = (tbs + nthr - 1) / nthr;
    const int b0 = tid * chunk, b1 = min(tbs, b0 + chunk);
    if (b0 < b1) {
        uint32_t r = 0;
        for (int b = b0; b < b1; ++b) {
            const uint32_t top = ((r >> 23) ^ src_bit(payload, b)) & 1u;
            r = ((r << 1) & 0xFFFFFFu) ^ (top ? kPoly24A : 0u);
        }
        if (r && tbs - b1 > 0) r = enc_mulmod(r, enc_xpow((uint64_t)(tbs - b1), kPoly24A), kPoly24A);
        if (r) atomicXor(&acc, r);
    }
    __syncthreads();
    const uint32_t p = acc;
    const int B = tbs + 24, nbytes = (B + 7) >> 3;
    for (int q = tid; q < nbytes; q += nthr) {
        uint32_t v = 0;
        for (int k = 0; k < 8; ++k) {
            const int b = 8 * q + k;
            uint32_t bit = 0;
            if (b < tbs) bit = src_bit(payload, b);
            else if (b < B) bit = (p >> (23 - (b - tbs))) & 1u;
            v = (v << 1) | bit;
        }
        out[q] = (uint8_t)v;
    }
}

int launch_tb_crc_attach(const uint8_t *payload, int32_t tbs, uint8_t *stream_bits,
                         const uint32_t *crc_tab, void *stream)
{
    (void)crc_tab;
    hipLaunchKernelGGL(tb_crc_attach_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream, payload,
                       tbs, stream_bits);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace tdec
