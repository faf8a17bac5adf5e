// enc_kernels.hip -- gfx950 kernels of the LTE turbo encoder.
//
// The paper's encoding function (Sec. IV-B, Fig. 3): a transport block is
// conditioned (CRC24A) and segmented into code blocks; each block b is
// encoded by two RSC encoders, the second one fed through the interleaver,
// giving (b, b', b'') at rate 1/3.  Constants per TS 36.212 5.1.3.2: RSC
// g0 = 1 + D^2 + D^3 (feedback), g1 = 1 + D + D^3 (parity), QPP
// interleaver, 3-step termination of each encoder.
//
// One work group of two waves per code block: the block's input bits are
// staged in LDS, the block CRC is computed by per-thread LFSR chunks combined
// with the x^m mod g table, and each wave runs one RSC encoder with its 64
// lanes on 64 consecutive chunks of the block.  An RSC encoder is linear over
// GF(2) (state s = (a_{k-1}, a_{k-2}, a_{k-3}), s' = A s + b u): every lane
// first runs its chunk from state 0 to get the chunk's zero-state end state
// e_j; the true start state of chunk l is the XOR over j < l of
// A^(L (l-1-j)) e_j, with A^7 = I because 1 + D^2 + D^3 is primitive; then
// every lane runs its chunk again from that state and writes its parity bits
// straight to the output (the block's LDS holds only its input bits, so 16
// blocks fit a CU).
// The start states come from a log-depth scan across the wave's lanes: with
// P(l) = XOR over j <= l of A^(L (l-j)) e_j, the step with offset d sets
// P(l) ^= A^(L d) P(l - d), and chunk l starts in P(l - 1).
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
// computed by the whole work group; result valid in every thread.  Each
// thread's chunk remainder is moved to the end by r(x) x^m mod g from the
// table T[m] = x^m mod g (m + 23 < kCrcTabN).
__device__ static uint32_t block_crc(const uint8_t *c, int n, uint32_t poly, const uint32_t *T,
                                     uint32_t *acc)
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
        uint32_t o = 0;
        const int m = n - b1;
#pragma unroll
        for (int i = 0; i < 24; ++i) o ^= ((r >> i) & 1u) ? T[m + i] : 0u;
        if (o) atomicXor(acc, o);
    }
    __syncthreads();
    return *acc;
}

// RSC state as 3 bits: bit 0 = a_{k-1}, bit 1 = a_{k-2}, bit 2 = a_{k-3}.
// One step with input u: feedback a = u ^ a_{k-2} ^ a_{k-3}, parity
// z = a ^ a_{k-1} ^ a_{k-3}.
__device__ static inline uint32_t rsc_step(uint32_t s, uint32_t u, uint32_t *z)
{
    const uint32_t a1 = s & 1u, a2 = (s >> 1) & 1u, a3 = (s >> 2) & 1u;
    const uint32_t a = u ^ a2 ^ a3;
    *z = a ^ a1 ^ a3;
    return a | (a1 << 1) | (a2 << 2);
}

// A^p s: p zero-input steps.
__device__ static inline uint32_t rsc_zero_steps(uint32_t s, int p)
{
    uint32_t z;
    for (int i = 0; i < p; ++i) s = rsc_step(s, 0u, &z);
    return s;
}

constexpr int kEncThreads = 128;  // two waves: encoder 1 and encoder 2

__global__ void __launch_bounds__(kEncThreads) turbo_encode_kernel(const EncCb *cbs,
                                                                   const uint8_t *src,
                                                                   uint8_t *out,
                                                                   const uint32_t *crc_tab)
{
    __shared__ uint8_t c[kKmax];
    __shared__ uint8_t raw[kKmax / 8 + 2];
    __shared__ uint8_t tl[2][6];
    __shared__ uint32_t acc;
    __shared__ uint8_t zt[7][8];  // zt[q][s] = A^q s
    const EncCb cb = cbs[blockIdx.x];
    const int K = cb.K, F = cb.F, L = cb.crc ? 24 : 0;
    const int tid = threadIdx.x, nthr = blockDim.x;
    // input bits: the payload bytes that hold bits src_bit .. src_bit + n - 1
    // are copied into LDS, then expanded to one bit per byte
    const int n = K - F - L;
    const int64_t byte0 = cb.src_bit >> 3;
    const int bo = (int)(cb.src_bit & 7);
    const int nbytes = (bo + n + 7) >> 3;  // <= kKmax / 8 + 1
    for (int i0 = tid; i0 < nbytes; i0 += 4 * nthr) {
        uint8_t v[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int i = i0 + m * nthr;
            v[m] = i < nbytes ? src[byte0 + i] : (uint8_t)0;
        }
#pragma unroll
        for (int m = 0; m < 4; ++m)
            if (i0 + m * nthr < nbytes) raw[i0 + m * nthr] = v[m];
    }
    if (tid < 56) zt[tid >> 3][tid & 7] = (uint8_t)rsc_zero_steps((uint32_t)(tid & 7), tid >> 3);
    __syncthreads();
    for (int k = tid; k < K; k += nthr) {
        const int b = bo + (k - F);
        c[k] = (k >= F && k < K - L) ? (uint8_t)((raw[b >> 3] >> (7 - (b & 7))) & 1u) : (uint8_t)0;
    }
    __syncthreads();
    if (L) {
        const uint32_t p = block_crc(c, K - L, cb.crc == 1 ? kPoly24A : kPoly24B,
                                     crc_tab + (cb.crc == 1 ? 0 : kCrcTabN), &acc);
        if (tid < 24) c[K - 24 + tid] = (uint8_t)((p >> (23 - tid)) & 1u);
        __syncthreads();
    }
    // wave w runs encoder w + 1 (w = 1: input c'_k = c_{pi(k)}); lane l the
    // steps [l Lc, min(K, (l + 1) Lc))
    const int w = tid >> 6, l = tid & 63;
    const int Lc = (K + 63) / 64;
    const int k0 = l * Lc, k1 = min(K, k0 + Lc);
    const uint32_t uK = (uint32_t)K;
    // QPP pi(k0) = (f1 k0 + f2 k0^2) mod K and its increment
    // g(k0) = pi(k0 + 1) - pi(k0) = f1 + f2 (2 k0 + 1) mod K
    const uint32_t pi0 = ((uint32_t)cb.f1 * (uint32_t)k0 % uK +
                          (uint32_t)cb.f2 * ((uint32_t)k0 * (uint32_t)k0 % uK) % uK) % uK;
    const uint32_t g0 = ((uint32_t)cb.f1 + (uint32_t)cb.f2 * (2u * (uint32_t)k0 + 1u)) % uK;
    const uint32_t f2x2 = (2u * (uint32_t)cb.f2) % uK;
    // The chunk's inputs, 8 steps at a time: the 8 reads go out before the
    // serial steps use them.
    auto inputs8 = [&](int k, uint32_t &pi, uint32_t &g, uint32_t u[8]) {
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            if (w == 0) {
                u[m] = k + m < k1 ? c[k + m] : 0u;
            } else {
                u[m] = k + m < k1 ? c[pi] : 0u;
                pi += g;
                if (pi >= uK) pi -= uK;
                g += f2x2;
                if (g >= uK) g -= uK;
            }
        }
    };
    // pass 1: end state of the chunk from state 0
    uint32_t s = 0, zz;
    {
        uint32_t pi = pi0, g = g0, u[8];
        for (int k = k0; k < k1; k += 8) {
            inputs8(k, pi, g, u);
#pragma unroll
            for (int m = 0; m < 8; ++m)
                if (k + m < k1) s = rsc_step(s, u[m], &zz);
        }
    }
    // start state of chunk l: chunks before it all have Lc steps, chunk j
    // contributes A^(Lc (l - 1 - j)) e_j (exponents mod 7); inclusive scan
    // of the wave, then the state of the lane before
    uint32_t s0;
    {
        uint32_t P = s;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t t = (uint32_t)__shfl_up((int)P, d, 64);
            if (l >= d) P ^= zt[(Lc * d) % 7][t];
        }
        s0 = (uint32_t)__shfl_up((int)P, 1, 64);
        if (l == 0) s0 = 0;
    }
    // pass 2: the chunk from its true start state; the parity bytes of 8
    // steps go straight to the encoder's output stream, as two words when
    // the destination is 4-byte aligned
    uint8_t *d = out + cb.out_off;
    const int N = K + 4;
    s = s0;
    {
        uint8_t *oz = d + (w + 1) * N;
        uint32_t pi = pi0, g = g0, u[8];
        for (int k = k0; k < k1; k += 8) {
            inputs8(k, pi, g, u);
            uint32_t zw[2] = {0u, 0u};
#pragma unroll
            for (int m = 0; m < 8; ++m)
                if (k + m < k1) {
                    s = rsc_step(s, u[m], &zz);
                    zw[m >> 2] |= zz << (8 * (m & 3));
                }
            uint8_t *o = oz + k;
            const int cnt = min(8, k1 - k);
            if (cnt == 8 && ((uint32_t)(uintptr_t)o & 3u) == 0) {
                *(uint32_t *)o = zw[0];
                *(uint32_t *)(o + 4) = zw[1];
            } else {
                for (int m = 0; m < cnt; ++m) o[m] = (uint8_t)(zw[m >> 2] >> (8 * (m & 3)));
            }
        }
    }
    if (k0 < K && k1 == K) {
        // termination after the last step: input = feedback, so a = 0
        for (int j = 0; j < 3; ++j) {
            const uint32_t u = ((s >> 1) ^ (s >> 2)) & 1u;
            s = rsc_step(s, u, &zz);
            tl[w][2 * j] = (uint8_t)u;
            tl[w][2 * j + 1] = (uint8_t)zz;
        }
    }
    __syncthreads();
    // the systematic stream's first K bytes: byte stores up to a 4-byte
    // boundary of the destination, then whole words assembled from LDS,
    // then the rest
    {
        uint8_t *o = d;
        const int head = min(K, (int)((4u - ((uint32_t)(uintptr_t)o & 3u)) & 3u));
        const int nw4 = (K - head) >> 2;
        if (tid < head) o[tid] = c[tid];
        for (int q = tid; q < nw4; q += nthr) {
            const int k = head + 4 * q;
            *(uint32_t *)(o + k) = (uint32_t)c[k] | ((uint32_t)c[k + 1] << 8) |
                                   ((uint32_t)c[k + 2] << 16) | ((uint32_t)c[k + 3] << 24);
        }
        for (int k = head + 4 * nw4 + tid; k < K; k += nthr) o[k] = c[k];
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
    if (n_cb <= 0) return 0;
    hipLaunchKernelGGL(turbo_encode_kernel, dim3(n_cb), dim3(kEncThreads), 0, (hipStream_t)stream,
                       cbs, src, out, crc_tab);
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
