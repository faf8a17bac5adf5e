// enc_kernels.hip -- gfx950 kernels of the LTE turbo encoder.
//
// The paper's encoding function (Sec. IV-B, Fig. 3): a transport block is
// conditioned (CRC24A) and segmented into code blocks; each block b is
// encoded by two RSC encoders, the second one fed through the interleaver,
// giving (b, b', b'') at rate 1/3.  Constants per TS 36.212 5.1.3.2: RSC
// g0 = 1 + D^2 + D^3 (feedback), g1 = 1 + D + D^3 (parity), QPP
// interleaver, 3-step termination of each encoder.
//
// One work group of two waves per code block.  The block's payload bytes are
// staged in LDS and turned into the input bits as 32-bit words (a bit array);
// the block CRC is computed over those words by 64-bit chunks per thread, 4
// bits per table step, combined with the x^m mod g table; and each wave runs
// one RSC encoder with its 64 lanes on 64 consecutive chunks of the block.
// An RSC encoder is linear over GF(2) (state s = (a_{k-1}, a_{k-2},
// a_{k-3}), s' = A s + b u), so a chunk's output is its zero-state response
// plus the zero-input response of its start state.  Each lane takes its
// chunk's input bits as a 128-bit word (encoder 1 straight from the bit
// array, encoder 2 gathered through the interleaver) and computes the
// zero-state response with word operations (the feedback's impulse response
// is 7-periodic); the start state of chunk l is the XOR over j < l of
// A^(L (l-1-j)) e_j, e_j being chunk j's zero-state end state, with A^7 = I
// because 1 + D^2 + D^3 is primitive.  The start states come from a
// log-depth scan across the wave's lanes: with P(l) = XOR over j <= l of
// A^(L (l-j)) e_j, the step with offset d sets P(l) ^= A^(L d) P(l - d), and
// chunk l starts in P(l - 1).  The zero-input parity from a state is
// 7-periodic too, so the true parity is one more XOR.  The parity bits are
// ORed into the encoder's LDS bit array, and the work group writes all three
// streams from the bit arrays with coalesced stores, 8 bits to 8 bytes through
// a 256-entry table (5.6 KB of LDS per block).
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
typedef unsigned __int128 u128;
constexpr int kBitWords = kKmax / 32 + 4;  // bit arrays; spare words for 64- and 128-bit reads

// One byte per bit of a 4-bit value: bit j of n becomes byte j.
__device__ static inline uint32_t spread4(uint32_t n)
{
    return (n & 1u) | ((n & 2u) << 7) | ((n & 4u) << 14) | ((n & 8u) << 21);
}

__global__ void __launch_bounds__(kEncThreads) turbo_encode_kernel(const EncCb *cbs,
                                                                   const uint8_t *src,
                                                                   uint8_t *out,
                                                                   const uint32_t *crc_tab)
{
    __shared__ uint8_t raw[kKmax / 8 + 2];
    __shared__ uint32_t cw[kBitWords];     // input bit c_k: bit k % 32 of cw[k / 32]
    __shared__ uint32_t pz[2][kBitWords];  // parity bit k of encoder w: bit k % 32 of pz[w][k / 32]
    __shared__ uint32_t t4[16];            // CRC register after 4 zero bits from v x^20
    __shared__ uint2 sp8[256];             // byte j of sp8[v] = bit j of v
    __shared__ uint8_t tl[2][6];
    __shared__ uint32_t acc;
    __shared__ uint8_t zt[7][8];  // zt[q][s] = A^q s
    const EncCb cb = cbs[blockIdx.x];
    const int K = cb.K, F = cb.F, L = cb.crc ? 24 : 0;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const uint32_t poly = cb.crc == 1 ? kPoly24A : kPoly24B;
    // input bits: the payload bytes that hold bits src_bit .. src_bit + n_in - 1
    // are copied into LDS
    const int n_in = K - F - L;
    const int64_t byte0 = cb.src_bit >> 3;
    const int bo = (int)(cb.src_bit & 7);
    const int nbytes = (bo + n_in + 7) >> 3;  // <= kKmax / 8 + 1
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
    if (tid < 16) {
        uint32_t r = (uint32_t)tid << 20;
        for (int i = 0; i < 4; ++i) r = ((r << 1) & 0xFFFFFFu) ^ (((r >> 23) & 1u) ? poly : 0u);
        t4[tid] = r;
    }
    for (int i = tid; i < 2 * kBitWords; i += nthr) pz[i / kBitWords][i % kBitWords] = 0u;
    for (int v = tid; v < 256; v += nthr) sp8[v] = make_uint2(spread4(v & 15u), spread4(v >> 4));
    if (tid == 0) acc = 0u;
    __syncthreads();
    // c as words: 0 for the F filler bits, then the payload, then 0 where the
    // CRC goes (and past K).  Word j holds c_{32j} .. c_{32j+31}, whose payload
    // bits start at q = bo + 32 j - F (negative inside the filler): five bytes
    // from q / 8 hold them most significant bit first.
    for (int j = tid; j < kBitWords; j += nthr) {
        const int k = 32 * j, lo = max(F, k), hi = min(K - L, k + 32);
        uint32_t v = 0;
        if (lo < hi) {
            const int q = bo + k - F, base = q >> 3, sh = q & 7;
            uint64_t B = 0;
#pragma unroll
            for (int i = 0; i < 5; ++i) {
                const int bi = base + i;
                B = (B << 8) | (uint64_t)((bi >= 0 && bi < nbytes) ? raw[bi] : (uint8_t)0);
            }
            v = __builtin_bitreverse32((uint32_t)(B >> (8 - sh)));  // bit i = payload bit q + i
            const uint32_t mhi = hi - k == 32 ? 0xFFFFFFFFu : (1u << (hi - k)) - 1u;
            v &= mhi & ~((1u << (lo - k)) - 1u);
        }
        cw[j] = v;
    }
    __syncthreads();
    if (L) {
        // CRC of c_0 .. c_{n-1}, n = K - 24 (the remainder of M(x) x^24 mod
        // g): each thread takes 64 bits (a multiple of 4 bits, as is n), 4 bits
        // per table step, and moves its remainder to the end by r(x) x^m mod g
        // from the table T[m] = x^m mod g (m + 23 < kCrcTabN).
        const int n = K - 24;
        const int b0 = 64 * tid, b1 = min(n, b0 + 64);
        if (b0 < b1) {
            uint32_t r = 0;
            for (int j = b0 >> 5; j < (b1 + 31) >> 5; ++j) {
                const uint32_t x = __builtin_bitreverse32(cw[j]);  // c_{32j} in bit 31
                const int nb = min(32, b1 - 32 * j) >> 2;
                for (int i = 0; i < nb; ++i)
                    r = ((r << 4) & 0xFFFFFFu) ^ t4[((r >> 20) ^ (x >> (28 - 4 * i))) & 15u];
            }
            const uint32_t *T = crc_tab + (cb.crc == 1 ? 0 : kCrcTabN);
            const int m = n - b1;
            uint32_t o = 0;
#pragma unroll
            for (int i = 0; i < 24; ++i) o ^= ((r >> i) & 1u) ? T[m + i] : 0u;
            if (o) atomicXor(&acc, o);
        }
        __syncthreads();
        if (tid < 24) {
            const int k = K - 24 + tid;
            if ((acc >> (23 - tid)) & 1u) atomicOr(&cw[k >> 5], 1u << (k & 31));
        }
        __syncthreads();
    }
    // wave w runs encoder w + 1 (w = 1: input c'_k = c_{pi(k)}); lane l the
    // n steps [l Lc, min(K, (l + 1) Lc)), Lc <= 96
    const int w = tid >> 6, l = tid & 63;
    const int Lc = (K + 63) / 64;
    const int k0 = l * Lc, n = max(0, min(K, k0 + Lc) - k0);
    const uint32_t uK = (uint32_t)K;
    // The chunk's input bits, bit k = input of step k0 + k; bits past n are
    // never used.  Encoder 1 takes them from the bit array (k0 <= 63 Lc <=
    // 6048, so the four words lie in it).  Encoder 2 gathers c_{pi(k)} with the
    // QPP pi(k0) = (f1 k0 + f2 k0^2) mod K and its increment g(k) = pi(k + 1) -
    // pi(k) = f1 + f2 (2 k + 1) mod K, which grows by 2 f2 per step; its reads
    // run on to a whole number of words, every index staying below K.
    u128 U;
    if (w == 0) {
        const int i = k0 >> 5;
        const u128 X = (u128)cw[i] | ((u128)cw[i + 1] << 32) | ((u128)cw[i + 2] << 64) |
                       ((u128)cw[i + 3] << 96);
        U = X >> (k0 & 31);
    } else {
        const uint32_t kk = (uint32_t)k0;
        uint32_t pi = ((uint32_t)cb.f1 * kk % uK + (uint32_t)cb.f2 * (kk * kk % uK) % uK) % uK;
        uint32_t g = ((uint32_t)cb.f1 + (uint32_t)cb.f2 * (2u * kk + 1u)) % uK;
        const uint32_t dg = (2u * (uint32_t)cb.f2) % uK;
        const int nw = (Lc + 31) >> 5;
        uint32_t wv[3] = {0u, 0u, 0u};
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            if (j < nw) {
                uint32_t x = 0;
#pragma unroll
                for (int m = 0; m < 32; ++m) {
                    x |= ((cw[pi >> 5] >> (pi & 31)) & 1u) << m;
                    pi = min(pi + g, pi + g - uK);  // both below K: one of the two is the sum mod K
                    g = min(g + dg, g + dg - uK);
                }
                wv[j] = x;
            }
        }
        U = (u128)wv[0] | ((u128)wv[1] << 32) | ((u128)wv[2] << 64);
    }
    // Zero-state response a = u / (1 + D^2 + D^3).  The feedback's impulse
    // response is periodic with period 7 (the polynomial is primitive), one
    // period being 1 0 1 1 1 0 0, so a_k = V_k + V_{k-2} + V_{k-3} + V_{k-4}
    // over GF(2) with V_k the sum of u_{k-7q}, q >= 0: a stride-7 prefix XOR
    // by doubling.  Bit k of a 128-bit word is step k.
    u128 V = U;
    V ^= V << 7;
    V ^= V << 14;
    V ^= V << 28;
    V ^= V << 56;
    V ^= V << 112;
    const u128 av = V ^ (V << 2) ^ (V << 3) ^ (V << 4);
    const u128 zs = av ^ (av << 1) ^ (av << 3);  // z_k = a_k + a_{k-1} + a_{k-3}
    // the chunk's end state from state 0: (a_{n-1}, a_{n-2}, a_{n-3}) as
    // state bits 0, 1, 2 (a_j = 0 for j < 0)
    const uint32_t t3 = (uint32_t)((av << 3) >> n) & 7u;
    const uint32_t e = ((t3 & 1u) << 2) | (t3 & 2u) | (t3 >> 2);
    // start state of chunk l: chunks before it all have Lc steps, chunk j
    // contributes A^(Lc (l - 1 - j)) e_j (exponents mod 7); inclusive scan
    // of the wave, then the state of the lane before
    uint32_t s0;
    {
        uint32_t P = e;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t t = (uint32_t)__shfl_up((int)P, d, 64);
            if (l >= d) P ^= zt[(Lc * d) % 7][t];
        }
        s0 = (uint32_t)__shfl_up((int)P, 1, 64);
        if (l == 0) s0 = 0;
    }
    // The true parity adds the zero-input response from s0, whose parity is
    // periodic with period 7 from the chunk's first step (A^7 = I).
    uint32_t zz, zp = 0, sz = s0;
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        sz = rsc_step(sz, 0u, &zz);
        zp |= zz << j;
    }
    u128 R = zp;
    R |= R << 7;
    R |= R << 14;
    R |= R << 28;
    R |= R << 56;
    R |= R << 112;
    uint8_t *d = out + cb.out_off;
    const int N = K + 4;
    if (n > 0) {
        // the n parity bits into the LDS bit array at k0: the words from
        // k0 / 32 to (k0 + n - 1) / 32, shared with the neighbouring chunks
        const u128 z = (zs ^ R) & (((u128)1 << n) - 1);
        const int off = k0 & 31;
        const u128 X = z << off;  // off + n <= 127
        const int nwo = (off + n + 31) >> 5;
        uint32_t *pw = pz[w] + (k0 >> 5);
        atomicOr(&pw[0], (uint32_t)X);
        if (nwo > 1) atomicOr(&pw[1], (uint32_t)(X >> 32));
        if (nwo > 2) atomicOr(&pw[2], (uint32_t)(X >> 64));
        if (nwo > 3) atomicOr(&pw[3], (uint32_t)(X >> 96));
    }
    if (n > 0 && k0 + n == K) {
        // termination after the last step, from the state A^n s0 + e there:
        // input = feedback, so a = 0
        uint32_t s = e ^ zt[n % 7][s0];
        for (int j = 0; j < 3; ++j) {
            const uint32_t u = ((s >> 1) ^ (s >> 2)) & 1u;
            s = rsc_step(s, u, &zz);
            tl[w][2 * j] = (uint8_t)u;
            tl[w][2 * j + 1] = (uint8_t)zz;
        }
    }
    __syncthreads();
    // the three streams' first K bytes from the bit arrays (the input bits,
    // then each encoder's parity): byte stores up to an 8-byte boundary of the
    // destination, then 8 bytes per store, then the rest
#pragma unroll
    for (int st = 0; st < 3; ++st) {
        uint8_t *o = d + st * N;
        const uint32_t *pw = st == 0 ? cw : pz[st - 1];
        const int head = min(K, (int)((8u - ((uint32_t)(uintptr_t)o & 7u)) & 7u));
        const int n8 = (K - head) >> 3;
        if (tid < head) o[tid] = (uint8_t)((pw[tid >> 5] >> (tid & 31)) & 1u);
        for (int q = tid; q < n8; q += nthr) {
            const int k = head + 8 * q;
            const uint64_t v = ((uint64_t)pw[(k >> 5) + 1] << 32) | pw[k >> 5];
            *(uint2 *)(o + k) = sp8[(uint32_t)(v >> (k & 31)) & 0xFFu];
        }
        for (int k = head + 8 * n8 + tid; k < K; k += nthr)
            o[k] = (uint8_t)((pw[k >> 5] >> (k & 31)) & 1u);
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
