// dec_kernels.hip -- gfx950 kernels of the LTE turbo decoder.
//
// Method (paper Sec. IV-B "Decoding function", Fig. 4): decoder 1 runs
// max-log-MAP over (systematic + a-priori, parity 1) in natural order; its
// extrinsic, scaled by 0.75, becomes decoder 2's a-priori in QPP-interleaved
// order; decoder 2 runs over (interleaved systematic + a-priori, parity 2)
// and its scaled extrinsic returns de-interleaved; each full iteration ends
// with a hard decision on decoder 2's a-posteriori values and, when asked, a
// CRC check that may stop the block early.
//
// Mapping to CDNA4 (one code block never leaves its work group):
//   * one lane = one trellis window; all 8 state metrics of the window live
//     in the lane as packed int16 pairs, so an add-compare-select step is 8
//     v_pk_add_i16 (saturating) + 4 v_pk_max_i16 with the broadcasts and
//     swaps folded into op_sel: no cross-lane traffic at all;
//   * forward metrics are kept as checkpoints every S steps (global scratch)
//     and recomputed segment by segment in registers during the backward
//     sweep, which computes the extrinsic from the stored segment;
//   * the extrinsic/a-priori array of a block lives in LDS for the whole
//     decode (padded one int16 per 64 to spread banks); decoder 2 reaches it
//     through the QPP address, generated per step by its second-order
//     recurrence;
//   * the channel LLRs are restaged once per block into a window-interleaved
//     layout in global scratch, so the 32 lanes of a block read one 128-byte
//     line per load (16 B per lane = 4 trellis steps);
//   * hard decisions are OR-ed into an LDS bitmap, the CRC is a per-window
//     LFSR combined across windows with x^n mod g tables.
//
// Metric layouts: alpha "P" = {(a0,a4),(a1,a5),(a2,a6),(a3,a7)},
// beta "Q" = {(b0,b1),(b2,b3),(b4,b5),(b6,b7)} with state s = 4 a_{k-1} +
// 2 a_{k-2} + a_{k-3}.  Branch metric pairs of a step: g00 = (0, Lsa+Lp),
// g01 = (Lp, Lsa); their swaps g11 and g10 complete the four values.
#include <hip/hip_runtime.h>

#include "tdec_internal.h"

namespace tdec {

typedef short s2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ s2 bcx(s2 v) { return (s2){v.x, v.x}; }
__device__ __forceinline__ s2 bcy(s2 v) { return (s2){v.y, v.y}; }
__device__ __forceinline__ s2 swp(s2 v) { return (s2){v.y, v.x}; }
__device__ __forceinline__ s2 adds(s2 a, s2 b) { return __builtin_elementwise_add_sat(a, b); }
__device__ __forceinline__ s2 subs(s2 a, s2 b) { return __builtin_elementwise_sub_sat(a, b); }
__device__ __forceinline__ s2 vmax(s2 a, s2 b) { return __builtin_elementwise_max(a, b); }
__device__ __forceinline__ s2 as_s2(uint32_t u) { return __builtin_bit_cast(s2, u); }
__device__ __forceinline__ uint32_t as_u(s2 v) { return __builtin_bit_cast(uint32_t, v); }

constexpr short kNeg = -32768;

// g00 = (0, Lp + Lsa) from g01 = (Lp, Lsa).
__device__ __forceinline__ s2 mk_g00(s2 g01)
{
    s2 x = g01 + swp(g01);  // |Lp + Lsa| <= 6141: no wrap
    return as_s2(as_u(x) & 0xFFFF0000u);
}

// Forward add-compare-select, P layout in and out.
__device__ __forceinline__ void acs_fwd(s2 A[4], s2 g00, s2 g01)
{
    const s2 g11 = swp(g00), g10 = swp(g01);
    const s2 n0 = vmax(adds(bcx(A[0]), g00), adds(bcx(A[1]), g11));
    const s2 n1 = vmax(adds(bcx(A[2]), g10), adds(bcx(A[3]), g01));
    const s2 n2 = vmax(adds(bcy(A[0]), g01), adds(bcy(A[1]), g10));
    const s2 n3 = vmax(adds(bcy(A[2]), g11), adds(bcy(A[3]), g00));
    A[0] = n0;
    A[1] = n1;
    A[2] = n2;
    A[3] = n3;
}

// Shift a metric vector so that its maximum is 0.
__device__ __forceinline__ void normalise(s2 V[4])
{
    s2 m = vmax(vmax(V[0], V[1]), vmax(V[2], V[3]));
    m = vmax(m, swp(m));
    V[0] = subs(V[0], m);
    V[1] = subs(V[1], m);
    V[2] = subs(V[2], m);
    V[3] = subs(V[3], m);
}

// Backward step: from beta_{k+1} (Q layout) and the forward metric alpha_k
// (Q layout) compute the extrinsic Le(k) and replace B by beta_k.
__device__ __forceinline__ int bwd_le(s2 B[4], const s2 AQ[4], s2 g00, s2 g01)
{
    const s2 g11 = swp(g00), g10 = swp(g01);
    // candidates beta_{k+1}(next) + gamma for the branches of states 2j, 2j+1
    const s2 c00 = adds(bcx(B[0]), g00), c01 = adds(bcx(B[2]), g11);
    const s2 c10 = adds(bcy(B[0]), g10), c11 = adds(bcy(B[2]), g01);
    const s2 c20 = adds(bcx(B[1]), g01), c21 = adds(bcx(B[3]), g10);
    const s2 c30 = adds(bcy(B[1]), g11), c31 = adds(bcy(B[3]), g00);
    // alpha + candidate: halves ordered (u=0, u=1) in n, (u=1, u=0) in s
    const s2 n = vmax(vmax(adds(AQ[0], c00), adds(AQ[1], c11)),
                      vmax(adds(AQ[2], c20), adds(AQ[3], c31)));
    const s2 s = vmax(vmax(adds(AQ[0], c01), adds(AQ[1], c10)),
                      vmax(adds(AQ[2], c21), adds(AQ[3], c30)));
    const s2 m = vmax(n, swp(s));
    B[0] = vmax(c00, c01);
    B[1] = vmax(c10, c11);
    B[2] = vmax(c20, c21);
    B[3] = vmax(c30, c31);
    // Le = M1 - M0 - Lsa, exact modulo 2^16 (the true value fits int16)
    return (int)(short)(m.y - m.x - g01.y);
}

__device__ __forceinline__ void to_q(const s2 A[4], s2 Q[4])
{
    Q[0] = (s2){A[0].x, A[1].x};
    Q[1] = (s2){A[2].x, A[3].x};
    Q[2] = (s2){A[0].y, A[1].y};
    Q[3] = (s2){A[2].y, A[3].y};
}

// 0.75 * e truncated toward zero, clamped to +-2047 (clamping e to +-2730
// first gives the same value and keeps 3e in int16 range).
__device__ __forceinline__ int scale_ext(int e)
{
    e = max(-2730, min(2730, e));
    const int t = 3 * e;
    return (t + ((t >> 31) & 3)) >> 2;
}

__device__ __forceinline__ int epad(int j) { return j + (j >> 6); }

__device__ __forceinline__ uint32_t modadd(uint32_t a, uint32_t b, uint32_t K)
{
    const uint32_t s = a + b;
    return min(s, s - K);
}

__device__ __forceinline__ uint4 pack4(const s2 V[4])
{
    return make_uint4(as_u(V[0]), as_u(V[1]), as_u(V[2]), as_u(V[3]));
}
__device__ __forceinline__ void unpack4(uint4 u, s2 V[4])
{
    V[0] = as_s2(u.x);
    V[1] = as_s2(u.y);
    V[2] = as_s2(u.z);
    V[3] = as_s2(u.w);
}

// Everything one lane needs for a constituent pass over its window.
struct LaneCtx {
    int K, W, nw, w, lo;
    uint32_t f2x2;      // 2 f2 mod K
    uint32_t pi0, g0;   // QPP position and increment at the window start
    short *E;           // LDS extrinsic / a-priori array of the block (padded)
    uint32_t *bm;       // LDS hard-decision bitmap of the block
    const int4 *R1;     // restaged (Lp1 | Ls << 16), [t/4][w] x 4 steps
    const uint2 *R2;    // restaged Lp2, [t/4][w] x 4 steps
    uint4 *ck_a;        // forward checkpoints [seg][lane]
    uint2 *ck_p;        // QPP state at the checkpoints [seg][lane]
    int lanes;          // lanes of the item (checkpoint stride)
    int lane;
    bool first, last;
};

// Forward metric step i (1-based, counted from the window start) is
// normalised for i <= 2 and for even i; window 0 re-pins the states that
// cannot be reached after 1 and 2 steps to minus infinity.
template <int S>
__device__ __forceinline__ void fwd_post(s2 A[4], int i0, int t, bool first)
{
    if ((t & 1) || (i0 == 0 && t == 0)) normalise(A);
    if (i0 == 0 && t < 2 && first) {
        const s2 neg = (s2){kNeg, kNeg};
        A[1] = neg;
        A[3] = neg;
        if (t == 0) A[2] = neg;
    }
}

// One constituent decoder pass over the lane's window.
//   DEC 1: natural order, systematic + a-priori from E, parity 1; writes
//          E[j] = Ls[j] + scaled Le[j] (decoder 2's systematic + a-priori).
//   DEC 2: interleaved order, E[pi(k)] holds Ls + La, parity 2; writes
//          E[pi(k)] = scaled Le[k] and the hard decision of pi(k).
// The window's boundary metrics go to the neighbours' slots for the next
// iteration (alpha at the window end, beta at the window start).
template <int DEC, int S>
__device__ void run_pass(const LaneCtx &c, const s2 Ainit[4], const s2 Binit[4], uint4 *bnd_a_out,
                         uint4 *bnd_b_out)
{
    const int nseg = c.W / S;
    s2 A[4] = {Ainit[0], Ainit[1], Ainit[2], Ainit[3]};
    uint32_t pi = c.pi0, g = c.g0;
    const uint32_t K = (uint32_t)c.K;

    // ---- forward sweep: checkpoints only
    for (int seg = 0; seg < nseg; ++seg) {
        const int i0 = seg * S;
        c.ck_a[seg * c.lanes + c.lane] = pack4(A);
        if (DEC == 2) c.ck_p[seg * c.lanes + c.lane] = make_uint2(pi, g);
        uint32_t r[S];
        if (DEC == 1) {
#pragma unroll
            for (int m = 0; m < S / 4; ++m) {
                const int4 q = c.R1[((i0 >> 2) + m) * c.nw + c.w];
                r[4 * m + 0] = q.x;
                r[4 * m + 1] = q.y;
                r[4 * m + 2] = q.z;
                r[4 * m + 3] = q.w;
            }
        } else {
#pragma unroll
            for (int m = 0; m < S / 4; ++m) {
                const uint2 q = c.R2[((i0 >> 2) + m) * c.nw + c.w];
                r[4 * m + 0] = q.x & 0xFFFFu;
                r[4 * m + 1] = q.x >> 16;
                r[4 * m + 2] = q.y & 0xFFFFu;
                r[4 * m + 3] = q.y >> 16;
            }
        }
#pragma unroll
        for (int t = 0; t < S; ++t) {
            s2 g01;
            if (DEC == 1) {
                const uint32_t e = (uint16_t)c.E[epad(c.lo + i0 + t)];
                g01 = as_s2(r[t] + (e << 16));
            } else {
                const uint32_t e = (uint16_t)c.E[epad((int)pi)];
                g01 = as_s2(r[t] | (e << 16));
                pi = modadd(pi, g, K);
                g = modadd(g, c.f2x2, K);
            }
            acs_fwd(A, mk_g00(g01), g01);
            fwd_post<S>(A, i0, t, c.first);
        }
    }
    if (!c.last) *bnd_a_out = pack4(A);

    // ---- backward sweep: recompute each segment's forward metrics, then
    //      run beta over it and emit the extrinsic
    s2 Bq[4] = {Binit[0], Binit[1], Binit[2], Binit[3]};
    for (int seg = nseg - 1; seg >= 0; --seg) {
        const int i0 = seg * S;
        unpack4(c.ck_a[seg * c.lanes + c.lane], A);
        if (DEC == 2) {
            const uint2 p = c.ck_p[seg * c.lanes + c.lane];
            pi = p.x;
            g = p.y;
        }
        uint32_t r[S];
        if (DEC == 1) {
#pragma unroll
            for (int m = 0; m < S / 4; ++m) {
                const int4 q = c.R1[((i0 >> 2) + m) * c.nw + c.w];
                r[4 * m + 0] = q.x;
                r[4 * m + 1] = q.y;
                r[4 * m + 2] = q.z;
                r[4 * m + 3] = q.w;
            }
        } else {
#pragma unroll
            for (int m = 0; m < S / 4; ++m) {
                const uint2 q = c.R2[((i0 >> 2) + m) * c.nw + c.w];
                r[4 * m + 0] = q.x & 0xFFFFu;
                r[4 * m + 1] = q.x >> 16;
                r[4 * m + 2] = q.y & 0xFFFFu;
                r[4 * m + 3] = q.y >> 16;
            }
        }
        s2 AQ[S][4];
        s2 G01[S];
        uint32_t aux[S];
#pragma unroll
        for (int t = 0; t < S; ++t) {
            s2 g01;
            if (DEC == 1) {
                const uint32_t e = (uint16_t)c.E[epad(c.lo + i0 + t)];
                g01 = as_s2(r[t] + (e << 16));
                aux[t] = r[t];
            } else {
                const uint32_t e = (uint16_t)c.E[epad((int)pi)];
                g01 = as_s2(r[t] | (e << 16));
                aux[t] = pi;
                pi = modadd(pi, g, K);
                g = modadd(g, c.f2x2, K);
            }
            G01[t] = g01;
            to_q(A, AQ[t]);
            acs_fwd(A, mk_g00(g01), g01);
            fwd_post<S>(A, i0, t, c.first);
        }
#pragma unroll
        for (int t = S - 1; t >= 0; --t) {
            const s2 g01 = G01[t];
            const int le = bwd_le(Bq, AQ[t], mk_g00(g01), g01);
            // beta at local position i0+t; steps from its init = W - i0 - t
            if (!(t & 1) || (seg == nseg - 1 && t >= S - 2)) normalise(Bq);
            const int q = scale_ext(le);
            if (DEC == 1) {
                const int ls = (int)(short)(aux[t] >> 16);
                c.E[epad(c.lo + i0 + t)] = (short)(ls + q);
            } else {
                const int p = (int)aux[t];
                c.E[epad(p)] = (short)q;
                if ((int)g01.y + le > 0) atomicOr(&c.bm[p >> 5], 0x80000000u >> (p & 31));
            }
        }
    }
    if (!c.first) *bnd_b_out = pack4(Bq);
}

// CRC (LFSR form, MSB first) of natural bits [b0, b1) of a block's bitmap.
__device__ uint32_t crc_range(const uint32_t *bm, int b0, int b1, uint32_t poly)
{
    uint32_t r = 0;
    int b = b0;
    while (b < b1) {
        uint32_t wd = bm[b >> 5] << (b & 31);
        const int n = min(32 - (b & 31), b1 - b);
        for (int q = 0; q < n; ++q) {
            const uint32_t top = ((r >> 23) ^ (wd >> 31)) & 1u;
            r = ((r << 1) & 0xFFFFFFu) ^ (top ? poly : 0u);
            wd <<= 1;
        }
        b += n;
    }
    return r;
}

// r(x) * x^n mod g from the table T[m] = x^m mod g.
__device__ uint32_t crc_shift(uint32_t r, int n, const uint32_t *T)
{
    uint32_t o = 0;
    for (int i = 0; i < 24; ++i)
        if ((r >> i) & 1u) o ^= T[n + i];
    return o;
}

__device__ __forceinline__ short clamp_llr(int v) { return (short)max(-kLlrMax, min(kLlrMax, v)); }

__global__ void __launch_bounds__(kMaxWgThreads) turbo_decode_kernel(DecArgs a)
{
    extern __shared__ __align__(16) char lds[];
    __shared__ uint32_t s_crc[kMaxSlotsPerWg];
    __shared__ int s_done[kMaxSlotsPerWg];
    __shared__ int s_iters[kMaxSlotsPerWg];
    __shared__ int s_ok[kMaxSlotsPerWg];

    const int tid = threadIdx.x, nthr = blockDim.x;
    char *scr = a.scratch + (int64_t)blockIdx.x * a.scratch_stride;

    for (int item_i = blockIdx.x; item_i < a.n_items; item_i += gridDim.x) {
        const DecItem it = a.items[item_i];
        const int K = it.K, nw = it.nw, W = it.W, ncb = it.ncb, S = it.S;
        const int lanes = ncb * nw;
        // global scratch layout of this item
        int4 *R1all = (int4 *)scr;                                   // ncb * K * 4 B
        uint16_t *R2all = (uint16_t *)(scr + (int64_t)ncb * K * 4);  // ncb * K * 2 B
        char *p = scr + (int64_t)ncb * K * 6;
        const int nseg = W / S;
        uint4 *ck_a = (uint4 *)p;
        p += (int64_t)nseg * lanes * 16;
        uint2 *ck_p = (uint2 *)p;
        p += ((int64_t)nseg * lanes * 8 + 15) & ~(int64_t)15;
        uint4 *bnd = (uint4 *)p;  // [dec 2][alpha/beta 2][lanes]

        // ---- restage the channel LLRs, clear the extrinsic arrays
        const int ewords = (epad(K - 1) + 2) / 2;  // int32 words of E
        const int bwords = (int)hard_words(K);
        for (int cs = 0; cs < ncb; ++cs) {
            const DecCb cb = a.cbs[it.cb0 + cs];
            const int16_t *src = a.llr + cb.llr_off;
            const int N = K + 4;
            short *r1h = (short *)(R1all) + (int64_t)cs * K * 2;
            uint16_t *r2 = R2all + (int64_t)cs * K;
            for (int pp = tid; pp < K; pp += nthr) {
                const int ww = pp / W, t = pp - ww * W;
                const int idx = ((t >> 2) * nw + ww) * 4 + (t & 3);
                short ls = clamp_llr(src[pp]), lp1 = clamp_llr(src[N + pp]);
                const short lp2 = clamp_llr(src[2 * N + pp]);
                if (pp < cb.F) ls = lp1 = -kLlrMax;
                r1h[2 * idx] = lp1;
                r1h[2 * idx + 1] = ls;
                r2[idx] = (uint16_t)lp2;
            }
            uint32_t *slot = (uint32_t *)(lds + (int64_t)cs * it.lds_slot);
            for (int q = tid; q < ewords + bwords; q += nthr) slot[q] = 0;
        }
        if (tid < ncb) {
            s_done[tid] = 0;
            s_iters[tid] = a.max_iters;
            s_ok[tid] = 0;
        }

        // ---- lane role
        const bool active = tid < lanes;
        const int cs = active ? tid / nw : 0;
        const int w = active ? tid - cs * nw : 0;
        const DecCb cb = a.cbs[it.cb0 + (active ? cs : 0)];
        LaneCtx lc;
        lc.K = K;
        lc.W = W;
        lc.nw = nw;
        lc.w = w;
        lc.lo = w * W;
        lc.f2x2 = (uint32_t)((2 * it.f2) % K);
        {
            const uint64_t k0 = (uint64_t)w * W;
            lc.pi0 = (uint32_t)(((uint64_t)it.f1 * k0 + (uint64_t)it.f2 * ((k0 * k0) % K)) % K);
            lc.g0 = (uint32_t)(((uint64_t)it.f1 + (uint64_t)it.f2 * (2 * k0 + 1)) % K);
        }
        lc.E = (short *)(lds + (int64_t)cs * it.lds_slot);
        lc.bm = (uint32_t *)(lds + (int64_t)cs * it.lds_slot) + ewords;
        lc.R1 = R1all + (int64_t)cs * K / 4;
        lc.R2 = (const uint2 *)(R2all + (int64_t)cs * K);
        lc.ck_a = ck_a;
        lc.ck_p = ck_p;
        lc.lanes = lanes;
        lc.lane = tid;
        lc.first = w == 0;
        lc.last = w == nw - 1;

        // trellis termination: beta_K of both encoders (Q layout), closed form
        // along the forced zero-feedback path from each state
        s2 tb[2][4];
        if (active && lc.last) {
            const int16_t *src = a.llr + cb.llr_off;
            const int N = K + 4;
            for (int d = 0; d < 2; ++d) {
                const int o = K + 2 * d;
                const int lx0 = clamp_llr(src[o]), lz0 = clamp_llr(src[N + o]),
                          lx1 = clamp_llr(src[2 * N + o]), lz1 = clamp_llr(src[o + 1]),
                          lx2 = clamp_llr(src[N + o + 1]), lz2 = clamp_llr(src[2 * N + o + 1]);
                short v[8];
                for (int s = 0; s < 8; ++s) {
                    const int s1 = (s >> 2) & 1, s2b = (s >> 1) & 1, s3 = s & 1;
                    v[s] = (short)((s2b ^ s3) * lx0 + (s1 ^ s3) * lz0 + (s1 ^ s2b) * lx1 +
                                   s2b * lz1 + s1 * lx2 + s1 * lz2);
                }
                for (int j = 0; j < 4; ++j) tb[d][j] = (s2){v[2 * j], v[2 * j + 1]};
                normalise(tb[d]);
            }
        }
        __syncthreads();

        // ---- turbo iterations
        const uint32_t poly = cb.crc == 1 ? kPoly24A : kPoly24B;
        const uint32_t *T = a.crc_tab + (cb.crc == 1 ? 0 : kCrcTabN);
        for (int iter = 1; iter <= a.max_iters; ++iter) {
            const bool run = active && !s_done[cs];
            const bool prev = a.win_init && iter > 1;
            if (run) {
                // clear this block's bitmap and CRC accumulator for decoder 2
                for (int q = w; q < bwords; q += nw) lc.bm[q] = 0;
                if (w == 0) s_crc[cs] = 0;
                s2 Ai[4], Bi[4];
                const s2 z = (s2){0, 0};
                if (lc.first) {
                    Ai[0] = (s2){0, kNeg};
                    Ai[1] = Ai[2] = Ai[3] = (s2){kNeg, kNeg};
                } else if (prev) {
                    unpack4(bnd[0 * lanes + tid], Ai);
                } else {
                    Ai[0] = Ai[1] = Ai[2] = Ai[3] = z;
                }
                if (lc.last) {
                    for (int j = 0; j < 4; ++j) Bi[j] = tb[0][j];
                } else if (prev) {
                    unpack4(bnd[1 * lanes + tid], Bi);
                } else {
                    Bi[0] = Bi[1] = Bi[2] = Bi[3] = z;
                }
                run_pass<1, 8>(lc, Ai, Bi, &bnd[0 * lanes + tid + 1], &bnd[1 * lanes + tid - 1]);
            }
            __syncthreads();
            if (run) {
                s2 Ai[4], Bi[4];
                const s2 z = (s2){0, 0};
                if (lc.first) {
                    Ai[0] = (s2){0, kNeg};
                    Ai[1] = Ai[2] = Ai[3] = (s2){kNeg, kNeg};
                } else if (prev) {
                    unpack4(bnd[2 * lanes + tid], Ai);
                } else {
                    Ai[0] = Ai[1] = Ai[2] = Ai[3] = z;
                }
                if (lc.last) {
                    for (int j = 0; j < 4; ++j) Bi[j] = tb[1][j];
                } else if (prev) {
                    unpack4(bnd[3 * lanes + tid], Bi);
                } else {
                    Bi[0] = Bi[1] = Bi[2] = Bi[3] = z;
                }
                run_pass<2, 8>(lc, Ai, Bi, &bnd[2 * lanes + tid + 1], &bnd[3 * lanes + tid - 1]);
            }
            __syncthreads();
            const bool check = run && cb.crc != 0 && (a.early_stop || iter == a.max_iters);
            if (check) {
                const int b0 = max((int)cb.F, lc.lo), b1 = lc.lo + W;
                uint32_t r = b0 < b1 ? crc_range(lc.bm, b0, b1, poly) : 0u;
                r = crc_shift(r, K - b1, T);
                if (r) atomicXor(&s_crc[cs], r);
            }
            __syncthreads();
            if (run && w == 0) {
                const bool pass = cb.crc == 0 || s_crc[cs] == 0;
                if (a.early_stop && cb.crc != 0 && pass) {
                    s_done[cs] = 1;
                    s_iters[cs] = iter;
                    s_ok[cs] = 1;
                } else if (iter == a.max_iters) {
                    s_iters[cs] = iter;
                    s_ok[cs] = pass;
                }
            }
            __syncthreads();
            if (!__syncthreads_or(active && !s_done[cs])) break;
        }

        // ---- outputs
        if (active) {
            const int L = cb.crc ? 24 : 0;
            if (cb.bits_off >= 0 && a.bits) {
                const int nbits = K - cb.F - L;
                const int nbytes = (nbits + 7) >> 3;
                uint8_t *out = a.bits + cb.bits_off;
                for (int bb = w; bb < nbytes; bb += nw) {
                    const int pos = cb.F + 8 * bb;
                    const uint64_t two = ((uint64_t)lc.bm[pos >> 5] << 32) | lc.bm[(pos >> 5) + 1];
                    uint32_t byte = (uint32_t)(two >> (56 - (pos & 31))) & 0xFFu;
                    const int valid = min(8, nbits - 8 * bb);
                    byte &= (0xFFu << (8 - valid)) & 0xFFu;
                    out[bb] = (uint8_t)byte;
                }
            }
            if (cb.hard_off >= 0 && a.hard) {
                uint32_t *h = a.hard + cb.hard_off;
                for (int q = w; q < bwords; q += nw) h[q] = lc.bm[q];
            }
            if (w == 0) {
                a.crc_ok[cb.out_idx] = (uint8_t)s_ok[cs];
                a.iters[cb.out_idx] = (uint8_t)s_iters[cs];
            }
        }
        __syncthreads();
    }
}

const void *decode_kernel_address() { return (const void *)turbo_decode_kernel; }

int launch_decode(const DecArgs &a, int grid, int wg_threads, int lds_bytes, void *stream)
{
    hipLaunchKernelGGL(turbo_decode_kernel, dim3(grid), dim3(wg_threads), lds_bytes,
                       (hipStream_t)stream, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ------------------------------------------------------------------------
// Transport block assembly: payload bits of the blocks (filler and CRC24B
// dropped) back to back, CRC24A over them, per-block flags into the result.

struct TbRes {
    int32_t tb_ok, max_iters_used, C, rsv;
    uint8_t cb_ok[64], cb_iters[64];
};

__device__ uint32_t gf_mulmod(uint32_t a, uint32_t b, uint32_t poly)
{
    uint32_t r = 0;
    for (int i = 23; i >= 0; --i) {
        const uint32_t top = (r >> 23) & 1u;
        r = ((r << 1) & 0xFFFFFFu) ^ (top ? poly : 0u);
        if ((b >> i) & 1u) r ^= a;
    }
    return r;
}

__device__ uint32_t gf_xpow(uint64_t n, uint32_t poly)
{
    uint32_t res = 1, base = 2;
    while (n) {
        if (n & 1) res = gf_mulmod(res, base, poly);
        base = gf_mulmod(base, base, poly);
        n >>= 1;
    }
    return res;
}

__global__ void __launch_bounds__(256) tb_assemble_kernel(const TbItem *items, const uint32_t *hard,
                                                          const uint8_t *crc_ok,
                                                          const uint8_t *iters, uint8_t *bits,
                                                          TbRes *res)
{
    __shared__ int64_t s_hoff[64];  // hard word offset of each block
    __shared__ int32_t s_start[65]; // first TB bit of each block's payload
    __shared__ int32_t s_F[64];
    __shared__ uint32_t s_crc;
    const TbItem tb = items[blockIdx.x];
    const int tid = threadIdx.x, nthr = blockDim.x;
    if (tid == 0) {
        int64_t h = tb.hard_off;
        int32_t st = 0;
        for (int r = 0; r < tb.C; ++r) {
            const int32_t K = r < tb.Cminus ? tb.Kminus : tb.Kplus;
            const int32_t F = r == 0 ? tb.F : 0;
            s_hoff[r] = h;
            s_start[r] = st;
            s_F[r] = F;
            h += hard_words(K);
            st += K - F - tb.L;
        }
        s_start[tb.C] = st;
        s_crc = 0;
    }
    __syncthreads();
    auto bit_at = [&](int b) -> uint32_t {
        int r = 0;
        while (r + 1 < tb.C && s_start[r + 1] <= b) ++r;
        const int pos = s_F[r] + (b - s_start[r]);
        return (hard[s_hoff[r] + (pos >> 5)] >> (31 - (pos & 31))) & 1u;
    };
    // payload bytes
    if (tb.bits_off >= 0 && bits) {
        const int nbytes = (tb.tbs + 7) >> 3;
        for (int q = tid; q < nbytes; q += nthr) {
            uint32_t v = 0;
            for (int k = 0; k < 8; ++k) {
                const int b = 8 * q + k;
                v = (v << 1) | (b < tb.tbs ? bit_at(b) : 0u);
            }
            bits[tb.bits_off + q] = (uint8_t)v;
        }
    }
    // CRC24A over the B reassembled bits: per-thread chunks, shifted into place
    const int chunk = (tb.B + nthr - 1) / nthr;
    const int b0 = tid * chunk, b1 = min(tb.B, b0 + chunk);
    if (b0 < b1) {
        uint32_t r = 0;
        for (int b = b0; b < b1; ++b) {
            const uint32_t top = ((r >> 23) ^ bit_at(b)) & 1u;
            r = ((r << 1) & 0xFFFFFFu) ^ (top ? kPoly24A : 0u);
        }
        if (r) r = gf_mulmod(r, gf_xpow((uint64_t)(tb.B - b1), kPoly24A), kPoly24A);
        if (r) atomicXor(&s_crc, r);
    }
    __syncthreads();
    if (tid == 0) {
        TbRes &o = res[tb.res_idx];
        int mx = 0;
        for (int r = 0; r < 64; ++r) {
            o.cb_ok[r] = r < tb.C ? crc_ok[tb.cb_idx0 + r] : 0;
            o.cb_iters[r] = r < tb.C ? iters[tb.cb_idx0 + r] : 0;
            if (r < tb.C) mx = max(mx, (int)iters[tb.cb_idx0 + r]);
        }
        o.tb_ok = s_crc == 0;
        o.max_iters_used = mx;
        o.C = tb.C;
        o.rsv = 0;
    }
}

int launch_tb_assemble(const TbItem *items, int n_tb, const uint32_t *hard, const uint8_t *crc_ok,
                       const uint8_t *iters, const uint32_t *crc_tab, uint8_t *bits, void *res,
                       void *stream)
{
    (void)crc_tab;
    if (n_tb <= 0) return 0;
    hipLaunchKernelGGL(tb_assemble_kernel, dim3(n_tb), dim3(256), 0, (hipStream_t)stream, items,
                       hard, crc_ok, iters, bits, (TbRes *)res);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace tdec
