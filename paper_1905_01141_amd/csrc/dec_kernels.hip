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
//   * all 8 state metrics of a trellis window live in one lane as packed
//     int16 pairs: an add-compare-select step is 8 saturating v_pk_add_i16 +
//     4 v_pk_max_i16 with the broadcasts and swaps folded into op_sel, and no
//     cross-lane traffic;
//   * every window has two lanes in two different waves ("X" schedule): the
//     forward-first lane runs the forward recursion over the first half of
//     the window while the backward-first lane runs the backward recursion
//     over the second half, both leaving checkpoints every 8 steps; then each
//     lane takes the other half, recomputes the other recursion segment by
//     segment from those checkpoints into registers and runs its own
//     recursion over it, emitting the extrinsic.  Each wave runs one code
//     path; the dependent chain per window is half its length;
//   * the extrinsic / a-priori array of a block lives in LDS for the whole
//     decode; decoder 1 reads it 8 steps per ds_read_b128, decoder 2 through
//     LDS addresses of the QPP permutation precomputed once per block;
//   * the channel LLRs are restaged once per block into a window-interleaved
//     layout in global scratch (one 16-byte load = 4 trellis steps of one
//     lane, the lanes of a wave reading consecutive 16-byte pieces), through
//     an LDS tile so that the planar input is read contiguously too;
//   * hard decisions ride in the low bit of decoder 2's output in the LDS
//     array; the CRC is a per-window LFSR combined across windows with
//     x^n mod g tables;
//   * a persistent grid takes work items dynamically, the claims spread over
//     one counter per set of work groups.
//
// Metric layouts: "P" = {(m0,m4),(m1,m5),(m2,m6),(m3,m7)},
// "Q" = {(m0,m1),(m2,m3),(m4,m5),(m6,m7)} with state s = 4 a_{k-1} +
// 2 a_{k-2} + a_{k-3}; forward metrics run in P, backward metrics in Q.
// Branch metric pairs of a step: g00 = (0, Lsa+Lp), g01 = (Lp, Lsa); their
// swaps g11 and g10 complete the four values u*Lsa + z*Lp.
//
// Fixed point: metrics are shifted so that their maximum is 0 after steps
// 1 and 2 of a recursion and after every even step, and left alone after odd
// steps from the third on; candidate sums saturate.  With the input clamps
// (|Lsa| <= 4094, |Lp| <= 2047) no value that decides a maximum ever leaves
// int16, so every result equals the exact (unbounded) max-log-MAP.
#include <hip/hip_runtime.h>

#include <mutex>

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
constexpr int S = kSeg;

// g00 = (0, Lp + Lsa) from g01 = (Lp, Lsa).  Built with v_perm so that the
// compiler keeps the pair opaque and folds the swapped uses into op_sel.
__device__ __forceinline__ s2 mk_g00(s2 g01)
{
    const s2 x = g01 + swp(g01);  // |Lp + Lsa| <= 6141: no wrap
    return as_s2(__builtin_amdgcn_perm(0u, as_u(x), 0x03020c0cu));
}

// The four branch metric pairs are g00, g01 and their swaps; a broadcast
// plus a swapped pair is the swap of the broadcast plus the pair, which puts
// every swap on an operand of a max or add where it folds into op_sel.

// Forward add-compare-select, P layout in and out.
__device__ __forceinline__ void acs_fwd(s2 A[4], s2 g00, s2 g01)
{
    const s2 n0 = vmax(adds(bcx(A[0]), g00), swp(adds(bcx(A[1]), g00)));
    const s2 n1 = vmax(swp(adds(bcx(A[2]), g01)), adds(bcx(A[3]), g01));
    const s2 n2 = vmax(adds(bcy(A[0]), g01), swp(adds(bcy(A[1]), g01)));
    const s2 n3 = vmax(swp(adds(bcy(A[2]), g00)), adds(bcy(A[3]), g00));
    A[0] = n0;
    A[1] = n1;
    A[2] = n2;
    A[3] = n3;
}

// Forward step that also returns the extrinsic maxima of the step: the
// candidate sums alpha_k(p) + gamma(p -> n) of the recursion, plus
// beta_{k+1}(n) (P layout), maximised per input bit u: (M0, M1).  The
// extrinsic is Le = M1 - M0 - Lsa modulo 2^16 (the true value fits int16).
__device__ __forceinline__ s2 acs_fwd_le(s2 A[4], s2 g00, s2 g01, const s2 BP[4])
{
    const s2 t0 = adds(bcx(A[0]), g00), t1 = swp(adds(bcx(A[1]), g00));
    const s2 t2 = swp(adds(bcx(A[2]), g01)), t3 = adds(bcx(A[3]), g01);
    const s2 t4 = adds(bcy(A[0]), g01), t5 = swp(adds(bcy(A[1]), g01));
    const s2 t6 = swp(adds(bcy(A[2]), g00)), t7 = adds(bcy(A[3]), g00);
    // halves (u=0, u=1) for p = 0, 3, 4, 7 and (u=1, u=0) for p = 1, 2, 5, 6
    const s2 n = vmax(vmax(adds(t0, BP[0]), adds(t3, BP[1])), vmax(adds(t4, BP[2]), adds(t7, BP[3])));
    const s2 s = vmax(vmax(adds(t1, BP[0]), adds(t2, BP[1])), vmax(adds(t5, BP[2]), adds(t6, BP[3])));
    const s2 m = vmax(n, swp(s));
    A[0] = vmax(t0, t1);
    A[1] = vmax(t2, t3);
    A[2] = vmax(t4, t5);
    A[3] = vmax(t6, t7);
    return m;
}

// Backward step, Q layout in and out.
__device__ __forceinline__ void acs_bwd(s2 B[4], s2 g00, s2 g01)
{
    const s2 c00 = adds(bcx(B[0]), g00), c01 = swp(adds(bcx(B[2]), g00));
    const s2 c10 = swp(adds(bcy(B[0]), g01)), c11 = adds(bcy(B[2]), g01);
    const s2 c20 = adds(bcx(B[1]), g01), c21 = swp(adds(bcx(B[3]), g01));
    const s2 c30 = swp(adds(bcy(B[1]), g00)), c31 = adds(bcy(B[3]), g00);
    B[0] = vmax(c00, c01);
    B[1] = vmax(c10, c11);
    B[2] = vmax(c20, c21);
    B[3] = vmax(c30, c31);
}

// Backward step that also returns the extrinsic maxima from alpha_k (Q
// layout): the candidate sums beta_{k+1}(n) + gamma(p -> n) plus alpha_k(p).
__device__ __forceinline__ s2 acs_bwd_le(s2 B[4], const s2 AQ[4], s2 g00, s2 g01)
{
    const s2 c00 = adds(bcx(B[0]), g00), c01 = swp(adds(bcx(B[2]), g00));
    const s2 c10 = swp(adds(bcy(B[0]), g01)), c11 = adds(bcy(B[2]), g01);
    const s2 c20 = adds(bcx(B[1]), g01), c21 = swp(adds(bcx(B[3]), g01));
    const s2 c30 = swp(adds(bcy(B[1]), g00)), c31 = adds(bcy(B[3]), g00);
    const s2 n = vmax(vmax(adds(AQ[0], c00), adds(AQ[1], c11)),
                      vmax(adds(AQ[2], c20), adds(AQ[3], c31)));
    const s2 s = vmax(vmax(adds(AQ[0], c01), adds(AQ[1], c10)),
                      vmax(adds(AQ[2], c21), adds(AQ[3], c30)));
    const s2 m = vmax(n, swp(s));
    B[0] = vmax(c00, c01);
    B[1] = vmax(c10, c11);
    B[2] = vmax(c20, c21);
    B[3] = vmax(c30, c31);
    return m;
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

__device__ __forceinline__ void p_to_q(const s2 A[4], s2 Q[4])
{
    Q[0] = (s2){A[0].x, A[1].x};
    Q[1] = (s2){A[2].x, A[3].x};
    Q[2] = (s2){A[0].y, A[1].y};
    Q[3] = (s2){A[2].y, A[3].y};
}

__device__ __forceinline__ void q_to_p(const s2 Q[4], s2 P[4])
{
    P[0] = (s2){Q[0].x, Q[2].x};
    P[1] = (s2){Q[0].y, Q[2].y};
    P[2] = (s2){Q[1].x, Q[3].x};
    P[3] = (s2){Q[1].y, Q[3].y};
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

// Forward step i = i0 + t + 1 (counted from the window start) is normalised
// for i <= 2 and for even i -- or, SPARSE, only for i a multiple of 4; in
// window 0 the states that cannot be reached after 1 and 2 steps are pinned
// back to minus infinity.  The recursion that runs beside the extrinsic is
// dense; phase 1 and the recomputation from checkpoints are sparse: an
// extrinsic sum then holds one metric at most 1 step and the other at most
// 3 steps past its last shift (or its normalised start), at most 6141 +
// 3 * 6141 + 6141 = 30705 and, for a winning sum, at least -32752
// (checkpoints and window ends, multiples of 8 steps from the window edges,
// are shifted in both forms).
template <bool SPARSE = false>
__device__ __forceinline__ void fwd_post(s2 A[4], int i0, int t, bool first)
{
    if (SPARSE ? (t & 3) == 3 : ((t & 1) != 0 || (i0 == 0 && t == 0))) normalise(A);
    if (i0 == 0 && t < 2 && first) {
        const s2 neg = (s2){kNeg, kNeg};
        A[1] = neg;
        A[3] = neg;
        if (t == 0) A[2] = neg;
    }
}

// Backward metric at local position i = i0 + t is normalised when W - i <= 2
// or W - i is even -- or, SPARSE, a multiple of 4 (W and i0 are multiples
// of 8; the forms are used as in fwd_post).
template <bool SPARSE = false>
__device__ __forceinline__ bool bwd_norm(int i0, int t, int W)
{
    return SPARSE ? (t & 3) == 0 : ((t & 1) == 0 || (i0 == W - S && t >= S - 2));
}

// Everything a lane needs for one constituent pass over its window.
struct Win {
    int W, M, lo, wi, lanes;
    int qs;              // units per row of the QPP address table (the item's window count)
    bool first, last;
    short *E;            // LDS extrinsic array of the block (padded)
    const uint4 *R;      // restaged input of the decoder: decoder 1 [t/4][lane] x 4
                         // steps of Lp1 | Ls << 16; decoder 2 [t/4][lane] x 4 int16 Lp2
    const uint2 *qt;     // QPP address table of the shape at this lane's window:
                         // unit t/4 at qt[(t/4) * qs], 4 LDS byte offsets in E
    uint4 *ck;           // checkpoints [segment][window]
    const unsigned short *mit;  // LDS entropy table (mutual-information stop only)
};

// The inputs of 8 steps starting at local step i0:
//   decoder 1: r[t] = Lp1 | Ls << 16 of step t;
//   decoder 2: r[0..3] = Lp2 of steps (0,1), (2,3), (4,5), (6,7) and r[4..7]
//              the LDS byte offsets of E[pi(k)] of the same step pairs.
template <int DEC>
__device__ __forceinline__ void load_seg(const Win &c, int i0, uint32_t r[S])
{
    if (DEC == 1) {
        const uint4 q0 = c.R[(size_t)(i0 >> 2) * c.lanes + c.wi];
        const uint4 q1 = c.R[(size_t)((i0 >> 2) + 1) * c.lanes + c.wi];
        r[0] = q0.x; r[1] = q0.y; r[2] = q0.z; r[3] = q0.w;
        r[4] = q1.x; r[5] = q1.y; r[6] = q1.z; r[7] = q1.w;
    } else {
        const uint2 *R2 = (const uint2 *)c.R;
        const uint2 p0 = R2[(size_t)(i0 >> 2) * c.lanes + c.wi];
        const uint2 p1 = R2[(size_t)((i0 >> 2) + 1) * c.lanes + c.wi];
        const uint2 a0 = c.qt[(i0 >> 2) * c.qs];
        const uint2 a1 = c.qt[((i0 >> 2) + 1) * c.qs];
        r[0] = p0.x; r[1] = p0.y; r[2] = p1.x; r[3] = p1.y;
        r[4] = a0.x; r[5] = a0.y; r[6] = a1.x; r[7] = a1.y;
    }
}

// LDS byte offset of step t's E[pi(k)] in a decoder-2 segment r.
__device__ __forceinline__ uint32_t qaddr(const uint32_t r[S], int t)
{
    const uint32_t w = r[4 + (t >> 1)];
    return (t & 1) ? (w >> 16) : (w & 0xFFFFu);
}

// Branch metric pairs g01 = (Lp, Lsa) of 8 steps.
//   decoder 1: r = Lp1 | Ls << 16 and Lsa = Ls + E[j] (natural order, one
//              ds_read_b128 for the 8 steps);
//   decoder 2: Lp2 from r[t/2] and Lsa = E[pi(k)] (decoder 1 stored Ls + La
//              there) at the step's LDS offset.
template <int DEC>
__device__ __forceinline__ void gammas(const Win &c, int i0, const uint32_t r[S], s2 g01[S])
{
    if (DEC == 1) {
        const uint4 e = *(const uint4 *)(c.E + epad(c.lo + i0));
        const uint32_t ew[4] = {e.x, e.y, e.z, e.w};
#pragma unroll
        for (int t = 0; t < S; ++t) {
            // E holds 2 La + hard bit (decoder 2's output); high half of the
            // sum: Ls + La (no carry between halves); low half: Lp
            const s2 la2 = as_s2(ew[t >> 1]) >> (s2){1, 1};
            const s2 ee = (t & 1) ? la2 : swp(la2);
            const s2 sum = as_s2(r[t]) + ee;
            g01[t] = as_s2(__builtin_amdgcn_perm(as_u(sum), r[t], 0x07060100u));
        }
    } else {
#pragma unroll
        for (int t = 0; t < S; ++t) {
            const uint32_t e = *(const uint16_t *)((const char *)c.E + qaddr(r, t));
            g01[t] = as_s2(__builtin_amdgcn_perm(e, r[t >> 1], (t & 1) ? 0x05040302u : 0x05040100u));
        }
    }
}

typedef unsigned short u2 __attribute__((ext_vector_type(2)));

// Output of two steps ta, ta + 1 (ta even) from their extrinsic maxima pairs
// (M0, M1) ma, mb, the segment's inputs r and branch metric pairs ga, gb, both
// steps packed in one register pair by pair:
//   Le = M1 - M0 - Lsa, modulo 2^16 (the true values fit int16);
//   q = 0.75 Le truncated toward zero and clamped to +-2047, formed as
//       (3 (x + [x < 0])) >> 2 with x = Le clamped to +-2730 (for x < 0 the
//       bias 3 turns the floor of 3x / 4 into its ceiling);
//   decoder 1 stores Ls + q (decoder 2's systematic + a-priori) at the two
//   natural positions, one 32-bit LDS store;
//   decoder 2 stores 2 q + the hard decision of pi(k), [L > 0] for the
//   a-posteriori L = Lsa + Le, at each step's LDS address.  The hard
//   decisions stay readable from the low bits until the next decoder-1
//   pass, i.e. through the CRC check and the output.  With MI, decoder 2
//   also adds the entropy of its hard decisions, h(|L|) from the LDS table,
//   to the lane's sum.
template <int DEC, bool MI = false>
__device__ __forceinline__ void emit2(const Win &c, int i0, int ta, const uint32_t r[S],
                                      s2 ga, s2 gb, s2 ma, s2 mb, int &acc)
{
    const s2 m1 = as_s2(__builtin_amdgcn_perm(as_u(mb), as_u(ma), 0x07060302u));   // (ma.y, mb.y)
    const s2 m0 = as_s2(__builtin_amdgcn_perm(as_u(mb), as_u(ma), 0x05040100u));   // (ma.x, mb.x)
    const s2 lsa = as_s2(__builtin_amdgcn_perm(as_u(gb), as_u(ga), 0x07060302u));  // (ga.y, gb.y)
    const s2 le = m1 - m0 - lsa;
    const s2 x = vmax(__builtin_elementwise_min(le, (s2){2730, 2730}), (s2){-2730, -2730});
    const s2 neg = __builtin_bit_cast(s2, __builtin_bit_cast(u2, x) >> (u2){15, 15});
    const s2 q = ((x + neg) * (s2){3, 3}) >> (s2){2, 2};
    if (DEC == 1) {
        const s2 ls = as_s2(__builtin_amdgcn_perm(r[ta + 1], r[ta], 0x07060302u));  // (Ls_a, Ls_b)
        *(s2 *)(c.E + epad(c.lo + i0) + ta) = ls + q;
    } else {
        const s2 lapp = lsa + le;
        const s2 bit = __builtin_bit_cast(s2, __builtin_bit_cast(u2, (s2){0, 0} - lapp) >> (u2){15, 15});
        const s2 o = q * (s2){2, 2} + bit;
        *(short *)((char *)c.E + qaddr(r, ta)) = o.x;
        *(short *)((char *)c.E + qaddr(r, ta + 1)) = o.y;
        if (MI)
            acc += c.mit[min(abs((int)lapp.x), kMiTabN - 1)] + c.mit[min(abs((int)lapp.y), kMiTabN - 1)];
    }
}

// Every phase loop prefetches the next segment's restaged inputs (and, in
// phase 2, its checkpoint) one segment ahead; the last segment reloads itself.

// ---- phase 1, forward-first lane: alpha over [0, M) with checkpoints.
template <int DEC>
__device__ void ph1_fwd(const Win &c, s2 A[4])
{
    if (c.M <= 0) return;
    uint32_t r[S];
    load_seg<DEC>(c, 0, r);
    for (int i0 = 0; i0 < c.M; i0 += S) {
        uint32_t rn[S];
        load_seg<DEC>(c, min(i0 + S, c.M - S), rn);
        c.ck[(size_t)(i0 / S) * c.lanes + c.wi] = pack4(A);
        s2 g[S];
        gammas<DEC>(c, i0, r, g);
#pragma unroll
        for (int t = 0; t < S; ++t) {
            acs_fwd(A, mk_g00(g[t]), g[t]);
            fwd_post<true>(A, i0, t, c.first);
        }
#pragma unroll
        for (int t = 0; t < S; ++t) r[t] = rn[t];
    }
}

// ---- phase 1, backward-first lane: beta over [M, W) with checkpoints
// (beta at the end of every segment).
template <int DEC>
__device__ void ph1_bwd(const Win &c, s2 B[4])
{
    uint32_t r[S];
    load_seg<DEC>(c, c.W - S, r);
    for (int i0 = c.W - S; i0 >= c.M; i0 -= S) {
        uint32_t rn[S];
        load_seg<DEC>(c, max(i0 - S, c.M), rn);
        c.ck[(size_t)(i0 / S) * c.lanes + c.wi] = pack4(B);
        s2 g[S];
        gammas<DEC>(c, i0, r, g);
#pragma unroll
        for (int t = S - 1; t >= 0; --t) {
            acs_bwd(B, mk_g00(g[t]), g[t]);
            if (bwd_norm<true>(i0, t, c.W)) normalise(B);
        }
#pragma unroll
        for (int t = 0; t < S; ++t) r[t] = rn[t];
    }
}

// Phase 2 is software-pipelined: the recomputation of the next segment (it
// depends only on that segment's checkpoint) is interleaved step by step with
// the extrinsic pass over the current segment, which doubles the independent
// work available to each wave.  Inputs are fetched two segments ahead.

__device__ __forceinline__ uint4 ck_at(const Win &c, int i0)
{
    return c.ck[(size_t)(i0 / S) * c.lanes + c.wi];
}

// ---- phase 2, forward-first lane: the upper half [M, W) in forward order.
// Per segment: beta recomputed backward from the checkpoint at its end, then
// alpha forward over it with the extrinsic.
// Returns the lane's entropy sum when MI (else 0).
template <int DEC, bool MI = false>
__device__ int ph2_fwd(const Win &c, s2 A[4])
{
    int acc = 0;
    if (c.M >= c.W) return acc;
    const int last = c.W - S;
    int i0 = c.M;
    uint32_t r[S], rn[S], rnn[S];
    s2 g[S], g0[S], BP[S][4], m[S];
    load_seg<DEC>(c, i0, r);
    uint4 ckn = ck_at(c, min(i0 + S, last));
    load_seg<DEC>(c, min(i0 + S, last), rn);
    {
        s2 B[4];
        unpack4(ck_at(c, i0), B);
        gammas<DEC>(c, i0, r, g);
#pragma unroll
        for (int t = S - 1; t >= 0; --t) {
            q_to_p(B, BP[t]);
            g0[t] = mk_g00(g[t]);
            acs_bwd(B, g0[t], g[t]);
            if (bwd_norm<true>(i0, t, c.W)) normalise(B);
        }
    }
    // two segments per trip: the hand-over of the next segment's values
    // (inputs, gammas, recomputed metrics) becomes register renaming
#pragma unroll 2
    for (; i0 < last; i0 += S) {
        const int i1 = i0 + S;
        load_seg<DEC>(c, min(i1 + S, last), rnn);
        const uint4 cknn = ck_at(c, min(i1 + S, last));
        s2 Bn[4], gn[S], g0n[S], BPn[S][4];
        unpack4(ckn, Bn);
        gammas<DEC>(c, i1, rn, gn);
#pragma unroll
        for (int t = 0; t < S; ++t) {
            const int u = S - 1 - t;  // recompute step of the next segment
            q_to_p(Bn, BPn[u]);
            g0n[u] = mk_g00(gn[u]);
            acs_bwd(Bn, g0n[u], gn[u]);
            if (bwd_norm<true>(i1, u, c.W)) normalise(Bn);
            m[t] = acs_fwd_le(A, g0[t], g[t], BP[t]);
            fwd_post(A, i0, t, c.first);
            if (t & 1) emit2<DEC, MI>(c, i0, t - 1, r, g[t - 1], g[t], m[t - 1], m[t], acc);
        }
#pragma unroll
        for (int t = 0; t < S; ++t) {
            r[t] = rn[t];
            rn[t] = rnn[t];
            g[t] = gn[t];
            g0[t] = g0n[t];
            BP[t][0] = BPn[t][0];
            BP[t][1] = BPn[t][1];
            BP[t][2] = BPn[t][2];
            BP[t][3] = BPn[t][3];
        }
        ckn = cknn;
    }
#pragma unroll
    for (int t = 0; t < S; ++t) {
        m[t] = acs_fwd_le(A, g0[t], g[t], BP[t]);
        fwd_post(A, i0, t, c.first);
        if (t & 1) emit2<DEC, MI>(c, i0, t - 1, r, g[t - 1], g[t], m[t - 1], m[t], acc);
    }
    return acc;
}

// ---- phase 2, backward-first lane: the lower half [0, M) in backward order.
// Per segment: alpha recomputed forward from the checkpoint at its start,
// then beta backward over it with the extrinsic.
// Returns the lane's entropy sum when MI (else 0).
template <int DEC, bool MI = false>
__device__ int ph2_bwd(const Win &c, s2 B[4])
{
    int acc = 0;
    if (c.M <= 0) return acc;
    int i0 = c.M - S;
    uint32_t r[S], rn[S], rnn[S];
    s2 g[S], g0[S], AQ[S][4], m[S];
    load_seg<DEC>(c, i0, r);
    uint4 ckn = ck_at(c, max(i0 - S, 0));
    load_seg<DEC>(c, max(i0 - S, 0), rn);
    {
        s2 A[4];
        unpack4(ck_at(c, i0), A);
        gammas<DEC>(c, i0, r, g);
#pragma unroll
        for (int t = 0; t < S; ++t) {
            p_to_q(A, AQ[t]);
            g0[t] = mk_g00(g[t]);
            acs_fwd(A, g0[t], g[t]);
            fwd_post<true>(A, i0, t, c.first);
        }
    }
    // two segments per trip: the hand-over of the next segment's values
    // (inputs, gammas, recomputed metrics) becomes register renaming
#pragma unroll 2
    for (; i0 > 0; i0 -= S) {
        const int i1 = i0 - S;
        load_seg<DEC>(c, max(i1 - S, 0), rnn);
        const uint4 cknn = ck_at(c, max(i1 - S, 0));
        s2 An[4], gn[S], g0n[S], AQn[S][4];
        unpack4(ckn, An);
        gammas<DEC>(c, i1, rn, gn);
#pragma unroll
        for (int t = 0; t < S; ++t) {
            p_to_q(An, AQn[t]);  // recompute step of the next segment
            g0n[t] = mk_g00(gn[t]);
            acs_fwd(An, g0n[t], gn[t]);
            fwd_post<true>(An, i1, t, c.first);
            const int u = S - 1 - t;
            m[u] = acs_bwd_le(B, AQ[u], g0[u], g[u]);
            if (bwd_norm(i0, u, c.W)) normalise(B);
            if (!(u & 1)) emit2<DEC, MI>(c, i0, u, r, g[u], g[u + 1], m[u], m[u + 1], acc);
        }
#pragma unroll
        for (int t = 0; t < S; ++t) {
            r[t] = rn[t];
            rn[t] = rnn[t];
            g[t] = gn[t];
            g0[t] = g0n[t];
            AQ[t][0] = AQn[t][0];
            AQ[t][1] = AQn[t][1];
            AQ[t][2] = AQn[t][2];
            AQ[t][3] = AQn[t][3];
        }
        ckn = cknn;
    }
#pragma unroll
    for (int u = S - 1; u >= 0; --u) {
        m[u] = acs_bwd_le(B, AQ[u], g0[u], g[u]);
        if (bwd_norm(i0, u, c.W)) normalise(B);
        if (!(u & 1)) emit2<DEC, MI>(c, i0, u, r, g[u], g[u + 1], m[u], m[u + 1], acc);
    }
    return acc;
}

// ---- exact window boundaries (win_init = 2)
//
// Full-length max-log-MAP computed window by window: before each half-
// iteration every window computes the max-plus transfer matrices of its steps
// (one forward run from each state at its start, one backward run from each
// state at its end), and a scan along the windows turns them into the exact
// forward metric at every window start and backward metric at every window
// end -- the values the full-length recursion has there, in its normalised
// form (maximum 0: window boundaries are multiples of 8 steps from both block
// ends, where the full-length recursion has just been normalised).  The
// windows then run from those boundaries, so every extrinsic equals the
// full-length decoder's (metrics that differ by a constant per step give the
// same extrinsic).

// Normalise as normalise() and return the amount subtracted.
__device__ __forceinline__ int normalise_acc(s2 V[4])
{
    s2 m = vmax(vmax(V[0], V[1]), vmax(V[2], V[3]));
    m = vmax(m, swp(m));
    V[0] = subs(V[0], m);
    V[1] = subs(V[1], m);
    V[2] = subs(V[2], m);
    V[3] = subs(V[3], m);
    return (int)m.x;
}

// Keep register `keep` (and `keep2`) of a metric vector, set the others to
// minus infinity: the states a run cannot have reached yet.
__device__ __forceinline__ void pin_regs(s2 V[4], int keep, int keep2)
{
    const s2 neg = (s2){kNeg, kNeg};
#pragma unroll
    for (int r = 0; r < 4; ++r)
        if (r != keep && r != keep2) V[r] = neg;
}

// Forward transfer runs over the whole window: for each start state i, the
// forward recursion from i (P layout: state i in register i & 3, half i >> 2)
// with the usual normalisation; out[2i] = the metrics at the window end,
// out[2i+1].x = the total subtracted by normalisation (int32), so that the
// best path metric from i to j is metric_j + total.  The states reachable from
// i after 1 step sit in register i >> 1, after 2 steps in i >> 2 and
// (i >> 2) | 2; the others are pinned to minus infinity until then.
template <int DEC>
__device__ void tf_fwd(const Win &c, uint4 *out)
{
    for (int i = 0; i < 8; ++i) {
        s2 A[4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
            A[r] = (s2){(short)((r == (i & 3) && i < 4) ? 0 : kNeg),
                        (short)((r == (i & 3) && i >= 4) ? 0 : kNeg)};
        int acc = 0;
        uint32_t r0[S];
        load_seg<DEC>(c, 0, r0);
        for (int i0 = 0; i0 < c.W; i0 += S) {
            uint32_t rn[S];
            load_seg<DEC>(c, min(i0 + S, c.W - S), rn);
            s2 g[S];
            gammas<DEC>(c, i0, r0, g);
#pragma unroll
            for (int t = 0; t < S; ++t) {
                acs_fwd(A, mk_g00(g[t]), g[t]);
                if ((t & 1) || (i0 == 0 && t == 0)) acc += normalise_acc(A);
                if (i0 == 0 && t == 0) pin_regs(A, i >> 1, i >> 1);
                if (i0 == 0 && t == 1) pin_regs(A, i >> 2, (i >> 2) | 2);
            }
#pragma unroll
            for (int t = 0; t < S; ++t) r0[t] = rn[t];
        }
        out[2 * i] = pack4(A);
        out[2 * i + 1] = make_uint4((uint32_t)acc, 0u, 0u, 0u);
    }
}

// Backward transfer runs: for each end state j, the backward recursion from j
// (Q layout: state j in register j >> 1, half j & 1) to the window start;
// out[2j] = the metrics at the window start, out[2j+1].x = the total
// subtracted.  The states that reach j in 1 step sit in register j & 3, in 2
// steps in registers 2 (j & 1) and 2 (j & 1) + 1.
template <int DEC>
__device__ void tf_bwd(const Win &c, uint4 *out)
{
    for (int j = 0; j < 8; ++j) {
        s2 B[4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
            B[r] = (s2){(short)((r == (j >> 1) && !(j & 1)) ? 0 : kNeg),
                        (short)((r == (j >> 1) && (j & 1)) ? 0 : kNeg)};
        int acc = 0;
        uint32_t r0[S];
        load_seg<DEC>(c, c.W - S, r0);
        for (int i0 = c.W - S; i0 >= 0; i0 -= S) {
            uint32_t rn[S];
            load_seg<DEC>(c, max(i0 - S, 0), rn);
            s2 g[S];
            gammas<DEC>(c, i0, r0, g);
#pragma unroll
            for (int t = S - 1; t >= 0; --t) {
                acs_bwd(B, mk_g00(g[t]), g[t]);
                if (bwd_norm(i0, t, c.W)) acc += normalise_acc(B);
                if (i0 == c.W - S && t == S - 1) pin_regs(B, j & 3, j & 3);
                if (i0 == c.W - S && t == S - 2) pin_regs(B, 2 * (j & 1), 2 * (j & 1) + 1);
            }
#pragma unroll
            for (int t = 0; t < S; ++t) r0[t] = rn[t];
        }
        out[2 * j] = pack4(B);
        out[2 * j + 1] = make_uint4((uint32_t)acc, 0u, 0u, 0u);
    }
}

// Windows whose transfer values one scan trip loads before it combines them.
constexpr int kScanB = 4;

// Max over the 8 lanes of a group (lanes 8g .. 8g+7 of a wave).
__device__ __forceinline__ int group8_max(int v)
{
    v = max(v, __shfl_xor(v, 1, 64));
    v = max(v, __shfl_xor(v, 2, 64));
    v = max(v, __shfl_xor(v, 4, 64));
    return v;
}

// Hard decisions (the low bit of E after decoder 2) of the 8 positions g..g+7 (g a multiple of 8, g + 7 < K),
// MSB first, from one 16-byte LDS read: position g + 2i is the low half of
// word i, g + 2i + 1 its high half.
__device__ __forceinline__ uint32_t hard8(const short *E, int g)
{
    const uint4 v = *(const uint4 *)(E + epad(g));
    return ((v.x & 1u) << 7) | ((v.x >> 10) & 0x40u) | ((v.y & 1u) << 5) | ((v.y >> 12) & 0x10u) |
           ((v.z & 1u) << 3) | ((v.z >> 14) & 0x04u) | ((v.w & 1u) << 1) | ((v.w >> 16) & 0x01u);
}

// CRC (LFSR form, MSB first) of natural bits [b0, b1) of a block.
__device__ uint32_t crc_range(const short *E, int b0, int b1, uint32_t poly)
{
    uint32_t r = 0;
    for (int j = b0 & ~7; j < b1; j += 8) {
        const uint4 v = *(const uint4 *)(E + epad(j));  // 8 positions, 16-byte aligned
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const uint32_t bit = (w[q >> 1] >> (16 * (q & 1))) & 1u;
            const uint32_t top = ((r >> 23) ^ bit) & 1u;
            const uint32_t nr = ((r << 1) & 0xFFFFFFu) ^ (top ? poly : 0u);
            r = (j + q >= b0 && j + q < b1) ? nr : r;
        }
    }
    return r;
}

// r(x) * x^n mod g from the table T[m] = x^m mod g (n + 23 < kCrcTabN).
// All 24 entries are loaded unconditionally, so the loads go out together
// instead of one round trip per set bit of r.
__device__ uint32_t crc_shift(uint32_t r, int n, const uint32_t *T)
{
    uint32_t t[24];
#pragma unroll
    for (int i = 0; i < 24; ++i) t[i] = T[n + i];
    uint32_t o = 0;
#pragma unroll
    for (int i = 0; i < 24; ++i) o ^= ((r >> i) & 1u) ? t[i] : 0u;
    return o;
}

__device__ __forceinline__ short clamp_llr(int v) { return (short)max(-kLlrMax, min(kLlrMax, v)); }

// Four consecutive int16 LLRs (8 bytes); one 8-byte load when the address is
// 8-byte aligned, else four 2-byte loads.  The channel LLRs are read once per
// launch, so the loads are non-temporal: they do not displace the restaged
// inputs and checkpoints that the iterations re-read from the caches.
// SYS (the ring kernel): system-scope loads instead, which read the LLRs
// from memory whatever this XCD's cache holds -- the ring kernel runs while
// the host and other kernels rewrite the LLR slots.
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
template <bool SYS = false>
__device__ __forceinline__ uint2 load4(const int16_t *p, bool aligned)
{
    if constexpr (SYS) {
        if (aligned) {
            const unsigned long long v = __hip_atomic_load((const unsigned long long *)p, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_SYSTEM);
            return make_uint2((uint32_t)v, (uint32_t)(v >> 32));
        }
        uint32_t h[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
            h[j] = __hip_atomic_load((const unsigned short *)(p + j), __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_SYSTEM);
        return make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
    }
    if (aligned) {
        const u32x2_t v = __builtin_nontemporal_load((const u32x2_t *)p);
        return make_uint2(v.x, v.y);
    }
    const uint32_t a = (uint16_t)__builtin_nontemporal_load(p);
    const uint32_t b = (uint16_t)__builtin_nontemporal_load(p + 1);
    const uint32_t c = (uint16_t)__builtin_nontemporal_load(p + 2);
    const uint32_t d = (uint16_t)__builtin_nontemporal_load(p + 3);
    return make_uint2(a | (b << 16), c | (d << 16));
}

// One restaged unit: 4 steps starting at natural position pos, from the
// systematic, parity 1 and parity 2 LLRs v[0..2] (4 int16 each).  Clamps to
// +-2047, overrides filler positions (known zeros: -2047 on systematic and
// parity 1), and writes decoder 1's word Lp1 | Ls << 16 per step and
// decoder 2's four Lp2 (its QPP addresses come from the shape's table).
__device__ __forceinline__ void restage_unit(const uint2 v[3], int pos, int F, uint4 *r1, uint2 *r2)
{
    const s2 lo = (s2){(short)-kLlrMax, (short)-kLlrMax};
    const s2 hi = (s2){(short)kLlrMax, (short)kLlrMax};
    uint32_t ls[2], lp[2], z[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        ls[h] = as_u(vmax(__builtin_elementwise_min(as_s2(h ? v[0].y : v[0].x), hi), lo));
        lp[h] = as_u(vmax(__builtin_elementwise_min(as_s2(h ? v[1].y : v[1].x), hi), lo));
        z[h] = as_u(vmax(__builtin_elementwise_min(as_s2(h ? v[2].y : v[2].x), hi), lo));
    }
    if (pos < F) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (pos + j < F) {
                const uint32_t msk = 0xFFFFu << (16 * (j & 1));
                const uint32_t neg = 0xF801F801u & msk;  // -2047 in that half
                ls[j >> 1] = (ls[j >> 1] & ~msk) | neg;
                lp[j >> 1] = (lp[j >> 1] & ~msk) | neg;
            }
    }
    *r1 = make_uint4(__builtin_amdgcn_perm(ls[0], lp[0], 0x05040100u),
                     __builtin_amdgcn_perm(ls[0], lp[0], 0x07060302u),
                     __builtin_amdgcn_perm(ls[1], lp[1], 0x05040100u),
                     __builtin_amdgcn_perm(ls[1], lp[1], 0x07060302u));
    *r2 = make_uint2(z[0], z[1]);
}

// Rows of the restage tile: the largest power of two R <= 32 with 4R <= W
// whose tile (3 streams x nw windows x (R + 1) uint2) fits `tile_words`
// 8-byte words; 0 when none does (the direct form is used then).
__device__ __forceinline__ int restage_rows(int tile_words, int nw, int W)
{
    const int maxR = tile_words / (3 * nw) - 1;
    int R = 0;
    for (int r = 1; r <= 32 && r <= maxR && 4 * r <= W; r <<= 1) R = r;
    return R;
}

// Restage one code block (LLRs at src, [3][K+4] int16, F filler bits) into
// the item's inputs R1v / R2v ([t/4][lane], lanes per row; the block's
// windows are lanes lane0 .. lane0 + nw - 1).  One unit = 4 trellis steps of
// one window, written as one 16-byte word (decoder 1) and one 8-byte word
// (decoder 2) so that the iterations read them coalesced.  Tiled form
// (R > 0): a chunk of 4R steps of every window and stream is read with
// contiguous loads into the LDS tile, then turned into units with
// consecutive threads on consecutive windows (rows of R uint2 plus one of
// padding).  Direct form (R = 0): consecutive threads take consecutive
// windows.  Every thread of the work group calls it (it holds barriers).
template <bool SYS>
__device__ void restage_block(const int16_t *src, int K, int F, int nw, int W, int lanes,
                              int lane0, uint4 *R1v, uint2 *R2v, uint2 *tile, int R, int tid,
                              int nthr)
{
    const int N = K + 4;
    // every load address is src plus a multiple of 4 elements
    const bool aligned = (((uintptr_t)src) & 7) == 0;
    if (R > 0) {
        const int lg = __builtin_ctz((unsigned)R), rs = R + 1, nl = nw * R;
        for (int c0 = 0; c0 < W; c0 += 4 * R) {
            const int Rc = min(R, (W - c0) >> 2);
            // the three streams' loads of 4 rows are all issued
            // before the first LDS store (12 loads in flight)
            for (int e0 = tid; e0 < nl; e0 += 4 * nthr) {
                uint2 v[3][4];
#pragma unroll
                for (int st = 0; st < 3; ++st)
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        const int e = e0 + m * nthr;
                        const int ww = e >> lg, j = e & (R - 1);
                        const int p = ww * W + c0 + 4 * j;
                        v[st][m] = make_uint2(0u, 0u);
                        if (e < nl && j < Rc && p < K) v[st][m] = load4<SYS>(src + st * N + p, aligned);
                    }
#pragma unroll
                for (int st = 0; st < 3; ++st)
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        const int e = e0 + m * nthr;
                        const int ww = e >> lg, j = e & (R - 1);
                        if (e < nl && j < Rc) tile[(st * nw + ww) * rs + j] = v[st][m];
                    }
            }
            __syncthreads();
            const int nu = nw * Rc;
            for (int e = tid; e < nu; e += nthr) {
                const int jj = e / nw, ww = e - jj * nw;
                const int t4 = (c0 >> 2) + jj;
                const uint2 v[3] = {tile[ww * rs + jj], tile[(nw + ww) * rs + jj],
                                    tile[(2 * nw + ww) * rs + jj]};
                restage_unit(v, ww * W + 4 * t4, F, R1v + (size_t)t4 * lanes + lane0 + ww,
                             R2v + (size_t)t4 * lanes + lane0 + ww);
            }
            __syncthreads();
        }
    } else {
        // 4 units of loads in flight
        const int units = (nw * W) >> 2;
        for (int u0 = tid; u0 < units; u0 += 4 * nthr) {
            uint2 v[4][3];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int u = min(u0 + m * nthr, units - 1);
                const int t4 = u / nw, ww = u - t4 * nw;
                const int p = ww * W + 4 * t4;
#pragma unroll
                for (int st = 0; st < 3; ++st)
                    v[m][st] = p < K ? load4<SYS>(src + st * N + p, aligned) : make_uint2(0u, 0u);
            }
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int u = u0 + m * nthr;
                if (u >= units) break;
                const int t4 = u / nw, ww = u - t4 * nw;
                restage_unit(v[m], ww * W + 4 * t4, F, R1v + (size_t)t4 * lanes + lane0 + ww,
                             R2v + (size_t)t4 * lanes + lane0 + ww);
            }
        }
    }
}

// Ring mode, thread 0: take a ticket and wait until the item of that number
// is published.  Tickets come from one fetch-and-add (ring_head[0]), so a
// burst of claims costs one atomic each.  Only the holder of the first
// unpublished ticket looks at the host's tail (and stop flag) over the bus,
// and mirrors what it sees into device memory (ring_head[16], ring_head[32])
// for the others.  The wait is bounded: it ends when the item is published,
// when the server stops, or after ring_idle_ticks of the wall clock (the
// ticket is then abandoned: the host, which stops the kernel itself long
// before that, rewinds the counter before the next launch).  A rewound
// counter hands out items that are done already: they are skipped.
// Returns the item's ring index, or -1 when the work group is to leave.
__device__ long long ring_claim(const RingArgs &a)
{
    unsigned long long *seen = a.head + 16;            // own 128-byte line
    unsigned int *stopm = (unsigned int *)(a.head + 32);
    for (;;) {
        const unsigned long long t = __hip_atomic_fetch_add(a.head, 1ull, __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t t0 = wall_clock64();
        int nap = 0;
        for (;;) {
            const unsigned long long m = __hip_atomic_load(seen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (t < m) break;
            const bool lead = t == m;
            if (lead) {
                const unsigned long long x =
                    __hip_atomic_load(&a.ctl->tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                if (x > m) {
                    __hip_atomic_fetch_max(seen, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (t < x) break;
                }
                if (__hip_atomic_load(&a.ctl->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM))
                    __hip_atomic_store(stopm, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            if (__hip_atomic_load(stopm, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return -1;
            if ((uint64_t)wall_clock64() - t0 > a.idle_ticks) return -1;
            // back off: 2^nap naps of 8 x 64 clocks, up to about 1 us for
            // the ticket holder that watches the host, 3.5 us for the others
            for (int k = 0; k < (1 << nap); ++k) __builtin_amdgcn_s_sleep(8);
            nap = min(nap + 1, lead ? 2 : 4);
        }
        if (__hip_atomic_load(&a.done[t & (unsigned long long)(a.cap - 1)], __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_SYSTEM) != (uint32_t)t + 1u)
            return (long long)t;
    }
}

// Ring mode, whole work group: claim an item and copy its entry (host
// memory) and its code blocks (device memory) into LDS at `ent`.  Returns
// the item's ring index, or -1 when the work group is to leave.
//
// Everything an item reads that someone else may have rewritten while the
// kernel runs -- its entry, its plan's code block list (uploaded by the
// host), the LLRs of its blocks (copied into reused slots) -- is read with
// system-scope loads, which go to memory past any stale copy in this XCD's
// cache; the host publishes an item only after all of it is in memory.  The
// QPP tables are only ever appended, on cache lines of their own, so no
// cache holds an old copy of a table the kernel has not read yet.
__device__ long long ring_take(const RingArgs &a, RingEntry *ent, int tid, int nthr)
{
    __shared__ long long s_claim;
    if (tid == 0) s_claim = ring_claim(a);
    __syncthreads();
    const long long i = s_claim;
    if (i < 0) return -1;
    constexpr int ew = (int)(sizeof(RingEntry) / 4);
    const uint32_t *src = (const uint32_t *)(a.ent + (i & (a.cap - 1)));
    if (tid < ew)
        ((uint32_t *)ent)[tid] = __hip_atomic_load(src + tid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __syncthreads();
    constexpr int cw = (int)(sizeof(DecCb) / 4);
    const int n = min(max(ent->item.ncb, 0), kMaxSlotsPerWg) * cw;
    const uint32_t *cs = (const uint32_t *)ent->cbs;
    uint32_t *dst = (uint32_t *)(ent + 1);
    for (int q = tid; q < n; q += nthr)
        dst[q] = __hip_atomic_load(cs + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __syncthreads();
    return i;
}

// Kernel arguments: DecArgs, and for the ring kernel RingArgs after them.
template <bool RING>
struct KernArgs : DecArgs {
};
template <>
struct KernArgs<true> : DecArgs {
    RingArgs ring;
};

// At most 168 VGPRs, so that three waves share a SIMD.  The compiler spills
// 136 of them (548 B of scratch per lane) in the uniform instantiation and
// 124-199 in the others, all in the code around the phase loops: the
// innermost loops (a segment of 8 steps in phase 1, two in phase 2) have no
// scratch access.  UNEVEN: some item's last window is shorter than the
// others, so window lengths are per lane; the even instantiation keeps them
// uniform (scalar loop bounds).  RING: items come from the serving loop's
// work ring (ring_take) and outputs are written through to memory.
template <bool UNEVEN, bool EXACT, bool MI, bool RING = false>
__global__ void __launch_bounds__(kMaxWgThreads, 3) turbo_decode_kernel(KernArgs<RING> a)
{
    // dynamic LDS: per-slot state (CRC, done, iterations, ok) for the most
    // blocks an item of this launch holds; with MI the entropy table and the
    // per-slot entropy sums of this and the previous iteration; then the
    // blocks' extrinsic arrays
    extern __shared__ __align__(16) char lds_all[];
    const int ss = a.state_slots;
    uint32_t *s_crc = (uint32_t *)lds_all;
    int *s_done = (int *)(lds_all + 4 * ss);
    int *s_iters = (int *)(lds_all + 8 * ss);
    int *s_ok = (int *)(lds_all + 12 * ss);
    unsigned short *s_mit = (unsigned short *)(lds_all + lds_state_bytes(ss));
    int *s_mi = (int *)(s_mit + kMiTabN);
    int *s_mip = s_mi + ss;
    char *lds = lds_all + lds_state_bytes(ss) + (MI ? lds_mi_bytes(ss) : 0);

    const int tid = threadIdx.x, nthr = blockDim.x, half = nthr >> 1;
    if (MI)
        for (int m = tid; m < kMiTabN; m += nthr) s_mit[m] = (unsigned short)a.mi_tab[m];
    const bool bwd_first = tid >= half;       // wave-uniform role
    const int wi = bwd_first ? tid - half : tid;  // window index within the item
    char *scr = a.scratch + (int64_t)blockIdx.x * a.scratch_stride;

    // Items are handed out dynamically: every work group starts with item
    // blockIdx.x and then claims the next unclaimed one, so blocks that stop
    // early free their work group for more work.  The claims are spread over
    // nset = min(8, grid) counters (one per XCD under round-robin dispatch),
    // each on its own 256-byte line: work group b belongs to set
    // xc = b % nset, whose items are xc, xc + nset, xc + 2 nset, ...; the
    // first gx of them start the set's gx work groups, the rest are claimed.
    // A single counter serialised the claims of all work groups, which all
    // finish their first item at about the same time.  The last work group
    // of a set to finish resets that set's counters for the next launch.
    const int nset = min((int)gridDim.x, kCtrSets);
    const int xc = (int)blockIdx.x % nset;
    const int gx = ((int)gridDim.x - xc + nset - 1) / nset;
    uint32_t *ctr_item = a.counter + xc * kCtrStride;
    uint32_t *ctr_done = a.counter + (kCtrSets + xc) * kCtrStride;
    __shared__ int s_next;
    // Ring mode: items are claimed from the host's ring instead, and each
    // claimed item is copied into LDS after the extrinsic arrays.
    RingEntry *r_ent = nullptr;
    long long ring_i = -1;
    if constexpr (RING) {
        r_ent = (RingEntry *)(lds_all + a.ring.lds);
        ring_i = ring_take(a.ring, r_ent, tid, nthr);
    }
    for (int item_i = blockIdx.x; RING ? ring_i >= 0 : item_i < a.n_items; item_i = RING ? 0 : s_next) {
        // the item, block i of it, its QPP tables and outputs: from the ring
        // entry's copy in ring mode, else from the plan and the arguments
        const DecItem it = [&] {
            if constexpr (RING) return r_ent->item;
            else return a.items[item_i];
        }();
        const auto cbat = [&](int i) -> DecCb {
            if constexpr (RING) return ((const DecCb *)(r_ent + 1))[i];
            else return a.cbs[it.cb0 + i];
        };
        const uint16_t *qtab = RING ? r_ent->qtab : a.qtab;
        uint32_t *o_hard = RING ? r_ent->hard : a.hard;
        uint8_t *o_ok = RING ? r_ent->crc_ok : a.crc_ok;
        uint8_t *o_it = RING ? r_ent->iters : a.iters;
        const int K = it.K, nw = it.nw, W = it.W, ncb = it.ncb;
        const int lanes = ncb * nw;
        // global scratch of this item: restaged inputs of both decoders,
        // checkpoints, window boundary metrics
        const int64_t rsz = (int64_t)lanes * W;                  // padded steps of the item
        uint32_t *R1 = (uint32_t *)scr;                          // rsz int32
        uint32_t *R2 = R1 + rsz;                                 // rsz int16
        uint4 *ck = (uint4 *)(R2 + rsz / 2);                     // (W/S)*lanes
        uint4 *bnd = ck + (int64_t)(W / S) * lanes;              // [4][lanes]
        // exact boundaries only: transfer runs, [lanes][8 states][2] each
        uint4 *tfA = bnd + (int64_t)4 * lanes;
        uint4 *tfB = tfA + (int64_t)16 * lanes;

        // ---- restage the channel LLRs, clear LDS.  The tile of the restage
        // is the item's extrinsic slots, unused until the iterations.
        {
            const int esz = lds_e_bytes(K);
            uint4 *R1v = (uint4 *)R1;
            uint2 *R2v = (uint2 *)R2;
            const int R = restage_rows((ncb * it.lds_slot) / 8, nw, W);
            for (int cs = 0; cs < ncb; ++cs) {
                const DecCb cb = cbat(cs);
                restage_block<RING>(a.llr + cb.llr_off, K, cb.F, nw, W, lanes, cs * nw, R1v, R2v,
                              (uint2 *)lds, R, tid, nthr);
            }
            __syncthreads();  // the tile's last reads come before the clear
            for (int cs = 0; cs < ncb; ++cs) {
                uint32_t *slot = (uint32_t *)(lds + (int64_t)cs * it.lds_slot);
                for (int q = tid; q < esz / 4; q += nthr) slot[q] = 0;
            }
        }
        if (tid < ncb) {
            s_done[tid] = 0;
            s_iters[tid] = a.max_iters;
            s_ok[tid] = 0;
            if (MI) s_mip[tid] = 0;
        }

        // ---- lane role within the item
        const bool active = wi < lanes;
        const int cs = active ? wi / nw : 0;
        const int w = active ? wi - cs * nw : 0;
        const DecCb cb = cbat(cs);
        Win c;
        // every window has W steps but the last, which has the rest of K
        c.W = (UNEVEN && w == nw - 1) ? K - (nw - 1) * W : W;
        c.M = win_split(c.W);
        c.lo = w * W;
        c.wi = wi;
        c.lanes = lanes;
        c.first = w == 0;
        c.last = w == nw - 1;
        c.E = (short *)(lds + (int64_t)cs * it.lds_slot);
        c.qt = (const uint2 *)(qtab + it.qtab) + w;
        c.qs = nw;
        c.ck = ck;
        c.mit = s_mit;

        // trellis termination of both encoders: beta_K (Q layout) in closed
        // form along the forced zero-feedback path from each state
        s2 tb[2][4];
        if (active && c.last && bwd_first) {
            const int16_t *src = a.llr + cb.llr_off;
            const int N = K + 4;
            const auto ld = [&](int q) -> int {
                if constexpr (RING)
                    return (short)__hip_atomic_load((const unsigned short *)(src + q), __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_SYSTEM);
                return src[q];
            };
            for (int d = 0; d < 2; ++d) {
                const int o = K + 2 * d;
                const int lx0 = clamp_llr(ld(o)), lz0 = clamp_llr(ld(N + o)),
                          lx1 = clamp_llr(ld(2 * N + o)), lz1 = clamp_llr(ld(o + 1)),
                          lx2 = clamp_llr(ld(N + o + 1)), lz2 = clamp_llr(ld(2 * N + o + 1));
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
            const bool prev = EXACT || (a.win_init && iter > 1);
            const s2 z = (s2){0, 0};
            s2 V[4];  // this lane's running metric (alpha or beta)
            int acc = 0;  // entropy sum of this lane's decoder-2 steps (MI)
#pragma unroll
            for (int dec = 1; dec <= 2; ++dec) {
                Win cd = c;
                cd.R = (const uint4 *)(dec == 1 ? R1 : R2);
                uint4 *bA = bnd + (dec - 1) * 2 * lanes;  // alpha boundaries of this decoder
                uint4 *bB = bA + lanes;                   // beta boundaries
                if (EXACT) {
                    // transfer runs of every window, then the scans that give
                    // the exact boundaries (8 lanes per block: lane q owns state q)
                    if (run) {
                        if (!bwd_first && !c.last) {
                            if (dec == 1) tf_fwd<1>(cd, tfA + (size_t)wi * 16);
                            else tf_fwd<2>(cd, tfA + (size_t)wi * 16);
                        } else if (bwd_first && !c.first) {
                            if (dec == 1) tf_bwd<1>(cd, tfB + (size_t)wi * 16);
                            else tf_bwd<2>(cd, tfB + (size_t)wi * 16);
                        }
                    }
                    __syncthreads();
                    const int tl = bwd_first ? tid - half : tid;  // lane within the half
                    const int q = tl & 7, lb = (tid & 63) & ~7;   // state; group base lane in the wave
                    for (int cs0 = 0; cs0 < ncb; cs0 += half >> 3) {
                        const int cg = cs0 + (tl >> 3);
                        if (cg >= ncb || s_done[cg]) continue;  // the same for the group's 8 lanes
                        if (!bwd_first) {
                            // alpha at the start of windows 1 .. nw-1, from state 0;
                            // the transfer values of kScanB windows are loaded per
                            // trip (each lane: its state's metric of the 8 runs and
                            // the 8 totals), then combined window by window
                            int av = q == 0 ? 0 : -(1 << 30);
                            const int h = 2 * (q & 3) + (q >> 2);  // P-layout halfword of state q
                            for (int w0 = 0; w0 < nw - 1; w0 += kScanB) {
                                int tv[kScanB][8];
#pragma unroll
                                for (int b = 0; b < kScanB; ++b) {
                                    const int ww = min(w0 + b, nw - 2);
                                    const uint32_t *Tm = (const uint32_t *)(tfA + (size_t)(cg * nw + ww) * 16);
#pragma unroll
                                    for (int i = 0; i < 8; ++i)
                                        tv[b][i] = (int)(short)(Tm[8 * i + (h >> 1)] >> (16 * (h & 1))) +
                                                   (int)Tm[8 * i + 4];
                                }
#pragma unroll
                                for (int b = 0; b < kScanB; ++b) {
                                    if (w0 + b >= nw - 1) break;
                                    int best = -0x7fffffff;
#pragma unroll
                                    for (int i = 0; i < 8; ++i) best = max(best, __shfl(av, lb | i, 64) + tv[b][i]);
                                    av = best - group8_max(best);
                                    ((short *)&bA[cg * nw + w0 + b + 1])[h] = (short)max(-32768, av);
                                }
                            }
                        } else {
                            // beta at the end of windows nw-2 .. 0, from the termination
                            const int16_t *src = a.llr + cbat(cg).llr_off;
                            const int N = K + 4, o = K + 2 * (dec - 1);
                            const int lx0 = clamp_llr(src[o]), lz0 = clamp_llr(src[N + o]),
                                      lx1 = clamp_llr(src[2 * N + o]), lz1 = clamp_llr(src[o + 1]),
                                      lx2 = clamp_llr(src[N + o + 1]), lz2 = clamp_llr(src[2 * N + o + 1]);
                            const int s1 = (q >> 2) & 1, s2b = (q >> 1) & 1, s3 = q & 1;
                            const int v0 = (s2b ^ s3) * lx0 + (s1 ^ s3) * lz0 + (s1 ^ s2b) * lx1 +
                                           s2b * lz1 + s1 * lx2 + s1 * lz2;
                            int bv = v0 - group8_max(v0);
                            for (int w0 = nw - 1; w0 >= 1; w0 -= kScanB) {
                                int tv[kScanB][8];
#pragma unroll
                                for (int b = 0; b < kScanB; ++b) {
                                    const int ww = max(w0 - b, 1);
                                    const uint32_t *U = (const uint32_t *)(tfB + (size_t)(cg * nw + ww) * 16);
#pragma unroll
                                    for (int j = 0; j < 8; ++j)  // Q layout: halfword q
                                        tv[b][j] = (int)(short)(U[8 * j + (q >> 1)] >> (16 * (q & 1))) +
                                                   (int)U[8 * j + 4];
                                }
#pragma unroll
                                for (int b = 0; b < kScanB; ++b) {
                                    if (w0 - b < 1) break;
                                    int best = -0x7fffffff;
#pragma unroll
                                    for (int j = 0; j < 8; ++j) best = max(best, __shfl(bv, lb | j, 64) + tv[b][j]);
                                    bv = best - group8_max(best);
                                    ((short *)&bB[cg * nw + w0 - b - 1])[q] = (short)max(-32768, bv);
                                }
                            }
                        }
                    }
                    __syncthreads();
                }
                if (run) {
                    if (dec == 1 && w == 0 && !bwd_first) {
                        s_crc[cs] = 0;
                        if (MI) s_mi[cs] = 0;
                    }
                    if (!bwd_first) {
                        if (c.first) {
                            V[0] = (s2){0, kNeg};
                            V[1] = V[2] = V[3] = (s2){kNeg, kNeg};
                        } else if (prev) {
                            unpack4(bA[wi], V);
                        } else {
                            V[0] = V[1] = V[2] = V[3] = z;
                        }
                        if (dec == 1) ph1_fwd<1>(cd, V); else ph1_fwd<2>(cd, V);
                    } else {
                        if (c.last) {
                            for (int j = 0; j < 4; ++j) V[j] = tb[dec - 1][j];
                        } else if (prev) {
                            unpack4(bB[wi], V);
                        } else {
                            V[0] = V[1] = V[2] = V[3] = z;
                        }
                        if (dec == 1) ph1_bwd<1>(cd, V); else ph1_bwd<2>(cd, V);
                    }
                }
                __syncthreads();
                if (run) {
                    if (!bwd_first) {
                        if (dec == 1) ph2_fwd<1>(cd, V); else acc = ph2_fwd<2, MI>(cd, V);
                        if (!EXACT && !c.last) bA[wi + 1] = pack4(V);  // alpha at the window end
                    } else {
                        if (dec == 1) ph2_bwd<1>(cd, V); else acc = ph2_bwd<2, MI>(cd, V);
                        if (!EXACT && !c.first) bB[wi - 1] = pack4(V);  // beta at the window start
                    }
                    if (MI && dec == 2) atomicAdd(&s_mi[cs], acc);
                }
                __syncthreads();
            }
            const bool check = run && !bwd_first && cb.crc != 0 && (a.early_stop || iter == a.max_iters);
            if (check) {
                const int b0 = max((int)cb.F, c.lo), b1 = c.lo + c.W;
                uint32_t r = b0 < b1 ? crc_range(c.E, b0, b1, poly) : 0u;
                r = crc_shift(r, K - b1, T);
                if (r) atomicXor(&s_crc[cs], r);
            }
            __syncthreads();
            if (run && w == 0 && !bwd_first) {
                const bool pass = cb.crc == 0 || s_crc[cs] == 0;
                bool stop = (a.early_stop & 1) && cb.crc != 0 && pass;
                if (MI) {
                    // converged: 1 - I within eps of 0, or changed by at most
                    // eps since the previous iteration (per bit, 2^-15 units)
                    const int sum = s_mi[cs], thr = K * a.mi_eps;
                    stop = stop || sum <= thr || (iter > 1 && abs(sum - s_mip[cs]) <= thr);
                    s_mip[cs] = sum;
                }
                if (stop) {
                    s_done[cs] = 1;
                    s_iters[cs] = iter;
                    s_ok[cs] = pass;
                    // a block that stops with a failed CRC fails its
                    // transport block (Algorithm 2): mark it for the siblings
                    if (!pass && a.tb_fail && cb.tb >= 0) atomicOr(&a.tb_fail[cb.tb], 1u);
                } else if (iter == a.max_iters) {
                    s_iters[cs] = iter;
                    s_ok[cs] = pass;
                } else if (a.tb_fail && cb.tb >= 0 &&
                           __hip_atomic_load(&a.tb_fail[cb.tb], __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT) != 0u) {
                    // a sibling failed: the rest of this block's work is purged
                    s_done[cs] = 1;
                    s_iters[cs] = 0;
                    s_ok[cs] = 0;
                }
            }
            __syncthreads();
            if (!__syncthreads_or(active && !s_done[cs])) break;
        }

        // ---- outputs (the forward-first lanes of each block)
        if (active && !bwd_first) {
            const int L = cb.crc ? 24 : 0;
            if (cb.bits_off >= 0 && a.bits) {
                const int nbits = K - cb.F - L;
                const int nbytes = (nbits + 7) >> 3;
                uint8_t *out = a.bits + cb.bits_off;
                for (int bb = w; bb < nbytes; bb += nw) {
                    // positions pos .. pos + valid - 1 (all < K - L)
                    const int pos = cb.F + 8 * bb;
                    const int valid = min(8, nbits - 8 * bb);
                    const int g = pos & ~7, o = pos & 7;
                    uint32_t byte = hard8(c.E, g);
                    if (o) {
                        const uint32_t nx = o + valid > 8 ? hard8(c.E, g + 8) : 0u;
                        byte = ((byte << 8) | nx) >> (8 - o);
                    }
                    out[bb] = (uint8_t)(byte & (0xFFu << (8 - valid)));
                }
            }
            if (cb.hard_off >= 0 && o_hard) {
                uint32_t *h = o_hard + cb.hard_off;
                const int hw = (int)hard_words(K);
                for (int q = w; q < hw; q += nw) {
                    // K is a multiple of 8: a group of 8 is all inside or all past K
                    uint32_t v = 0;
#pragma unroll
                    for (int k = 0; k < 32; k += 8)
                        v = (v << 8) | (32 * q + k < K ? hard8(c.E, 32 * q + k) : 0u);
                    // ring: written through to memory, so the assembly
                    // kernel reads them without this XCD's cache written back
                    if constexpr (RING)
                        __hip_atomic_store(h + q, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    else
                        h[q] = v;
                }
            }
            if (w == 0) {
                if constexpr (RING) {
                    __hip_atomic_store(o_ok + cb.out_idx, (uint8_t)s_ok[cs], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_SYSTEM);
                    __hip_atomic_store(o_it + cb.out_idx, (uint8_t)s_iters[cs], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_SYSTEM);
                } else {
                    o_ok[cb.out_idx] = (uint8_t)s_ok[cs];
                    o_it[cb.out_idx] = (uint8_t)s_iters[cs];
                }
            }
        }
        if constexpr (RING) {
            // every wave's write-through output stores have completed
            // before the barrier, so they are in memory before the host can
            // see the item's done mark
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            if (tid == 0)
                __hip_atomic_store(&a.ring.done[ring_i & (a.ring.cap - 1)], (uint32_t)ring_i + 1u,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            ring_i = ring_take(a.ring, r_ent, tid, nthr);
        } else {
            __syncthreads();
            if (tid == 0) s_next = xc + nset * (gx + (int)atomicAdd(ctr_item, 1u));
            __syncthreads();
        }
    }
    // Every claim of this work group has returned (its last one ended the
    // loop) before it counts itself done, so the last of the set resets the
    // set's counters after all of the set's claims.
    if constexpr (!RING) {
        if (tid == 0 && atomicAdd(ctr_done, 1u) == (uint32_t)gx - 1) {
            atomicExch(ctr_item, 0u);
            atomicExch(ctr_done, 0u);
        }
    }
}

using DecodeKernel = void (*)(KernArgs<false>);

// The eight instantiations, indexed by uneven + 2 exact + 4 mi.
static DecodeKernel decode_kernel(bool uneven, bool exact, bool mi)
{
    static const DecodeKernel k[8] = {
        turbo_decode_kernel<false, false, false>, turbo_decode_kernel<true, false, false>,
        turbo_decode_kernel<false, true, false>,  turbo_decode_kernel<true, true, false>,
        turbo_decode_kernel<false, false, true>,  turbo_decode_kernel<true, false, true>,
        turbo_decode_kernel<false, true, true>,   turbo_decode_kernel<true, true, true>};
    return k[(uneven ? 1 : 0) + (exact ? 2 : 0) + (mi ? 4 : 0)];
}

const void *decode_kernel_address(bool uneven, bool exact, bool mi)
{
    return (const void *)decode_kernel(uneven, exact, mi);
}

int launch_decode(const DecArgs &a, bool uneven, bool exact, bool mi, int grid, int wg_threads,
                  int lds_bytes, void *stream)
{
    KernArgs<false> k;
    static_cast<DecArgs &>(k) = a;
    hipLaunchKernelGGL(decode_kernel(uneven, exact, mi), dim3(grid), dim3(wg_threads), lds_bytes,
                       (hipStream_t)stream, k);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

const void *ring_kernel_address() { return (const void *)turbo_decode_kernel<true, false, false, true>; }

int launch_ring_decode(const DecArgs &a, const RingArgs &r, int grid, int lds_bytes, void *stream)
{
    KernArgs<true> k;
    static_cast<DecArgs &>(k) = a;
    k.ring = r;
    hipLaunchKernelGGL((turbo_decode_kernel<true, false, false, true>), dim3(grid), dim3(kRingWg),
                       lds_bytes, (hipStream_t)stream, k);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ------------------------------------------------------------------------
// Fixed device scratch of the allocation-free decode entry point: the claim
// counters (kCtrBytes) and then the per-work-group scratch.  Each device that
// loads the library holds one copy for the life of the process; its address
// comes from hipGetSymbolAddress (host code never passes the symbol itself).

static __device__ __align__(256) char scratch[kStaticScratchBytes];

namespace {
std::mutex g_static_mu;
char *g_static_ptr[kMaxDevices] = {};
}  // namespace

int static_scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return -1;
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (g_static_ptr[device]) return 0;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != device) return -1;
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return -1;
    g_static_ptr[device] = (char *)p;
    return 0;
}

char *static_scratch_ptr(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_static_mu);
    return g_static_ptr[device];
}

__global__ void __launch_bounds__(256) zero_words_kernel(uint32_t *p, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

int launch_zero_words(uint32_t *p, int n, void *stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(zero_words_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, p, n);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ------------------------------------------------------------------------
// Transport block assembly: payload bits of the blocks (filler and CRC24B
// dropped) back to back, CRC24A over them, per-block flags into the result.

struct TbRes {
    int32_t tb_ok, max_iters_used, C, rsv;
    uint8_t cb_ok[64], cb_iters[64];
};

// a * b mod g over GF(2), 24-bit operands
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

// `n` bits (1..32) of a block's hard-decision words starting at bit `pos`,
// left-aligned; reads one word past the last full one (every block keeps a
// spare word for this).
__device__ __forceinline__ uint32_t take_bits(const uint32_t *h, int pos, int n)
{
    const int i = pos >> 5, sh = pos & 31;
    uint32_t x = h[i] << sh;
    if (sh) x |= h[i + 1] >> (32 - sh);
    return n >= 32 ? x : (x & ~(0xFFFFFFFFu >> n));
}


// The B = tbs + 24 reassembled bits of a transport block (every block's bits
// F..K-L-1, in block order) are gathered into LDS words; the CRC24A
// remainder of that message, zero-padded to whole words, is the XOR of each
// thread's word-chunk remainder times x^(32 * words after the chunk) (table
// X32).  Padding multiplies the remainder by a power of x, which is
// invertible modulo the generator (its constant term is 1), so the padded
// remainder is zero exactly when the message's is.
__global__ void __launch_bounds__(256) tb_assemble_kernel(const TbItem *items, int n_tb,
                                                                  const uint32_t *hard,
                                                                  const uint8_t *crc_ok,
                                                                  const uint8_t *iters,
                                                                  const uint32_t *tb_fail,
                                                                  uint8_t *bits, TbRes *res,
                                                                  const uint32_t *x32)
{
    extern __shared__ uint32_t msg[];
    __shared__ int64_t s_hoff[64];   // hard word offset of each block
    __shared__ int32_t s_start[65];  // first message bit of each block
    __shared__ int32_t s_F[64];
    __shared__ uint32_t s_t8[256];   // byte table of CRC24A
    __shared__ uint32_t s_crc;
    const int tid = threadIdx.x, nthr = blockDim.x;
    for (int e = tid; e < 256; e += nthr) {
        // byte step of the MSB-first CRC: the remainder of e * x^24 after 8 shifts
        uint32_t r = (uint32_t)e << 16;
        for (int k = 0; k < 8; ++k) r = ((r << 1) & 0xFFFFFFu) ^ ((r & 0x800000u) ? kPoly24A : 0u);
        s_t8[e] = r;
    }
    for (int t = blockIdx.x; t < n_tb; t += gridDim.x) {
        const TbItem tb = items[t];
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
            s_start[tb.C] = st;  // = B
            s_crc = 0;
        }
        __syncthreads();
        const int B = tb.B;
        const int nwd = (B + 31) >> 5;
        // each thread builds a run of consecutive message words (the run it
        // takes for the CRC below): a run inside one block reads its hard
        // words in order, eight at a time with every load issued before the
        // first is used; runs across a block boundary go word by word
        const int cw0 = (nwd + nthr - 1) / nthr;
        const int g0 = tid * cw0, g1 = min(nwd, g0 + cw0);
        if (g0 < g1) {
            const int b0 = g0 << 5;
            int lo = 0, hi = tb.C - 1;  // block holding bit b0: the last r with s_start[r] <= b0
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_start[mid] <= b0) lo = mid;
                else hi = mid - 1;
            }
            if (min(B, g1 << 5) <= s_start[lo + 1]) {
                const int pos = s_F[lo] + (b0 - s_start[lo]);
                const uint32_t *h = hard + s_hoff[lo] + (pos >> 5);
                const int sh = pos & 31;
                // the last word may read past the block's bits: the extra
                // bits are dropped below, and the block's spare word keeps
                // the read inside its hard-decision words
                for (int w = g0; w < g1; w += 8) {
                    uint32_t hw[9];
#pragma unroll
                    for (int k = 0; k < 9; ++k) hw[k] = (w + k <= g1) ? h[w - g0 + k] : 0u;
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        if (w + k >= g1) break;
                        uint32_t v = sh ? (hw[k] << sh) | (hw[k + 1] >> (32 - sh)) : hw[k];
                        const int left = B - ((w + k) << 5);  // message bits from this word on
                        if (left < 32) v &= ~(0xFFFFFFFFu >> left);
                        msg[w + k] = v;
                    }
                }
            } else {
                for (int w = g0; w < g1; ++w) {
                    int b = w << 5;
                    int r = lo;
                    while (s_start[r + 1] <= b) ++r;
                    int got = 0;
                    uint32_t v = 0;
                    while (got < 32 && b < B) {
                        const int n = min(32 - got, s_start[r + 1] - b);
                        const uint32_t c = take_bits(hard + s_hoff[r], s_F[r] + (b - s_start[r]), n);
                        v |= c >> got;
                        got += n;
                        b += n;
                        ++r;
                    }
                    msg[w] = v;
                }
            }
        }
        __syncthreads();
        // payload bytes (the first tbs bits)
        if (tb.bits_off >= 0 && bits) {
            const int nbytes = (tb.tbs + 7) >> 3;
            for (int q = tid; q < nbytes; q += nthr) {
                uint32_t v = (msg[q >> 2] >> (24 - 8 * (q & 3))) & 0xFFu;
                const int keep = tb.tbs - 8 * q;  // payload bits in this byte
                if (keep < 8) v &= 0xFFu << (8 - keep);
                bits[tb.bits_off + q] = (uint8_t)v;
            }
        }
        // CRC24A over the zero-padded message: word chunks per thread
        const int cw = (nwd + nthr - 1) / nthr;
        const int w0 = tid * cw, w1 = min(nwd, w0 + cw);
        if (w0 < w1) {
            uint32_t r = 0;
            for (int w = w0; w < w1; ++w) {
                const uint32_t v = msg[w];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const uint32_t byte = (v >> (24 - 8 * k)) & 0xFFu;
                    r = ((r << 8) & 0xFFFFFFu) ^ s_t8[((r >> 16) ^ byte) & 0xFFu];
                }
            }
            if (r) r = gf_mulmod(r, x32[nwd - w1], kPoly24A);
            if (r) atomicXor(&s_crc, r);
        }
        __syncthreads();
        if (tid < 64) {
            TbRes &o = res[tb.res_idx];
            const int r = tid;
            o.cb_ok[r] = r < tb.C ? crc_ok[tb.cb_idx0 + r] : 0;
            o.cb_iters[r] = r < tb.C ? iters[tb.cb_idx0 + r] : 0;
            int mx = r < tb.C ? (int)iters[tb.cb_idx0 + r] : 0;
            // wave-wide maximum (the 64 threads are one wave)
            for (int d = 32; d > 0; d >>= 1) mx = max(mx, __shfl_xor(mx, d));
            if (tid == 0) {
                // a transport block marked failed by a purge fails (Algorithm 2)
                o.tb_ok = s_crc == 0 && !(tb_fail && tb_fail[t]);
                o.max_iters_used = mx;
                o.C = tb.C;
                o.rsv = 0;
            }
        }
        __syncthreads();  // the shared state is rewritten for the next block
    }
}

int launch_tb_assemble(const TbItem *items, int n_tb, int max_words, const uint32_t *hard,
                       const uint8_t *crc_ok, const uint8_t *iters, const uint32_t *tb_fail,
                       const uint32_t *crc_tab, uint8_t *bits, void *res, int small_grid,
                       void *stream)
{
    if (n_tb <= 0) return 0;
    // one work group of 256 threads per transport block, or small_grid work
    // groups of two waves (each fits the slot of a decode work group)
    const int grid = small_grid > 0 ? min(n_tb, small_grid) : n_tb;
    hipLaunchKernelGGL(tb_assemble_kernel, dim3(grid), dim3(small_grid > 0 ? 128 : 256),
                       (size_t)max_words * 4, (hipStream_t)stream, items, n_tb, hard, crc_ok, iters,
                       tb_fail, bits, (TbRes *)res, crc_tab + 2 * kCrcTabN);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace tdec
