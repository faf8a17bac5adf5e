/*
 * oracle.c -- plain CPU reference of the LTE turbo decoding path.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Written for obviousness, not for
 * speed: every trellis quantity is recomputed from the generator
 * polynomials, every maximum is taken over an explicit list of branches, and
 * the decoder keeps whole alpha/beta arrays per window.
 *
 * Sources:
 *   paper Sec. IV-B "Encoding function"  -- two RSC encoders separated by an
 *     interleaver, rate 1/3 output (b, b', b'') of size 3T, code blocks
 *     created by segmentation before encoding;
 *   paper Sec. IV-B "Decoding function"  -- LLR = log P(1)/P(0); decoder 1
 *     (systematic + parity 1 + a-priori) produces extrinsic information that
 *     is interleaved into decoder 2 (interleaved systematic + parity 2), whose
 *     extrinsic is de-interleaved back into decoder 1; iterate up to a
 *     maximum, final hard decision;
 *   paper Algorithm 1 -- code blocks of at most CB_MAX_SIZE = 6120 payload
 *     bits; Algorithm 2 -- a transport block succeeds only if all of its code
 *     blocks do;
 *   3GPP TS 36.212 5.1.1 (CRC polynomials), 5.1.2 (segmentation),
 *   5.1.3.2 (RSC polynomials, termination, QPP) for the constants the paper
 *   does not print.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ===================================================================== */
/* CRC (TS 36.212 5.1.1)                                                  */
/* ===================================================================== */

/* g24A(D) = D^24+D^23+D^18+D^17+D^14+D^11+D^10+D^7+D^6+D^5+D^4+D^3+D+1 */
#define OR_G24A 0x864CFBu
/* g24B(D) = D^24+D^23+D^6+D^5+D+1 */
#define OR_G24B 0x800063u

uint32_t or_crc24(const uint8_t *bits, int64_t n, int which)
{
    uint32_t g;
    if (which == OR_CRC24A) g = OR_G24A;
    else if (which == OR_CRC24B) g = OR_G24B;
    else return 0xFFFFFFFFu;
    /* Long division of M(D) * D^24 by g(D): shift one message bit in per step;
     * when the bit leaving degree 23 (xor the incoming bit) is 1, subtract g. */
    uint32_t r = 0;
    for (int64_t i = 0; i < n; ++i) {
        uint32_t top = ((r >> 23) & 1u) ^ (uint32_t)(bits[i] & 1u);
        r = (r << 1) & 0xFFFFFFu;
        if (top) r ^= g;
    }
    return r;
}

/* ===================================================================== */
/* Block sizes and QPP coefficients (TS 36.212 Table 5.1.3-3)             */
/* ===================================================================== */

/* {K, f1, f2}; transcribed from the standard.  The tests check that the K
 * column follows the table's step rule and that every row is a permutation. */
static const int32_t OR_QPP_TAB[OR_NUM_K][3] = {
    {40, 3, 10},      {48, 7, 12},      {56, 19, 42},     {64, 7, 16},
    {72, 7, 18},      {80, 11, 20},     {88, 5, 22},      {96, 11, 24},
    {104, 7, 26},     {112, 41, 84},    {120, 103, 90},   {128, 15, 32},
    {136, 9, 34},     {144, 17, 108},   {152, 9, 38},     {160, 21, 120},
    {168, 101, 84},   {176, 21, 44},    {184, 57, 46},    {192, 23, 48},
    {200, 13, 50},    {208, 27, 52},    {216, 11, 36},    {224, 27, 56},
    {232, 85, 58},    {240, 29, 60},    {248, 33, 62},    {256, 15, 32},
    {264, 17, 198},   {272, 33, 68},    {280, 103, 210},  {288, 19, 36},
    {296, 19, 74},    {304, 37, 76},    {312, 19, 78},    {320, 21, 120},
    {328, 21, 82},    {336, 115, 84},   {344, 193, 86},   {352, 21, 44},
    {360, 133, 90},   {368, 81, 46},    {376, 45, 94},    {384, 23, 48},
    {392, 243, 98},   {400, 151, 40},   {408, 155, 102},  {416, 25, 52},
    {424, 51, 106},   {432, 47, 72},    {440, 91, 110},   {448, 29, 168},
    {456, 29, 114},   {464, 247, 58},   {472, 29, 118},   {480, 89, 180},
    {488, 91, 122},   {496, 157, 62},   {504, 55, 84},    {512, 31, 64},
    {528, 17, 66},    {544, 35, 68},    {560, 227, 420},  {576, 65, 96},
    {592, 19, 74},    {608, 37, 76},    {624, 41, 234},   {640, 39, 80},
    {656, 185, 82},   {672, 43, 252},   {688, 21, 86},    {704, 155, 44},
    {720, 79, 120},   {736, 139, 92},   {752, 23, 94},    {768, 217, 48},
    {784, 25, 98},    {800, 17, 80},    {816, 127, 102},  {832, 25, 52},
    {848, 239, 106},  {864, 17, 48},    {880, 137, 110},  {896, 215, 112},
    {912, 29, 114},   {928, 15, 58},    {944, 147, 118},  {960, 29, 60},
    {976, 59, 122},   {992, 65, 124},   {1008, 55, 84},   {1024, 31, 64},
    {1056, 17, 66},   {1088, 171, 204}, {1120, 67, 140},  {1152, 35, 72},
    {1184, 19, 74},   {1216, 39, 76},   {1248, 19, 78},   {1280, 199, 240},
    {1312, 21, 82},   {1344, 211, 252}, {1376, 21, 86},   {1408, 43, 88},
    {1440, 149, 60},  {1472, 45, 92},   {1504, 49, 846},  {1536, 71, 48},
    {1568, 13, 28},   {1600, 17, 80},   {1632, 25, 102},  {1664, 183, 104},
    {1696, 55, 954},  {1728, 127, 96},  {1760, 27, 110},  {1792, 29, 112},
    {1824, 29, 114},  {1856, 57, 116},  {1888, 45, 354},  {1920, 31, 120},
    {1952, 59, 610},  {1984, 185, 124}, {2016, 113, 420}, {2048, 31, 64},
    {2112, 17, 66},   {2176, 171, 136}, {2240, 209, 420}, {2304, 253, 216},
    {2368, 367, 444}, {2432, 265, 456}, {2496, 181, 468}, {2560, 39, 80},
    {2624, 27, 164},  {2688, 127, 504}, {2752, 143, 172}, {2816, 43, 88},
    {2880, 29, 300},  {2944, 45, 92},   {3008, 157, 188}, {3072, 47, 96},
    {3136, 13, 28},   {3200, 111, 240}, {3264, 443, 204}, {3328, 51, 104},
    {3392, 51, 212},  {3456, 451, 192}, {3520, 257, 220}, {3584, 57, 336},
    {3648, 313, 228}, {3712, 271, 232}, {3776, 179, 236}, {3840, 331, 120},
    {3904, 363, 244}, {3968, 375, 248}, {4032, 127, 168}, {4096, 31, 64},
    {4160, 33, 130},  {4224, 43, 264},  {4288, 33, 134},  {4352, 477, 408},
    {4416, 35, 138},  {4480, 233, 280}, {4544, 357, 142}, {4608, 337, 480},
    {4672, 37, 146},  {4736, 71, 444},  {4800, 71, 120},  {4864, 37, 152},
    {4928, 39, 462},  {4992, 127, 234}, {5056, 39, 158},  {5120, 39, 80},
    {5184, 31, 96},   {5248, 113, 902}, {5312, 41, 166},  {5376, 251, 336},
    {5440, 43, 170},  {5504, 21, 86},   {5568, 43, 174},  {5632, 45, 176},
    {5696, 45, 178},  {5760, 161, 120}, {5824, 89, 182},  {5888, 323, 184},
    {5952, 47, 186},  {6016, 23, 94},   {6080, 47, 190},  {6144, 263, 480},
};

void or_k_table(int32_t out[OR_NUM_K])
{
    for (int i = 0; i < OR_NUM_K; ++i) out[i] = OR_QPP_TAB[i][0];
}

int or_k_index(int32_t K)
{
    for (int i = 0; i < OR_NUM_K; ++i)
        if (OR_QPP_TAB[i][0] == K) return i;
    return -1;
}

int or_qpp_params(int32_t K, int32_t *f1, int32_t *f2)
{
    int i = or_k_index(K);
    if (i < 0) return -1;
    *f1 = OR_QPP_TAB[i][1];
    *f2 = OR_QPP_TAB[i][2];
    return 0;
}

int or_qpp(int32_t K, int32_t *pi)
{
    int32_t f1, f2;
    if (or_qpp_params(K, &f1, &f2)) return -1;
    for (int64_t i = 0; i < K; ++i)
        pi[i] = (int32_t)(((int64_t)f1 * i + (int64_t)f2 * i * i) % K);
    return 0;
}

/* ===================================================================== */
/* Segmentation (TS 36.212 5.1.2; paper Algorithm 1, CB_MAX_SIZE = 6120)   */
/* ===================================================================== */

int or_segment(int32_t tbs, or_seg *s)
{
    if (tbs < 1 || tbs > (1 << 20)) return -1;
    const int32_t Z = 6144;
    int32_t B = tbs + 24, C, L, Bp;
    if (B <= Z) {
        L = 0;
        C = 1;
        Bp = B;
    } else {
        L = 24;
        C = (B + (Z - L) - 1) / (Z - L);
        Bp = B + C * L;
    }
    int32_t Kp = -1, Km = 0, Cp, Cm;
    for (int i = 0; i < OR_NUM_K; ++i) {
        if ((int64_t)C * OR_QPP_TAB[i][0] >= Bp) {
            Kp = OR_QPP_TAB[i][0];
            if (i > 0) Km = OR_QPP_TAB[i - 1][0];
            break;
        }
    }
    if (Kp < 0) return -1;
    if (C == 1) {
        Cp = 1;
        Km = 0;
        Cm = 0;
    } else {
        int32_t dK = Kp - Km;
        Cm = (C * Kp - Bp) / dK;
        Cp = C - Cm;
    }
    s->B = B;
    s->C = C;
    s->L = L;
    s->Kplus = Kp;
    s->Kminus = Km;
    s->Cplus = Cp;
    s->Cminus = Cm;
    s->F = Cp * Kp + Cm * Km - Bp;
    return 0;
}

int32_t or_seg_k(const or_seg *s, int32_t r)
{
    return r < s->Cminus ? s->Kminus : s->Kplus;
}

/* ===================================================================== */
/* The constituent code (TS 36.212 5.1.3.2.1)                             */
/* ===================================================================== */
/* Transfer function [1, g1(D)/g0(D)], g0 = 1 + D^2 + D^3 (feedback),
 * g1 = 1 + D + D^3 (parity).  Shift register a_{k-1}, a_{k-2}, a_{k-3}; the
 * state index is s = 4*a_{k-1} + 2*a_{k-2} + a_{k-3}.  With input u:
 *   a = u ^ a_{k-2} ^ a_{k-3},   parity z = a ^ a_{k-1} ^ a_{k-3},
 *   next state = (a, a_{k-1}, a_{k-2}).                                     */
static int or_next(int s, int u, int *z)
{
    int s1 = (s >> 2) & 1, s2 = (s >> 1) & 1, s3 = s & 1;
    int a = (u ^ s2 ^ s3) & 1;
    *z = a ^ s1 ^ s3;
    return (a << 2) | (s1 << 1) | s2;
}

/* One RSC encoder with its 3-step termination (input = feedback, so a = 0). */
static void or_rsc(const uint8_t *c, int32_t K, uint8_t *z, uint8_t tx[3], uint8_t tz[3])
{
    int s = 0, zz;
    for (int32_t k = 0; k < K; ++k) {
        s = or_next(s, c[k] & 1, &zz);
        z[k] = (uint8_t)zz;
    }
    for (int j = 0; j < 3; ++j) {
        int u = ((s >> 1) ^ s) & 1; /* a_{k-2} ^ a_{k-3} */
        s = or_next(s, u, &zz);
        tx[j] = (uint8_t)u;
        tz[j] = (uint8_t)zz;
    }
}

int or_turbo_encode_cb(const uint8_t *c, int32_t K, uint8_t *d)
{
    if (or_k_index(K) < 0) return -1;
    int32_t *pi = (int32_t *)malloc(sizeof(int32_t) * K);
    uint8_t *ci = (uint8_t *)calloc((size_t)K, 1);
    uint8_t *z1 = (uint8_t *)malloc(K), *z2 = (uint8_t *)malloc(K);
    uint8_t x1t[3], z1t[3], x2t[3], z2t[3];
    if (!pi || !ci || !z1 || !z2) {
        free(pi);
        free(ci);
        free(z1);
        free(z2);
        return -2;
    }
    or_qpp(K, pi);
    for (int32_t k = 0; k < K; ++k) ci[k] = c[pi[k]] & 1; /* c'_k = c_{pi(k)} */
    or_rsc(c, K, z1, x1t, z1t);
    or_rsc(ci, K, z2, x2t, z2t);
    const int32_t N = K + 4;
    uint8_t *d0 = d, *d1 = d + N, *d2 = d + 2 * N;
    for (int32_t k = 0; k < K; ++k) {
        d0[k] = c[k] & 1;
        d1[k] = z1[k];
        d2[k] = z2[k];
    }
    /* Termination bits, read round robin x_K z_K x_K+1 z_K+1 x_K+2 z_K+2 into
     * d0, d1, d2 (TS 36.212 5.1.3.2.2), encoder 1 first, then encoder 2. */
    d0[K] = x1t[0];     d1[K] = z1t[0];     d2[K] = x1t[1];
    d0[K + 1] = z1t[1]; d1[K + 1] = x1t[2]; d2[K + 1] = z1t[2];
    d0[K + 2] = x2t[0]; d1[K + 2] = z2t[0]; d2[K + 2] = x2t[1];
    d0[K + 3] = z2t[1]; d1[K + 3] = x2t[2]; d2[K + 3] = z2t[2];
    free(pi);
    free(ci);
    free(z1);
    free(z2);
    return 0;
}

int or_tb_encode(const uint8_t *payload, int32_t tbs, uint8_t *d_out, uint8_t *cb_bits_out)
{
    or_seg sg;
    if (or_segment(tbs, &sg)) return -1;
    const int32_t B = sg.B;
    uint8_t *b = (uint8_t *)malloc(B);
    for (int32_t i = 0; i < tbs; ++i) b[i] = payload[i] & 1;
    uint32_t pa = or_crc24(b, tbs, OR_CRC24A);
    for (int i = 0; i < 24; ++i) b[tbs + i] = (uint8_t)((pa >> (23 - i)) & 1u);
    int32_t pos = 0; /* next unread bit of b */
    int64_t doff = 0, coff = 0;
    for (int32_t r = 0; r < sg.C; ++r) {
        const int32_t K = or_seg_k(&sg, r);
        const int32_t F = r == 0 ? sg.F : 0;
        uint8_t *c = (uint8_t *)calloc(K, 1);
        int32_t n = K - sg.L - F;
        for (int32_t i = 0; i < n; ++i) c[F + i] = b[pos + i];
        pos += n;
        if (sg.C > 1) {
            /* CRC24B over the K - 24 bits before it; the leading filler zeros
             * do not change the remainder. */
            uint32_t pb = or_crc24(c, K - 24, OR_CRC24B);
            for (int i = 0; i < 24; ++i) c[K - 24 + i] = (uint8_t)((pb >> (23 - i)) & 1u);
        }
        or_turbo_encode_cb(c, K, d_out + doff);
        if (cb_bits_out) memcpy(cb_bits_out + coff, c, K);
        doff += 3 * (int64_t)(K + 4);
        coff += K;
        free(c);
    }
    free(b);
    return pos == B ? sg.C : -1;
}

/* ===================================================================== */
/* Constituent max-log-MAP decoder, exact (int64)                          */
/* ===================================================================== */
/* Branch metric of (state s, input u) at a step with LLRs (Lsa, Lp):
 *   gamma = u*Lsa + z*Lp  (the log-probability form b*L + const of the
 * positive-means-1 convention, in which both bits of a branch contribute).
 * alpha_{k+1}(s') = max over branches (s,u) -> s' of alpha_k(s) + gamma,
 * beta_k(s) = max over u of beta_{k+1}(next(s,u)) + gamma,
 * Le(k) = max over u=1 branches of (alpha_k(s) + z*Lp + beta_{k+1}(s'))
 *       - max over u=0 branches of the same.                                */

#define OR_NEG (-(((int64_t)1) << 40)) /* minus infinity; never overflows */

static int64_t or_max64(int64_t a, int64_t b) { return a > b ? a : b; }

/* beta_K from the three termination steps: beta_{K+3} = (0, -inf, ...) and
 * the ordinary backward recursion over the tail, whose systematic bits carry
 * no a-priori information.  tail = (x0, z0, x1, z1, x2, z2). */
static void or_tail_beta(const int64_t tail[6], int64_t out[8])
{
    int64_t bn[8], bk[8];
    for (int s = 0; s < 8; ++s) bn[s] = s == 0 ? 0 : OR_NEG;
    for (int j = 2; j >= 0; --j) {
        for (int s = 0; s < 8; ++s) {
            int64_t best = 0;
            for (int u = 0; u < 2; ++u) {
                int z, ns = or_next(s, u, &z);
                int64_t v = bn[ns] + u * tail[2 * j] + z * tail[2 * j + 1];
                best = u == 0 ? v : or_max64(best, v);
            }
            bk[s] = best;
        }
        memcpy(bn, bk, sizeof bn);
    }
    memcpy(out, bn, sizeof bn);
}

/* Window partition of a K-step trellis into nw windows of W = 8 ceil(K / (8 nw))
 * steps: window w covers steps [w W, min(K, (w+1) W)), so only the last one
 * may be shorter (when 8 nw divides K every window has K / nw steps).  One
 * window is the whole trellis.  Returns W, or 0 when some window would be
 * empty. */
int32_t or_win_len(int32_t K, int32_t nw)
{
    if (K < 1 || nw < 1) return 0;
    if (nw == 1) return K;
    const int32_t W = 8 * ((K + 8 * nw - 1) / (8 * nw));
    if ((int64_t)(nw - 1) * W >= K) return 0;
    return W;
}

int or_constituent(int32_t K, const int64_t *lsa, const int64_t *lp, const int64_t tail[6],
                   int32_t nw, const int64_t *a_in, const int64_t *b_in,
                   int64_t *a_out, int64_t *b_out, int64_t *le)
{
    if (nw > 1 && (!a_in || !b_in)) return -1;
    const int32_t W = or_win_len(K, nw);
    if (!W) return -1;
    int64_t(*A)[8] = malloc(sizeof(int64_t[8]) * (W + 1));
    int64_t(*Bt)[8] = malloc(sizeof(int64_t[8]) * (W + 1));
    int64_t btail[8];
    or_tail_beta(tail, btail);
    for (int32_t w = 0; w < nw; ++w) {
        const int32_t lo = w * W, n = w == nw - 1 ? K - lo : W;
        /* forward recursion */
        for (int s = 0; s < 8; ++s)
            A[0][s] = w == 0 ? (s == 0 ? 0 : OR_NEG) : a_in[w * 8 + s];
        for (int32_t i = 0; i < n; ++i) {
            const int32_t k = lo + i;
            int64_t nx[8];
            int have[8] = {0};
            for (int s = 0; s < 8; ++s)
                for (int u = 0; u < 2; ++u) {
                    int z, ns = or_next(s, u, &z);
                    int64_t v = A[i][s] + u * lsa[k] + z * lp[k];
                    nx[ns] = have[ns] ? or_max64(nx[ns], v) : v;
                    have[ns] = 1;
                }
            memcpy(A[i + 1], nx, sizeof nx);
        }
        if (a_out && w < nw - 1)
            for (int s = 0; s < 8; ++s) a_out[(w + 1) * 8 + s] = A[n][s];
        /* backward recursion */
        for (int s = 0; s < 8; ++s) Bt[n][s] = w == nw - 1 ? btail[s] : b_in[w * 8 + s];
        for (int32_t i = n - 1; i >= 0; --i) {
            const int32_t k = lo + i;
            for (int s = 0; s < 8; ++s) {
                int64_t best = 0;
                for (int u = 0; u < 2; ++u) {
                    int z, ns = or_next(s, u, &z);
                    int64_t v = Bt[i + 1][ns] + u * lsa[k] + z * lp[k];
                    best = u == 0 ? v : or_max64(best, v);
                }
                Bt[i][s] = best;
            }
        }
        if (b_out && w > 0)
            for (int s = 0; s < 8; ++s) b_out[(w - 1) * 8 + s] = Bt[0][s];
        /* extrinsic */
        for (int32_t i = 0; i < n; ++i) {
            const int32_t k = lo + i;
            int64_t m[2] = {0, 0};
            int have[2] = {0, 0};
            for (int s = 0; s < 8; ++s)
                for (int u = 0; u < 2; ++u) {
                    int z, ns = or_next(s, u, &z);
                    int64_t v = A[i][s] + z * lp[k] + Bt[i + 1][ns];
                    m[u] = have[u] ? or_max64(m[u], v) : v;
                    have[u] = 1;
                }
            le[k] = m[1] - m[0];
        }
    }
    free(A);
    free(Bt);
    return 0;
}

/* ===================================================================== */
/* The int16 twin                                                         */
/* ===================================================================== */
/* Same recursion with every metric stored in int16:
 *  - candidate sums (metric + gamma) saturate to [-32768, 32767];
 *  - a state vector is shifted so that its maximum is 0 after every step
 *    whose count from the window edge is a multiple of the recursion's
 *    period (period 2: also after steps 1 and 2), and left alone after the
 *    others.
 *    The GPU kernel shifts the recursion that runs beside the extrinsic
 *    every 2 steps and the recursion it recomputes from checkpoints every 4
 *    (forward or backward, depending on the lane), so the twin runs with
 *    the periods (4, 2) and (2, 4) for (forward, backward).  The largest
 *    extrinsic sum is then 6141 (one unshifted step) + 3 * 6141 (three) +
 *    6141 (the branch) = 30705, and a winning one is at least -32752, so no
 *    value that decides a result leaves int16 -- the twin counts any that
 *    would;
 *  - minus infinity is -32768; in window 0 the states that cannot be reached
 *    after one step (all but 0 and 4) and after two steps (odd states) are
 *    pinned back to -32768;
 *  - the extrinsic is (max over u=1 of sat(alpha + sat(beta + gamma)))
 *    - (max over u=0 of the same) - Lsa, taken modulo 2^16.
 * A saturated maximum is counted in *sat: it would change a result. */

static int16_t or_sat16(int32_t v, int *clipped)
{
    if (v > 32767) { *clipped = 1; return 32767; }
    if (v < -32768) { *clipped = 1; return -32768; }
    *clipped = 0;
    return (int16_t)v;
}

static void or16_normalise(int16_t v[8])
{
    int16_t m = v[0];
    for (int s = 1; s < 8; ++s) if (v[s] > m) m = v[s];
    for (int s = 0; s < 8; ++s) {
        int32_t t = (int32_t)v[s] - m;
        v[s] = (int16_t)(t < -32768 ? -32768 : t);
    }
}

/* Shift after step t (counted from 1 at the window edge) of a recursion
 * with the given period: period 2 also shifts after steps 1 and 2, a longer
 * period only after its multiples. */
static int or16_norm_step(int32_t t, int32_t period)
{
    return period <= 2 ? (t <= 2 || t % 2 == 0) : t % period == 0;
}

int or16_constituent(int32_t K, const int64_t *lsa, const int64_t *lp, const int64_t tail[6],
                     int32_t nw, const int64_t *a_in, const int64_t *b_in,
                     int64_t *a_out, int64_t *b_out, int64_t *le, int64_t *sat)
{
    return or16_constituent_sched(K, lsa, lp, tail, nw, a_in, b_in, a_out, b_out, le, 4, 2, sat);
}

int or16_constituent_sched(int32_t K, const int64_t *lsa, const int64_t *lp,
                           const int64_t tail[6], int32_t nw, const int64_t *a_in,
                           const int64_t *b_in, int64_t *a_out, int64_t *b_out, int64_t *le,
                           int32_t a_period, int32_t b_period, int64_t *sat)
{
    if (a_period < 1 || b_period < 1) return -1;
    if (nw > 1 && (!a_in || !b_in)) return -1;
    const int32_t W = or_win_len(K, nw);
    if (!W) return -1;
    int16_t(*A)[8] = malloc(sizeof(int16_t[8]) * (W + 1));
    int16_t(*Bt)[8] = malloc(sizeof(int16_t[8]) * (W + 1));
    int64_t bt64[8];
    int16_t btail[8];
    int64_t nsat = 0;
    int clip;
    or_tail_beta(tail, bt64); /* |value| <= 6*2047, fits int16 */
    for (int s = 0; s < 8; ++s) btail[s] = or_sat16((int32_t)bt64[s], &clip), nsat += clip;
    or16_normalise(btail);
    for (int32_t k = 0; k < K; ++k)
        if (lsa[k] < -4094 || lsa[k] > 4094 || lp[k] < -2047 || lp[k] > 2047) ++nsat;
    for (int32_t w = 0; w < nw; ++w) {
        const int32_t lo = w * W, n = w == nw - 1 ? K - lo : W;
        for (int s = 0; s < 8; ++s) {
            if (w == 0) A[0][s] = s == 0 ? 0 : -32768;
            else A[0][s] = or_sat16((int32_t)a_in[w * 8 + s], &clip), nsat += clip;
        }
        if (w > 0) or16_normalise(A[0]);
        for (int32_t i = 0; i < n; ++i) {
            const int32_t k = lo + i;
            const int16_t Ls = (int16_t)lsa[k], Lp = (int16_t)lp[k];
            int16_t nx[8];
            int32_t ex[8];
            int have[8] = {0};
            for (int s = 0; s < 8; ++s)
                for (int u = 0; u < 2; ++u) {
                    int z, ns = or_next(s, u, &z);
                    int16_t g = (int16_t)(u * Ls + z * Lp);
                    int32_t e = (int32_t)A[i][s] + g;
                    int16_t v = or_sat16(e, &clip);
                    if (!have[ns] || v > nx[ns]) nx[ns] = v;
                    if (!have[ns] || e > ex[ns]) ex[ns] = e;
                    have[ns] = 1;
                }
            for (int s = 0; s < 8; ++s) {
                int pinned = w == 0 && ((i == 0 && s != 0 && s != 4) || (i == 1 && (s & 1)));
                if (!pinned && (int32_t)nx[s] != ex[s]) ++nsat;
            }
            if (or16_norm_step(i + 1, a_period)) or16_normalise(nx);
            if (w == 0 && i == 0)
                for (int s = 0; s < 8; ++s) if (s != 0 && s != 4) nx[s] = -32768;
            if (w == 0 && i == 1)
                for (int s = 0; s < 8; ++s) if (s & 1) nx[s] = -32768;
            memcpy(A[i + 1], nx, sizeof nx);
        }
        if (a_out && w < nw - 1) {
            int16_t t[8];
            memcpy(t, A[n], sizeof t);
            or16_normalise(t);
            for (int s = 0; s < 8; ++s) a_out[(w + 1) * 8 + s] = t[s];
        }
        for (int s = 0; s < 8; ++s) {
            if (w == nw - 1) Bt[n][s] = btail[s];
            else Bt[n][s] = or_sat16((int32_t)b_in[w * 8 + s], &clip), nsat += clip;
        }
        if (w < nw - 1) or16_normalise(Bt[n]);
        for (int32_t i = n - 1; i >= 0; --i) {
            const int32_t k = lo + i;
            const int16_t Ls = (int16_t)lsa[k], Lp = (int16_t)lp[k];
            int16_t cand[8][2];
            int32_t ecand[8][2];
            /* branch candidates beta_{k+1}(next) + gamma, shared with Le */
            for (int s = 0; s < 8; ++s)
                for (int u = 0; u < 2; ++u) {
                    int z, ns = or_next(s, u, &z);
                    int16_t g = (int16_t)(u * Ls + z * Lp);
                    ecand[s][u] = (int32_t)Bt[i + 1][ns] + g;
                    cand[s][u] = or_sat16(ecand[s][u], &clip);
                }
            /* extrinsic */
            int16_t m[2] = {0, 0};
            int32_t em[2] = {0, 0};
            int have[2] = {0, 0};
            for (int s = 0; s < 8; ++s)
                for (int u = 0; u < 2; ++u) {
                    int32_t e = (int32_t)A[i][s] + cand[s][u];
                    int16_t v = or_sat16(e, &clip);
                    int32_t ee = (int32_t)A[i][s] + ecand[s][u];
                    if (!have[u] || v > m[u]) m[u] = v;
                    if (!have[u] || ee > em[u]) em[u] = ee;
                    have[u] = 1;
                }
            if ((int32_t)m[0] != em[0] || (int32_t)m[1] != em[1]) ++nsat;
            le[k] = (int16_t)(uint16_t)((uint32_t)(uint16_t)m[1] - (uint32_t)(uint16_t)m[0] -
                                        (uint32_t)(uint16_t)Ls);
            /* beta */
            int16_t nb[8];
            for (int s = 0; s < 8; ++s) {
                nb[s] = cand[s][0] > cand[s][1] ? cand[s][0] : cand[s][1];
                int32_t e = ecand[s][0] > ecand[s][1] ? ecand[s][0] : ecand[s][1];
                if ((int32_t)nb[s] != e) ++nsat;
            }
            if (or16_norm_step(n - i, b_period)) or16_normalise(nb);
            memcpy(Bt[i], nb, sizeof nb);
        }
        if (b_out && w > 0) {
            int16_t t[8];
            memcpy(t, Bt[0], sizeof t);
            or16_normalise(t);
            for (int s = 0; s < 8; ++s) b_out[(w - 1) * 8 + s] = t[s];
        }
    }
    free(A);
    free(Bt);
    if (sat) *sat += nsat;
    return 0;
}

/* ===================================================================== */
/* Turbo decoder (paper Sec. IV-B "Decoding function")                     */
/* ===================================================================== */

static int64_t or_clamp(int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : v > hi ? hi : v; }

/* Extrinsic scaling by 0.75 with truncation toward zero, then the a-priori
 * clamp.  C99 division truncates toward zero. */
static int64_t or_scale(int64_t e) { return or_clamp((3 * e) / 4, -OR_LLR_MAX, OR_LLR_MAX); }

static uint32_t or_crc_bits(const uint8_t *hard, int32_t K, int32_t F, int32_t crc)
{
    return crc == OR_CRC_NONE ? 0u : or_crc24(hard + F, K - F, crc);
}

/* ---- mutual-information stop (paper Sec. IV-B, "Decoding function") ---- */

/* Binary entropy of the error probability p = 1 / (1 + e^x) of a decision
 * on an LLR of magnitude x nats:
 *   h(p) = -(1-p) log2(1-p) - p log2(p) = log2(1 + e^-x) + p x / ln 2. */
void or_mi_table(int32_t out[OR_MI_TAB_N])
{
    for (int m = 0; m < OR_MI_TAB_N; ++m) {
        const double x = (double)m / 8.0, p = 1.0 / (1.0 + exp(x));
        const double h = -(1.0 - p) * log2(1.0 - p) - (p > 0.0 ? p * log2(p) : 0.0);
        out[m] = (int32_t)llround(32768.0 * h);
    }
}

int64_t or_mi_sum(const int64_t *L, int32_t K)
{
    int32_t T[OR_MI_TAB_N];
    or_mi_table(T);
    int64_t s = 0;
    for (int32_t k = 0; k < K; ++k) {
        const int64_t m = L[k] < 0 ? -L[k] : L[k];
        s += T[m < OR_MI_TAB_N - 1 ? m : OR_MI_TAB_N - 1];
    }
    return s;
}

int or_mi_converged(int64_t s, int64_t s_prev, int32_t it, int32_t K, int32_t eps)
{
    const int64_t thr = (int64_t)K * eps;
    const int64_t d = s - s_prev;
    return s <= thr || (it >= 2 && (d < 0 ? -d : d) <= thr);
}

static int or_params_ok(const or_params *p, int32_t K)
{
    if (!p) return 0;
    if (p->max_iters < 1 || p->max_iters > 16) return 0;
    if (p->early_stop < 0 || p->early_stop > 3 || p->mi_eps < 0 || p->mi_eps > 32768) return 0;
    const int32_t W = or_win_len(K, p->n_windows);
    if (!W || W < 8 || K - (p->n_windows - 1) * W < 8) return 0;
    return 1;
}

int or_cb_decode_ex(const int16_t *llr, int32_t K, int32_t F, int32_t crc, const or_params *p,
                    uint8_t *bits, int64_t *lapp, int32_t *ok, int32_t *iters,
                    int32_t use16, int64_t *sat_count)
{
    if (!llr || or_k_index(K) < 0 || F < 0 || F >= K) return -1;
    if (crc < OR_CRC_NONE || crc > OR_CRC24B || !or_params_ok(p, K)) return -1;
    if (crc != OR_CRC_NONE && K - F < 24) return -1;
    const int32_t N = K + 4, nw = p->n_windows;
    const int16_t *d0 = llr, *d1 = llr + N, *d2 = llr + 2 * N;
    int64_t *Ls = malloc(8 * (size_t)K), *Lp1 = malloc(8 * (size_t)K), *Lp2 = malloc(8 * (size_t)K);
    int64_t *La1 = calloc(K, 8), *La2 = malloc(8 * (size_t)K), *lsa = malloc(8 * (size_t)K);
    int64_t *Le = malloc(8 * (size_t)K), *L2 = malloc(8 * (size_t)K);
    int32_t *pi = malloc(4 * (size_t)K);
    uint8_t *hard = malloc(K);
    /* window boundary metrics per decoder: current inputs and fresh outputs */
    int64_t *ain[2], *bin[2], *aout[2], *bout[2], *zero;
    zero = calloc((size_t)nw * 8, 8);
    for (int d = 0; d < 2; ++d) {
        ain[d] = calloc((size_t)nw * 8, 8);
        bin[d] = calloc((size_t)nw * 8, 8);
        aout[d] = calloc((size_t)nw * 8, 8);
        bout[d] = calloc((size_t)nw * 8, 8);
    }
    or_qpp(K, pi);
    /* channel LLRs: clamp; the filler positions of d0/d1 are known zeros */
    for (int32_t k = 0; k < K; ++k) {
        Ls[k] = or_clamp(d0[k], -OR_LLR_MAX, OR_LLR_MAX);
        Lp1[k] = or_clamp(d1[k], -OR_LLR_MAX, OR_LLR_MAX);
        Lp2[k] = or_clamp(d2[k], -OR_LLR_MAX, OR_LLR_MAX);
        if (k < F) Ls[k] = Lp1[k] = -OR_LLR_MAX;
    }
    /* termination LLRs (x0, z0, x1, z1, x2, z2) of each encoder */
    int64_t t1[6], t2[6];
    t1[0] = d0[K];     t1[1] = d1[K];     t1[2] = d2[K];
    t1[3] = d0[K + 1]; t1[4] = d1[K + 1]; t1[5] = d2[K + 1];
    t2[0] = d0[K + 2]; t2[1] = d1[K + 2]; t2[2] = d2[K + 2];
    t2[3] = d0[K + 3]; t2[4] = d1[K + 3]; t2[5] = d2[K + 3];
    for (int j = 0; j < 6; ++j) {
        t1[j] = or_clamp(t1[j], -OR_LLR_MAX, OR_LLR_MAX);
        t2[j] = or_clamp(t2[j], -OR_LLR_MAX, OR_LLR_MAX);
    }
    int32_t it, passed = 0, done_iters = p->max_iters;
    int64_t mi_prev = 0;
    for (it = 1; it <= p->max_iters; ++it) {
        /* decoder 1: natural order */
        for (int32_t k = 0; k < K; ++k) lsa[k] = Ls[k] + La1[k];
        const int64_t *ai = p->win_init ? ain[0] : zero, *bi = p->win_init ? bin[0] : zero;
        if (use16) or16_constituent(K, lsa, Lp1, t1, nw, ai, bi, aout[0], bout[0], Le, sat_count);
        else or_constituent(K, lsa, Lp1, t1, nw, ai, bi, aout[0], bout[0], Le);
        memcpy(ain[0], aout[0], (size_t)nw * 64);
        memcpy(bin[0], bout[0], (size_t)nw * 64);
        /* interleave the scaled extrinsic into decoder 2's a-priori */
        for (int32_t k = 0; k < K; ++k) La2[k] = or_scale(Le[pi[k]]);
        /* decoder 2: interleaved systematic, parity 2 */
        for (int32_t k = 0; k < K; ++k) lsa[k] = Ls[pi[k]] + La2[k];
        ai = p->win_init ? ain[1] : zero;
        bi = p->win_init ? bin[1] : zero;
        if (use16) or16_constituent(K, lsa, Lp2, t2, nw, ai, bi, aout[1], bout[1], Le, sat_count);
        else or_constituent(K, lsa, Lp2, t2, nw, ai, bi, aout[1], bout[1], Le);
        memcpy(ain[1], aout[1], (size_t)nw * 64);
        memcpy(bin[1], bout[1], (size_t)nw * 64);
        /* de-interleave back into decoder 1; a-posteriori and hard decision */
        for (int32_t k = 0; k < K; ++k) {
            La1[pi[k]] = or_scale(Le[k]);
            L2[pi[k]] = lsa[k] + Le[k];
            hard[pi[k]] = L2[pi[k]] > 0;
        }
        passed = crc == OR_CRC_NONE ? 1 : or_crc_bits(hard, K, F, crc) == 0;
        int stop = (p->early_stop & 1) && crc != OR_CRC_NONE && passed;
        if (p->early_stop & 2) {
            const int64_t mi = or_mi_sum(L2, K);
            stop = stop || or_mi_converged(mi, mi_prev, it, K, p->mi_eps);
            mi_prev = mi;
        }
        if (stop) {
            done_iters = it;
            break;
        }
    }
    if (bits) memcpy(bits, hard, K);
    if (lapp) memcpy(lapp, L2, 8 * (size_t)K);
    if (ok) *ok = passed;
    if (iters) *iters = done_iters;
    free(Ls); free(Lp1); free(Lp2); free(La1); free(La2); free(lsa); free(Le); free(L2);
    free(pi); free(hard); free(zero);
    for (int d = 0; d < 2; ++d) { free(ain[d]); free(bin[d]); free(aout[d]); free(bout[d]); }
    return 0;
}

static void or_pack_msb(const uint8_t *src, int64_t n, uint8_t *dst)
{
    for (int64_t i = 0; i < (n + 7) / 8; ++i) dst[i] = 0;
    for (int64_t i = 0; i < n; ++i)
        if (src[i] & 1) dst[i >> 3] |= (uint8_t)(0x80u >> (i & 7));
}

int or_cb_decode_batch(int32_t n_cb, const or_cb_desc *desc, const int16_t *llr,
                       const or_params *p, uint8_t *bits, uint8_t *crc_ok, uint8_t *iters)
{
    if (n_cb < 0 || (n_cb > 0 && (!desc || !llr))) return -1;
    for (int32_t i = 0; i < n_cb; ++i) {
        const or_cb_desc *d = &desc[i];
        uint8_t *hard = malloc(d->K > 0 ? d->K : 1);
        int32_t ok = 0, it = 0;
        if (or_cb_decode_ex(llr + d->llr_off, d->K, d->F, d->crc, p, hard, NULL, &ok, &it, 0, NULL)) {
            free(hard);
            return -1;
        }
        const int32_t L = d->crc == OR_CRC_NONE ? 0 : 24;
        if (bits) or_pack_msb(hard + d->F, d->K - d->F - L, bits + d->bits_off);
        if (crc_ok) crc_ok[i] = (uint8_t)ok;
        if (iters) iters[i] = (uint8_t)it;
        free(hard);
    }
    return 0;
}

int or_tb_decode(const int16_t *llr, int32_t tbs, const or_params *p, uint8_t *bits,
                 or_tb_result *res)
{
    return or_tb_decode_w(llr, tbs, p, NULL, bits, res);
}

int or_tb_decode_w(const int16_t *llr, int32_t tbs, const or_params *p, const int32_t *nw,
                   uint8_t *bits, or_tb_result *res)
{
    or_seg sg;
    if (!llr || !res || or_segment(tbs, &sg) || sg.C > 64) return -1;
    uint8_t *b = malloc(sg.B);
    int32_t pos = 0, maxit = 0;
    int64_t off = 0;
    memset(res, 0, sizeof *res);
    res->C = sg.C;
    for (int32_t r = 0; r < sg.C; ++r) {
        const int32_t K = or_seg_k(&sg, r), F = r == 0 ? sg.F : 0;
        const int32_t crc = sg.C > 1 ? OR_CRC24B : OR_CRC24A;
        uint8_t *hard = malloc(K);
        int32_t ok = 0, it = 0;
        or_params pr = *p;
        if (nw) pr.n_windows = nw[r];
        if (or_cb_decode_ex(llr + off, K, F, crc, &pr, hard, NULL, &ok, &it, 0, NULL)) {
            free(hard);
            free(b);
            return -1;
        }
        /* reassembly: drop the filler and the code block CRC */
        const int32_t n = K - F - sg.L;
        memcpy(b + pos, hard + F, n);
        pos += n;
        res->cb_ok[r] = (uint8_t)ok;
        res->cb_iters[r] = (uint8_t)it;
        if (it > maxit) maxit = it;
        off += 3 * (int64_t)(K + 4);
        free(hard);
    }
    res->tb_ok = or_crc24(b, sg.B, OR_CRC24A) == 0;
    res->max_iters_used = maxit;
    if (bits) or_pack_msb(b, tbs, bits);
    free(b);
    return 0;
}

/* ---- rate matching (TS 36.212 5.1.4.1) --------------------------------- */

/* Inter-column permutation of the 32-column sub-block interleaver. */
static const int32_t OR_SB_PERM[32] = {0,  16, 8,  24, 4,  20, 12, 28, 2,  18, 10,
                                       26, 6,  22, 14, 30, 1,  17, 9,  25, 5,  21,
                                       13, 29, 3,  19, 11, 27, 7,  23, 15, 31};

void or_subblock_perm(int32_t out[32])
{
    for (int i = 0; i < 32; ++i) out[i] = OR_SB_PERM[i];
}

int32_t or_rm_kw(int32_t K) { return 3 * 32 * ((K + 4 + 31) / 32); }

/* The circular buffer w of a code block, as indices into its [3][K+4] array
 * (stream * (K+4) + k), -1 for a <NULL>: the dummy bits that pad each
 * stream to R x 32 in front, and the filler positions of streams 0 and 1.
 * Streams 0 and 1 go through the column-permuted matrix read column by
 * column; stream 2 through pi(k) = (P[k / R] + 32 (k mod R) + 1) mod (32 R);
 * w = v0, then v1 and v2 interlaced. */
static void or_rm_buffer(int32_t K, int32_t F, int32_t *w)
{
    const int32_t D = K + 4, R = (D + 31) / 32, KP = 32 * R, ND = KP - D;
    for (int32_t i = 0; i < 3; ++i)
        for (int32_t k = 0; k < KP; ++k) {
            int32_t y; /* position in y (row-major matrix of R x 32) */
            if (i < 2) {
                const int32_t col = k / R, row = k % R;
                y = row * 32 + OR_SB_PERM[col];
            } else {
                y = (OR_SB_PERM[k / R] + 32 * (k % R) + 1) % KP;
            }
            int32_t idx = -1;
            if (y >= ND) {
                const int32_t dk = y - ND; /* index into d(i) */
                if (!(i < 2 && dk < F)) idx = i * D + dk;
            }
            const int32_t pos = i == 0 ? k : KP + 2 * k + (i - 1);
            w[pos] = idx;
        }
}

int32_t or_rm_k0(int32_t K, int32_t Ncb, int32_t rv)
{
    const int32_t R = (K + 4 + 31) / 32;
    return R * (2 * ((Ncb + 8 * R - 1) / (8 * R)) * rv + 2);
}

/* Bit selection: the E positions (indices into [3][K+4]) that rv transmits,
 * in transmission order, reading the buffer circularly from k0 over its
 * first Ncb entries and skipping <NULL>s.  Returns 0, -1 on bad arguments. */
static int or_rm_select(int32_t K, int32_t F, int32_t E, int32_t rv, int32_t Ncb, int32_t *sel)
{
    const int32_t Kw = or_rm_kw(K);
    if (or_k_index(K) < 0 || F < 0 || F >= K || E < 0 || rv < 0 || rv > 3 || Ncb < 1 ||
        Ncb > Kw)
        return -1;
    int32_t *w = malloc(sizeof(int32_t) * Kw);
    or_rm_buffer(K, F, w);
    int32_t nn = 0;
    for (int32_t j = 0; j < Ncb; ++j) nn += w[j] >= 0;
    if (nn == 0 && E > 0) {
        free(w);
        return -1;
    }
    const int32_t k0 = or_rm_k0(K, Ncb, rv);
    for (int32_t k = 0, j = 0; k < E; ++j) {
        const int32_t v = w[(k0 + j) % Ncb];
        if (v >= 0) sel[k++] = v;
    }
    free(w);
    return 0;
}

int or_rate_match(const uint8_t *d, int32_t K, int32_t F, int32_t E, int32_t rv, int32_t Ncb,
                  uint8_t *e)
{
    int32_t *sel = malloc(sizeof(int32_t) * (E > 0 ? E : 1));
    const int rc = or_rm_select(K, F, E, rv, Ncb, sel);
    if (rc == 0)
        for (int32_t k = 0; k < E; ++k) e[k] = d[sel[k]];
    free(sel);
    return rc;
}

int or_derate_match(const int16_t *e, int32_t E, int32_t K, int32_t F, int32_t rv, int32_t Ncb,
                    int16_t *soft)
{
    int32_t *sel = malloc(sizeof(int32_t) * (E > 0 ? E : 1));
    const int rc = or_rm_select(K, F, E, rv, Ncb, sel);
    if (rc == 0)
        for (int32_t k = 0; k < E; ++k) {
            /* soft combining in transmission order, saturating at int16 */
            int32_t v = (int32_t)soft[sel[k]] + e[k];
            soft[sel[k]] = (int16_t)(v > 32767 ? 32767 : v < -32767 ? -32767 : v);
        }
    free(sel);
    return rc;
}
