// tables.cpp -- code block sizes, QPP coefficients, segmentation and CRC
// shift tables of libtdec (host side).
//
// Code block sizes and QPP coefficients: TS 36.212 Table 5.1.3-3.  The sizes
// follow the table's step rule (40..512 step 8, 528..1024 step 16,
// 1056..2048 step 32, 2112..6144 step 64); f1/f2 are listed per table row.
// Segmentation: TS 36.212 5.1.2 (Z = 6144), which is the rule behind the
// paper's Algorithm 1 cap of 6120 payload bits per code block.
#include <algorithm>
#include <cmath>

#include "tdec_internal.h"

namespace tdec {

static const int16_t kF1[kNumK] = {
    3,   7,   19,  7,   7,   11,  5,   11,  7,   41,  103, 15,  9,   17,  9,   21,  101, 21,  57,
    23,  13,  27,  11,  27,  85,  29,  33,  15,  17,  33,  103, 19,  19,  37,  19,  21,  21,  115,
    193, 21,  133, 81,  45,  23,  243, 151, 155, 25,  51,  47,  91,  29,  29,  247, 29,  89,  91,
    157, 55,  31,  17,  35,  227, 65,  19,  37,  41,  39,  185, 43,  21,  155, 79,  139, 23,  217,
    25,  17,  127, 25,  239, 17,  137, 215, 29,  15,  147, 29,  59,  65,  55,  31,  17,  171, 67,
    35,  19,  39,  19,  199, 21,  211, 21,  43,  149, 45,  49,  71,  13,  17,  25,  183, 55,  127,
    27,  29,  29,  57,  45,  31,  59,  185, 113, 31,  17,  171, 209, 253, 367, 265, 181, 39,  27,
    127, 143, 43,  29,  45,  157, 47,  13,  111, 443, 51,  51,  451, 257, 57,  313, 271, 179, 331,
    363, 375, 127, 31,  33,  43,  33,  477, 35,  233, 357, 337, 37,  71,  71,  37,  39,  127, 39,
    39,  31,  113, 41,  251, 43,  21,  43,  45,  45,  161, 89,  323, 47,  23,  47,  263};

static const int16_t kF2[kNumK] = {
    10,  12,  42,  16,  18,  20,  22,  24,  26,  84,  90,  32,  34,  108, 38,  120, 84,  44,  46,
    48,  50,  52,  36,  56,  58,  60,  62,  32,  198, 68,  210, 36,  74,  76,  78,  120, 82,  84,
    86,  44,  90,  46,  94,  48,  98,  40,  102, 52,  106, 72,  110, 168, 114, 58,  118, 180, 122,
    62,  84,  64,  66,  68,  420, 96,  74,  76,  234, 80,  82,  252, 86,  44,  120, 92,  94,  48,
    98,  80,  102, 52,  106, 48,  110, 112, 114, 58,  118, 60,  122, 124, 84,  64,  66,  204, 140,
    72,  74,  76,  78,  240, 82,  252, 86,  88,  60,  92,  846, 48,  28,  80,  102, 104, 954, 96,
    110, 112, 114, 116, 354, 120, 610, 124, 420, 64,  66,  136, 420, 216, 444, 456, 468, 80,  164,
    504, 172, 88,  300, 92,  188, 96,  28,  240, 204, 104, 212, 192, 220, 336, 228, 232, 236, 120,
    244, 248, 168, 64,  130, 264, 134, 408, 138, 280, 142, 480, 146, 444, 120, 152, 462, 234, 158,
    80,  96,  902, 166, 336, 170, 86,  174, 176, 178, 120, 182, 184, 186, 94,  190, 480};

int32_t k_of_index(int i)
{
    if (i < 60) return 40 + 8 * i;
    if (i < 92) return 528 + 16 * (i - 60);
    if (i < 124) return 1056 + 32 * (i - 92);
    return 2112 + 64 * (i - 124);
}

int k_index(int32_t K)
{
    int i;
    if (K >= 40 && K <= 512 && K % 8 == 0) i = (K - 40) / 8;
    else if (K >= 528 && K <= 1024 && K % 16 == 0) i = 60 + (K - 528) / 16;
    else if (K >= 1056 && K <= 2048 && K % 32 == 0) i = 92 + (K - 1056) / 32;
    else if (K >= 2112 && K <= 6144 && K % 64 == 0) i = 124 + (K - 2112) / 64;
    else return -1;
    return i;
}

void qpp_coeffs(int i, int32_t *f1, int32_t *f2)
{
    *f1 = kF1[i];
    *f2 = kF2[i];
}

int segment(int32_t tbs, int32_t seg[8])
{
    if (tbs < 1 || tbs > (1 << 20)) return -1;
    const int32_t Z = 6144;
    const int32_t B = tbs + 24;
    int32_t C, L;
    if (B <= Z) {
        C = 1;
        L = 0;
    } else {
        L = 24;
        C = (B + Z - L - 1) / (Z - L);
    }
    const int32_t Bp = B + C * L;
    // smallest table size K+ with C * K+ >= B': round ceil(B' / C) up to the
    // table's step at that size
    const int32_t t = (Bp + C - 1) / C;
    int32_t Kp;
    if (t <= 40) Kp = 40;
    else if (t <= 512) Kp = (t + 7) & ~7;
    else if (t <= 1024) Kp = std::max(528, (t + 15) & ~15);
    else if (t <= 2048) Kp = std::max(1056, (t + 31) & ~31);
    else if (t <= 6144) Kp = std::max(2112, (t + 63) & ~63);
    else return -1;
    const int ip = k_index(Kp);
    int32_t Km = 0, Cm = 0, Cp = 1;
    if (C > 1) {
        Km = k_of_index(ip - 1);
        Cm = (C * Kp - Bp) / (Kp - Km);
        Cp = C - Cm;
    }
    seg[0] = B;
    seg[1] = C;
    seg[2] = L;
    seg[3] = Kp;
    seg[4] = Km;
    seg[5] = Cp;
    seg[6] = Cm;
    seg[7] = Cp * Kp + Cm * Km - Bp;
    return 0;
}

void crc_shift_table(uint32_t poly, uint32_t *out, int n)
{
    // x^0 = 1; x^(m+1) = x * x^m mod g (shift, reduce when degree 24 appears)
    uint32_t v = 1;
    for (int m = 0; m < n; ++m) {
        out[m] = v;
        v <<= 1;
        if (v & 0x1000000u) v = (v ^ poly) & 0xFFFFFFu;
    }
}

void crc_x32_table(uint32_t poly, uint32_t *out, int n)
{
    // x^(32(j+1)) = x^32 * x^(32j) mod g: 32 reduced shifts per entry
    uint32_t v = 1;
    for (int j = 0; j < n; ++j) {
        out[j] = v;
        for (int k = 0; k < 32; ++k) {
            v <<= 1;
            if (v & 0x1000000u) v = (v ^ poly) & 0xFFFFFFu;
        }
    }
}

// Entropy table of the mutual-information stop (paper Sec. IV-B, decoding
// function).  A hard decision on an LLR of magnitude x nats errs with
// probability p = 1 / (1 + e^x); the table holds its binary entropy
// h(p) = -p log2 p - (1 - p) log2 (1 - p) in units of 2^-15 bit for x = m / 8
// (the decoder's LLR unit).  1 - (sum of h over a block's a-posteriori values)
// / K estimates the block's average mutual information (Land and Hoeher's
// estimator for consistent LLRs, which needs no reference bits).
void mi_table(uint32_t *out)
{
    for (int m = 0; m < kMiTabN; ++m) {
        const double x = m / 8.0;
        const double p = 1.0 / (1.0 + std::exp(x)), q = 1.0 - p;
        double h = -q * std::log2(q);
        if (p > 0.0) h -= p * std::log2(p);
        out[m] = (uint32_t)std::lround(32768.0 * h);
    }
}

// Rate matching circular buffer (TS 36.212 5.1.4.1).  Each of the three
// streams (D = K + 4 bits) is written row by row into an R x 32 matrix after
// 32R - D leading <NULL>s; streams 0 and 1 are read column by column in the
// column order given by 5-bit bit reversal, stream 2 through
// (col(k / R) + 32 (k mod R) + 1) mod 32R.  The buffer holds stream 0, then
// streams 1 and 2 alternating.  Filler bits of streams 0 and 1 are <NULL>.
static int32_t bitrev5(int32_t c)
{
    int32_t r = 0;
    for (int b = 0; b < 5; ++b) r |= ((c >> b) & 1) << (4 - b);
    return r;
}

int32_t rm_buffer(int32_t K, int32_t F, int32_t *w)
{
    const int32_t D = K + 4, rows = (D + 31) / 32, cols = 32, kp = rows * cols, pad = kp - D;
    for (int32_t k = 0; k < kp; ++k) {
        const int32_t col = k / rows, row = k - col * rows;
        const int32_t m01 = row * cols + bitrev5(col);               // streams 0 and 1
        const int32_t m2 = (bitrev5(col) + cols * row + 1) % kp;     // stream 2
        const int32_t j01 = m01 - pad, j2 = m2 - pad;
        w[k] = (j01 >= F) ? j01 : -1;                                  // j01 < 0 is a dummy
        w[kp + 2 * k] = (j01 >= F) ? D + j01 : -1;
        w[kp + 2 * k + 1] = (j2 >= 0) ? 2 * D + j2 : -1;
    }
    return 3 * kp;
}

}  // namespace tdec
