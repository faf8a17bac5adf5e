/*
 * oracle.h -- plain CPU reference of the LTE turbo decoding path.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the oracle that the GPU decoder
 * is checked against.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the product path never does.
 * It shares no source with the GPU library (its own tables, its own trellis,
 * its own CRC), so that agreement between the two means something.
 *
 * What it computes (citations are to the paper "Higher aggregation of
 * gNodeBs in Cloud-RAN architectures via parallel computing", Sec. IV-B
 * "Encoding function" / "Decoding function", and to 3GPP TS 36.212 for the
 * constants the paper leaves out):
 *   - CRC24A / CRC24B attach and check (TS 36.212 5.1.1)
 *   - code block segmentation with filler bits (TS 36.212 5.1.2; the paper's
 *     Algorithm 1 splits a TB into code blocks of at most 6120 payload bits)
 *   - the QPP interleaver (TS 36.212 5.1.3.2.3)
 *   - the rate-1/3 turbo encoder: two 8-state RSC encoders with trellis
 *     termination (paper Sec. IV-B "Encoding function", Fig. 3)
 *   - the iterative turbo decoder: decoder 1 -> extrinsic -> interleave ->
 *     decoder 2 -> de-interleave -> decoder 1 ..., max-log-MAP constituent
 *     decoders, hard decision, CRC check (paper Sec. IV-B "Decoding function",
 *     Fig. 4)
 *
 * Fixed-point contract (exact integer arithmetic, clamps only where named):
 *   channel LLR   Lc = clamp(x, -2047, 2047)            (units of 1/8 nat)
 *   a-priori      La = clamp(trunc(3*Le/4), -2047, 2047) (extrinsic scale 0.75)
 *   LLR sign      positive means bit 1 (paper: log P(1)/P(0))
 *   hard decision bit = 1 iff L > 0
 * The decoder core runs in int64 with -2^40 standing for minus infinity, so
 * nothing saturates.  A second build of the constituent decoder (the "int16
 * twin") stores every metric in int16 with saturating adds, renormalises the
 * state metrics, and counts any saturation of a value that decides a result;
 * the tests require both to agree bit for bit.
 *
 * Pins (tests/test_oracle_*.py): CRC check values of the public catalogue,
 * polynomial long division, linearity; the K step rule; worked segmentation
 * examples and invariants; QPP bijection, recurrence form and two spot values;
 * the encoder's impulse response and parity identity; the constituent decoder
 * against brute force over all codewords; window plumbing against full
 * length; the int16 twin against the exact build; noiseless round trip and
 * codeword-translation symmetry of the full decoder.
 * Parity unpinned (conformance of constants only): the full table of QPP
 * coefficients and the order of the 12 tail bits follow TS 36.212 as recalled
 * here; no copy of the standard is at hand to check them against, so a
 * consistent misreading shared by encoder and decoder would pass every test.
 */
#ifndef TDEC_ORACLE_H
#define TDEC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_CRC_NONE = 0, OR_CRC24A = 1, OR_CRC24B = 2 };

#define OR_LLR_MAX 2047
#define OR_NUM_K 188

/* ---- CRC (TS 36.212 5.1.1) -------------------------------------------- */
/* Remainder of bits[0..n-1] * D^24 modulo g24A / g24B, MSB (first bit) first,
 * initial value 0, no reflection, no final XOR.  bits[] holds one bit per
 * byte (0/1).  Appending the 24 returned bits (MSB first) to the message
 * gives a word whose remainder is 0.  Returns 0xFFFFFFFF for a bad `which`. */
uint32_t or_crc24(const uint8_t *bits, int64_t n, int which);

/* ---- block sizes, segmentation, QPP ------------------------------------ */
/* The 188 code block sizes K (TS 36.212 Table 5.1.3-3), ascending. */
void or_k_table(int32_t out[OR_NUM_K]);
/* Index of K in that table, or -1. */
int or_k_index(int32_t K);
/* QPP coefficients for K; returns 0 on success, -1 if K is not a table size. */
int or_qpp_params(int32_t K, int32_t *f1, int32_t *f2);
/* pi[i] = (f1*i + f2*i*i) mod K for i < K, computed in 64-bit. */
int or_qpp(int32_t K, int32_t *pi);

typedef struct {
    int32_t B, C, L, Kplus, Kminus, Cplus, Cminus, F;
} or_seg;
/* Segmentation of a transport block of `tbs` payload bits (CRC24A is added
 * here, so B = tbs + 24).  Returns 0, or -1 when tbs < 1 or tbs > 1<<20. */
int or_segment(int32_t tbs, or_seg *out);
/* Size of code block r (the K- blocks come first). */
int32_t or_seg_k(const or_seg *s, int32_t r);

/* ---- encoder (support: builds test inputs) ------------------------------ */
/* Turbo-encode one code block c[0..K-1] (filler bits, if any, are the first F
 * entries and must be 0).  d is [3][K+4] (d0 systematic, d1 parity 1,
 * d2 parity 2, trellis termination at indices K..K+3 of each stream).
 * Returns 0, -1 if K is not a table size, or -2 if an allocation fails. */
int or_turbo_encode_cb(const uint8_t *c, int32_t K, uint8_t *d);

/* Transport block encoder: attaches CRC24A to payload[0..tbs-1], segments,
 * attaches CRC24B per block when C > 1, inserts F zero filler bits at the
 * start of block 0 and encodes every block.  d_out receives the blocks'
 * [3][K_r+4] arrays one after the other (K- blocks first); cb_bits_out, if
 * not NULL, receives every block's K_r input bits one after the other.
 * Returns the number of code blocks, or -1 on bad input. */
int or_tb_encode(const uint8_t *payload, int32_t tbs, uint8_t *d_out, uint8_t *cb_bits_out);

/* ---- decoder ------------------------------------------------------------ */
typedef struct {
    int32_t max_iters;   /* 1..16 */
    int32_t early_stop;  /* bit 0: stop after the first full iteration whose CRC passes;
                            bit 1: stop once the average mutual information of the
                            a-posteriori values has converged (or_mi_converged) */
    int32_t n_windows;   /* >= 1, divides K, K/n_windows >= 8; 1 = full length */
    int32_t win_init;    /* 1: window boundaries start from the previous iteration's metrics */
    int32_t mi_eps;      /* convergence threshold of the mutual-information stop, in
                            2^-15 bit per code block bit, 0..32768 */
} or_params;

/* ---- mutual-information stop (paper Sec. IV-B, "Decoding function") ----
 * The paper stops the iterations when the average mutual information of the
 * LLRs converges.  Its estimate here is the estimator of Land, Hoeher et al.
 * for consistent LLRs that needs no reference bits:
 *   I = 1 - mean_k h(p_k),  p_k = 1 / (1 + e^|L_k|)  (L in nats),
 * h the binary entropy function and p_k the error probability of the hard
 * decision on L_k.  In integers, with L in the decoder's unit of 1/8 nat:
 *   T[m] = round(2^15 h(1 / (1 + e^(m/8)))) for m < OR_MI_TAB_N, 0 beyond
 *          (T[m] is 0 well before m = OR_MI_TAB_N - 1);
 *   S    = sum over the K a-posteriori values of T[min(|L_k|, OR_MI_TAB_N-1)],
 *          so that 1 - I = S / (2^15 K). */
#define OR_MI_TAB_N 128
void or_mi_table(int32_t out[OR_MI_TAB_N]);
int64_t or_mi_sum(const int64_t *L, int32_t K);
/* Convergence after full iteration `it` (1-based) with sums s (this
 * iteration) and s_prev (the one before): 1 - I within eps of 1, or a change
 * of at most eps since the previous iteration (both per bit):
 *   s <= K eps  or  (it >= 2 and |s - s_prev| <= K eps). */
int or_mi_converged(int64_t s, int64_t s_prev, int32_t it, int32_t K, int32_t eps);

/* One constituent max-log-MAP pass (exact, int64).
 *   lsa[k] = Ls[k] + La[k], lp[k] parity LLR, k < K;
 *   tail[6] = (x0, z0, x1, z1, x2, z2) termination LLRs of this encoder;
 *   nw windows of W = K/nw steps;
 *   a_in[w*8+s]  : alpha at step w*W used to start window w (w >= 1);
 *   b_in[w*8+s]  : beta at step (w+1)*W used to start window w (w <= nw-2);
 *   a_out, b_out : the values this pass computes at the same boundaries;
 *   le[k]        : extrinsic output.
 * a_in/b_in/a_out/b_out may be NULL when nw == 1.  Returns 0 or -1. */
/* Window partition: windows of W = 8 ceil(K / (8 nw)) steps (K for one
 * window), window w covering [w W, min(K, (w+1) W)), so that only the last
 * may be shorter.  Returns W, or 0 when a window would be empty. */
int32_t or_win_len(int32_t K, int32_t nw);
int or_constituent(int32_t K, const int64_t *lsa, const int64_t *lp, const int64_t tail[6],
                   int32_t nw, const int64_t *a_in, const int64_t *b_in,
                   int64_t *a_out, int64_t *b_out, int64_t *le);

/* The int16 twin of or_constituent: identical interface, metrics stored in
 * int16 with saturating candidate adds and renormalisation.  *sat_count is
 * increased by the number of saturated values that could decide a result.
 * The forward metric is shifted to maximum 0 after every a_period-th step
 * of a window (with period 2 also after steps 1 and 2), the backward metric
 * likewise with b_period; or16_constituent uses (4, 2). */
int or16_constituent(int32_t K, const int64_t *lsa, const int64_t *lp, const int64_t tail[6],
                     int32_t nw, const int64_t *a_in, const int64_t *b_in,
                     int64_t *a_out, int64_t *b_out, int64_t *le, int64_t *sat_count);
int or16_constituent_sched(int32_t K, const int64_t *lsa, const int64_t *lp,
                           const int64_t tail[6], int32_t nw, const int64_t *a_in,
                           const int64_t *b_in, int64_t *a_out, int64_t *b_out, int64_t *le,
                           int32_t a_period, int32_t b_period, int64_t *sat_count);

/* Decode one code block.
 *   llr      : [3][K+4] int16 channel LLRs (clamped here to +-2047; the F
 *              filler positions of d0 and d1 are ignored and taken as known 0)
 *   crc      : OR_CRC_NONE / OR_CRC24A / OR_CRC24B, checked over bits F..K-1
 *   bits     : K hard decisions, natural order, one per byte (may be NULL)
 *   lapp     : K final decoder-2 a-posteriori values in natural order (may be NULL)
 *   ok,iters : CRC pass flag (1 when crc is NONE) and iterations run
 *   use16    : 0 = exact int64 core, 1 = int16 twin core
 *   sat_count: saturation counter for the int16 core (may be NULL)
 * Returns 0, or -1 on bad arguments. */
int or_cb_decode_ex(const int16_t *llr, int32_t K, int32_t F, int32_t crc, const or_params *p,
                    uint8_t *bits, int64_t *lapp, int32_t *ok, int32_t *iters,
                    int32_t use16, int64_t *sat_count);

/* Same descriptor as the GPU library: one code block of a batch. */
typedef struct {
    int64_t llr_off;   /* element offset of this block's [3][K+4] LLR array */
    int64_t bits_off;  /* byte offset of its packed payload output */
    int32_t K;
    int16_t F;
    int8_t crc;        /* OR_CRC_NONE / OR_CRC24A / OR_CRC24B */
    int8_t rsv;
} or_cb_desc;

/* Batch form: for each block writes its payload bits F..K-L-1 (L = 24 when
 * crc != NONE), packed MSB first, at bits + bits_off, plus crc_ok and iters. */
int or_cb_decode_batch(int32_t n_cb, const or_cb_desc *desc, const int16_t *llr,
                       const or_params *p, uint8_t *bits, uint8_t *crc_ok, uint8_t *iters);

typedef struct {
    int32_t tb_ok, max_iters_used, C, rsv;
    uint8_t cb_ok[64], cb_iters[64];
} or_tb_result;

/* Transport block form: llr holds the C blocks' [3][K_r+4] arrays in order;
 * bits receives the tbs payload bits packed MSB first (ceil(tbs/8) bytes);
 * tb_ok is the CRC24A check of the reassembled block payloads. */
int or_tb_decode(const int16_t *llr, int32_t tbs, const or_params *p, uint8_t *bits,
                 or_tb_result *res);
/* The same with one window count per code block (nw[r] for block r; NULL =
 * p->n_windows for every block), as a decoder that picks windows per size
 * runs it. */
int or_tb_decode_w(const int16_t *llr, int32_t tbs, const or_params *p, const int32_t *nw,
                   uint8_t *bits, or_tb_result *res);

/* ---- rate matching (TS 36.212 5.1.4.1; the paper's puncturing, Sec. IV-B
 * "Encoding function", and the soft bits that a retransmission adds to,
 * Sec. V) ------------------------------------------------------------------ */
/* The sub-block interleaver's inter-column permutation (32 entries). */
void or_subblock_perm(int32_t out[32]);
/* Circular buffer length 3 * 32 * ceil((K+4)/32). */
int32_t or_rm_kw(int32_t K);
/* Start of redundancy version rv in a buffer of Ncb entries. */
int32_t or_rm_k0(int32_t K, int32_t Ncb, int32_t rv);
/* Transmitter: the E bits (one per byte) that redundancy version rv sends
 * from a block's [3][K+4] coded bits d (F filler bits); Ncb <= or_rm_kw(K). */
int or_rate_match(const uint8_t *d, int32_t K, int32_t F, int32_t E, int32_t rv, int32_t Ncb,
                  uint8_t *e);
/* Receiver: add the E soft values e (same order) into soft, the block's
 * [3][K+4] int16 soft buffer (HARQ combining; clear it first for a first
 * transmission), saturating at +-32767; positions never sent stay as they
 * are.  Returns 0, or -1 on bad arguments. */
int or_derate_match(const int16_t *e, int32_t E, int32_t K, int32_t F, int32_t rv, int32_t Ncb,
                    int16_t *soft);

#ifdef __cplusplus
}
#endif
#endif
