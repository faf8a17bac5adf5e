/*
 * tdec.h -- C ABI of the MI355X (gfx950) LTE turbo decoder library, libtdec.
 *
 * The library decodes LTE turbo code blocks and transport blocks on the GPU.
 * It implements the decoding function of the paper "Higher aggregation of
 * gNodeBs in Cloud-RAN architectures via parallel computing" (Sec. IV-B,
 * "Decoding function", Fig. 4): received data is de-multiplexed into the
 * systematic and the two parity streams; decoder 1 computes extrinsic LLRs
 * and passes them (interleaved) to decoder 2, which also takes the
 * interleaved systematic LLRs and parity 2, and feeds its extrinsic LLRs back
 * de-interleaved; the loop runs up to a maximum number of iterations and ends
 * with a hard decision.  The constituent decoders are max-log-MAP (BCJR in
 * the max-plus semiring) over the 8-state RSC trellis of TS 36.212 5.1.3.2;
 * code blocks come from the segmentation of TS 36.212 5.1.2 (the paper's
 * Algorithm 1 caps a block at 6120 payload bits) and carry CRC24B, the
 * transport block CRC24A (TS 36.212 5.1.1).  A transport block succeeds only
 * if it passes CRC24A (the paper's Algorithm 2: all code blocks must decode).
 *
 * Arithmetic contract (every result is exact; nothing is left to rounding):
 *   - input LLRs are int16 in units of 1/8 nat, positive meaning bit 1 (the
 *     paper defines the LLR as log P(1)/P(0)); values outside +-2047 are
 *     clamped, not rejected;
 *   - state metrics are int16 max-plus sums; extrinsic values are scaled by
 *     0.75 with truncation toward zero and clamped to +-2047 before they
 *     become a-priori values of the other decoder;
 *   - hard decision: bit = 1 iff the decoder-2 a-posteriori value is > 0;
 *   - windowed decoding: a code block of K bits is cut into n_windows
 *     windows that run concurrently, each of W = 8*ceil(K/(8*n_windows))
 *     trellis steps but the last, which takes the rest (W = K/n_windows when
 *     8*n_windows divides K); a window starts its forward (backward)
 *     recursion from all-zero metrics,
 *     or, with win_init = 1 and from the second iteration on, from the metric
 *     its left (right) neighbour computed at the shared boundary in the
 *     previous iteration of the same constituent decoder; window 0 always
 *     starts in state 0 and the last window always from the trellis
 *     termination; n_windows = 1 is exact full-length max-log-MAP;
 *   - exact boundaries (win_init = 2): before each constituent decoder every
 *     window computes the max-plus transfer matrices of its steps (one forward
 *     run from each of the 8 states at its start, one backward run from each
 *     state at its end) and a scan along the windows gives the full-length
 *     recursions' metrics at every window boundary, so the output equals
 *     full-length decoding (n_windows = 1) with the latency of the windows;
 *     the transfer runs cost about 8 times the window's own forward and
 *     backward work, so this is for latency-bound decodes, not throughput;
 *   - the CRC of a code block is checked over bits F..K-1 (the filler bits are
 *     known zeros) after each full iteration (CRC24B when the block belongs to
 *     a transport block of several blocks, CRC24A when it is the only one).
 *
 * Memory: "d_" arguments are device pointers (HIP device memory of the
 * context's device), every other pointer is host memory.  The caller owns
 * all input and output buffers.  The context owns a workspace allocated by
 * tdec_create; calls that fit in it allocate nothing.
 *
 * Asynchrony: calls validate their arguments on the host, enqueue work on
 * `stream` and return; outputs are valid once the stream has synchronised.
 * A context may be used by one host thread at a time and its calls must not
 * overlap in time on different streams (they share the workspace).
 *
 * Errors: on a non-zero return nothing has been enqueued and no output is
 * written.  A code block that fails its CRC is not an error: it is reported
 * through crc_ok = 0.
 */
#ifndef TDEC_H
#define TDEC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TDEC_OK = 0,
    TDEC_EINVAL = -1,  /* bad pointer, size, K, window count or parameter */
    TDEC_ERANGE = -2,  /* transport block size out of range */
    TDEC_ENOMEM = -3,  /* the call does not fit in the context's workspace */
    TDEC_EDEVICE = -4, /* a HIP runtime error (launch or copy failed) */
    TDEC_EBUSY = -5    /* reserved */
} tdec_status;

enum { TDEC_CRC_NONE = 0, TDEC_CRC24A = 1, TDEC_CRC24B = 2 };

enum { TDEC_STOP_CRC = 1, TDEC_STOP_MI = 2, TDEC_STOP_PURGE = 4 }; /* bits of tdec_params.early_stop */

/* Decoder parameters. */
typedef struct {
    int32_t max_iters;  /* 1..16 full iterations (decoder 1 + decoder 2) */
    int32_t early_stop; /* 0: run exactly max_iters; otherwise a block stops after the
                           first full iteration that meets one of the rules set:
                           TDEC_STOP_CRC: its CRC passes (blocks without CRC never stop
                             on this rule);
                           TDEC_STOP_MI: the average mutual information of its
                             a-posteriori values has converged (paper Sec. IV-B,
                             decoding function).  The estimate is
                             1 - I = (1/K) sum_k h(1 / (1 + e^|L_k|)), h the binary
                             entropy and L_k decoder 2's a-posteriori value in nats
                             (consistent-LLR estimator without reference bits), summed
                             in units of 2^-15 bit from a table over |L| in the
                             decoder's 1/8-nat unit, clipped at 127:
                             T[m] = round(2^15 h(1 / (1 + e^(m/8)))).  With S_i the
                             sum after iteration i, the block stops when
                             S_i <= K mi_eps, or i >= 2 and |S_i - S_(i-1)| <= K mi_eps.
                           crc_ok reports the CRC at the iteration the block stopped.
                           TDEC_STOP_PURGE (transport block calls only, with TDEC_STOP_MI:
                             the paper's Algorithm 2, a transport block fails when any of its
                             code blocks fails): a block that stops on a rule while its CRC
                             fails marks its transport block failed, and the block's siblings
                             still iterating stop at the end of their current iteration
                             (purged: cb_iters = 0, cb_ok = 0).  Such a transport block has
                             tb_ok = 0; its payload bits and its other blocks' flags depend
                             on timing (a sibling may finish before it sees the mark).  Code
                             block calls ignore the bit. */
    int32_t n_windows;  /* windows per code block, 1..128: every window but the last has
                           W = 8*ceil(K/(8n)) steps (K for n = 1), the last the rest, which
                           must be non-empty; 0 = the library's choice for each K
                           (tdec_pick_windows) */
    int32_t win_init;   /* 0: windows start from zero metrics every iteration;
                           1: from the neighbours' previous-iteration boundary metrics;
                           2: from the exact boundary metrics (see below): the result
                              equals n_windows = 1 for any window count */
    int32_t mi_eps;     /* threshold of TDEC_STOP_MI in 2^-15 bit per code block bit,
                           0..32768; ignored without it.  Max-log-MAP a-posteriori
                           values are overconfident, so thresholds above a few units
                           can stop blocks that still hold errors: 1 is a safe choice */
} tdec_params;

/* ---------------------------------------------------------------- host-only helpers */

/* Segmentation of a transport block of `tbs` payload bits (TS 36.212 5.1.2):
 * B = tbs + 24 (CRC24A), C code blocks, L = 24 CRC24B bits per block when
 * C > 1, Cminus blocks of Kminus bits first, then Cplus blocks of Kplus bits,
 * F filler bits at the start of block 0.  1 <= tbs <= 1<<20, else ERANGE. */
typedef struct {
    int32_t B, C, L, Kplus, Kminus, Cplus, Cminus, F;
} tdec_seg;
tdec_status tdec_segment(int32_t tbs, tdec_seg *out);

/* Number of int16 LLRs of a transport block: 3 * sum_r (K_r + 4); -1 if tbs is out of range. */
int64_t tdec_tb_llr_count(int32_t tbs);

/* The 188 code block sizes (TS 36.212 Table 5.1.3-3), ascending; returns 188. */
int32_t tdec_k_table(int32_t *out188);

/* QPP interleaver of size K (TS 36.212 5.1.3.2.3): pi[i] = (f1*i + f2*i^2) mod K;
 * writes K entries to pi (host memory) and the coefficients to f1/f2 (each may be NULL). */
tdec_status tdec_qpp(int32_t K, int32_t *pi, int32_t *f1, int32_t *f2);

/* ---------------------------------------------------------------- context */

typedef struct tdec_ctx tdec_ctx;

/* Create a context on HIP device `device`.  hbm_budget_bytes bounds the
 * workspace the context allocates (0 = 1 GiB); calls that would need more
 * return ENOMEM. */
tdec_status tdec_create(int device, size_t hbm_budget_bytes, tdec_ctx **out);
void tdec_destroy(tdec_ctx *ctx);

/* Window count the library uses for code block size K when
 * tdec_params.n_windows == 0 (always a valid count for K). */
int32_t tdec_pick_windows(const tdec_ctx *ctx, int32_t K);

/* Limit the library's window choice (tuned or built in) to at most max_nw
 * windows per code block, 1..128, or lift the limit (0): a larger choice
 * becomes the most windows <= max_nw that are valid for K.  The serving
 * loop's ring mode decodes with at most 64 (tdec_server.h).  EINVAL for a
 * value out of range. */
tdec_status tdec_set_max_windows(tdec_ctx *ctx, int32_t max_nw);

/* ---------------------------------------------------------------- decoding */

/* One code block of a batch.
 *   llr_off : element offset (int16 units) of the block's [3][K+4] LLR array
 *             in d_llr: row 0 systematic d0, row 1 parity 1 d1, row 2 parity 2
 *             d2, each with the trellis termination LLRs at indices K..K+3 in
 *             the TS 36.212 5.1.3.2.2 order (d0: x_K z_K+1 x'_K z'_K+1,
 *             d1: z_K x_K+2 z'_K x'_K+2, d2: x_K+1 z_K+2 x'_K+1 z'_K+2);
 *             the first F entries of rows 0 and 1 (filler) are ignored;
 *   bits_off: byte offset in d_bits where the block's K-F-L payload bits are
 *             written packed MSB first (L = 24 when crc != NONE, else 0);
 *   K       : code block size, one of the 188 table sizes;
 *   F       : filler bits at the start of the block, 0 <= F < K;
 *   crc     : TDEC_CRC_NONE / TDEC_CRC24A / TDEC_CRC24B (K - F >= 24 when not NONE). */
typedef struct {
    int64_t llr_off;
    int64_t bits_off;
    int32_t K;
    int16_t F;
    int8_t crc;
    int8_t rsv;
} tdec_cb_desc;

/* Decode n_cb independent code blocks in one launch.
 *   desc     : n_cb descriptors in HOST memory (the library plans the launch
 *              from them; a repeated identical batch reuses its plan);
 *   d_llr    : int16 LLRs (device);
 *   d_bits   : packed payload output (device); may be NULL;
 *   d_crc_ok : n_cb bytes, 1 if the block's CRC passed (1 for crc NONE);
 *   d_iters  : n_cb bytes, iterations run (max_iters unless it stopped early).
 * n_cb = 0 is a no-op.  EINVAL for a bad descriptor, bad parameters or a
 * window count that does not suit some K; ENOMEM if the batch needs more
 * workspace than the context holds. */
tdec_status cb_decode_batch(tdec_ctx *ctx, int32_t n_cb, const tdec_cb_desc *desc,
                            const int16_t *d_llr, const tdec_params *params, uint8_t *d_bits,
                            uint8_t *d_crc_ok, uint8_t *d_iters, void *stream);

/* cb_decode_batch for callers that cannot allocate device memory while they
 * run (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, same results, bit for bit.  The decode
 * kernel's scratch (its claim counters and per-work-group restaged inputs,
 * checkpoints and window boundaries) lives in a fixed device array of
 * TDEC_FIXED_SCRATCH_BYTES that the library's code object carries on every
 * GPU it runs on, held until the process ends; the call allocates nothing
 * (no hipMalloc, no hipFree).  The context's tables and plan slots, made by
 * tdec_create, are used as by cb_decode_batch.
 *   The array bounds how many work groups run at once (fewer than
 *   cb_decode_batch runs for large batches, so a large batch takes longer);
 *   any batch is accepted as long as one work group's scratch fits: ENOMEM
 *   when it does not (the planner keeps a work group's scratch under 256 KiB,
 *   far below the array, so valid calls do not meet it).
 *   Every call on a GPU shares that GPU's one array, whatever the context:
 *   calls whose launches overlap in time on one GPU (other streams, other
 *   threads, other contexts) race on it and give undefined results.  Each call
 *   clears the counters it needs with a fill kernel on `stream` before its
 *   decode kernel, so no state carries from one call to the next. */
#define TDEC_FIXED_SCRATCH_BYTES ((size_t)64 << 20)
tdec_status cb_decode_batch_fixed(tdec_ctx *ctx, int32_t n_cb, const tdec_cb_desc *desc,
                                  const int16_t *d_llr, const tdec_params *params,
                                  uint8_t *d_bits, uint8_t *d_crc_ok, uint8_t *d_iters,
                                  void *stream);

/* Result of one transport block (device memory, written by the decoder). */
typedef struct {
    int32_t tb_ok;          /* 1 iff the reassembled payload passes CRC24A */
    int32_t max_iters_used; /* largest iteration count over the code blocks */
    int32_t C;              /* number of code blocks */
    int32_t rsv;
    uint8_t cb_ok[64];      /* per code block CRC flag */
    uint8_t cb_iters[64];   /* per code block iteration count */
} tdec_tb_result;

/* Decode one transport block of `tbs` payload bits (C <= 64, i.e. tbs <= 391656).
 *   d_llr  : the C blocks' [3][K_r+4] LLR arrays back to back (K- blocks first),
 *            tdec_tb_llr_count(tbs) int16 values;
 *   d_bits : ceil(tbs/8) bytes, the payload packed MSB first (CRC24A removed);
 *   d_res  : one tdec_tb_result (device). */
tdec_status tb_decode(tdec_ctx *ctx, const int16_t *d_llr, int32_t tbs, const tdec_params *params,
                      uint8_t *d_bits, tdec_tb_result *d_res, void *stream);

/* Decode n_tb transport blocks in one launch.
 *   tbs, llr_off, bits_off : n_tb entries each, HOST memory: payload size,
 *                            element offset of the TB's LLRs in d_llr, byte
 *                            offset of its packed payload in d_bits;
 *   d_res                  : n_tb results (device). */
tdec_status tb_decode_batch(tdec_ctx *ctx, int32_t n_tb, const int32_t *tbs, const int64_t *llr_off,
                            const int64_t *bits_off, const int16_t *d_llr,
                            const tdec_params *params, uint8_t *d_bits, tdec_tb_result *d_res,
                            void *stream);

/* ---------------------------------------------------------------- captured launches */
/* A fixed batch, planned once and captured (with its own device copy of the
 * plan) into a HIP graph that replays the whole decode -- one persistent
 * launch for code blocks, decode + transport block assembly for transport
 * blocks -- with a single hipGraphLaunch.  It serves the case the paper's
 * scheduler is built for: every TTI brings a batch of the same shape (the
 * same cells and allocations), so the launch can be prepared once.
 *
 * The graph binds every pointer given at capture time; a replay decodes the
 * current contents of d_llr into the same outputs.  It uses the context's
 * workspace, so replays obey the context's rule: no two calls (direct or
 * replayed) of one context run at the same time.  The kernels reset their
 * own work counter, so the graph holds no memset node.  Arguments and errors
 * are those of cb_decode_batch / tb_decode_batch; ENOMEM also when the
 * plan's device copy cannot be allocated. */
typedef struct tdec_graph tdec_graph;
tdec_status tdec_graph_cb_decode(tdec_ctx *ctx, int32_t n_cb, const tdec_cb_desc *desc,
                                 const int16_t *d_llr, const tdec_params *params, uint8_t *d_bits,
                                 uint8_t *d_crc_ok, uint8_t *d_iters, tdec_graph **out);
tdec_status tdec_graph_tb_decode(tdec_ctx *ctx, int32_t n_tb, const int32_t *tbs,
                                 const int64_t *llr_off, const int64_t *bits_off,
                                 const int16_t *d_llr, const tdec_params *params, uint8_t *d_bits,
                                 tdec_tb_result *d_res, tdec_graph **out);
/* Enqueue one replay on `stream`. */
tdec_status tdec_graph_launch(tdec_graph *g, void *stream);
void tdec_graph_destroy(tdec_graph *g);

/* ---------------------------------------------------------------- autotuner */
/* Choose the window count of each code block size by measurement: for every
 * K in Ks (host array of n_k table sizes), time a batch of
 * max(1, batch_bits / K) blocks (at most 16384) at max_iters iterations
 * without early stop (the decode time does not depend on the LLR values
 * then, so the batch holds zeros) for the window counts n <= 128 whose
 * windows come closest above min_W, 1.5, 2, 3 and 4 times min_W, plus n = 1
 * and the built-in choice, and keep the fastest per decoded bit.  min_W
 * (>= 8) is the error-rate floor: shorter windows decode worse (the last
 * window of an uneven partition may be shorter; it starts from the known
 * termination).  The choice becomes what n_windows = 0 and tdec_pick_windows use on
 * this context; out_nw / out_ns_per_kbit (host, n_k entries, each may be
 * NULL) receive the choice and its time in ns per 1000 code block bits.
 * Runs on `stream` and synchronises it; allocates and frees temporary
 * device buffers. */
tdec_status tdec_autotune(tdec_ctx *ctx, int32_t n_k, const int32_t *Ks, int32_t min_W,
                          int32_t max_iters, int64_t batch_bits, int32_t *out_nw,
                          float *out_ns_per_kbit, void *stream);
/* Forget every tuned choice (back to the built-in rule): window counts and
 * the launch knobs below. */
void tdec_autotune_reset(tdec_ctx *ctx);

/* Launch knobs of a context: the planner choices that decide how one batch
 * (the paper's code block parallelism inside a TTI, Sec. IV-B, with the
 * FIFO queue of Algorithms 1 and 2 replaced by a persistent grid claiming
 * work items) is spread over the compute units.
 *   lds_budget  LDS bytes per work group the planner fills with code blocks
 *               of one size (packing: more blocks per work item use more of
 *               the work group's lanes but fewer work groups fit a compute
 *               unit); 1..163840, default 30720;
 *   order       order in which the grid claims the work items:
 *               TDEC_ORDER_K_DESC (largest blocks first, the default),
 *               TDEC_ORDER_K_ASC, or TDEC_ORDER_REQUEST (the request's own
 *               order, as the paper's FIFO queue; equal neighbours still
 *               share items);
 *   win_target  window length target of every code block size: a size K
 *               decodes in the most windows (<= 64) whose length is at least
 *               win_target (one window if K is shorter); 0 = the built-in
 *               rule; -1 = keep the per-size choices (tdec_autotune or the
 *               rule).  Applies where tdec_params.n_windows is 0.
 *   grid_cap    most work groups of a decode launch, 0 = as many as the
 *               device holds at once (the default; the batch tuner keeps
 *               it); the work groups claim the work items in turn.
 *   us          set by tdec_autotune_batch: that candidate's launch time in
 *               microseconds (ignored by tdec_set_knobs). */
enum { TDEC_ORDER_K_DESC = 0, TDEC_ORDER_K_ASC = 1, TDEC_ORDER_REQUEST = 2 };
typedef struct {
    int32_t lds_budget;
    int32_t order;
    int32_t win_target;
    int32_t grid_cap;
    float us;
} tdec_knobs;

/* The built-in knobs: {30720, TDEC_ORDER_K_DESC, 0, 0}. */
void tdec_default_knobs(tdec_knobs *out);

/* Set the knobs of a context (EINVAL when out of range: win_target must be
 * -1, 0 or 8..6144, grid_cap >= 0).  Plans made afterwards follow them; the window counts
 * win_target gives become what n_windows = 0 and tdec_pick_windows use. */
tdec_status tdec_set_knobs(tdec_ctx *ctx, const tdec_knobs *k);

/* The knobs in force (win_target reads -1: window counts are per size). */
tdec_status tdec_get_knobs(const tdec_ctx *ctx, tdec_knobs *out);

/* Choose the knobs by measurement on one representative batch of transport
 * blocks (tbs, llr_off, d_llr as for tb_decode_batch, the LLRs real ones:
 * the decode time depends on them where early stopping is on).  Every
 * combination of lds_budget in {8192, 16384, 30720, 49152, 81920}, the three
 * orders, and win_target in {-1, 0, and min_W times 1, 1.5, 2, 3, 4} (the
 * window choices only where params->n_windows is 0; min_W >= 8) decodes the
 * batch once untimed and three times timed on `stream`; the five fastest
 * and the built-in knobs are timed again, ten launches each, and the
 * fastest of those is set on the context as by tdec_set_knobs.  out (host,
 * max_out entries, may be NULL) receives every candidate timed in the first
 * pass with its time, *n_out (may be NULL) their count; *best and *rule
 * (may be NULL) the chosen knobs and the built-in knobs with their
 * second-pass times.  Synchronises `stream`; allocates and frees temporary
 * device buffers for the bits and results. */
tdec_status tdec_autotune_batch(tdec_ctx *ctx, int32_t n_tb, const int32_t *tbs,
                                const int64_t *llr_off, const int16_t *d_llr,
                                const tdec_params *params, int32_t min_W, tdec_knobs *out,
                                int32_t max_out, int32_t *n_out, tdec_knobs *best,
                                tdec_knobs *rule, void *stream);

/* ---------------------------------------------------------------- rate matching */
/* TS 36.212 5.1.4.1: the three coded streams of a block go through the
 * 32-column sub-block interleaver into a circular buffer of
 * Kw = 3 * 32 * ceil((K+4)/32) entries; redundancy version rv sends E bits
 * read circularly over the first Ncb entries from k0 = R (2 ceil(Ncb/8R) rv + 2)
 * (R = ceil((K+4)/32)), skipping the <NULL> entries (the dummy bits and the
 * filler bits of streams 0 and 1).  E below the buffer's non-<NULL> count
 * punctures (the paper's "puncturing procedure", Sec. IV-B), above it repeats.
 *
 * The receiver adds each of the E soft values to the block's [3][K+4] int16
 * soft buffer -- the decoder's input -- at the position its bit was taken
 * from, saturating at +-32767 and in transmission order.  Keeping that buffer
 * resident between transmissions is HARQ combining: a block that fails is
 * decoded again after the next redundancy version has been added (the paper's
 * retransmission of data that could not be decoded, Sec. V). */
typedef struct {
    int64_t e_off;    /* element offset of the block's E values in d_e */
    int64_t soft_off; /* element offset of its [3][K+4] soft buffer (receiver) or
                         coded bits (transmitter) */
    int32_t K;        /* one of the 188 sizes */
    int16_t F;        /* filler bits, 0 <= F < K */
    int8_t rv;        /* redundancy version 0..3 */
    int8_t rsv;
    int32_t E;        /* values sent, >= 0 */
    int32_t Ncb;      /* circular buffer length used, 1..Kw; 0 = Kw */
} tdec_rm_desc;

/* Receiver.  d_e: soft values (device), int8 (e_bytes = 1) or int16
 * (e_bytes = 2), units of 1/8 nat, positive = 1.  d_soft: int16 soft buffers
 * (device).  combine = 0 clears each block's buffer first (a first
 * transmission), 1 adds to it (a retransmission).  The buffers can be passed
 * to cb_decode_batch / tb_decode as they are (the decoder clamps to +-2047).
 * EINVAL for a bad descriptor; ENOMEM when the context's table arena is full. */
tdec_status tdec_derate_batch(tdec_ctx *ctx, int32_t n, const tdec_rm_desc *desc, const void *d_e,
                              int32_t e_bytes, int16_t *d_soft, int32_t combine, void *stream);

/* Transmitter: the E bits (one per byte, 0/1) that rv sends, from coded
 * bits in the [3][K+4] layout of cb_encode_batch (at soft_off). */
tdec_status tdec_rate_match_batch(tdec_ctx *ctx, int32_t n, const tdec_rm_desc *desc,
                                  const uint8_t *d_coded, uint8_t *d_e, void *stream);

/* ---------------------------------------------------------------- encoding */
/* The rate-1/3 turbo encoder of the paper's encoding function (Sec. IV-B,
 * Fig. 3): two RSC encoders separated by the QPP interleaver, output
 * (systematic, parity 1, parity 2) with trellis termination. */

/* Encode n_cb code blocks.  For block i, desc[i] (host memory) gives K, F and
 * crc as for decoding; its K-F-L payload bits are read packed MSB first from
 * d_payload + bits_off; the encoder puts F zero filler bits in front, appends
 * the block CRC when crc != NONE (computed over the K-24 bits before it), and
 * writes the coded bits as one byte per bit (0/1) to d_coded + llr_off in the
 * same [3][K+4] layout the decoder reads (filler positions of rows 0/1 hold 0). */
tdec_status cb_encode_batch(tdec_ctx *ctx, int32_t n_cb, const tdec_cb_desc *desc,
                            const uint8_t *d_payload, uint8_t *d_coded, void *stream);

/* Encode one transport block: CRC24A over the tbs payload bits (packed MSB
 * first), segmentation, CRC24B per block when C > 1, filler, turbo encoding.
 * d_coded receives tdec_tb_llr_count(tbs) bytes (0/1), blocks back to back. */
tdec_status tb_encode(tdec_ctx *ctx, const uint8_t *d_payload, int32_t tbs, uint8_t *d_coded,
                      void *stream);

#ifdef __cplusplus
}
#endif
#endif
