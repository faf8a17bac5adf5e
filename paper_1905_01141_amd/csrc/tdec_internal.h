// tdec_internal.h -- structures shared by the host planner and the kernels of
// libtdec.  Nothing here is part of the public C ABI (include/tdec.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tdec.h"

namespace tdec {

constexpr int kNumK = 188;
constexpr int kKmax = 6144;
constexpr int kLlrMax = 2047;
// x^n mod g for n = 0 .. kCrcTabN-1 (covers every shift a code block needs)
constexpr int kCrcTabN = kKmax + 32;
// x^(32 j) mod g24A for j = 0 .. kX32N-1 (transport blocks of up to 64 blocks)
constexpr int kX32N = 64 * kKmax / 32 + 2;
// layout of the CRC table in device memory: [x^m mod g24A][x^m mod g24B][x^(32j) mod g24A]
constexpr int kCrcTabWords = 2 * kCrcTabN + kX32N;
// mutual-information stop: entries of the entropy table, which follows the
// CRC tables in the same device buffer (one word per entry)
constexpr int kMiTabN = 128;
constexpr int kTabWords = kCrcTabWords + kMiTabN;
constexpr uint32_t kPoly24A = 0x864CFBu;  // D^24+D^23+D^18+D^17+D^14+D^11+D^10+D^7+D^6+D^5+D^4+D^3+D+1
constexpr uint32_t kPoly24B = 0x800063u;  // D^24+D^23+D^6+D^5+D+1
constexpr int kMaxSlotsPerWg = 64;        // code blocks per work group
constexpr int kMaxWgThreads = 256;
constexpr int kSeg = 8;  // trellis steps per checkpoint segment

// Host-side tables (tables.cpp).
int k_index(int32_t K);             // index in the size table or -1
int32_t k_of_index(int i);          // size of table entry i
void qpp_coeffs(int i, int32_t *f1, int32_t *f2);
int segment(int32_t tbs, int32_t seg[8]);  // B C L K+ K- C+ C- F; 0 ok, -1 range
void crc_shift_table(uint32_t poly, uint32_t *out, int n);  // out[m] = x^m mod g
void crc_x32_table(uint32_t poly, uint32_t *out, int n);    // out[j] = x^(32 j) mod g
// out[m] = round(2^15 h(1 / (1 + e^(m/8)))), m < kMiTabN, h the binary entropy
void mi_table(uint32_t *out);

// One work item of the decode kernel: `ncb` code blocks of the same size K,
// each cut into `nw` windows of W steps; lane l < ncb*nw of the work group
// runs window l % nw of block slot l / nw.
struct DecItem {
    int32_t K, nw, W, ncb;  // W: length of every window but the last (win_len)
    int32_t cb0;     // first entry of this item in the code block list
    int32_t f1, f2;  // QPP coefficients
    int32_t lds_slot;  // LDS bytes per code block slot (extrinsic array)
    int32_t qtab;      // element offset of this shape's QPP address table in DecArgs::qtab
};

// One code block of the decode kernel's list.
struct DecCb {
    int64_t llr_off;   // element offset of the [3][K+4] int16 LLRs
    int64_t bits_off;  // byte offset of the packed payload output, -1 = none
    int64_t hard_off;  // word offset of the full hard decision (TB assembly), -1 = none
    int32_t out_idx;   // index into crc_ok / iters
    int16_t F;
    int8_t crc;        // 0 none, 1 CRC24A, 2 CRC24B
    int8_t rsv;
    int32_t tb;        // index of its transport block in the plan (purge marks), -1 = none
};

// Work distribution counters of the decode kernel: kCtrSets sets of work
// groups, a claim counter and a done counter per set, each on its own
// 256-byte line.
constexpr int kCtrSets = 8;
constexpr int kCtrStride = 64;  // uint32 words
constexpr int kCtrBytes = 2 * kCtrSets * kCtrStride * 4;

// Work ring of the serving loop's ring mode.  The host appends work items
// to a ring in pinned host memory while one persistent decode kernel runs;
// its work groups claim items through a device counter and mark each item
// done in host memory once its outputs are written.
struct RingCtl {
    uint64_t tail;  // items published (written by the host, release order)
    uint32_t stop;  // set by the host: work groups leave once nothing is left to claim
    uint32_t rsv;
};
// One ring item: a work item of a plan uploaded by the host, with the device
// buffers of the context that planned it.
struct RingEntry {
    DecItem item;          // its cb0 is unused: cbs points at the item's first block
    int32_t rsv[2];
    const DecCb *cbs;      // device: the item's ncb code blocks
    const uint16_t *qtab;  // device: QPP address tables (item.qtab is an offset here)
    uint32_t *hard;        // device outputs (hard_off / out_idx of the blocks index these)
    uint8_t *crc_ok;
    uint8_t *iters;
};
// LDS bytes of the ring kernel's copy of one item: the entry, then up to
// kMaxSlotsPerWg code blocks.
constexpr int kRingCtrBytes = 384;
constexpr int kRingLdsBytes = (int)(sizeof(RingEntry) + kMaxSlotsPerWg * sizeof(DecCb) + 63) & ~63;

struct DecArgs {
    const DecItem *items;
    int32_t n_items;
    const DecCb *cbs;
    const int16_t *llr;
    uint8_t *bits;
    uint8_t *crc_ok;
    uint8_t *iters;
    uint32_t *hard;
    const uint32_t *crc_tab;  // [2][kCrcTabN]: 24A then 24B
    char *scratch;
    int64_t scratch_stride;   // bytes of global scratch per work group
    uint32_t *counter;        // kCtrSets claim counters then kCtrSets done counters, one
                              // per kCtrStride words (zero between launches)
    // QPP address tables, one per (K, windows) shape: for unit u = t4 * nw + w
    // (4 trellis steps of window w) the LDS byte offsets 2 * epad(pi(k)),
    // k = w * W + 4 * t4 + j, j = 0..3, relative to the block's slot
    const uint16_t *qtab;
    const uint32_t *mi_tab;  // kMiTabN entropy table entries (mutual-information stop)
    int32_t max_iters, early_stop, win_init, mi_eps;
    int32_t state_slots;  // most blocks of any item (size of the per-slot LDS state)
    uint32_t *tb_fail;    // per transport block failure marks (purge), null = no purge
};

// The ring kernel's further arguments (its items come from the ring, not
// DecArgs::items).
struct RingArgs {
    const RingCtl *ctl;        // host
    const RingEntry *ent;      // host, cap entries
    uint32_t *done;            // host, cap marks: item i writes i + 1 when done
    unsigned long long *head;  // device, kRingCtrBytes: [0] tickets handed out, [16] the
                               // host's tail as last seen, [32] (32 bits) its stop flag as seen
    int32_t cap;               // a power of two
    int32_t lds;               // LDS byte offset of the item copy (kRingLdsBytes)
    uint64_t idle_ticks;       // a work group that waits this many wall-clock ticks for
                               // its item gives up and leaves the kernel
};

// One transport block for the assembly kernel (after the code blocks are decoded).
struct TbItem {
    int32_t tbs, B, C, F, L;
    int32_t Kminus, Cminus, Kplus;
    int64_t hard_off;   // word offset of block 0's hard bits; block r follows at
                        // hard_off + sum_{q<r} hard_words(K_q)
    int64_t bits_off;   // byte offset of the payload output, -1 = none
    int32_t cb_idx0;    // index of block 0 in crc_ok / iters
    int32_t res_idx;    // index into the result array
};

// Words of hard-decision storage per code block: the K bits plus one spare word.
__host__ __device__ inline int64_t hard_words(int32_t K) { return (K + 31) / 32 + 1; }

// LDS layout of one code block slot of the decode kernel: the extrinsic
// array (int16, padded with 8 entries after every 128 so that windows start in
// different banks; a K = 6144 slot is 13 KB, and 12 fit a CU beside their
// state).  After decoder 2 its low bits hold the hard decisions.
__host__ __device__ inline int32_t epad(int32_t j) { return j + ((j >> 7) << 3); }
__host__ __device__ inline int32_t lds_e_bytes(int32_t K) { return ((epad(K - 1) + 1) * 2 + 15) & ~15; }
__host__ __device__ inline int32_t lds_slot_bytes(int32_t K) { return (lds_e_bytes(K) + 63) & ~63; }
// LDS bytes of the per-slot state that precedes the extrinsic arrays.
__host__ __device__ inline int32_t lds_state_bytes(int32_t slots) { return (16 * slots + 63) & ~63; }
// With the mutual-information stop, the entropy table (16-bit entries) and
// two sums per slot follow the state.
__host__ __device__ inline int32_t lds_mi_bytes(int32_t slots) { return (2 * kMiTabN + 8 * slots + 63) & ~63; }
// Window length of K steps cut into nw windows: all windows but the last
// have W = 8 ceil(K / (8 nw)) steps (K for one window), the last the rest;
// 0 when some window would be empty.
__host__ __device__ inline int32_t win_len(int32_t K, int32_t nw)
{
    if (K < 1 || nw < 1) return 0;
    if (nw == 1) return K;
    const int32_t W = 8 * ((K + 8 * nw - 1) / (8 * nw));
    return (int64_t)(nw - 1) * W < K ? W : 0;
}

// Split point of a window of W steps between its forward-first lane
// (steps [0, M)) and its backward-first lane (steps [M, W)).
__host__ __device__ inline int32_t win_split(int32_t W) { return (W / 16) * 8; }

// One code block for the encoder kernel.
struct EncCb {
    int64_t src_bit;   // bit offset of the payload in the packed source
    int64_t out_off;   // byte offset of the [3][K+4] output
    int32_t K, f1, f2;
    int16_t F;
    int8_t crc;
    int8_t rsv;
};

// One code block of a rate matching launch.
struct RmItem {
    int64_t e_off;     // element offset of its E transmitted values
    int64_t soft_off;  // element offset of its [3][K+4] soft buffer / coded bits
    int64_t tab_off;   // offset of its rank table in the context's table arena
    int32_t K, E;
    int32_t n_valid;   // non-<NULL> entries among the first Ncb of the circular buffer
    int32_t r0;        // rank of the first non-<NULL> entry at or after k0(rv)
};
// max_k: the largest K among the items (sizes the LDS staging buffer).
int launch_derate(const RmItem *items, int n, int max_k, const void *e, int e_bytes,
                  int16_t *soft, const uint16_t *tab, int combine, void *stream);
int launch_rate_match(const RmItem *items, int n, int max_k, const uint8_t *coded, uint8_t *e,
                      const uint16_t *tab, void *stream);
// Host: the circular buffer of a block as [3][K+4] indices, -1 for <NULL>
// (tables.cpp); returns its length 3 * 32 * ceil((K+4)/32).
int32_t rm_buffer(int32_t K, int32_t F, int32_t *w);

// Device-to-device staging of the serving loop: up to kGatherMax copies per
// launch, passed by value (kernel arguments stay under 4 KB).
constexpr int kGatherMax = 200;
struct GatherItem {
    const int16_t *src;  // caller's device LLRs
    uint32_t dst_blk;    // destination offset in 256-byte units from dst_base
    uint32_t n;          // int16 elements
};
struct GatherArgs {
    int32_t n;
    int16_t *dst_base;
    GatherItem it[kGatherMax];
};
int launch_gather(const GatherArgs &g, void *stream);

// Launches of ctx leave `n` resident work group slots free for the launches
// beside them (the serving loop's launch lanes): the persistent decode grid
// is at most the resident capacity minus n.  small_asm: transport block
// assembly in kAsmGrid small work groups, which fit the slots that such a
// launch leaves.
void ctx_set_launch_reserve(tdec_ctx *ctx, int n, bool small_asm);

// Ring mode of the serving loop.  A plan of transport blocks built and
// uploaded (on `st`) as for tdec_tb_decode_batch, for the ring kernel: its
// items, whose code block lists start at d_cbs + cb0, are published on the
// ring by the caller once `ready` has fired (the upload, and that of any QPP
// table the plan added, are complete then), and its transport blocks are
// assembled by ring_assemble once every item is done.  The plan stays valid
// until the context plans again.
struct RingPlan {
    const DecItem *items = nullptr;  // host copy
    int n_items = 0, n_cb = 0, n_tb = 0, asm_words = 0;
    const DecCb *d_cbs = nullptr;
    const TbItem *d_tbs = nullptr;
    int wg = 0;            // threads per work group the plan's window counts need
    int max_item_lds = 0;  // LDS bytes of the largest item's extrinsic arrays
    int64_t stride = 0;    // scratch bytes per work group of the largest item
    bool exact = false, mi = false;
    hipEvent_t ready = nullptr;
    // the planning context's device buffers, with their sizes (elements)
    const uint16_t *d_qtab = nullptr;
    int64_t qtab_entries = 0;
    uint32_t *d_hard = nullptr;
    int64_t hard_words = 0;
    uint8_t *d_ok = nullptr, *d_it = nullptr;
    int64_t flags = 0;
};
tdec_status ring_plan(tdec_ctx *ctx, int32_t n_tb, const int32_t *tbs, const int64_t *llr_off,
                      const int64_t *bits_off, const tdec_params *params, hipStream_t st,
                      RingPlan *out);
// Transport block assembly of a ring plan whose items are all done, in
// kAsmGrid small work groups (beside the resident ring kernel).
tdec_status ring_assemble(tdec_ctx *ctx, const RingPlan &r, const tdec_params *params,
                          uint8_t *d_bits, tdec_tb_result *d_res, hipStream_t st);
// Plans of ctx with at most max_nw windows per block (the ring kernel's
// work groups hold 64 windows) and items of at most lds_budget LDS bytes.
void ctx_set_ring_shape(tdec_ctx *ctx, int max_nw, int lds_budget);
// Scratch bytes per work group that covers every item such plans can hold.
int64_t ring_max_stride(int max_nw, int lds_budget);
const uint32_t *ctx_crc_tab(const tdec_ctx *ctx);
int ctx_num_cus(const tdec_ctx *ctx);

// A new context on src's device with src's workspace budget and window
// choices (the serving loop's further launch lanes, each with a workspace of
// its own so that their launches can run at the same time).
tdec_status ctx_clone(const tdec_ctx *src, tdec_ctx **out);

// The ranges tdec.h gives for every field of tdec_params (the window count
// is checked against each block size where it is used).
bool params_valid(const tdec_params *p);

// tb_decode_batch that also records ev_start (hipEvent_t, may be null) just
// before the decode kernel and ev_mid between it and the assembly kernel.
tdec_status tb_decode_batch_timed(tdec_ctx *ctx, int32_t n_tb, const int32_t *tbs,
                                  const int64_t *llr_off, const int64_t *bits_off,
                                  const int16_t *d_llr, const tdec_params *params, uint8_t *d_bits,
                                  tdec_tb_result *d_res, void *stream, void *ev_start,
                                  void *ev_mid);

// Launchers (dec_kernels.hip / enc_kernels.hip).
// uneven: some item's windows are not all of equal length (per-lane lengths)
// exact: exact window boundaries (win_init = 2)
// mi: the mutual-information stop is on (early_stop bit 1)
const void *decode_kernel_address(bool uneven, bool exact, bool mi);
int launch_decode(const DecArgs &a, bool uneven, bool exact, bool mi, int grid, int wg_threads,
                  int lds_bytes, void *stream);
// The ring kernel (uneven windows allowed, window boundaries from the
// previous iteration, no mutual-information stop), kRingWg threads per work
// group; it runs until its work groups have found nothing to claim for
// ring_idle_ticks, or the ring's stop flag is set and nothing is left.
constexpr int kRingWg = 128;
const void *ring_kernel_address();
int launch_ring_decode(const DecArgs &a, const RingArgs &r, int grid, int lds_bytes, void *stream);
// Fixed scratch of the allocation-free decode entry point (a file-scope
// device array of kStaticScratchBytes per device: kCtrBytes of claim counters,
// then per-work-group scratch).  static_scratch_init, called with `device`
// current, looks up and keeps that device's address (0 ok, -1 error);
// static_scratch_ptr returns it (null before the init).
constexpr size_t kStaticScratchBytes = TDEC_FIXED_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
int static_scratch_init(int device);
char *static_scratch_ptr(int device);
// Zero n words with a fill kernel (no memset node when the stream is captured).
int launch_zero_words(uint32_t *p, int n, void *stream);
// Work groups of the assembly launch: each takes transport blocks t, t +
// grid, ...  So few small work groups fit the compute unit slots that a
// decode launch beside them leaves free (the serving loop keeps that many
// free), and the assembly of one launch never waits for the decode of the
// next.
constexpr int kAsmGrid = 64;
// The ring kernel leaves one CU per XCD free: eight CUs hold about 14 such
// work groups each (their LDS is bounded by the largest transport block).
constexpr int kRingAsmGrid = 112;
// max_words: the largest (B + 31) / 32 of the transport blocks (LDS per work group)
// small_grid > 0: that many work groups of 128 threads (kAsmGrid beside a
// launch lane's decode, kRingAsmGrid on the CUs the ring kernel leaves
// free), each taking transport blocks in turn; 0: one work group of 256
// threads per transport block.
// tb_fail: the decode launch's failure marks (purge), a marked block fails
// without its CRC24A being checked; null = no purge.
int launch_tb_assemble(const TbItem *items, int n_tb, int max_words, const uint32_t *hard,
                       const uint8_t *crc_ok, const uint8_t *iters, const uint32_t *tb_fail,
                       const uint32_t *crc_tab, uint8_t *bits, void *res, int small_grid,
                       void *stream);
int launch_encode(const EncCb *cbs, int n_cb, const uint8_t *src, uint8_t *out,
                  const uint32_t *crc_tab, void *stream);
int launch_tb_crc_attach(const uint8_t *payload, int32_t tbs, uint8_t *stream_bits,
                         const uint32_t *crc_tab, void *stream);

}  // namespace tdec
