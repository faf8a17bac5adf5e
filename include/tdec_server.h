/*
 * tdec_server.h -- serving loop of libtdec (C ABI).
 *
 * The GPU counterpart of the paper's channel coding thread pool (Sec. IV-B
 * "Thread-pool", Sec. IV-C "Queuing principles", Algorithms 1 and 2): every
 * TTI a batch of transport blocks arrives; the paper queues their code blocks
 * and lets free cores pick them up in FIFO order, each running a whole decode
 * without preemption.  Here a native dispatcher thread takes everything that
 * is waiting and decodes it as one persistent launch (code block parallelism
 * inside the launch, as in the paper's finest granularity), without waiting
 * for the launches already running: up to max_inflight launches are in
 * flight at once, each on a lane of its own (a decoder context with its own
 * workspace, a stream, mapped result staging).  The next batch is taken and
 * enqueued while the launch before it still runs (once that launch is
 * predicted to end within a quarter of its length, at most 200 us), with no
 * host round trip between the two on the device.  Behind a launch of at
 * most 256 transport blocks, its work groups take the compute units as the
 * finishing launch's work groups leave them (its persistent grid leaves
 * free the few slots that the finishing launch's transport block assembly
 * needs); behind a larger launch its decode kernel waits on the device for
 * that launch's assembly.  A completer thread hands each launch's bits and
 * flags back in host memory as soon as it finishes, in any order.  The paper's performance captor (Sec. IV-D) becomes the per-TB
 * latency record: arrival to results in host memory, with p50/p99 and the
 * count of deadline misses.
 *
 * Admission happens at submission:
 *   - budget: the TB's LLRs must fit in the server's device-resident slot
 *     arena (hbm budget); otherwise it is rejected (TDEC_SERVE_REJ_BUDGET);
 *   - deadline: with admission bit TDEC_ADMIT_DEADLINE set, a TB whose
 *     predicted completion (the work in flight and queued ahead of it plus
 *     its own decode, from a service-time model learned from past launches)
 *     lies beyond its arrival plus 0.9 deadline_us is rejected
 *     (TDEC_SERVE_REJ_DEADLINE); the last tenth is a guard against the
 *     prediction's error.  An idle server admits any block.  A TB that is
 *     admitted and still finishes late counts as a deadline miss.
 * Admitted TBs have their LLRs copied asynchronously into their slot on a
 * copy stream; the decode launch waits for those copies on the device.
 *
 * Threading: submit, poll and stats may be called from any host thread (the
 * server serialises them); the server's threads are the only users of the
 * decoder context it was given, which must not be used by anyone else while
 * the server exists (lanes past the first get contexts the server creates
 * with the same workspace budget and window choices, so tune the context's
 * windows before creating the server).
 *
 * Ring mode (TDEC_SERVE_RING): the dispatcher does not launch a decode
 * kernel per batch.  One persistent decode kernel stays resident while work
 * arrives, and every batch is appended to a work ring in pinned host memory
 * as it is taken (up to max_inflight batches in flight): the batch is
 * planned, its plan uploaded, and its work items (1-64 code blocks of one
 * size each) published by advancing the ring's tail.  A work group of the
 * kernel that has finished an item claims the next published one through a
 * device counter, so blocks that arrive while the kernel runs start as soon
 * as a work group is free, with no launch and no host round trip between
 * them and the work already running.  Each item's work group marks it done
 * in host memory after its outputs; once all items of a batch are done the
 * completer assembles its transport blocks (a small kernel in slots the ring
 * kernel leaves free) and hands the results back.  Every wait of the kernel
 * is bounded: a work group with nothing to claim leaves after ring_idle_us,
 * or at once when the server is destroyed, and the kernel is launched again
 * when work arrives after it has ended.  This mode decodes with window
 * boundaries from the previous iteration or none (win_init 0 or 1), without
 * the mutual-information stop, and with at most 64 windows per block (the
 * context's window choices are capped there; n_windows must be 0 or <= 64);
 * other configurations are rejected with EINVAL.
 *
 * Modelled executor: tdec_server_create_model runs the same queueing,
 * admission, batching and statistics with no device at all.  Its device runs
 * the launches' work one after another at ns_per_kbit per 1000 code block
 * bits, and no launch ends before lat_ns after it was dispatched: a launch
 * dispatched at t ends at max(t + lat_ns, max(t, end of the work before it)
 * + ns_per_kbit * K-kbits / 1000).  Every TB is reported decoded (tb_ok = 1).
 * It exists to test the scheduler and to plan capacity on a host without a
 * GPU.
 */
#ifndef TDEC_SERVER_H
#define TDEC_SERVER_H

#include <stddef.h>
#include <stdint.h>

#include "tdec.h"

#ifdef __cplusplus
extern "C" {
#endif

enum {
    TDEC_SERVE_CONTINUOUS = 0, /* decode everything waiting as one launch whenever a lane is free */
    TDEC_SERVE_PER_TB = 1,     /* one launch per TB in arrival order (the plain form, for comparison) */
    TDEC_SERVE_RING = 2        /* one persistent decode kernel fed from a work ring (see below) */
};
enum { TDEC_ADMIT_BUDGET = 1, TDEC_ADMIT_DEADLINE = 2 };
enum {
    TDEC_SERVE_DONE = 0,         /* decoded; tb_ok tells whether CRC24A passed */
    TDEC_SERVE_REJ_BUDGET = 1,   /* rejected at submission: slot arena full */
    TDEC_SERVE_REJ_DEADLINE = 2, /* rejected at submission: predicted to miss its deadline */
    TDEC_SERVE_REJ_INVALID = 3,  /* rejected at submission: tbs out of range or C > 64 */
    TDEC_SERVE_ERROR = 4         /* admitted, but its launch failed (a HIP error) */
};

typedef struct {
    size_t slot_budget_bytes; /* device bytes for resident LLR slots (0 = 1 GiB) */
    int32_t deadline_us;      /* arrival-to-results deadline (HARQ), e.g. 3000 */
    int32_t max_batch_cb;     /* most code blocks per launch (0 = 8192) */
    int32_t mode;             /* TDEC_SERVE_CONTINUOUS or TDEC_SERVE_PER_TB */
    int32_t admission;        /* OR of TDEC_ADMIT_* (the budget check is always on) */
    int64_t model_lat_ns;     /* service model prior: duration of a small launch */
    int64_t model_ns_per_kbit;/* service model prior: ns per 1000 code block bits */
    tdec_params params;       /* decoder parameters of every launch */
    int32_t max_inflight;     /* launches in flight at once, 1..8 (0 = 2; ring
                                 mode: batches in flight, 0 = 4); the per-TB
                                 mode always runs one at a time */
    int32_t ring_idle_us;     /* ring mode: the ring kernel ends once its work
                                 groups have found nothing to claim for this
                                 long (0 = 20000, at most 10^7); the next
                                 batch launches it again */
} tdec_server_cfg;

typedef struct {
    uint64_t tag;        /* the caller's tag from submission */
    int32_t tbs;         /* payload bits */
    int32_t status;      /* TDEC_SERVE_* */
    int32_t tb_ok;       /* CRC24A pass (DONE only) */
    int32_t max_iters_used;
    int32_t C;           /* code blocks */
    int32_t batch_tbs;   /* TBs in the launch that decoded it */
    int64_t t_arrive_ns; /* as given at submission (CLOCK_MONOTONIC, tdec_now_ns) */
    int64_t t_done_ns;   /* bits and flags in host memory; t_arrive_ns for rejections */
} tdec_server_result;

typedef struct {
    int64_t submitted, admitted, rej_budget, rej_deadline, rej_invalid;
    int64_t completed, tb_fail, deadline_miss, batches;
    int64_t payload_bits;      /* sum of tbs over completed TBs */
    int64_t busy_ns;           /* time with at least one launch in flight (the union
                                  of the launches' take-to-results intervals) */
    int64_t lat_p50_ns, lat_p99_ns, lat_p999_ns, lat_max_ns, lat_mean_ns; /* completed TBs */
    int64_t model_lat_ns, model_ns_per_kbit;  /* the service model as learned so far */
    int64_t slots_in_use_bytes, slots_peak_bytes;
    /* per launch, the paper's performance captor delays: pre-processing
     * (host: batch formation, plan, enqueue), coding (decode kernel), and
     * post-processing (transport block assembly, copies back, copy-out) */
    int64_t mean_pre_ns, mean_coding_ns, mean_post_ns;
    double mean_batch_tbs, mean_batch_cbs;
    int64_t ring_launches;     /* ring mode: launches of the ring kernel since creation */
    int64_t ring_grid;         /* ring mode: work groups of the ring kernel */
} tdec_serve_stats;

/* One launch of the serving loop, as the paper's performance captor
 * (Sec. IV-D) records a processed subframe: when the dispatcher took the
 * batch, the three delays, and what the batch held.  Records of launches in
 * flight at the same time overlap in time. */
typedef struct {
    int64_t t_start_ns;     /* dispatcher took the batch (tdec_now_ns clock) */
    int64_t t_end_ns;       /* results in host memory */
    int64_t pre_ns, coding_ns, post_ns; /* as in tdec_serve_stats */
    int64_t copy_ns;        /* part of post_ns spent in the copies back to host memory */
    int64_t oldest_wait_ns; /* t_start_ns minus the arrival of the batch's oldest TB */
    int32_t n_tb, n_cb;
    int64_t cb_bits;        /* sum of K over the batch's code blocks */
    int64_t copyout_ns;     /* host copy of the payload bits into the callers' buffers
                               (part of t_end_ns - t_start_ns, after post_ns) */
} tdec_launch_rec;

typedef struct tdec_server tdec_server;

/* CLOCK_MONOTONIC in nanoseconds: the time base of arrivals and completions. */
int64_t tdec_now_ns(void);

/* Create a server that decodes on `ctx` (the server allocates its slot arena
 * and staging buffers on the context's device).  EINVAL for a bad config,
 * ENOMEM when the arena cannot be allocated. */
tdec_status tdec_server_create(tdec_ctx *ctx, const tdec_server_cfg *cfg, tdec_server **out);

/* The same server with the modelled executor (no device is touched). */
tdec_status tdec_server_create_model(const tdec_server_cfg *cfg, int64_t lat_ns,
                                     int64_t ns_per_kbit, tdec_server **out);

/* Submit n transport blocks that arrived at t_arrive_ns (one TTI's batch).
 * For block i: tags[i] is returned with its result, tbs[i] its payload size,
 * h_llr[i] its tdec_tb_llr_count(tbs[i]) int16 LLRs (host memory, best
 * pinned; read asynchronously), h_bits[i] where ceil(tbs/8) payload bytes are
 * written (may be NULL).  Both buffers must stay valid until the block's
 * result has been polled.  status[i] (may be NULL) receives TDEC_SERVE_DONE
 * for admitted blocks or the rejection reason; rejected blocks also produce
 * a result.  Returns the number admitted, or a negative tdec_status. */
int32_t tdec_server_submit(tdec_server *s, int32_t n, const uint64_t *tags, const int32_t *tbs,
                           const int16_t *const *h_llr, uint8_t *const *h_bits,
                           int64_t t_arrive_ns, int32_t *status);

/* The same for LLRs already in device memory (for instance written there by
 * a demodulator running on the GPU): d_llr[i] are device pointers of the
 * context's device.  The blocks are copied into the server's slots by one
 * gather launch per 200 blocks on the copy stream, instead of one host copy
 * each; the caller's buffers must stay valid until the results are polled. */
int32_t tdec_server_submit_dev(tdec_server *s, int32_t n, const uint64_t *tags,
                               const int32_t *tbs, const int16_t *const *d_llr,
                               uint8_t *const *h_bits, int64_t t_arrive_ns, int32_t *status);

/* Load generator for measurements: submit a precomputed arrival schedule of
 * device-resident transport blocks from the calling thread, one arrival
 * batch per tick, with no interpreter or other host work between ticks.
 * Tick k is at t_first_ns + k * period_ns (tdec_now_ns clock); the thread
 * spins until each tick and submits counts[k] blocks stamped with the tick
 * as their arrival time, through tdec_server_submit_dev.  tbs, d_llr and
 * h_bits (may be NULL, and may hold NULL entries) have one entry per
 * arrival, all ticks' arrivals in order; arrival i gets tag tag_base + i.
 * late_max_ns (may be NULL): how far after its tick the latest batch went
 * in; submit_max_ns (may be NULL): the longest submission call.  Returns
 * after the last tick's submission (results are polled as usual). */
tdec_status tdec_server_replay(tdec_server *s, int32_t n_ticks, int64_t t_first_ns,
                               int64_t period_ns, const int32_t *counts, const int32_t *tbs,
                               const int16_t *const *d_llr, uint8_t *const *h_bits,
                               uint64_t tag_base, int64_t *late_max_ns, int64_t *submit_max_ns);

/* Move up to `max` finished results (completion order) into out; waits up
 * to wait_us for the first one when none is ready.  Returns the count. */
int32_t tdec_server_poll(tdec_server *s, tdec_server_result *out, int32_t max, int32_t wait_us);

/* Wait until every admitted block has completed (or timeout_ms passed:
 * then EBUSY). */
tdec_status tdec_server_drain(tdec_server *s, int32_t timeout_ms);

/* Counters and latency percentiles of completed blocks since creation (or
 * the last reset). */
tdec_status tdec_server_stats(tdec_server *s, tdec_serve_stats *out);
void tdec_server_reset_stats(tdec_server *s);

/* Copy the records of the most recent launches, oldest first, into out
 * (at most max; the server keeps the last 4096 since creation or the last
 * tdec_server_reset_stats).  Returns the count, or a negative tdec_status. */
int32_t tdec_server_launches(tdec_server *s, tdec_launch_rec *out, int32_t max);

/* Drain, stop the server's threads and free its device memory and contexts. */
void tdec_server_destroy(tdec_server *s);

#ifdef __cplusplus
}
#endif
#endif
