// server.cpp -- serving loop of libtdec: admission, device-resident LLR
// slots, continuous batching and the per-TB latency record (tdec_server.h).
//
// The paper runs channel decoding as jobs of a thread pool fed by a FIFO
// queue (Sec. IV-B "Thread-pool", Algorithm 1 appends the code blocks of
// every UE's transport block; Sec. IV-C, Algorithm 2 lets the next free core
// take the next job and run it to completion).  On one GPU the unit of
// dispatch is a launch, not a core: a dispatcher thread drains the queue
// into a persistent decode launch on whichever launch lane is free, without
// waiting for the launches already in flight, and a completer thread
// retires each launch the moment its events say it has finished.  Blocks
// that arrive while launches run therefore go out at once on another lane,
// and the hardware dispatcher starts their work groups as the earlier
// launches' work groups leave the compute units: the device is shared by
// every launch in flight, as the paper's cores are shared by its jobs.
#include <hip/hip_runtime.h>
#include <string.h>
#include <time.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <mutex>
#include <set>
#include <thread>
#include <vector>

#include "tdec.h"
#include "tdec_internal.h"
#include "tdec_server.h"

// the ring kernel copies ring entries and block lists word by word
static_assert(sizeof(tdec::RingEntry) % 4 == 0 && sizeof(tdec::DecCb) % 4 == 0, "word copies");

namespace {

int64_t mono_ns()
{
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (int64_t)ts.tv_sec * 1000000000LL + ts.tv_nsec;
}

// Best-fit allocator over [0, cap) bytes with coalescing of free extents;
// extents are 256-byte aligned.  Free extents are indexed by offset (for
// coalescing) and by (size, offset) (for the fit), so both calls are
// O(log extents) however fragmented the arena gets.
class Arena {
public:
    void init(int64_t cap)
    {
        cap_ = cap;
        by_off_.clear();
        by_size_.clear();
        if (cap > 0) add(0, cap);
        used_ = peak_ = 0;
    }
    int64_t alloc(int64_t n)
    {
        n = (n + 255) & ~(int64_t)255;
        auto f = by_size_.lower_bound({n, (int64_t)-1});
        if (f == by_size_.end()) return -1;
        const int64_t off = f->second, size = f->first;
        remove(off, size);
        if (size > n) add(off + n, size - n);
        used_ += n;
        peak_ = std::max(peak_, used_);
        return off;
    }
    void release(int64_t off, int64_t n)
    {
        n = (n + 255) & ~(int64_t)255;
        used_ -= n;
        auto nx = by_off_.lower_bound(off);
        if (nx != by_off_.end() && off + n == nx->first) {
            const int64_t o = nx->first, z = nx->second;
            remove(o, z);
            n += z;
        }
        nx = by_off_.lower_bound(off);
        if (nx != by_off_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == off) {
                const int64_t o = pv->first, z = pv->second;
                remove(o, z);
                off = o;
                n += z;
            }
        }
        add(off, n);
    }
    // Release many extents at once: sorted by offset, adjacent ones are
    // merged first, so a launch's slots (mostly allocated one after another)
    // cost a few index operations instead of a few per slot.  `ext` holds
    // (offset, bytes) pairs and is reordered.
    void release_many(std::vector<std::pair<int64_t, int64_t>> &ext)
    {
        if (ext.empty()) return;
        for (auto &e : ext) e.second = (e.second + 255) & ~(int64_t)255;
        std::sort(ext.begin(), ext.end());
        int64_t off = ext[0].first, n = ext[0].second;
        for (size_t i = 1; i < ext.size(); ++i) {
            if (ext[i].first == off + n) {
                n += ext[i].second;
            } else {
                release(off, n);
                off = ext[i].first;
                n = ext[i].second;
            }
        }
        release(off, n);
    }
    int64_t used() const { return used_; }
    int64_t peak() const { return peak_; }
    void reset_peak() { peak_ = used_; }
    size_t extents() const { return by_off_.size(); }

private:
    void add(int64_t off, int64_t n)
    {
        by_off_[off] = n;
        by_size_.insert({n, off});
    }
    void remove(int64_t off, int64_t n)
    {
        by_off_.erase(off);
        by_size_.erase({n, off});
    }
    std::map<int64_t, int64_t> by_off_;             // offset -> size
    std::set<std::pair<int64_t, int64_t>> by_size_;  // (size, offset)
    int64_t cap_ = 0, used_ = 0, peak_ = 0;
};

struct Pending {
    uint64_t tag;
    int32_t tbs, C;
    int64_t kbits;  // sum of K over the code blocks (bits)
    int64_t slot_off, slot_bytes;
    uint8_t *h_bits;
    int64_t t_arrive;
    uint64_t copy_seq;    // copy event that covers this block's upload
    int64_t pred_dur;     // per-TB mode: predicted launch duration counted in the queue
};

constexpr int kCopyEvents = 64;
constexpr int64_t kLaunchRing = 4096;  // launch records kept
constexpr int kMaxLanes = 8;
// Result staging: pinned host memory mapped into the device (the assembly
// kernel writes it over PCIe) and coarse-grained, so that the host reads it
// through its caches; the writes are visible to the host once the launch's
// completion event has fired (the kernel's end releases them at system scope).
constexpr unsigned kStageFlags = hipHostMallocMapped | hipHostMallocNonCoherent;

// One launch lane: a decoder context (workspace), a stream, events and
// mapped result staging of its own, so that the launches of different lanes
// can be in flight -- and run on the device -- at the same time.
struct Lane {
    tdec_ctx *ctx = nullptr;
    bool own_ctx = false;  // lanes past the first use contexts the server made
    hipStream_t st = nullptr;
    hipEvent_t ev_s = nullptr, ev_m = nullptr;  // around the decode kernel (timing)
    hipEvent_t ev_c = nullptr;                  // after the assembly kernel (timing)
    hipEvent_t done_ev = nullptr;
    // results land in mapped pinned host memory: the assembly kernel writes
    // the payload bits and per-TB records straight over PCIe (device
    // addresses hd_*), so no copy back follows the launch
    uint8_t *h_bits = nullptr, *hd_bits = nullptr;
    tdec_tb_result *h_res = nullptr, *hd_res = nullptr;
    // the launch in flight (owned by the dispatcher until `launched`, then
    // by the completer until the lane is free again)
    bool busy = false, launched = false, ok = true;
    bool small_asm = false;  // its transport blocks are assembled in kAsmGrid work groups
    std::vector<Pending> b;
    std::vector<int64_t> bo;  // byte offset of each TB's bits in h_bits
    int64_t t0 = 0, t_enq = 0, kb = 0, cbs = 0, model_end = 0;
    uint64_t seq = 0;  // dispatch order
    // ring mode: the batch's items on the ring ([ring_first, ring_first +
    // ring_n)), the first not yet seen done, and whether its assembly is
    // enqueued; t_items: when every item was seen done
    tdec::RingPlan rp;
    uint64_t ring_first = 0, ring_chk = 0;
    int ring_n = 0;
    bool items_done = true;  // every item seen done (under ring_mu)
    bool asm_enq = false;
    int64_t t_items = 0;
};

}  // namespace

struct tdec_server {
    tdec_server_cfg cfg{};
    tdec_ctx *ctx = nullptr;
    bool model = false;
    int64_t sim_lat = 0, sim_npk = 0;
    int64_t sim_busy_until = 0;  // modelled device: when its queued work ends
    int device = 0;
    // device resources
    int16_t *d_arena = nullptr;
    hipStream_t copy_st = nullptr;
    hipEvent_t copy_ev[kCopyEvents] = {};
    uint64_t copy_seq = 0;  // events recorded so far
    size_t bits_cap = 0;
    int32_t res_cap = 0;
    int n_lanes = 1;
    Lane lanes[kMaxLanes];
    std::mutex submit_mu;  // serialises submitters (held across their copies)
    // queue state (under mu)
    std::mutex mu;
    std::condition_variable cv_work, cv_done, cv_retire;
    std::deque<Pending> queue;
    std::deque<tdec_server_result> done;
    Arena arena;
    int64_t inflight = 0;       // admitted, not yet completed
    int64_t queued_kbits = 0;   // bits of code blocks waiting in the queue
    int64_t queued_dur_ns = 0;  // per-TB mode: predicted durations of the queue
    int64_t queued_cbs = 0;
    int64_t lanes_busy = 0;
    int64_t gpu_end_pred = 0;   // predicted end of the launches in flight (0 = idle)
    int64_t gpu_begin = 0;      // dispatch of the oldest launch in flight
    uint64_t dispatch_seq = 0;
    int last_lane = -1;         // lane of the most recent dispatch
    int64_t last_retire = 0;    // completion time of the last retired launch
    int64_t busy_until = 0;     // end of the union of launch intervals so far
    double m_lat = 0, m_npk = 0;  // service model: max(m_lat, m_npk * kbits)
    // statistics (under mu)
    tdec_serve_stats st{};
    int64_t batch_tbs_sum = 0, batch_cbs_sum = 0;
    int64_t pre_sum = 0, coding_sum = 0, post_sum = 0;  // per-launch delays (ns)
    std::deque<int64_t> lat;   // chunked: appending never moves what is stored
    std::vector<tdec_launch_rec> ring;  // last kLaunchRing launches
    int64_t ring_n = 0;                 // launches recorded since the last reset
    bool stop = false;
    std::thread dispatcher, completer;
    // ring mode: one persistent decode kernel takes the lanes' items from a
    // work ring in pinned host memory; the lanes plan, upload and assemble
    // on one side stream
    bool ring_mode = false;
    tdec::RingCtl *ring_ctl = nullptr;
    tdec::RingEntry *ring_ent = nullptr;
    uint32_t *ring_done = nullptr;
    tdec::RingCtl *hd_ring_ctl = nullptr;   // device addresses of the three
    tdec::RingEntry *hd_ring_ent = nullptr;
    uint32_t *hd_ring_done = nullptr;
    unsigned long long *d_ring_head = nullptr;  // the kernel's ticket counter and mirrors
    char *ring_stage = nullptr;                 // pinned: their values for the next launch
    char *d_ring_scratch = nullptr;
    int64_t ring_stride = 0;
    int ring_cap = 0, ring_grid = 0, ring_lds = 0, ring_item_lds = 0;
    uint64_t ring_idle_ticks = 0;
    hipStream_t ring_st = nullptr, side_st = nullptr;
    hipEvent_t ring_ev = nullptr;
    bool ring_live = false;  // a ring kernel was launched (ring_ev marks its end)
    uint64_t ring_pub = 0;   // items published
    int ring_outstanding = 0;  // lanes with items not all done
    std::atomic<int64_t> ring_launches{0};
    std::mutex ring_mu;      // publishing and (re)launching the ring kernel

    int64_t dur(int64_t kbits) const
    {
        return (int64_t)std::max(m_lat, m_npk * (double)kbits / 1000.0);
    }
    // how long before the predicted end of the work in flight the next
    // launch may be dispatched: a quarter of that work, at most 200 us
    int64_t lead() const
    {
        return std::min<int64_t>(200000, std::max<int64_t>(0, gpu_end_pred - gpu_begin) / 4);
    }
    int free_lane() const
    {
        for (int i = 0; i < n_lanes; ++i)
            if (!lanes[i].busy) return i;
        return -1;
    }
};

namespace {

struct Segm {
    int32_t C = 0;
    int64_t kbits = 0, n_llr = 0;
};

bool seg_of(int32_t tbs, Segm *o)
{
    tdec_seg s;
    if (tdec_segment(tbs, &s) != TDEC_OK || s.C > 64) return false;
    o->C = s.C;
    o->kbits = (int64_t)s.Cplus * s.Kplus + (int64_t)s.Cminus * s.Kminus;
    o->n_llr = tdec_tb_llr_count(tbs);
    return true;
}

// Lane L's batch as the decoder's arrays: payload sizes, LLR offsets in the
// slot arena, and (into L.bo) the byte offset of each TB's bits in the
// lane's staging; returns the copy event that covers the batch's slots.
uint64_t batch_arrays(Lane &L, std::vector<int32_t> &tbs, std::vector<int64_t> &lo)
{
    const int n = (int)L.b.size();
    tbs.resize(n);
    lo.resize(n);
    L.bo.resize(n);
    uint64_t seq = 0;
    int64_t bytes = 0;
    for (int i = 0; i < n; ++i) {
        tbs[i] = L.b[i].tbs;
        lo[i] = L.b[i].slot_off / 2;
        L.bo[i] = bytes;
        bytes += (L.b[i].tbs + 7) / 8;
        seq = std::max(seq, L.b[i].copy_seq);
    }
    return seq;
}

// Enqueue lane L's batch on its stream: wait for the batch's slot copies
// and (`after`, may be null) for an earlier launch's assembly, then decode +
// transport block assembly into the lane's mapped staging, events for the
// delays and the completion.  Returns without waiting.
void enqueue_device(tdec_server *s, Lane &L, hipEvent_t after)
{
    std::vector<int32_t> tbs;
    std::vector<int64_t> lo;
    const uint64_t seq = batch_arrays(L, tbs, lo);
    const int n = (int)tbs.size();
    bool ok = hipStreamWaitEvent(L.st, s->copy_ev[seq % kCopyEvents], 0) == hipSuccess;
    if (after) ok = ok && hipStreamWaitEvent(L.st, after, 0) == hipSuccess;
    ok = ok && tdec::tb_decode_batch_timed(L.ctx, n, tbs.data(), lo.data(), L.bo.data(),
                                           s->d_arena, &s->cfg.params, L.hd_bits, L.hd_res, L.st,
                                           L.ev_s, L.ev_m) == TDEC_OK;
    L.t_enq = mono_ns();
    ok = ok && hipEventRecord(L.ev_c, L.st) == hipSuccess;
    ok = ok && hipEventRecord(L.done_ev, L.st) == hipSuccess;
    L.ok = ok;
}

// Ring mode (under ring_mu): launch the ring kernel unless one is running.
// A ring kernel ends once its work groups have found nothing to claim for
// the idle time (or on stop), so a publication may find it ended, or it may
// end with items published after its work groups' last look: the caller
// publishing and the completer (which sees items outstanding) both call this.
bool ring_launch_locked(tdec_server *s)
{
    if (s->ring_live && hipEventQuery(s->ring_ev) == hipErrorNotReady) return true;
    // No work group of an earlier launch runs any more: the ticket counter
    // restarts at the oldest published item that is not done (tickets that
    // work groups abandoned when they left are handed out again; done items
    // below it are skipped by the kernel), the mirrors at the same point.
    uint64_t floor = s->ring_pub;
    for (int i = 0; i < s->n_lanes; ++i) {
        const Lane &L = s->lanes[i];
        if (!L.items_done) floor = std::min(floor, L.ring_first);
    }
    memset(s->ring_stage, 0, tdec::kRingCtrBytes);
    ((uint64_t *)s->ring_stage)[0] = floor;
    ((uint64_t *)s->ring_stage)[16] = floor;
    if (hipMemcpyAsync(s->d_ring_head, s->ring_stage, tdec::kRingCtrBytes, hipMemcpyHostToDevice,
                       s->ring_st) != hipSuccess)
        return false;
    tdec::DecArgs a{};
    const uint32_t *tab = tdec::ctx_crc_tab(s->lanes[0].ctx);
    a.llr = s->d_arena;
    a.crc_tab = tab;
    a.mi_tab = tab + tdec::kCrcTabWords;
    a.scratch = s->d_ring_scratch;
    a.scratch_stride = s->ring_stride;
    a.max_iters = s->cfg.params.max_iters;
    a.early_stop = s->cfg.params.early_stop;
    a.win_init = s->cfg.params.win_init;
    a.mi_eps = s->cfg.params.mi_eps;
    a.state_slots = tdec::kMaxSlotsPerWg;
    tdec::RingArgs r{};
    r.ctl = s->hd_ring_ctl;
    r.ent = s->hd_ring_ent;
    r.done = s->hd_ring_done;
    r.head = s->d_ring_head;
    r.cap = s->ring_cap;
    r.lds = tdec::lds_state_bytes(tdec::kMaxSlotsPerWg) + s->ring_item_lds;
    r.idle_ticks = s->ring_idle_ticks;
    if (tdec::launch_ring_decode(a, r, s->ring_grid, s->ring_lds, s->ring_st) != 0 ||
        hipEventRecord(s->ring_ev, s->ring_st) != hipSuccess)
        return false;
    s->ring_live = true;
    ++s->ring_launches;
    return true;
}

// Ring mode: plan lane L's batch with its context, wait for the batch's
// slot copies and the plan's upload, then publish its items on the ring.
// Returns without waiting for any decoding.
void enqueue_ring(tdec_server *s, Lane &L)
{
    std::vector<int32_t> tbs;
    std::vector<int64_t> lo;
    const uint64_t seq = batch_arrays(L, tbs, lo);
    const int n = (int)tbs.size();
    L.asm_enq = false;
    L.ring_n = 0;
    // the items are claimed by a kernel that is already running: everything
    // they read must be in device memory before they are published (the plan
    // is built and its upload enqueued while the slot copies still run)
    bool ok = tdec::ring_plan(L.ctx, n, tbs.data(), lo.data(), L.bo.data(), &s->cfg.params, L.st,
                              &L.rp) == TDEC_OK;
    ok = ok && hipEventSynchronize(s->copy_ev[seq % kCopyEvents]) == hipSuccess;
    const tdec::RingPlan &r = L.rp;
    // the ring kernel's shape: two waves, the LDS and scratch it was sized for
    ok = ok && r.wg == tdec::kRingWg && r.max_item_lds <= s->ring_item_lds &&
         r.stride <= s->ring_stride && !r.exact && !r.mi && r.n_items <= s->ring_cap / kMaxLanes;
    ok = ok && hipEventSynchronize(r.ready) == hipSuccess;
    if (ok) {
        std::lock_guard<std::mutex> g(s->ring_mu);
        // the ring never wraps onto an item that is published but not done:
        // its entry may still be claimed (in flight there are at most
        // max_inflight batches of max_batch_cb items, which the ring holds)
        uint64_t oldest = s->ring_pub;
        for (int i = 0; i < s->n_lanes; ++i)
            if (!s->lanes[i].items_done) oldest = std::min(oldest, s->lanes[i].ring_first);
        if (s->ring_pub + (uint64_t)r.n_items - oldest > (uint64_t)s->ring_cap) {
            L.t_enq = mono_ns();
            L.ok = false;
            return;
        }
        L.ring_first = L.ring_chk = s->ring_pub;
        for (int k = 0; k < r.n_items; ++k) {
            tdec::RingEntry &e = s->ring_ent[(s->ring_pub + (uint64_t)k) & (uint64_t)(s->ring_cap - 1)];
            e.item = r.items[k];
            e.cbs = r.d_cbs + r.items[k].cb0;
            e.qtab = r.d_qtab;
            e.hard = r.d_hard;
            e.crc_ok = r.d_ok;
            e.iters = r.d_it;
        }
        s->ring_pub += (uint64_t)r.n_items;
        L.ring_n = r.n_items;
        L.items_done = false;
        ++s->ring_outstanding;
        __atomic_store_n(&s->ring_ctl->tail, s->ring_pub, __ATOMIC_RELEASE);
        ok = ring_launch_locked(s);
    }
    L.t_enq = mono_ns();
    L.ok = ok;
}

// Has lane L's launch finished?  (A launch whose enqueue failed has.)  In
// ring mode a lane finishes in two steps: once all its items are marked
// done, its assembly is enqueued here; then its completion event fires.
bool lane_finished(tdec_server *s, Lane &L, int64_t now)
{
    if (s->model) return now >= L.model_end;
    if (!L.ok) return true;
    if (s->ring_mode && !L.asm_enq) {
        const uint64_t end = L.ring_first + (uint64_t)L.ring_n;
        while (L.ring_chk < end &&
               __atomic_load_n(&s->ring_done[L.ring_chk & (uint64_t)(s->ring_cap - 1)],
                               __ATOMIC_ACQUIRE) == (uint32_t)(L.ring_chk + 1))
            ++L.ring_chk;
        {
            std::lock_guard<std::mutex> g(s->ring_mu);
            if (L.ring_chk < end) {
                // items outstanding: the kernel must be running (it may have
                // ended with them published after its work groups left)
                if (!ring_launch_locked(s)) L.ok = false;
                return !L.ok;
            }
            L.items_done = true;
            --s->ring_outstanding;
        }
        L.t_items = mono_ns();
        bool ok = hipEventRecord(L.ev_m, L.st) == hipSuccess &&
                  tdec::ring_assemble(L.ctx, L.rp, &s->cfg.params, L.hd_bits, L.hd_res, L.st) ==
                      TDEC_OK &&
                  hipEventRecord(L.ev_c, L.st) == hipSuccess &&
                  hipEventRecord(L.done_ev, L.st) == hipSuccess;
        L.asm_enq = true;
        L.ok = ok;
        return !ok;
    }
    const hipError_t e = hipEventQuery(L.done_ev);
    return e != hipErrorNotReady;
}

// Results of lane L's finished launch into `res`; lat = pre-processing,
// coding, post-processing and copy delays; t1 = when the results are in
// host memory.
void collect(tdec_server *s, Lane &L, std::vector<tdec_server_result> &res, int64_t lat[5],
             int64_t *t1)
{
    const int n = (int)L.b.size();
    res.assign((size_t)n, tdec_server_result{});
    if (s->model) {
        for (auto &r : res) {
            r.status = TDEC_SERVE_DONE;
            r.tb_ok = 1;
            r.max_iters_used = s->cfg.params.max_iters;
        }
        *t1 = mono_ns();
        lat[0] = lat[2] = lat[3] = lat[4] = 0;
        lat[1] = *t1 - L.t0;
        return;
    }
    bool ok = L.ok && hipEventSynchronize(L.done_ev) == hipSuccess;
    float coding_ms = 0.f, post_ms = 0.f, copy_ms = 0.f;
    if (ok) {
        // ring mode: coding runs from publication until every item was
        // seen done (host clock)
        if (s->ring_mode) coding_ms = (float)((double)(L.t_items - L.t_enq) * 1e-6);
        else (void)hipEventElapsedTime(&coding_ms, L.ev_s, L.ev_m);
        (void)hipEventElapsedTime(&post_ms, L.ev_m, L.done_ev);
        (void)hipEventElapsedTime(&copy_ms, L.ev_c, L.done_ev);
    }
    const int64_t tc = mono_ns();
    for (int i = 0; i < n; ++i) {
        tdec_server_result &r = res[i];
        if (!ok) {
            r.status = TDEC_SERVE_ERROR;
            continue;
        }
        if (L.b[i].h_bits)
            memcpy(L.b[i].h_bits, L.h_bits + L.bo[i], (size_t)(L.b[i].tbs + 7) / 8);
        r.status = TDEC_SERVE_DONE;
        r.tb_ok = L.h_res[i].tb_ok;
        r.max_iters_used = L.h_res[i].max_iters_used;
    }
    *t1 = mono_ns();
    lat[4] = *t1 - tc;
    lat[0] = L.t_enq - L.t0;
    lat[1] = (int64_t)(coding_ms * 1e6f);
    lat[2] = (int64_t)(post_ms * 1e6f);
    lat[3] = (int64_t)(copy_ms * 1e6f);
}

// The dispatcher: whenever blocks wait and a lane is free, it forms a batch
// and enqueues it on that lane, without waiting for any launch to finish --
// blocks that arrive while launches run go out on the next free lane and
// their work shares the device with the launches already there.
void dispatcher_main(tdec_server *s)
{
    if (!s->model) (void)hipSetDevice(s->device);
    for (;;) {
        std::unique_lock<std::mutex> lk(s->mu);
        // A waiting batch goes out on a free lane when nothing is in flight,
        // or once the work in flight is predicted to end within the lead:
        // its work groups then take the compute units that the finishing
        // launches leave (the hand-over from one launch to the next is
        // hidden) without sharing them with those launches for long, which
        // would delay their older blocks.
        // In ring mode a batch goes out as soon as a lane is free: its items
        // join the running kernel, whose work groups take them as they free up.
        const auto ready = [&] {
            if (s->stop || s->queue.empty() || s->free_lane() < 0) return s->stop;
            return s->ring_mode || s->lanes_busy == 0 || mono_ns() >= s->gpu_end_pred - s->lead();
        };
        while (!ready()) {
            if (!s->queue.empty() && s->free_lane() >= 0 && s->lanes_busy > 0)
                s->cv_work.wait_for(lk, std::chrono::nanoseconds(
                                            std::max<int64_t>(s->gpu_end_pred - s->lead() - mono_ns(), 1000)));
            else
                s->cv_work.wait(lk);
        }
        if (s->queue.empty()) {
            if (s->stop) break;
            continue;
        }
        Lane &L = s->lanes[s->free_lane()];
        L.b.clear();
        int64_t kb = 0, cbs = 0;
        // Take the oldest block, then more while the launch stays within
        // max_batch_cb and is predicted to end before the oldest block's
        // deadline (if even that block alone cannot make it, its deadline
        // is lost anyway and the launch is filled for throughput).  The
        // prediction queues the launch behind the work already in flight.
        const int64_t now = mono_ns();
        const int64_t start = std::max(now, s->gpu_end_pred);
        const int64_t dl = s->queue.front().t_arrive + (int64_t)s->cfg.deadline_us * 1000;
        const bool feasible = start + s->dur(s->queue.front().kbits) <= dl;
        do {
            const Pending &p = s->queue.front();
            L.b.push_back(p);
            kb += p.kbits;
            cbs += p.C;
            s->queue.pop_front();
        } while (s->cfg.mode != TDEC_SERVE_PER_TB && !s->queue.empty() &&
                 cbs + s->queue.front().C <= s->cfg.max_batch_cb &&
                 (!feasible || start + s->dur(kb + s->queue.front().kbits) <= dl));
        s->queued_kbits -= kb;
        s->queued_cbs -= cbs;
        if (s->cfg.mode == TDEC_SERVE_PER_TB)
            for (auto &p : L.b) s->queued_dur_ns -= p.pred_dur;
        L.busy = true;
        L.launched = false;
        L.kb = kb;
        L.cbs = cbs;
        L.t0 = mono_ns();
        L.seq = ++s->dispatch_seq;
        if (s->lanes_busy == 0) s->gpu_begin = L.t0;
        s->gpu_end_pred = std::max(L.t0, s->gpu_end_pred) + s->dur(kb);
        // A launch with few transport blocks assembles them in kAsmGrid small
        // work groups, and a launch dispatched while it runs leaves that many
        // slots of its persistent grid free: its work groups then take the
        // compute units as the running launch's leave, and the running
        // launch's assembly never waits for them.  Behind a launch with many
        // transport blocks (whose assembly needs the whole device to be
        // quick) the next decode kernel waits on the device for that
        // assembly to end instead: the host side of the next launch still
        // overlaps, and no host round trip separates the two.
        L.small_asm = s->n_lanes > 1 && (int)L.b.size() <= 4 * tdec::kAsmGrid;
        int reserve = 0;
        hipEvent_t after = nullptr;
        if (s->lanes_busy > 0 && s->last_lane >= 0 && s->lanes[s->last_lane].busy) {
            const Lane &P = s->lanes[s->last_lane];
            if (P.small_asm) reserve = tdec::kAsmGrid;
            else after = P.ev_c;
        }
        s->last_lane = (int)(&L - s->lanes);
        ++s->lanes_busy;
        lk.unlock();
        if (s->model) {
            // the modelled device: a launch takes at least sim_lat and the
            // device completes sim_npk ns of work per kbit, launches in turn
            s->sim_busy_until = std::max(L.t0 + s->sim_lat,
                                         std::max(s->sim_busy_until, L.t0) +
                                             (int64_t)((double)s->sim_npk * kb / 1000.0));
            L.model_end = s->sim_busy_until;
        } else if (s->ring_mode) {
            enqueue_ring(s, L);
        } else {
            tdec::ctx_set_launch_reserve(L.ctx, reserve, L.small_asm);
            enqueue_device(s, L, after);
        }
        lk.lock();
        L.launched = true;
        lk.unlock();
        s->cv_retire.notify_one();
    }
}

// Account one finished launch (under mu): results, slots, statistics,
// launch record, service model.
void retire_locked(tdec_server *s, Lane &L, std::vector<tdec_server_result> &res,
                   const int64_t lat3[5], int64_t t1)
{
    const std::vector<Pending> &b = L.b;
    std::vector<std::pair<int64_t, int64_t>> ext;
    ext.reserve(b.size());
    for (size_t i = 0; i < b.size(); ++i) {
        tdec_server_result &r = res[i];
        r.tag = b[i].tag;
        r.tbs = b[i].tbs;
        r.C = b[i].C;
        r.batch_tbs = (int32_t)b.size();
        r.t_arrive_ns = b[i].t_arrive;
        r.t_done_ns = t1;
        ext.emplace_back(b[i].slot_off, b[i].slot_bytes);
        if (r.status == TDEC_SERVE_DONE) {
            ++s->st.completed;
            s->st.payload_bits += r.tbs;
            if (!r.tb_ok) ++s->st.tb_fail;
            const int64_t l = t1 - r.t_arrive_ns;
            s->lat.push_back(l);
            if (l > (int64_t)s->cfg.deadline_us * 1000) ++s->st.deadline_miss;
        }
        s->done.push_back(r);
    }
    s->arena.release_many(ext);
    s->inflight -= (int64_t)b.size();
    ++s->st.batches;
    s->batch_tbs_sum += (int64_t)b.size();
    s->batch_cbs_sum += L.cbs;
    // busy time: the union of the launches' [take, results] intervals
    s->st.busy_ns += std::max<int64_t>(0, t1 - std::max(L.t0, s->busy_until));
    s->busy_until = std::max(s->busy_until, t1);
    s->pre_sum += lat3[0];
    s->coding_sum += lat3[1];
    s->post_sum += lat3[2];
    tdec_launch_rec lr{};
    lr.t_start_ns = L.t0;
    lr.t_end_ns = t1;
    lr.pre_ns = lat3[0];
    lr.coding_ns = lat3[1];
    lr.post_ns = lat3[2];
    lr.copy_ns = lat3[3];
    lr.copyout_ns = lat3[4];
    int64_t oldest = L.t0;
    for (const Pending &p : b) oldest = std::min(oldest, p.t_arrive);
    lr.oldest_wait_ns = L.t0 - oldest;
    lr.n_tb = (int32_t)b.size();
    lr.n_cb = (int32_t)L.cbs;
    lr.cb_bits = L.kb;
    s->ring[(size_t)(s->ring_n++ % kLaunchRing)] = lr;
    // service model: the launch's own share of the time, from when its
    // oldest block arrived or the previous launch finished, whichever is
    // later (the time before that belonged to the launches ahead of it; the
    // hand-over from a finished launch to the next dispatch is counted, as
    // the blocks wait through it).  One observation moves the model by at
    // most a factor of 4 (a cold first launch must not stall admission for
    // long).
    const int64_t own = t1 - std::max(oldest, s->last_retire);
    s->last_retire = std::max(s->last_retire, t1);
    const double d = std::min((double)std::max<int64_t>(own, 1), 4.0 * (double)s->dur(L.kb));
    if (s->m_npk * (double)L.kb / 1000.0 < s->m_lat)
        s->m_lat = 0.8 * s->m_lat + 0.2 * d;
    else
        s->m_npk = 0.8 * s->m_npk + 0.2 * d * 1000.0 / (double)std::max<int64_t>(L.kb, 1);
    L.busy = false;
    L.launched = false;
    if (--s->lanes_busy == 0) s->gpu_end_pred = 0;
}

// Ring mode: end the ring kernel (it has had no work for the idle time):
// its work groups, all waiting for unpublished tickets, leave once the stop
// flag is seen, within microseconds.  Under ring_mu, so that nothing is
// published meanwhile; a later publication launches the kernel again.
void ring_stop_idle(tdec_server *s)
{
    std::lock_guard<std::mutex> g(s->ring_mu);
    if (!s->ring_live || s->ring_outstanding > 0) return;
    __atomic_store_n(&s->ring_ctl->stop, 1u, __ATOMIC_RELEASE);
    (void)hipEventSynchronize(s->ring_ev);
    s->ring_live = false;
    __atomic_store_n(&s->ring_ctl->stop, 0u, __ATOMIC_RELEASE);
}

// The completer: watches the lanes' launches, oldest first, and retires each
// as soon as it finishes (in whatever order they finish).
void completer_main(tdec_server *s)
{
    if (!s->model) (void)hipSetDevice(s->device);
    std::vector<tdec_server_result> res;
    std::vector<int> cand;
    for (;;) {
        cand.clear();
        {
            std::unique_lock<std::mutex> lk(s->mu);
            const auto pending = [&] {
                for (int i = 0; i < s->n_lanes; ++i)
                    if (s->lanes[i].launched) return true;
                return s->stop && s->lanes_busy == 0;
            };
            if (s->ring_mode && !s->model && !pending()) {
                // nothing in flight: after the idle time, end the ring kernel
                if (!s->cv_retire.wait_for(lk, std::chrono::microseconds(s->cfg.ring_idle_us), pending)) {
                    lk.unlock();
                    ring_stop_idle(s);
                    continue;
                }
            }
            s->cv_retire.wait(lk, pending);
            for (int i = 0; i < s->n_lanes; ++i)
                if (s->lanes[i].launched) cand.push_back(i);
            if (cand.empty()) break;  // stop, nothing in flight
        }
        std::sort(cand.begin(), cand.end(),
                  [&](int a, int b) { return s->lanes[a].seq < s->lanes[b].seq; });
        // wait for the first of them to finish: spin on the events (a launch
        // lasts tens of microseconds to milliseconds); the modelled device
        // sleeps until its earliest completion
        int fin = -1;
        for (int spins = 0; fin < 0; ++spins) {
            const int64_t now = mono_ns();
            int64_t soonest = INT64_MAX;
            for (int i : cand) {
                if (lane_finished(s, s->lanes[i], now)) {
                    fin = i;
                    break;
                }
                soonest = std::min(soonest, s->lanes[i].model_end);
            }
            if (fin >= 0) break;
            if (s->model) {
                std::this_thread::sleep_for(std::chrono::nanoseconds(std::max<int64_t>(soonest - now, 1000)));
            } else if (spins > 64) {
                // a newer launch may have joined the lanes being watched
                std::this_thread::yield();
                if (spins % 256 == 0) break;
            }
        }
        if (fin < 0) continue;
        Lane &L = s->lanes[fin];
        int64_t lat3[5] = {0, 0, 0, 0, 0};
        int64_t t1 = 0;
        collect(s, L, res, lat3, &t1);
        {
            std::lock_guard<std::mutex> lk(s->mu);
            retire_locked(s, L, res, lat3, t1);
        }
        s->cv_work.notify_one();
        s->cv_done.notify_all();
    }
}

void free_device(tdec_server *s)
{
    if (s->model) return;
    (void)hipSetDevice(s->device);
    if (s->ring_ctl) {
        // the ring kernel's work groups leave at their next look at the ring
        __atomic_store_n(&s->ring_ctl->stop, 1u, __ATOMIC_RELEASE);
        if (s->ring_st) (void)hipStreamSynchronize(s->ring_st);
    }
    for (int i = 0; i < kMaxLanes; ++i) {
        Lane &L = s->lanes[i];
        if (L.st == s->side_st) L.st = nullptr;  // shared, destroyed below
        if (L.st) (void)hipStreamSynchronize(L.st);
        if (L.h_bits) (void)hipHostFree(L.h_bits);
        if (L.h_res) (void)hipHostFree(L.h_res);
        for (hipEvent_t e : {L.ev_s, L.ev_m, L.ev_c, L.done_ev})
            if (e) (void)hipEventDestroy(e);
        if (L.st) (void)hipStreamDestroy(L.st);
        if (L.own_ctx && L.ctx) tdec_destroy(L.ctx);
        else if (L.ctx) tdec::ctx_set_launch_reserve(L.ctx, 0, false);  // the caller's context
        L = Lane{};
    }
    if (s->side_st) {
        (void)hipStreamSynchronize(s->side_st);
        (void)hipStreamDestroy(s->side_st);
    }
    if (s->ring_ev) (void)hipEventDestroy(s->ring_ev);
    if (s->ring_st) (void)hipStreamDestroy(s->ring_st);
    if (s->ring_ctl) (void)hipHostFree(s->ring_ctl);
    if (s->ring_ent) (void)hipHostFree(s->ring_ent);
    if (s->ring_done) (void)hipHostFree(s->ring_done);
    if (s->ring_stage) (void)hipHostFree(s->ring_stage);
    if (s->d_ring_head) (void)hipFree(s->d_ring_head);
    if (s->d_ring_scratch) (void)hipFree(s->d_ring_scratch);
    if (s->d_arena) (void)hipFree(s->d_arena);
    for (auto &e : s->copy_ev)
        if (e) (void)hipEventDestroy(e);
    if (s->copy_st) (void)hipStreamDestroy(s->copy_st);
}

// Ring mode: the work ring (pinned host memory, fine-grained so that both
// sides see each other's writes while the kernel runs), the claim counter,
// the ring kernel's scratch and shape, and the streams.
bool ring_setup(tdec_server *s)
{
    constexpr unsigned kRingFlags = hipHostMallocMapped | hipHostMallocCoherent;
    s->ring_mode = true;
    int cap = 1;
    while (cap < kMaxLanes * s->cfg.max_batch_cb) cap <<= 1;
    s->ring_cap = cap;
    // LDS: the per-slot state of 64 blocks, the item's extrinsic arrays, the
    // item's copy; 26 KB in all (with the kernel's static LDS under 27 KB),
    // so that six two-wave work groups share a CU's 160 KB
    s->ring_lds = 26624;
    s->ring_item_lds = s->ring_lds - tdec::lds_state_bytes(tdec::kMaxSlotsPerWg) - tdec::kRingLdsBytes;
    s->ring_stride = tdec::ring_max_stride(tdec::kRingWg / 2, s->ring_item_lds);
    int occ = 0, khz = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, tdec::ring_kernel_address(), tdec::kRingWg,
                                                     s->ring_lds) != hipSuccess ||
        occ < 1 ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, s->device) != hipSuccess || khz < 1)
        return false;
    // The ring kernel's stream masks out one compute unit per eighth of the
    // device (which is one per XCD whether the CU numbering runs XCD by XCD
    // or round-robin over them): the transport block assembly, the gather
    // and copy launches of the other streams always find room there.  A
    // stream with a CU mask also gets a hardware queue of its own, so that
    // no other stream's work queues up behind the resident ring kernel.
    const int ncu = tdec::ctx_num_cus(s->ctx);
    // (ncu words: enough whether the runtime counts the mask's size in bits
    // or in 32-bit words; words past the CU count are ignored)
    std::vector<uint32_t> mask((size_t)std::max(ncu, 1), 0u);
    int used = 0;
    for (int c = 0; c < ncu; ++c) {
        const int blk = ncu / 8, k = blk > 0 ? c / blk : 8;
        if (ncu >= 64 && k < 8 && c == k * blk + blk - 1 - k) continue;
        mask[(size_t)c / 32] |= 1u << (c % 32);
        ++used;
    }
    s->ring_grid = std::max(1, occ * used);
    // a work group gives up a wait after four idle times and 100 ms more:
    // the host ends an idle kernel itself long before that, so the bound
    // only matters if the host stops looking after the ring
    s->ring_idle_ticks = ((uint64_t)s->cfg.ring_idle_us * 4u + 100000u) * (uint64_t)khz / 1000u;
    bool ok = hipHostMalloc(&s->ring_ctl, sizeof(tdec::RingCtl), kRingFlags) == hipSuccess &&
              hipHostMalloc(&s->ring_ent, sizeof(tdec::RingEntry) * (size_t)cap, kRingFlags) == hipSuccess &&
              hipHostMalloc(&s->ring_done, sizeof(uint32_t) * (size_t)cap, kRingFlags) == hipSuccess &&
              hipHostMalloc(&s->ring_stage, tdec::kRingCtrBytes, hipHostMallocDefault) == hipSuccess;
    if (!ok) return false;
    memset(s->ring_ctl, 0, sizeof(tdec::RingCtl));
    memset(s->ring_ent, 0, sizeof(tdec::RingEntry) * (size_t)cap);
    memset(s->ring_done, 0, sizeof(uint32_t) * (size_t)cap);
    ok = hipHostGetDevicePointer((void **)&s->hd_ring_ctl, s->ring_ctl, 0) == hipSuccess &&
         hipHostGetDevicePointer((void **)&s->hd_ring_ent, s->ring_ent, 0) == hipSuccess &&
         hipHostGetDevicePointer((void **)&s->hd_ring_done, s->ring_done, 0) == hipSuccess &&
         hipMalloc(&s->d_ring_head, tdec::kRingCtrBytes) == hipSuccess &&
         hipMalloc(&s->d_ring_scratch, (size_t)s->ring_stride * (size_t)s->ring_grid) == hipSuccess &&
         hipExtStreamCreateWithCUMask(&s->ring_st, (uint32_t)mask.size(), mask.data()) == hipSuccess &&
         hipStreamCreateWithFlags(&s->side_st, hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&s->ring_ev, hipEventDisableTiming) == hipSuccess &&
         hipDeviceSynchronize() == hipSuccess;
    return ok;
}

tdec_status create_common(const tdec_server_cfg *cfg, tdec_server *s)
{
    if (!cfg || cfg->deadline_us <= 0 || cfg->max_batch_cb < 0 ||
        (cfg->mode != TDEC_SERVE_CONTINUOUS && cfg->mode != TDEC_SERVE_PER_TB &&
         cfg->mode != TDEC_SERVE_RING) ||
        cfg->ring_idle_us < 0 || cfg->ring_idle_us > 10000000 ||
        !tdec::params_valid(&cfg->params) || cfg->model_lat_ns < 0 ||
        cfg->model_ns_per_kbit < 0 || cfg->max_inflight < 0 || cfg->max_inflight > kMaxLanes)
        return TDEC_EINVAL;
    s->cfg = *cfg;
    if (!s->cfg.slot_budget_bytes) s->cfg.slot_budget_bytes = (size_t)1 << 30;
    if (!s->cfg.max_batch_cb) s->cfg.max_batch_cb = 8192;
    s->cfg.max_batch_cb = std::max(s->cfg.max_batch_cb, 64);  // a TB has at most 64 blocks
    // the plain per-TB form runs one launch at a time
    s->n_lanes = s->cfg.mode == TDEC_SERVE_PER_TB
                     ? 1
                     : (s->cfg.max_inflight ? s->cfg.max_inflight
                                            : (s->cfg.mode == TDEC_SERVE_RING ? 4 : 2));
    if (!s->cfg.ring_idle_us) s->cfg.ring_idle_us = 20000;
    s->ring_mode = s->cfg.mode == TDEC_SERVE_RING;
    s->cfg.max_inflight = s->n_lanes;
    s->arena.init((int64_t)s->cfg.slot_budget_bytes);
    s->m_lat = (double)(cfg->model_lat_ns ? cfg->model_lat_ns : 300000);
    s->m_npk = (double)(cfg->model_ns_per_kbit ? cfg->model_ns_per_kbit : 50);
    s->ring.resize((size_t)kLaunchRing);
    return TDEC_OK;
}

void start_threads(tdec_server *s)
{
    s->dispatcher = std::thread(dispatcher_main, s);
    s->completer = std::thread(completer_main, s);
}

}  // namespace

extern "C" {

int64_t tdec_now_ns(void) { return mono_ns(); }

tdec_status tdec_server_create(tdec_ctx *ctx, const tdec_server_cfg *cfg, tdec_server **out)
{
    if (!out || !ctx) return TDEC_EINVAL;
    *out = nullptr;
    tdec_server *s = new tdec_server();
    tdec_status st = create_common(cfg, s);
    if (st != TDEC_OK) {
        delete s;
        return st;
    }
    s->ctx = ctx;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return TDEC_EDEVICE;
    }
    s->bits_cap = (size_t)s->cfg.max_batch_cb * 768 + 64;
    s->res_cap = s->cfg.max_batch_cb;
    bool ok = hipMalloc(&s->d_arena, s->cfg.slot_budget_bytes) == hipSuccess &&
              hipStreamCreateWithFlags(&s->copy_st, hipStreamNonBlocking) == hipSuccess;
    for (auto &e : s->copy_ev)
        ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
    // every copy event starts recorded, so that a wait on it never blocks on nothing
    for (auto &e : s->copy_ev) ok = ok && hipEventRecord(e, s->copy_st) == hipSuccess;
    tdec_status cs = TDEC_OK;
    const bool ring = s->cfg.mode == TDEC_SERVE_RING;
    if (ring) {
        // the ring kernel holds 64 windows per work group (two waves)
        ok = ok && s->cfg.params.win_init != 2 && !(s->cfg.params.early_stop & 2) &&
             s->cfg.params.n_windows <= tdec::kRingWg / 2;
        if (!ok) cs = TDEC_EINVAL;
        ok = ok && ring_setup(s);
    }
    for (int i = 0; i < s->n_lanes && ok; ++i) {
        Lane &L = s->lanes[i];
        if (i == 0 && !ring) {
            L.ctx = ctx;
        } else {
            // ring mode plans with contexts of the ring kernel's shape, so
            // the caller's context is left as it was
            cs = tdec::ctx_clone(ctx, &L.ctx);
            ok = cs == TDEC_OK;
            L.own_ctx = ok;
            if (ok && ring) tdec::ctx_set_ring_shape(L.ctx, tdec::kRingWg / 2, s->ring_item_lds);
        }
        if (ring) L.st = s->side_st;
        ok = ok &&
             hipHostMalloc(&L.h_bits, s->bits_cap, kStageFlags) == hipSuccess &&
             hipHostMalloc(&L.h_res, sizeof(tdec_tb_result) * (size_t)s->res_cap,
                           kStageFlags) == hipSuccess &&
             hipHostGetDevicePointer((void **)&L.hd_bits, L.h_bits, 0) == hipSuccess &&
             hipHostGetDevicePointer((void **)&L.hd_res, L.h_res, 0) == hipSuccess &&
             (ring || hipStreamCreateWithFlags(&L.st, hipStreamNonBlocking) == hipSuccess) &&
             hipEventCreate(&L.done_ev) == hipSuccess && hipEventCreate(&L.ev_s) == hipSuccess &&
             hipEventCreate(&L.ev_m) == hipSuccess && hipEventCreate(&L.ev_c) == hipSuccess;
    }
    if (!ok) {
        free_device(s);
        delete s;
        return cs == TDEC_EDEVICE || cs == TDEC_EINVAL ? cs : TDEC_ENOMEM;
    }
    start_threads(s);
    *out = s;
    return TDEC_OK;
}

tdec_status tdec_server_create_model(const tdec_server_cfg *cfg, int64_t lat_ns,
                                     int64_t ns_per_kbit, tdec_server **out)
{
    if (!out || lat_ns < 0 || ns_per_kbit < 0) return TDEC_EINVAL;
    *out = nullptr;
    tdec_server *s = new tdec_server();
    tdec_status st = create_common(cfg, s);
    if (st != TDEC_OK) {
        delete s;
        return st;
    }
    s->model = true;
    s->sim_lat = lat_ns;
    s->sim_npk = ns_per_kbit;
    start_threads(s);
    *out = s;
    return TDEC_OK;
}

// Submission runs in three steps so that the dispatcher never waits behind the
// copies: (1) under the server mutex, admission and slot allocation (the
// admitted blocks already count in the queue's totals); (2) under the
// submitters' own mutex only, the copies into the slots and the event that
// covers them; (3) under the server mutex again, the blocks join the queue,
// each naming that event, so the dispatcher can only launch them behind it.
static int32_t submit_impl(tdec_server *s, int32_t n, const uint64_t *tags, const int32_t *tbs,
                           const int16_t *const *h_llr, uint8_t *const *h_bits,
                           int64_t t_arrive_ns, int32_t *status, bool dev)
{
    if (!s || n < 0) return TDEC_EINVAL;
    if (n == 0) return 0;
    if (!tags || !tbs || !h_llr) return TDEC_EINVAL;
    if (!s->model && hipSetDevice(s->device) != hipSuccess) return TDEC_EDEVICE;
    std::lock_guard<std::mutex> sub(s->submit_mu);
    std::vector<Pending> adm;
    std::vector<int32_t> idx;  // caller index of each admitted block
    adm.reserve((size_t)n);
    idx.reserve((size_t)n);
    auto reject = [&](int32_t i, int32_t why, int32_t C) {
        if (status) status[i] = why;
        tdec_server_result r{};
        r.tag = tags[i];
        r.tbs = tbs[i];
        r.status = why;
        r.C = C;
        r.t_arrive_ns = r.t_done_ns = t_arrive_ns;
        s->done.push_back(r);
    };
    // (1) admission
    {
        std::lock_guard<std::mutex> lk(s->mu);
        const int64_t now = mono_ns();
        const int64_t deadline = t_arrive_ns + (int64_t)s->cfg.deadline_us * 1000;
        // One extent for the whole call when every block is valid and it
        // fits: the blocks take consecutive pieces of it, each released on
        // its own later (and merged back); otherwise one extent per block.
        int64_t big = -1, big_at = 0;
        if (n > 1) {
            int64_t tot = 0;
            bool valid = true;
            for (int32_t i = 0; i < n && valid; ++i) {
                Segm g;
                valid = seg_of(tbs[i], &g) && h_llr[i];
                tot += (g.n_llr * 2 + 255) & ~(int64_t)255;
            }
            if (valid) big = s->arena.alloc(tot);
        }
        std::vector<std::pair<int64_t, int64_t>> unused;  // pieces of refused blocks
        for (int32_t i = 0; i < n; ++i) {
            ++s->st.submitted;
            Segm g;
            int32_t why = TDEC_SERVE_DONE;
            int64_t off = -1, bytes = 0;
            if (!seg_of(tbs[i], &g) || !h_llr[i]) {
                why = TDEC_SERVE_REJ_INVALID;
            } else {
                bytes = g.n_llr * 2;
                if (big >= 0) {
                    off = big + big_at;
                    big_at += (bytes + 255) & ~(int64_t)255;
                } else {
                    off = s->arena.alloc(bytes);
                    if (off < 0) why = TDEC_SERVE_REJ_BUDGET;
                }
            }
            if (why == TDEC_SERVE_DONE && (s->cfg.admission & TDEC_ADMIT_DEADLINE)) {
                // the block joins the next launch after the running one (or
                // a later one once the queue exceeds a launch)
                const int64_t start = std::max(now, s->gpu_end_pred);
                int64_t pred;
                int64_t limit = deadline;
                if (s->cfg.mode != TDEC_SERVE_PER_TB) {
                    const int64_t launches =
                        (s->queued_cbs + g.C + s->cfg.max_batch_cb - 1) / s->cfg.max_batch_cb;
                    pred = start + s->dur(s->queued_kbits + g.kbits) +
                           (launches - 1) * (int64_t)s->m_lat;
                    // joining the same launch as the oldest waiting block
                    // must not push that block past its own deadline
                    // (submitters are serialised, so the waiting blocks
                    // are the queue's, then this call's)
                    const bool waiting = !s->queue.empty() || !adm.empty();
                    const int64_t oldest =
                        !s->queue.empty() ? s->queue.front().t_arrive : t_arrive_ns;
                    if (launches == 1 && waiting)
                        limit = std::min(limit, oldest + (int64_t)s->cfg.deadline_us * 1000);
                } else {
                    pred = start + s->queued_dur_ns + s->dur(g.kbits);
                }
                // an idle server always admits: the prediction only judges
                // the wait behind other work (and an overestimating model
                // must still see launches to correct itself)
                const bool busy = s->lanes_busy != 0 || !s->queue.empty() || !adm.empty();
                // a tenth of the deadline is kept in hand: blocks go out at
                // once on free lanes, so admission alone decides how close
                // to the deadline a launch ends, and the prediction is noisy
                if (busy && pred > limit - (int64_t)s->cfg.deadline_us * 100) {
                    why = TDEC_SERVE_REJ_DEADLINE;
                    unused.emplace_back(off, bytes);
                }
            }
            if (why != TDEC_SERVE_DONE) {
                if (why == TDEC_SERVE_REJ_BUDGET) ++s->st.rej_budget;
                if (why == TDEC_SERVE_REJ_DEADLINE) ++s->st.rej_deadline;
                if (why == TDEC_SERVE_REJ_INVALID) ++s->st.rej_invalid;
                reject(i, why, g.C);
                continue;
            }
            if (status) status[i] = TDEC_SERVE_DONE;
            Pending p{};
            p.tag = tags[i];
            p.tbs = tbs[i];
            p.C = g.C;
            p.kbits = g.kbits;
            p.slot_off = off;
            p.slot_bytes = bytes;
            p.h_bits = h_bits ? h_bits[i] : nullptr;
            p.t_arrive = t_arrive_ns;
            p.pred_dur = s->cfg.mode == TDEC_SERVE_PER_TB ? s->dur(g.kbits) : 0;
            s->queued_kbits += g.kbits;
            s->queued_cbs += g.C;
            s->queued_dur_ns += p.pred_dur;
            ++s->inflight;
            adm.push_back(p);
            idx.push_back(i);
        }
        s->arena.release_many(unused);
    }
    // (2) copies: host sources one asynchronous copy each, device sources
    // batched into gather launches; fail[k] marks blocks whose copy failed
    std::vector<char> fail(adm.size(), 0);
    uint64_t seq = 0;
    if (!s->model && !adm.empty()) {
        tdec::GatherArgs ga;
        ga.n = 0;
        ga.dst_base = s->d_arena;
        size_t g0 = 0;  // first block of the pending gather
        for (size_t k = 0; k < adm.size(); ++k) {
            const Pending &p = adm[k];
            const int32_t i = idx[k];
            if (!dev) {
                fail[k] = hipMemcpyAsync(s->d_arena + p.slot_off / 2, h_llr[i],
                                         (size_t)p.slot_bytes, hipMemcpyHostToDevice,
                                         s->copy_st) != hipSuccess;
                continue;
            }
            ga.it[ga.n].src = h_llr[i];
            ga.it[ga.n].dst_blk = (uint32_t)(p.slot_off / 256);
            ga.it[ga.n].n = (uint32_t)(p.slot_bytes / 2);
            if (++ga.n == tdec::kGatherMax || k + 1 == adm.size()) {
                if (tdec::launch_gather(ga, s->copy_st) != 0)
                    for (size_t q = g0; q <= k; ++q) fail[q] = 1;
                ga.n = 0;
                g0 = k + 1;
            }
        }
        // record after this call's copies; the dispatcher waits for it before
        // it launches any of these blocks
        seq = ++s->copy_seq;
        if (hipEventRecord(s->copy_ev[seq % kCopyEvents], s->copy_st) != hipSuccess)
            std::fill(fail.begin(), fail.end(), 1);
    }
    // (3) queue
    int32_t admitted = 0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (size_t k = 0; k < adm.size(); ++k) {
            Pending &p = adm[k];
            if (fail[k]) {
                s->arena.release(p.slot_off, p.slot_bytes);
                s->queued_kbits -= p.kbits;
                s->queued_cbs -= p.C;
                s->queued_dur_ns -= p.pred_dur;
                --s->inflight;
                reject(idx[k], TDEC_SERVE_ERROR, p.C);
                continue;
            }
            p.copy_seq = seq;
            s->queue.push_back(p);
            ++s->st.admitted;
            ++admitted;
        }
    }
    s->cv_work.notify_one();
    s->cv_done.notify_all();
    return admitted;
}

int32_t tdec_server_submit(tdec_server *s, int32_t n, const uint64_t *tags, const int32_t *tbs,
                           const int16_t *const *h_llr, uint8_t *const *h_bits,
                           int64_t t_arrive_ns, int32_t *status)
{
    return submit_impl(s, n, tags, tbs, h_llr, h_bits, t_arrive_ns, status, false);
}

int32_t tdec_server_submit_dev(tdec_server *s, int32_t n, const uint64_t *tags,
                               const int32_t *tbs, const int16_t *const *d_llr,
                               uint8_t *const *h_bits, int64_t t_arrive_ns, int32_t *status)
{
    return submit_impl(s, n, tags, tbs, d_llr, h_bits, t_arrive_ns, status, true);
}

tdec_status tdec_server_replay(tdec_server *s, int32_t n_ticks, int64_t t_first_ns,
                               int64_t period_ns, const int32_t *counts, const int32_t *tbs,
                               const int16_t *const *d_llr, uint8_t *const *h_bits,
                               uint64_t tag_base, int64_t *late_max_ns, int64_t *submit_max_ns)
{
    if (!s || n_ticks < 0 || period_ns <= 0 || (n_ticks && (!counts || !tbs || !d_llr)))
        return TDEC_EINVAL;
    int32_t most = 1;
    for (int32_t k = 0; k < n_ticks; ++k) {
        if (counts[k] < 0) return TDEC_EINVAL;
        most = std::max(most, counts[k]);
    }
    // one tick's tags at a time: nothing proportional to the whole schedule
    // is built between the caller's clock reading and the first tick
    std::vector<uint64_t> tags((size_t)most);
    int64_t late = 0, smax = 0, at = 0;
    for (int32_t k = 0; k < n_ticks; ++k) {
        const int64_t tick = t_first_ns + (int64_t)k * period_ns;
        while (mono_ns() < tick) {
        }
        late = std::max(late, mono_ns() - tick);
        if (counts[k]) {
            for (int32_t j = 0; j < counts[k]; ++j) tags[(size_t)j] = tag_base + (uint64_t)(at + j);
            const int64_t t0 = mono_ns();
            const int32_t r = submit_impl(s, counts[k], tags.data(), tbs + at, d_llr + at,
                                          h_bits ? h_bits + at : nullptr, tick, nullptr, true);
            if (r < 0) return (tdec_status)r;
            smax = std::max(smax, mono_ns() - t0);
        }
        at += counts[k];
    }
    if (late_max_ns) *late_max_ns = late;
    if (submit_max_ns) *submit_max_ns = smax;
    return TDEC_OK;
}

int32_t tdec_server_poll(tdec_server *s, tdec_server_result *out, int32_t max, int32_t wait_us)
{
    if (!s || !out || max <= 0) return 0;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->done.empty() && wait_us > 0)
        s->cv_done.wait_for(lk, std::chrono::microseconds(wait_us),
                            [&] { return !s->done.empty(); });
    int32_t k = 0;
    while (k < max && !s->done.empty()) {
        out[k++] = s->done.front();
        s->done.pop_front();
    }
    return k;
}

tdec_status tdec_server_drain(tdec_server *s, int32_t timeout_ms)
{
    if (!s) return TDEC_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    const bool ok = s->cv_done.wait_for(lk, std::chrono::milliseconds(std::max(timeout_ms, 0)),
                                        [&] { return s->inflight == 0; });
    return ok ? TDEC_OK : TDEC_EBUSY;
}

tdec_status tdec_server_stats(tdec_server *s, tdec_serve_stats *out)
{
    if (!s || !out) return TDEC_EINVAL;
    std::vector<int64_t> v;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        *out = s->st;
        v.assign(s->lat.begin(), s->lat.end());
        out->ring_launches = s->ring_launches;
        out->ring_grid = s->ring_grid;
        out->model_lat_ns = (int64_t)s->m_lat;
        out->model_ns_per_kbit = (int64_t)s->m_npk;
        out->slots_in_use_bytes = s->arena.used();
        out->slots_peak_bytes = s->arena.peak();
        out->mean_batch_tbs = s->st.batches ? (double)s->batch_tbs_sum / s->st.batches : 0.0;
        out->mean_batch_cbs = s->st.batches ? (double)s->batch_cbs_sum / s->st.batches : 0.0;
        if (s->st.batches) {
            out->mean_pre_ns = s->pre_sum / s->st.batches;
            out->mean_coding_ns = s->coding_sum / s->st.batches;
            out->mean_post_ns = s->post_sum / s->st.batches;
        }
    }
    if (!v.empty()) {
        std::sort(v.begin(), v.end());
        const size_t n = v.size();
        // nearest-rank percentiles
        auto q = [&](double f) {
            size_t r = (size_t)((double)n * f + 0.999999999);
            r = std::min(std::max<size_t>(r, 1), n);
            return v[r - 1];
        };
        out->lat_p50_ns = q(0.50);
        out->lat_p99_ns = q(0.99);
        out->lat_p999_ns = q(0.999);
        out->lat_max_ns = v.back();
        long double sum = 0;
        for (int64_t x : v) sum += x;
        out->lat_mean_ns = (int64_t)(sum / n);
    }
    return TDEC_OK;
}

void tdec_server_reset_stats(tdec_server *s)
{
    if (!s) return;
    std::lock_guard<std::mutex> lk(s->mu);
    s->st = tdec_serve_stats{};
    s->lat.clear();
    s->batch_tbs_sum = s->batch_cbs_sum = 0;
    s->pre_sum = s->coding_sum = s->post_sum = 0;
    s->ring_n = 0;
    s->arena.reset_peak();
}

int32_t tdec_server_launches(tdec_server *s, tdec_launch_rec *out, int32_t max)
{
    if (!s || max < 0 || (max > 0 && !out)) return TDEC_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    const int64_t kept = std::min<int64_t>(s->ring_n, kLaunchRing);
    const int64_t n = std::min<int64_t>(kept, max);
    for (int64_t i = 0; i < n; ++i)
        out[i] = s->ring[(size_t)((s->ring_n - n + i) % kLaunchRing)];
    return (int32_t)n;
}

void tdec_server_destroy(tdec_server *s)
{
    if (!s) return;
    (void)tdec_server_drain(s, 60000);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    s->cv_retire.notify_all();
    if (s->dispatcher.joinable()) s->dispatcher.join();
    if (s->completer.joinable()) s->completer.join();
    free_device(s);
    delete s;
}

}  // extern "C"
