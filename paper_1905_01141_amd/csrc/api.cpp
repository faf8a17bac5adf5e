// api.cpp -- the C ABI of libtdec (include/tdec.h): argument checking,
// launch planning, workspace management and kernel launches.
//
// A decode call becomes one persistent launch of the decode kernel over a
// list of work items (code blocks of one size grouped so that their windows
// fill the work group's lanes and their extrinsic arrays fit the LDS budget),
// plus, for transport blocks, one launch of the assembly kernel.  Plans are
// cached by the content of the request, so a repeated batch costs no host
// planning and no upload.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "tdec.h"
#include "tdec_internal.h"

using namespace tdec;

namespace {

constexpr int kPlanSlots = 8;
constexpr size_t kPlanSlotBytes = 8u << 20;
constexpr int kLdsPerCu = 160 * 1024;
constexpr size_t kQtabEntries = 4u << 20;  // QPP table arena (8 MiB): every size at ~11 window counts
constexpr size_t kRmEntries = 8u << 20;    // rate matching table arena (16 MiB, >= 450 tables)
constexpr int kDefaultLdsBudget = 30 * 1024;
constexpr int kTbFailWords = 1 << 16;  // transport blocks per purge launch

struct PlanSlot {
    std::string key;
    char *d_buf = nullptr;   // device copy of the plan
    char *h_buf = nullptr;   // pinned staging
    hipEvent_t ev = nullptr; // completion of the last upload from h_buf
    uint64_t last_use = 0;
    // decoded plan
    int n_items = 0, grid = 0, wg = 0, lds = 0;
    int resident = 0;   // work groups the device holds at once (occupancy x CUs)
    int64_t stride = 0;
    int n_cb = 0, n_tb = 0;
    int asm_words = 0;  // largest (B + 31) / 32 of the plan's transport blocks
    int max_k = 0;      // rate matching plans: the largest K
    int state_slots = 1;  // most blocks of any item
    bool uneven = false;  // some item's last window is shorter
    bool exact = false;   // exact window boundaries (win_init = 2): transfer-run scratch
    bool mi = false;      // mutual-information stop (early_stop bit 1): LDS table and sums
    size_t off_items = 0, off_cbs = 0, off_tbs = 0, off_enc = 0;
};

}  // namespace

struct tdec_ctx {
    int device = 0;
    int num_cus = 0;
    size_t budget = 0;
    uint32_t *d_crc_tab = nullptr;
    char *d_scratch = nullptr;
    size_t scratch_bytes = 0;
    uint32_t *d_hard = nullptr;
    size_t hard_words_cap = 0;
    uint8_t *d_ok = nullptr, *d_it = nullptr;
    size_t flags_cap = 0;
    uint8_t *d_encbuf = nullptr;
    size_t encbuf_bytes = 0;
    uint32_t *d_counter = nullptr;  // work distribution counters of the decode kernel (kCtrBytes)
    uint32_t *d_tbfail = nullptr;   // per transport block failure marks (purge), kTbFailWords
    // QPP LDS-address tables, one per (K, windows) shape, appended on first
    // use and kept for the context's lifetime; the pinned mirror is never
    // rewritten, so its asynchronous uploads need no synchronisation
    uint16_t *d_qtab = nullptr;
    uint16_t *h_qtab = nullptr;
    size_t qtab_cap = 0, qtab_used = 0;
    std::map<int64_t, int64_t> qtab_off;
    PlanSlot slots[kPlanSlots];
    uint64_t clock = 0;
    int32_t tuned_nw[kNumK] = {};  // autotuned window count per size (0 = default rule)
    uint32_t tune_gen = 0;         // bumped whenever tuned_nw changes (enters plan keys)
    std::map<int64_t, int> occ_cache;  // resident decode work groups per CU by (threads, LDS)
    // rate matching rank tables by (K, F, Ncb), appended like the QPP tables
    struct RmTab {
        int64_t off;
        int32_t n_valid, r0[4];
    };
    uint16_t *d_rmtab = nullptr;
    uint16_t *h_rmtab = nullptr;
    size_t rm_cap = 0, rm_used = 0;
    std::map<int64_t, RmTab> rm_tabs;
    int lds_budget = kDefaultLdsBudget;  // LDS bytes per work group the planner aims for
    int item_order = TDEC_ORDER_K_DESC;  // order of the work items (TDEC_ORDER_*)
    int grid_cap = 0;            // 0: occupancy-derived persistent grid
    int launch_reserve = 0;      // resident slots a launch leaves free (launch lanes)
    int max_nw = 0;              // most windows per block (0 = no limit; the ring kernel's shape)
    bool small_asm = false;      // transport block assembly in kAsmGrid small work groups
};

namespace {

bool params_ok(const tdec_params *p) { return tdec::params_valid(p); }

int32_t pick_windows(int32_t K)
{
    // Aim for windows of ~192 steps (the shape at which 32 windows of a
    // 6144-bit block fill a wave): the largest window count with W a
    // multiple of 8 and W >= 192, else full length.
    int best = 1;
    for (int nw = 1; nw <= 64; ++nw)
        if (K % nw == 0 && (K / nw) % 8 == 0 && K / nw >= 192) best = nw;
    return best;
}

bool windows_ok(int32_t K, int32_t nw)
{
    if (nw < 1 || nw > kMaxWgThreads / 2) return false;
    const int32_t W = win_len(K, nw);
    return W > 0 && W % kSeg == 0 && (K - (nw - 1) * W) % kSeg == 0;
}

int32_t ctx_windows(const tdec_ctx *ctx, int32_t K)
{
    const int i = k_index(K);
    int32_t nw = ctx && i >= 0 && ctx->tuned_nw[i] > 0 ? ctx->tuned_nw[i] : pick_windows(K);
    // a window limit takes the most windows it allows (one always does)
    if (ctx && ctx->max_nw > 0 && nw > ctx->max_nw) {
        nw = ctx->max_nw;
        while (nw > 1 && !windows_ok(K, nw)) --nw;
    }
    return nw;
}

struct CbReq {
    int32_t K, nw;
    DecCb cb;
};

// Rank table of (K, F, Ncb): the [3][K+4] index of every non-<NULL> entry
// among the first Ncb of the circular buffer, in buffer order, and for each
// redundancy version the rank at which its reading starts.  Added (upload
// on `st`) on first use; null when the arena is full.
const tdec_ctx::RmTab *rm_get(tdec_ctx *ctx, int32_t K, int32_t F, int32_t Ncb, hipStream_t st)
{
    const int64_t key = ((int64_t)K << 40) | ((int64_t)F << 20) | Ncb;
    auto f = ctx->rm_tabs.find(key);
    if (f != ctx->rm_tabs.end()) return &f->second;
    std::vector<int32_t> w(3 * 32 * ((K + 4 + 31) / 32));
    rm_buffer(K, F, w.data());
    size_t n = 0;
    for (int32_t j = 0; j < Ncb; ++j) n += w[j] >= 0;
    const size_t na = (n + 7) & ~(size_t)7;
    if (n == 0 || ctx->rm_used + na > ctx->rm_cap) return nullptr;
    tdec_ctx::RmTab t;
    t.off = (int64_t)ctx->rm_used;
    t.n_valid = (int32_t)n;
    uint16_t *h = ctx->h_rmtab + t.off;
    int32_t r = 0;
    for (int32_t j = 0; j < Ncb; ++j)
        if (w[j] >= 0) h[r++] = (uint16_t)w[j];
    const int32_t R = (K + 4 + 31) / 32;
    for (int rv = 0; rv < 4; ++rv) {
        const int32_t k0 = (R * (2 * ((Ncb + 8 * R - 1) / (8 * R)) * rv + 2)) % Ncb;
        int32_t c = 0;
        for (int32_t j = 0; j < k0; ++j) c += w[j] >= 0;
        t.r0[rv] = c % t.n_valid;
    }
    if (hipMemcpyAsync(ctx->d_rmtab + t.off, h, n * 2, hipMemcpyHostToDevice, st) != hipSuccess)
        return nullptr;
    ctx->rm_used += na;
    return &(ctx->rm_tabs[key] = t);
}

// Fill the QPP address table of shape (K, nw) into dst: unit u = t4 * nw + w
// holds the LDS byte offsets 2 * epad(pi(k)) of steps k = w * W + 4 * t4 + j.
// Units past K (the pad of a shorter last window) hold 0 and are never read.
void qtab_fill(int32_t K, int32_t nw, uint16_t *dst)
{
    const int32_t W = win_len(K, nw);
    std::vector<int32_t> pi(K);
    tdec_qpp(K, pi.data(), nullptr, nullptr);
    for (int u = 0; u < nw * W / 4; ++u) {
        const int t4 = u / nw, w = u % nw;
        for (int j = 0; j < 4; ++j) {
            const int k = w * W + 4 * t4 + j;
            dst[4 * u + j] = k < K ? (uint16_t)(2 * epad(pi[k])) : 0;
        }
    }
}

size_t qtab_entries(int32_t K, int32_t nw) { return (size_t)nw * win_len(K, nw); }

// Element offset of the (K, nw) table in the context's table arena, adding
// it (upload enqueued on `st`) on first use; -1 when the arena is full.
int64_t qtab_get(tdec_ctx *ctx, int32_t K, int32_t nw, hipStream_t st)
{
    const int64_t key = (int64_t)K * 1024 + nw;
    auto f = ctx->qtab_off.find(key);
    if (f != ctx->qtab_off.end()) return f->second;
    // tables start on 128-byte lines: a table added while a persistent
    // kernel runs shares no cache line with the tables it has read
    const size_t ne = qtab_entries(K, nw), n = (ne + 63) & ~(size_t)63;
    if (ctx->qtab_used + n > ctx->qtab_cap) return -1;
    const int64_t off = (int64_t)ctx->qtab_used;
    qtab_fill(K, nw, ctx->h_qtab + off);
    if (hipMemcpyAsync(ctx->d_qtab + off, ctx->h_qtab + off, ne * 2, hipMemcpyHostToDevice,
                       st) != hipSuccess)
        return -1;
    ctx->qtab_used += n;
    ctx->qtab_off[key] = off;
    return off;
}

// Global scratch bytes of one work item of `lanes` windows of W steps:
// restaged inputs, checkpoints, boundaries, and with exact boundaries the
// transfer runs (2 directions x 8 states x 32 bytes per lane).
int64_t item_scratch(int lanes, int W, bool exact)
{
    const int64_t need = (int64_t)lanes * W * 6 + (int64_t)(W / kSeg) * lanes * 16 +
                         (int64_t)4 * lanes * 16 + (exact ? (int64_t)lanes * 512 : 0) + 256;
    return (need + 255) & ~(int64_t)255;
}

// Build the decode plan (items + code block list) from a request.
// scratch_cap: bytes of per-work-group scratch the launch may use (the
// context's workspace, or the fixed scratch of the allocation-free entry).
tdec_status build_decode_plan(tdec_ctx *ctx, std::vector<CbReq> &reqs, PlanSlot &ps,
                              std::vector<char> &blob, const std::vector<TbItem> *tbs,
                              hipStream_t st, bool exact, bool mi, size_t scratch_cap)
{
    // group by (K, nw), biggest blocks first (or smallest first), request
    // order within a group: a counting sort over the size table (a size has
    // one window count per plan; mixed counts for one size fall back to a
    // comparison sort); or keep the request's order
    std::vector<int> order(reqs.size());
    const bool asc = ctx->item_order == TDEC_ORDER_K_ASC;
    if (ctx->item_order == TDEC_ORDER_REQUEST) {
        // the request's own order: runs of equal (K, nw) become items
        for (size_t i = 0; i < reqs.size(); ++i) order[i] = (int)i;
    } else {
        int cnt[kNumK + 1] = {}, nw_of[kNumK];
        bool mixed = false;
        for (const CbReq &r : reqs) {
            const int ki = k_index(r.K);
            if (cnt[ki + 1]++ == 0) nw_of[ki] = r.nw;
            else mixed = mixed || nw_of[ki] != r.nw;
        }
        if (!mixed) {
            int pos[kNumK], at = 0;
            for (int j = 0; j < kNumK; ++j) {
                const int ki = asc ? j : kNumK - 1 - j;
                pos[ki] = at;
                at += cnt[ki + 1];
            }
            for (size_t i = 0; i < reqs.size(); ++i) order[pos[k_index(reqs[i].K)]++] = (int)i;
        } else {
            for (size_t i = 0; i < reqs.size(); ++i) order[i] = (int)i;
            std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
                if (reqs[a].K != reqs[b].K) return asc ? reqs[a].K < reqs[b].K : reqs[a].K > reqs[b].K;
                return reqs[a].nw < reqs[b].nw;
            });
        }
    }
    int max_nw = 1;
    for (auto &r : reqs) max_nw = std::max(max_nw, r.nw);
    // two lanes per window, in two halves of the work group (forward-first
    // and backward-first waves)
    const int half = ((max_nw + 63) / 64) * 64;
    const int wg = 2 * half;
    if (wg > kMaxWgThreads) return TDEC_EINVAL;
    std::vector<DecItem> items;
    std::vector<DecCb> cbl;
    cbl.reserve(reqs.size());
    int lds = 0, max_n = 1;
    bool uneven = false;
    int64_t stride = 0;
    size_t i = 0;
    items.reserve(reqs.size());
    // per-size constants, computed once per run of equal (K, nw)
    DecItem proto{};
    int cap = 0, gK = -1, gnw = -1;
    while (i < order.size()) {
        const CbReq &r0 = reqs[order[i]];
        if (r0.K != gK || r0.nw != gnw) {
            gK = r0.K;
            gnw = r0.nw;
            const int sb = lds_slot_bytes(gK);
            cap = std::min(half / gnw, kMaxSlotsPerWg);
            cap = std::min(cap, std::max(1, ctx->lds_budget / sb));
            proto.K = gK;
            proto.nw = gnw;
            proto.W = win_len(gK, gnw);
            int32_t f1, f2;
            qpp_coeffs(k_index(gK), &f1, &f2);
            proto.f1 = f1;
            proto.f2 = f2;
            proto.lds_slot = sb;
            const int64_t off = qtab_get(ctx, gK, gnw, st);
            if (off < 0) return TDEC_ENOMEM;
            proto.qtab = (int32_t)off;
        }
        const int K = gK, nw = gnw, W = proto.W, sb = proto.lds_slot;
        DecItem it = proto;
        it.cb0 = (int)cbl.size();
        int n = 0;
        while (i < order.size() && n < cap && reqs[order[i]].K == K && reqs[order[i]].nw == nw) {
            cbl.push_back(reqs[order[i]].cb);
            ++i;
            ++n;
        }
        it.ncb = n;
        items.push_back(it);
        uneven = uneven || (int64_t)nw * W != K;
        lds = std::max(lds, n * sb);
        max_n = std::max(max_n, n);
        stride = std::max(stride, item_scratch(n * nw, W, exact));
    }
    lds += lds_state_bytes(max_n) + (mi ? lds_mi_bytes(max_n) : 0);
    // persistent grid: as many work groups as can be resident
    int occ = 0;
    const int64_t okey = (int64_t)mi << 44 | (int64_t)wg << 34 | (int64_t)exact << 33 |
                         (int64_t)uneven << 32 | (uint32_t)lds;
    auto oc = ctx->occ_cache.find(okey);
    if (oc != ctx->occ_cache.end()) {
        occ = oc->second;
    } else {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, decode_kernel_address(uneven, exact, mi), wg,
                                                         lds) !=
                hipSuccess ||
            occ < 1)
            occ = std::max(1, kLdsPerCu / std::max(lds, 1));
        ctx->occ_cache[okey] = occ;
    }
    int grid = std::min<int64_t>((int64_t)items.size(), (int64_t)occ * ctx->num_cus);
    if (ctx->grid_cap > 0) grid = std::min(grid, ctx->grid_cap);
    const int64_t fit = (int64_t)(scratch_cap / (size_t)stride);
    if (fit < 1) return TDEC_ENOMEM;
    grid = (int)std::min<int64_t>(grid, fit);
    grid = std::max(grid, 1);

    // serialise: [items][cbs][tbs]
    ps.off_items = 0;
    ps.off_cbs = (items.size() * sizeof(DecItem) + 255) & ~(size_t)255;
    ps.off_tbs = ps.off_cbs + ((cbl.size() * sizeof(DecCb) + 255) & ~(size_t)255);
    const size_t ntb = tbs ? tbs->size() : 0;
    const size_t total = ps.off_tbs + ntb * sizeof(TbItem);
    if (total > kPlanSlotBytes) return TDEC_ENOMEM;
    blob.assign(total, 0);
    memcpy(blob.data() + ps.off_items, items.data(), items.size() * sizeof(DecItem));
    memcpy(blob.data() + ps.off_cbs, cbl.data(), cbl.size() * sizeof(DecCb));
    if (ntb) memcpy(blob.data() + ps.off_tbs, tbs->data(), ntb * sizeof(TbItem));
    ps.n_items = (int)items.size();
    ps.n_cb = (int)cbl.size();
    ps.n_tb = (int)ntb;
    ps.asm_words = 0;
    for (size_t t = 0; t < ntb; ++t) ps.asm_words = std::max(ps.asm_words, ((*tbs)[t].B + 31) / 32);
    ps.grid = grid;
    ps.resident = (int)std::min<int64_t>((int64_t)occ * ctx->num_cus, 1 << 30);
    ps.wg = wg;
    ps.lds = lds;
    ps.state_slots = max_n;
    ps.uneven = uneven;
    ps.exact = exact;
    ps.mi = mi;
    ps.stride = stride;
    return TDEC_OK;
}

// Find a cached plan for `key`, or claim the least recently used slot.
PlanSlot *lookup(tdec_ctx *ctx, const std::string &key, bool *hit)
{
    ++ctx->clock;
    for (auto &s : ctx->slots)
        if (!s.key.empty() && s.key == key) {
            s.last_use = ctx->clock;
            *hit = true;
            return &s;
        }
    PlanSlot *v = &ctx->slots[0];
    for (auto &s : ctx->slots)
        if (s.last_use < v->last_use) v = &s;
    *hit = false;
    return v;
}

tdec_status upload(tdec_ctx *ctx, PlanSlot *ps, const std::string &key, const std::vector<char> &blob,
                   hipStream_t st)
{
    if (hipEventSynchronize(ps->ev) != hipSuccess) return TDEC_EDEVICE;
    memcpy(ps->h_buf, blob.data(), blob.size());
    if (hipMemcpyAsync(ps->d_buf, ps->h_buf, blob.size(), hipMemcpyHostToDevice, st) != hipSuccess)
        return TDEC_EDEVICE;
    if (hipEventRecord(ps->ev, st) != hipSuccess) return TDEC_EDEVICE;
    ps->key = key;
    ps->last_use = ctx->clock;
    return TDEC_OK;
}

// fixed: the fixed scratch of the allocation-free entry (counters, then
// per-work-group scratch) instead of the context's workspace.
tdec_status launch_plan(tdec_ctx *ctx, PlanSlot *ps, const int16_t *d_llr,
                        const tdec_params *p, uint8_t *d_bits, uint8_t *d_ok, uint8_t *d_it,
                        bool hard, hipStream_t st, char *fixed = nullptr)
{
    DecArgs a;
    a.items = (const DecItem *)(ps->d_buf + ps->off_items);
    a.n_items = ps->n_items;
    a.cbs = (const DecCb *)(ps->d_buf + ps->off_cbs);
    a.llr = d_llr;
    a.bits = d_bits;
    a.crc_ok = d_ok;
    a.iters = d_it;
    a.hard = hard ? ctx->d_hard : nullptr;
    a.crc_tab = ctx->d_crc_tab;
    a.scratch = fixed ? fixed + kCtrBytes : ctx->d_scratch;
    a.scratch_stride = ps->stride;
    a.counter = fixed ? (uint32_t *)fixed : ctx->d_counter;
    a.qtab = ctx->d_qtab;
    a.mi_tab = ctx->d_crc_tab + kCrcTabWords;
    a.max_iters = p->max_iters;
    a.early_stop = p->early_stop;
    a.win_init = p->win_init;
    a.mi_eps = p->mi_eps;
    a.state_slots = ps->state_slots;
    // purge (transport block plans): the failure marks start clear
    const bool purge = (p->early_stop & TDEC_STOP_PURGE) && ps->n_tb > 0 && !fixed;
    a.tb_fail = purge ? ctx->d_tbfail : nullptr;
    // the plan's scratch and LDS layouts
    if ((p->win_init == 2) != ps->exact || ((p->early_stop & 2) != 0) != ps->mi) return TDEC_EINVAL;
    // the fixed counters start every call at zero (another call may have
    // left them set if it overlapped this one, which the header forbids)
    if (fixed && launch_zero_words((uint32_t *)fixed, kCtrBytes / 4, st)) return TDEC_EDEVICE;
    if (purge && ps->n_tb > kTbFailWords) return TDEC_ENOMEM;
    if (purge && launch_zero_words(ctx->d_tbfail, ps->n_tb, st)) return TDEC_EDEVICE;
    int grid = ps->grid;
    if (ctx->launch_reserve > 0) grid = std::max(1, std::min(grid, ps->resident - ctx->launch_reserve));
    if (launch_decode(a, ps->uneven, ps->exact, ps->mi, grid, ps->wg, ps->lds, st))
        return TDEC_EDEVICE;
    return TDEC_OK;
}

// Plan cache keys: everything the plan depends on (the tuned window table
// enters through its generation counter).
std::string cb_key(int32_t n_cb, const tdec_cb_desc *desc, const tdec_params *p, bool bits,
                   uint32_t gen)
{
    std::string key(1, 'C');
    key.append((const char *)&p->n_windows, sizeof(int32_t));
    key.push_back((p->win_init == 2 ? 1 : 0) | ((p->early_stop & 2) ? 2 : 0));
    key.append((const char *)&gen, sizeof gen);
    key.push_back(bits ? 1 : 0);
    key.append((const char *)desc, sizeof(tdec_cb_desc) * (size_t)n_cb);
    return key;
}

std::string tb_key(int32_t n_tb, const int32_t *tbs, const int64_t *llr_off,
                   const int64_t *bits_off, const tdec_params *p, uint32_t gen)
{
    std::string key(1, 'T');
    key.append((const char *)&p->n_windows, sizeof(int32_t));
    key.push_back((p->win_init == 2 ? 1 : 0) | ((p->early_stop & 2) ? 2 : 0));
    key.append((const char *)&gen, sizeof gen);
    key.push_back(bits_off ? 1 : 0);
    key.append((const char *)tbs, sizeof(int32_t) * (size_t)n_tb);
    key.append((const char *)llr_off, sizeof(int64_t) * (size_t)n_tb);
    if (bits_off) key.append((const char *)bits_off, sizeof(int64_t) * (size_t)n_tb);
    return key;
}

// Validate code block descriptors and turn them into plan requests.
tdec_status make_cb_reqs(const tdec_ctx *ctx, int32_t n_cb, const tdec_cb_desc *desc,
                         const tdec_params *params, bool bits, std::vector<CbReq> &reqs)
{
    reqs.resize((size_t)n_cb);
    for (int32_t i = 0; i < n_cb; ++i) {
        const tdec_cb_desc &d = desc[i];
        if (k_index(d.K) < 0 || d.F < 0 || d.F >= d.K || d.crc < 0 || d.crc > 2 || d.llr_off < 0)
            return TDEC_EINVAL;
        if (d.crc && d.K - d.F < 24) return TDEC_EINVAL;
        if (bits && d.bits_off < 0) return TDEC_EINVAL;
        const int32_t nw = params->n_windows ? params->n_windows : ctx_windows(ctx, d.K);
        if (!windows_ok(d.K, nw)) return TDEC_EINVAL;
        CbReq &r = reqs[i];
        r.K = d.K;
        r.nw = nw;
        r.cb.llr_off = d.llr_off;
        r.cb.bits_off = bits ? d.bits_off : -1;
        r.cb.hard_off = -1;
        r.cb.out_idx = i;
        r.cb.F = d.F;
        r.cb.crc = d.crc;
        r.cb.rsv = 0;
        r.cb.tb = -1;
    }
    return TDEC_OK;
}

// Segment transport blocks into plan requests plus the assembly list.
tdec_status make_tb_reqs(const tdec_ctx *ctx, int32_t n_tb, const int32_t *tbs,
                         const int64_t *llr_off, const int64_t *bits_off,
                         const tdec_params *params, std::vector<CbReq> &reqs,
                         std::vector<TbItem> &tbl)
{
    tbl.assign((size_t)n_tb, TbItem{});
    reqs.clear();
    reqs.reserve((size_t)n_tb * 2);
    int64_t hard = 0;
    int32_t cbi = 0;
    for (int32_t t = 0; t < n_tb; ++t) {
        int32_t s[8];
        if (segment(tbs[t], s)) return TDEC_ERANGE;
        if (s[1] > 64) return TDEC_ERANGE;
        if (llr_off[t] < 0 || (bits_off && bits_off[t] < 0)) return TDEC_EINVAL;
        TbItem &ti = tbl[t];
        ti.tbs = tbs[t];
        ti.B = s[0];
        ti.C = s[1];
        ti.L = s[2];
        ti.Kplus = s[3];
        ti.Kminus = s[4];
        ti.Cminus = s[6];
        ti.F = s[7];
        ti.hard_off = hard;
        ti.bits_off = bits_off ? bits_off[t] : -1;
        ti.cb_idx0 = cbi;
        ti.res_idx = t;
        int64_t off = llr_off[t];
        for (int r = 0; r < s[1]; ++r) {
            const int32_t K = r < s[6] ? s[4] : s[3];
            const int32_t nw = params->n_windows ? params->n_windows : ctx_windows(ctx, K);
            if (!windows_ok(K, nw)) return TDEC_EINVAL;
            CbReq q;
            q.K = K;
            q.nw = nw;
            q.cb.llr_off = off;
            q.cb.bits_off = -1;
            q.cb.hard_off = hard;
            q.cb.out_idx = cbi;
            q.cb.F = (int16_t)(r == 0 ? s[7] : 0);
            q.cb.crc = (int8_t)(s[1] > 1 ? TDEC_CRC24B : TDEC_CRC24A);
            q.cb.rsv = 0;
            q.cb.tb = t;
            reqs.push_back(q);
            off += 3 * (int64_t)(K + 4);
            hard += hard_words(K);
            ++cbi;
        }
    }
    if ((size_t)hard > ctx->hard_words_cap || (size_t)cbi > ctx->flags_cap) return TDEC_ENOMEM;
    return TDEC_OK;
}

// Decode + assemble launches of a transport block plan whose device copy is at d_plan.
tdec_status launch_tb_plan(tdec_ctx *ctx, PlanSlot *ps, char *d_plan, const int16_t *d_llr,
                           const tdec_params *params, uint8_t *d_bits, tdec_tb_result *d_res,
                           hipStream_t st, hipEvent_t ev_start = nullptr,
                           hipEvent_t ev_mid = nullptr)
{
    PlanSlot v = *ps;
    v.d_buf = d_plan;
    if (ev_start && hipEventRecord(ev_start, st) != hipSuccess) return TDEC_EDEVICE;
    tdec_status s = launch_plan(ctx, &v, d_llr, params, nullptr, ctx->d_ok, ctx->d_it, true, st);
    if (s != TDEC_OK) return s;
    if (ev_mid && hipEventRecord(ev_mid, st) != hipSuccess) return TDEC_EDEVICE;
    if (launch_tb_assemble((const TbItem *)(d_plan + ps->off_tbs), ps->n_tb, ps->asm_words,
                           ctx->d_hard, ctx->d_ok, ctx->d_it,
                           (params->early_stop & TDEC_STOP_PURGE) ? ctx->d_tbfail : nullptr,
                           ctx->d_crc_tab, d_bits, d_res, ctx->small_asm ? kAsmGrid : 0, st))
        return TDEC_EDEVICE;
    return TDEC_OK;
}

}  // namespace

struct tdec_graph {
    tdec_ctx *ctx = nullptr;
    char *d_plan = nullptr;
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
};

namespace {

void graph_free(tdec_graph *g)
{
    if (!g) return;
    if (g->ge) (void)hipGraphExecDestroy(g->ge);
    if (g->g) (void)hipGraphDestroy(g->g);
    if (g->d_plan) (void)hipFree(g->d_plan);
    delete g;
}

// Build a plan into a private device copy, then capture `body` on a private
// stream into an instantiated graph.
template <class F>
tdec_status graph_capture(tdec_ctx *ctx, std::vector<CbReq> &reqs,
                                 const std::vector<TbItem> *tbl, bool exact, bool mi, F body,
                                 tdec_graph **out)
{
    PlanSlot ps;
    std::vector<char> blob;
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return TDEC_EDEVICE;
    tdec_status s = build_decode_plan(ctx, reqs, ps, blob, tbl, cs, exact, mi, ctx->scratch_bytes);
    tdec_graph *g = nullptr;
    if (s == TDEC_OK) {
        g = new tdec_graph();
        g->ctx = ctx;
        if (hipMalloc(&g->d_plan, blob.size()) != hipSuccess ||
            hipMemcpyAsync(g->d_plan, blob.data(), blob.size(), hipMemcpyHostToDevice, cs) !=
                hipSuccess ||
            hipStreamSynchronize(cs) != hipSuccess)
            s = TDEC_ENOMEM;
    }
    if (s == TDEC_OK) {
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            s = TDEC_EDEVICE;
        } else {
            s = body(ps, g->d_plan, cs);
            hipGraph_t gr = nullptr;
            const bool ended = hipStreamEndCapture(cs, &gr) == hipSuccess;
            g->g = gr;
            if (s == TDEC_OK && (!ended || !gr ||
                                 hipGraphInstantiate(&g->ge, gr, nullptr, nullptr, 0) != hipSuccess))
                s = TDEC_EDEVICE;
        }
    }
    (void)hipStreamDestroy(cs);
    if (s != TDEC_OK) {
        graph_free(g);
        return s;
    }
    *out = g;
    return TDEC_OK;
}

}  // namespace

extern "C" {

tdec_status tdec_segment(int32_t tbs, tdec_seg *out)
{
    if (!out) return TDEC_EINVAL;
    int32_t s[8];
    if (segment(tbs, s)) return TDEC_ERANGE;
    out->B = s[0];
    out->C = s[1];
    out->L = s[2];
    out->Kplus = s[3];
    out->Kminus = s[4];
    out->Cplus = s[5];
    out->Cminus = s[6];
    out->F = s[7];
    return TDEC_OK;
}

int64_t tdec_tb_llr_count(int32_t tbs)
{
    int32_t s[8];
    if (segment(tbs, s)) return -1;
    return 3 * ((int64_t)s[5] * (s[3] + 4) + (int64_t)s[6] * (s[4] + 4));
}

int32_t tdec_k_table(int32_t *out188)
{
    if (out188)
        for (int i = 0; i < kNumK; ++i) out188[i] = k_of_index(i);
    return kNumK;
}

tdec_status tdec_qpp(int32_t K, int32_t *pi, int32_t *f1, int32_t *f2)
{
    const int i = k_index(K);
    if (i < 0) return TDEC_EINVAL;
    int32_t a, b;
    qpp_coeffs(i, &a, &b);
    if (f1) *f1 = a;
    if (f2) *f2 = b;
    if (pi) {
        // second-order recurrence: pi(i+1) = pi(i) + g(i), g(i+1) = g(i) + 2 f2
        int64_t p = 0, g = (a + b) % K;
        for (int32_t k = 0; k < K; ++k) {
            pi[k] = (int32_t)p;
            p = (p + g) % K;
            g = (g + 2 * b) % K;
        }
    }
    return TDEC_OK;
}

tdec_status tdec_create(int device, size_t hbm_budget_bytes, tdec_ctx **out)
{
    if (!out) return TDEC_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return TDEC_EDEVICE;
    if (hipSetDevice(device) != hipSuccess) return TDEC_EDEVICE;
    // the device address of the fixed scratch (allocation-free entry point)
    if (static_scratch_init(device) != 0) return TDEC_EDEVICE;
    tdec_ctx *c = new tdec_ctx();
    c->device = device;
    c->budget = hbm_budget_bytes ? hbm_budget_bytes : ((size_t)1 << 30);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        delete c;
        return TDEC_EDEVICE;
    }
    c->num_cus = prop.multiProcessorCount;
    const size_t tab_bytes = kTabWords * sizeof(uint32_t);
    c->flags_cap = 1 << 20;
    c->encbuf_bytes = 1 << 20;
    const size_t plan_bytes = (size_t)kPlanSlots * kPlanSlotBytes;
    c->qtab_cap = kQtabEntries;
    c->rm_cap = kRmEntries;
    const size_t fixed = tab_bytes + 2 * c->flags_cap + c->encbuf_bytes + plan_bytes +
                         c->qtab_cap * 2 + c->rm_cap * 2 + (size_t)kTbFailWords * 4;
    if (c->budget < fixed + (16u << 20)) {
        delete c;
        return TDEC_ENOMEM;
    }
    const size_t rest = c->budget - fixed;
    c->hard_words_cap = std::min<size_t>(rest / 8, (size_t)128 << 20) / 4;
    c->scratch_bytes = rest - c->hard_words_cap * 4;
    bool ok = hipMalloc(&c->d_crc_tab, tab_bytes) == hipSuccess &&
              hipMalloc(&c->d_scratch, c->scratch_bytes) == hipSuccess &&
              hipMalloc(&c->d_hard, c->hard_words_cap * 4) == hipSuccess &&
              hipMalloc(&c->d_ok, c->flags_cap) == hipSuccess &&
              hipMalloc(&c->d_it, c->flags_cap) == hipSuccess &&
              hipMalloc(&c->d_encbuf, c->encbuf_bytes) == hipSuccess &&
              hipMalloc(&c->d_counter, kCtrBytes) == hipSuccess &&
              hipMalloc(&c->d_tbfail, (size_t)kTbFailWords * 4) == hipSuccess &&
              hipMemset(c->d_counter, 0, kCtrBytes) == hipSuccess &&
              hipMalloc(&c->d_qtab, c->qtab_cap * 2) == hipSuccess &&
              hipHostMalloc(&c->h_qtab, c->qtab_cap * 2, hipHostMallocDefault) == hipSuccess &&
              hipMalloc(&c->d_rmtab, c->rm_cap * 2) == hipSuccess &&
              hipHostMalloc(&c->h_rmtab, c->rm_cap * 2, hipHostMallocDefault) == hipSuccess;
    for (auto &s : c->slots) {
        ok = ok && hipMalloc(&s.d_buf, kPlanSlotBytes) == hipSuccess &&
             hipHostMalloc(&s.h_buf, kPlanSlotBytes, hipHostMallocDefault) == hipSuccess &&
             hipEventCreateWithFlags(&s.ev, hipEventDisableTiming) == hipSuccess;
    }
    if (ok) {
        std::vector<uint32_t> tab(kTabWords);
        crc_shift_table(kPoly24A, tab.data(), kCrcTabN);
        crc_shift_table(kPoly24B, tab.data() + kCrcTabN, kCrcTabN);
        crc_x32_table(kPoly24A, tab.data() + 2 * kCrcTabN, kX32N);
        mi_table(tab.data() + kCrcTabWords);
        ok = hipMemcpy(c->d_crc_tab, tab.data(), tab_bytes, hipMemcpyHostToDevice) == hipSuccess;
    }
    if (ok) {
        // the tables of every size at its default window count
        for (int i = 0; i < kNumK; ++i) {
            const int32_t K = k_of_index(i), nw = pick_windows(K);
            const int64_t off = (int64_t)c->qtab_used;
            qtab_fill(K, nw, c->h_qtab + off);
            c->qtab_off[(int64_t)K * 1024 + nw] = off;
            c->qtab_used += (qtab_entries(K, nw) + 7) & ~(size_t)7;
        }
        ok = hipMemcpy(c->d_qtab, c->h_qtab, c->qtab_used * 2, hipMemcpyHostToDevice) == hipSuccess;
    }
    if (!ok) {
        tdec_destroy(c);
        return TDEC_ENOMEM;
    }
    *out = c;
    return TDEC_OK;
}

void tdec_destroy(tdec_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(c->d_crc_tab);
    (void)hipFree(c->d_scratch);
    (void)hipFree(c->d_hard);
    (void)hipFree(c->d_ok);
    (void)hipFree(c->d_it);
    (void)hipFree(c->d_encbuf);
    (void)hipFree(c->d_counter);
    (void)hipFree(c->d_tbfail);
    if (c->d_qtab) (void)hipFree(c->d_qtab);
    if (c->h_qtab) (void)hipHostFree(c->h_qtab);
    if (c->d_rmtab) (void)hipFree(c->d_rmtab);
    if (c->h_rmtab) (void)hipHostFree(c->h_rmtab);
    for (auto &s : c->slots) {
        if (s.d_buf) (void)hipFree(s.d_buf);
        if (s.h_buf) (void)hipHostFree(s.h_buf);
        if (s.ev) (void)hipEventDestroy(s.ev);
    }
    delete c;
}

}  // extern "C"

void tdec::ctx_set_launch_reserve(tdec_ctx *ctx, int n, bool small_asm)
{
    if (!ctx) return;
    ctx->launch_reserve = std::max(0, n);
    ctx->small_asm = small_asm;
}

void tdec::ctx_set_ring_shape(tdec_ctx *ctx, int max_nw, int lds_budget)
{
    if (!ctx) return;
    ctx->max_nw = std::max(0, max_nw);
    ctx->lds_budget = std::max(1, lds_budget);
    ++ctx->tune_gen;
}

tdec_status tdec::ring_plan(tdec_ctx *ctx, int32_t n_tb, const int32_t *tbs, const int64_t *llr_off,
                            const int64_t *bits_off, const tdec_params *params, hipStream_t st,
                            RingPlan *out)
{
    if (!ctx || !out || n_tb <= 0 || !tbs || !llr_off || !params_ok(params)) return TDEC_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return TDEC_EDEVICE;
    const std::string key = tb_key(n_tb, tbs, llr_off, bits_off, params, ctx->tune_gen);
    bool hit;
    PlanSlot *ps = lookup(ctx, key, &hit);
    if (!hit) {
        std::vector<CbReq> reqs;
        std::vector<TbItem> tbl;
        tdec_status s = make_tb_reqs(ctx, n_tb, tbs, llr_off, bits_off, params, reqs, tbl);
        if (s != TDEC_OK) return s;
        std::vector<char> blob;
        s = build_decode_plan(ctx, reqs, *ps, blob, &tbl, st, params->win_init == 2,
                              (params->early_stop & 2) != 0, ctx->scratch_bytes);
        if (s == TDEC_OK) s = upload(ctx, ps, key, blob, st);
        if (s != TDEC_OK) {
            ps->key.clear();
            return s;
        }
    }
    RingPlan &r = *out;
    r.items = (const DecItem *)(ps->h_buf + ps->off_items);
    r.n_items = ps->n_items;
    r.d_cbs = (const DecCb *)(ps->d_buf + ps->off_cbs);
    r.n_cb = ps->n_cb;
    r.d_tbs = (const TbItem *)(ps->d_buf + ps->off_tbs);
    r.n_tb = ps->n_tb;
    r.asm_words = ps->asm_words;
    r.wg = ps->wg;
    r.max_item_lds = 0;
    for (int i = 0; i < ps->n_items; ++i)
        r.max_item_lds = std::max(r.max_item_lds, r.items[i].ncb * r.items[i].lds_slot);
    r.stride = ps->stride;
    r.exact = ps->exact;
    r.mi = ps->mi;
    r.ready = ps->ev;
    r.d_qtab = ctx->d_qtab;
    r.qtab_entries = (int64_t)ctx->qtab_used;
    r.d_hard = ctx->d_hard;
    r.hard_words = (int64_t)ctx->hard_words_cap;
    r.d_ok = ctx->d_ok;
    r.d_it = ctx->d_it;
    r.flags = (int64_t)ctx->flags_cap;
    return TDEC_OK;
}

tdec_status tdec::ring_assemble(tdec_ctx *ctx, const RingPlan &r, const tdec_params *params,
                                uint8_t *d_bits, tdec_tb_result *d_res, hipStream_t st)
{
    if (!ctx || !d_res || !params_ok(params)) return TDEC_EINVAL;
    if (launch_tb_assemble(r.d_tbs, r.n_tb, r.asm_words, ctx->d_hard, ctx->d_ok, ctx->d_it, nullptr,
                           ctx->d_crc_tab, d_bits, d_res, kRingAsmGrid, st))
        return TDEC_EDEVICE;
    return TDEC_OK;
}

int64_t tdec::ring_max_stride(int max_nw, int lds_budget)
{
    // every size, every window count a plan may use, as many blocks per
    // item as the planner packs (see build_decode_plan)
    int64_t m = 0;
    for (int i = 0; i < kNumK; ++i) {
        const int32_t K = k_of_index(i);
        for (int nw = 1; nw <= max_nw; ++nw) {
            if (!windows_ok(K, nw)) continue;
            const int half = ((nw + 63) / 64) * 64;
            int cap = std::min(half / nw, kMaxSlotsPerWg);
            cap = std::min(cap, std::max(1, lds_budget / lds_slot_bytes(K)));
            m = std::max(m, item_scratch(cap * nw, win_len(K, nw), false));
        }
    }
    return m;
}

const uint32_t *tdec::ctx_crc_tab(const tdec_ctx *ctx) { return ctx ? ctx->d_crc_tab : nullptr; }

int tdec::ctx_num_cus(const tdec_ctx *ctx) { return ctx ? ctx->num_cus : 0; }

tdec_status tdec::ctx_clone(const tdec_ctx *src, tdec_ctx **out)
{
    if (!src || !out) return TDEC_EINVAL;
    tdec_status s = tdec_create(src->device, src->budget, out);
    if (s != TDEC_OK) return s;
    tdec_ctx *c = *out;
    c->lds_budget = src->lds_budget;
    c->item_order = src->item_order;
    c->grid_cap = src->grid_cap;
    c->max_nw = src->max_nw;
    for (int i = 0; i < kNumK; ++i) c->tuned_nw[i] = src->tuned_nw[i];
    ++c->tune_gen;
    return TDEC_OK;
}

extern "C" {

tdec_status tdec_set_max_windows(tdec_ctx *ctx, int32_t max_nw)
{
    if (!ctx || max_nw < 0 || max_nw > kMaxWgThreads / 2) return TDEC_EINVAL;
    ctx->max_nw = max_nw;
    ++ctx->tune_gen;
    return TDEC_OK;
}

int32_t tdec_pick_windows(const tdec_ctx *ctx, int32_t K)
{
    (void)ctx;
    if (k_index(K) < 0) return 0;
    return ctx_windows(ctx, K);
}

tdec_status cb_decode_batch(tdec_ctx *ctx, int32_t n_cb, const tdec_cb_desc *desc,
                            const int16_t *d_llr, const tdec_params *params, uint8_t *d_bits,
                            uint8_t *d_crc_ok, uint8_t *d_iters, void *stream)
{
    if (!ctx || n_cb < 0 || !params_ok(params)) return TDEC_EINVAL;
    if (n_cb == 0) return TDEC_OK;
    if (!desc || !d_llr || !d_crc_ok || !d_iters) return TDEC_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    if (hipSetDevice(ctx->device) != hipSuccess) return TDEC_EDEVICE;
    // a batch identical to a cached one reuses its (validated) plan
    const std::string key = cb_key(n_cb, desc, params, d_bits != nullptr, ctx->tune_gen);
    bool hit;
    PlanSlot *ps = lookup(ctx, key, &hit);
    if (hit) return launch_plan(ctx, ps, d_llr, params, d_bits, d_crc_ok, d_iters, false, st);
    std::vector<CbReq> reqs;
    tdec_status s = make_cb_reqs(ctx, n_cb, desc, params, d_bits != nullptr, reqs);
    if (s != TDEC_OK) return s;
    std::vector<char> blob;
    s = build_decode_plan(ctx, reqs, *ps, blob, nullptr, st, params->win_init == 2,
                          (params->early_stop & 2) != 0, ctx->scratch_bytes);
    if (s == TDEC_OK) s = upload(ctx, ps, key, blob, st);
    if (s != TDEC_OK) {
        ps->key.clear();
        return s;
    }
    return launch_plan(ctx, ps, d_llr, params, d_bits, d_crc_ok, d_iters, false, st);
}

tdec_status cb_decode_batch_fixed(tdec_ctx *ctx, int32_t n_cb, const tdec_cb_desc *desc,
                                  const int16_t *d_llr, const tdec_params *params,
                                  uint8_t *d_bits, uint8_t *d_crc_ok, uint8_t *d_iters,
                                  void *stream)
{
    if (!ctx || n_cb < 0 || !params_ok(params)) return TDEC_EINVAL;
    if (n_cb == 0) return TDEC_OK;
    if (!desc || !d_llr || !d_crc_ok || !d_iters) return TDEC_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    if (hipSetDevice(ctx->device) != hipSuccess) return TDEC_EDEVICE;
    char *fixed = static_scratch_ptr(ctx->device);
    if (!fixed) return TDEC_EDEVICE;
    // plans of this entry differ from cb_decode_batch's in their grid (the
    // fixed scratch holds fewer work groups), so their keys differ too
    const std::string key = "F" + cb_key(n_cb, desc, params, d_bits != nullptr, ctx->tune_gen);
    bool hit;
    PlanSlot *ps = lookup(ctx, key, &hit);
    if (hit) return launch_plan(ctx, ps, d_llr, params, d_bits, d_crc_ok, d_iters, false, st, fixed);
    std::vector<CbReq> reqs;
    tdec_status s = make_cb_reqs(ctx, n_cb, desc, params, d_bits != nullptr, reqs);
    if (s != TDEC_OK) return s;
    std::vector<char> blob;
    // ENOMEM when one work group's scratch exceeds the fixed array
    s = build_decode_plan(ctx, reqs, *ps, blob, nullptr, st, params->win_init == 2,
                          (params->early_stop & 2) != 0, kStaticScratchBytes - kCtrBytes);
    if (s == TDEC_OK) s = upload(ctx, ps, key, blob, st);
    if (s != TDEC_OK) {
        ps->key.clear();
        return s;
    }
    return launch_plan(ctx, ps, d_llr, params, d_bits, d_crc_ok, d_iters, false, st, fixed);
}

tdec_status tb_decode_batch(tdec_ctx *ctx, int32_t n_tb, const int32_t *tbs, const int64_t *llr_off,
                            const int64_t *bits_off, const int16_t *d_llr,
                            const tdec_params *params, uint8_t *d_bits, tdec_tb_result *d_res,
                            void *stream)
{
    return tdec::tb_decode_batch_timed(ctx, n_tb, tbs, llr_off, bits_off, d_llr, params, d_bits,
                                       d_res, stream, nullptr, nullptr);
}

}  // extern "C"

bool tdec::params_valid(const tdec_params *p)
{
    return p && p->max_iters >= 1 && p->max_iters <= 16 && p->early_stop >= 0 &&
           p->early_stop <= 7 && p->n_windows >= 0 && p->n_windows <= 128 && p->win_init >= 0 &&
           p->win_init <= 2 && p->mi_eps >= 0 && p->mi_eps <= 32768;
}

tdec_status tdec::tb_decode_batch_timed(tdec_ctx *ctx, int32_t n_tb, const int32_t *tbs,
                                        const int64_t *llr_off, const int64_t *bits_off,
                                        const int16_t *d_llr, const tdec_params *params,
                                        uint8_t *d_bits, tdec_tb_result *d_res, void *stream,
                                        void *ev_start, void *ev_mid)
{
    if (!ctx || n_tb < 0 || !params_ok(params)) return TDEC_EINVAL;
    if (n_tb == 0) return TDEC_OK;
    if (!tbs || !llr_off || !d_llr || !d_res) return TDEC_EINVAL;
    if (d_bits && !bits_off) return TDEC_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    if (hipSetDevice(ctx->device) != hipSuccess) return TDEC_EDEVICE;
    const std::string key =
        tb_key(n_tb, tbs, llr_off, d_bits ? bits_off : nullptr, params, ctx->tune_gen);
    bool hit;
    PlanSlot *ps = lookup(ctx, key, &hit);
    if (!hit) {
        std::vector<CbReq> reqs;
        std::vector<TbItem> tbl;
        tdec_status s = make_tb_reqs(ctx, n_tb, tbs, llr_off, d_bits ? bits_off : nullptr, params,
                                     reqs, tbl);
        if (s != TDEC_OK) return s;
        std::vector<char> blob;
        s = build_decode_plan(ctx, reqs, *ps, blob, &tbl, st, params->win_init == 2,
                              (params->early_stop & 2) != 0, ctx->scratch_bytes);
        if (s == TDEC_OK) s = upload(ctx, ps, key, blob, st);
        if (s != TDEC_OK) {
            ps->key.clear();
            return s;
        }
    }
    return launch_tb_plan(ctx, ps, ps->d_buf, d_llr, params, d_bits, d_res, st,
                          (hipEvent_t)ev_start, (hipEvent_t)ev_mid);
}

extern "C" {

tdec_status tb_decode(tdec_ctx *ctx, const int16_t *d_llr, int32_t tbs, const tdec_params *params,
                      uint8_t *d_bits, tdec_tb_result *d_res, void *stream)
{
    const int64_t lo = 0, bo = 0;
    return tb_decode_batch(ctx, 1, &tbs, &lo, &bo, d_llr, params, d_bits, d_res, stream);
}


// ---------------------------------------------------------------- graphs

tdec_status tdec_graph_cb_decode(tdec_ctx *ctx, int32_t n_cb, const tdec_cb_desc *desc,
                                 const int16_t *d_llr, const tdec_params *params, uint8_t *d_bits,
                                 uint8_t *d_crc_ok, uint8_t *d_iters, tdec_graph **out)
{
    if (!out) return TDEC_EINVAL;
    *out = nullptr;
    if (!ctx || n_cb <= 0 || !params_ok(params) || !desc || !d_llr || !d_crc_ok || !d_iters)
        return TDEC_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return TDEC_EDEVICE;
    std::vector<CbReq> reqs;
    tdec_status s = make_cb_reqs(ctx, n_cb, desc, params, d_bits != nullptr, reqs);
    if (s != TDEC_OK) return s;
    const tdec_params p = *params;
    return graph_capture(ctx, reqs, nullptr, p.win_init == 2, (p.early_stop & 2) != 0,
                         [&](PlanSlot &ps, char *d_plan, hipStream_t cs) {
                             PlanSlot v = ps;
                             v.d_buf = d_plan;
                             return launch_plan(ctx, &v, d_llr, &p, d_bits, d_crc_ok, d_iters,
                                                false, cs);
                         },
                         out);
}

tdec_status tdec_graph_tb_decode(tdec_ctx *ctx, int32_t n_tb, const int32_t *tbs,
                                 const int64_t *llr_off, const int64_t *bits_off,
                                 const int16_t *d_llr, const tdec_params *params, uint8_t *d_bits,
                                 tdec_tb_result *d_res, tdec_graph **out)
{
    if (!out) return TDEC_EINVAL;
    *out = nullptr;
    if (!ctx || n_tb <= 0 || !params_ok(params) || !tbs || !llr_off || !d_llr || !d_res)
        return TDEC_EINVAL;
    if (d_bits && !bits_off) return TDEC_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return TDEC_EDEVICE;
    std::vector<CbReq> reqs;
    std::vector<TbItem> tbl;
    tdec_status s =
        make_tb_reqs(ctx, n_tb, tbs, llr_off, d_bits ? bits_off : nullptr, params, reqs, tbl);
    if (s != TDEC_OK) return s;
    const tdec_params p = *params;
    return graph_capture(ctx, reqs, &tbl, p.win_init == 2, (p.early_stop & 2) != 0,
                         [&](PlanSlot &ps, char *d_plan, hipStream_t cs) {
                             return launch_tb_plan(ctx, &ps, d_plan, d_llr, &p, d_bits, d_res, cs);
                         },
                         out);
}

tdec_status tdec_graph_launch(tdec_graph *g, void *stream)
{
    if (!g || !g->ge) return TDEC_EINVAL;
    if (hipSetDevice(g->ctx->device) != hipSuccess) return TDEC_EDEVICE;
    return hipGraphLaunch(g->ge, (hipStream_t)stream) == hipSuccess ? TDEC_OK : TDEC_EDEVICE;
}

void tdec_graph_destroy(tdec_graph *g)
{
    if (!g) return;
    (void)hipSetDevice(g->ctx->device);
    graph_free(g);
}

// ---------------------------------------------------------------- autotuner

tdec_status tdec_autotune(tdec_ctx *ctx, int32_t n_k, const int32_t *Ks, int32_t min_W,
                          int32_t max_iters, int64_t batch_bits, int32_t *out_nw,
                          float *out_ns_per_kbit, void *stream)
{
    if (!ctx || n_k < 0 || (n_k && !Ks) || min_W < 8 || max_iters < 1 || max_iters > 16 ||
        batch_bits < 0)
        return TDEC_EINVAL;
    for (int32_t i = 0; i < n_k; ++i)
        if (k_index(Ks[i]) < 0) return TDEC_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return TDEC_EDEVICE;
    hipStream_t st = (hipStream_t)stream;
    const int64_t max_cb = std::min<int64_t>((int64_t)ctx->flags_cap, 16384);
    int64_t max_llr = 0;
    for (int32_t i = 0; i < n_k; ++i) {
        const int64_t n = std::min<int64_t>(max_cb, std::max<int64_t>(1, batch_bits / Ks[i]));
        max_llr = std::max<int64_t>(max_llr, n * 3 * (Ks[i] + 4));
    }
    int16_t *d_llr = nullptr;
    uint8_t *d_ok = nullptr, *d_it = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    tdec_status rs = TDEC_OK;
    if (hipMalloc(&d_llr, (size_t)std::max<int64_t>(max_llr, 1) * 2) != hipSuccess ||
        hipMalloc(&d_ok, (size_t)max_cb) != hipSuccess ||
        hipMalloc(&d_it, (size_t)max_cb) != hipSuccess ||
        hipMemsetAsync(d_llr, 0, (size_t)std::max<int64_t>(max_llr, 1) * 2, st) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        rs = TDEC_ENOMEM;
    for (int32_t i = 0; i < n_k && rs == TDEC_OK; ++i) {
        const int32_t K = Ks[i];
        const int64_t n = std::min<int64_t>(max_cb, std::max<int64_t>(1, batch_bits / K));
        std::vector<tdec_cb_desc> desc((size_t)n);
        for (int64_t c = 0; c < n; ++c) {
            desc[c].llr_off = c * 3 * (K + 4);
            desc[c].bits_off = 0;
            desc[c].K = K;
            desc[c].F = 0;
            desc[c].crc = TDEC_CRC_NONE;
            desc[c].rsv = 0;
        }
        int32_t best_nw = pick_windows(K);
        float best = -1.f;
        // candidates: full length, the built-in rule, and the counts whose
        // windows come closest above min_W, 1.5, 2, 3 and 4 times min_W
        std::vector<int32_t> cand = {1, pick_windows(K)};
        for (int f2 : {2, 3, 4, 6, 8}) {
            const int32_t target = std::max(8, min_W * f2 / 2);
            int32_t nw = std::max(1, K / target);
            while (nw > 1 && (!windows_ok(K, nw) || win_len(K, nw) < min_W)) --nw;
            cand.push_back(nw);
        }
        std::sort(cand.begin(), cand.end());
        cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
        for (int32_t nw : cand) {
            if (rs != TDEC_OK) break;
            if (!windows_ok(K, nw) || (nw > 1 && win_len(K, nw) < min_W)) continue;
            const tdec_params p = {max_iters, 0, nw, 1};
            // one untimed launch builds and uploads the plan; then three
            // launches between one pair of events (host clock as a fallback
            // should the events report nothing)
            tdec_status s =
                cb_decode_batch(ctx, (int32_t)n, desc.data(), d_llr, &p, nullptr, d_ok, d_it, st);
            if (s == TDEC_ENOMEM) continue;  // this shape does not fit the workspace
            if (s != TDEC_OK || hipStreamSynchronize(st) != hipSuccess) {
                rs = s != TDEC_OK ? s : TDEC_EDEVICE;
                break;
            }
            float ms = 0.f;
            const auto h0 = std::chrono::steady_clock::now();
            bool ev = hipEventRecord(e0, st) == hipSuccess;
            for (int rep = 0; rep < 3 && rs == TDEC_OK; ++rep)
                rs = cb_decode_batch(ctx, (int32_t)n, desc.data(), d_llr, &p, nullptr, d_ok, d_it, st);
            if (rs != TDEC_OK) break;
            ev = ev && hipEventRecord(e1, st) == hipSuccess;
            if (hipStreamSynchronize(st) != hipSuccess) {
                rs = TDEC_EDEVICE;
                break;
            }
            const auto h1 = std::chrono::steady_clock::now();
            if (!(ev && hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms > 0.f))
                ms = std::chrono::duration<float, std::milli>(h1 - h0).count();
            ms /= 3.f;
            if (rs != TDEC_OK || ms <= 0.f) continue;
            const float ns_kbit = ms * 1e6f / ((float)n * (float)K / 1000.f);
            if (best < 0.f || ns_kbit < best) {
                best = ns_kbit;
                best_nw = nw;
            }
        }
        if (rs != TDEC_OK) break;
        ctx->tuned_nw[k_index(K)] = best_nw;
        if (out_nw) out_nw[i] = best_nw;
        if (out_ns_per_kbit) out_ns_per_kbit[i] = best;
    }
    ++ctx->tune_gen;
    (void)hipStreamSynchronize(st);
    if (d_llr) (void)hipFree(d_llr);
    if (d_ok) (void)hipFree(d_ok);
    if (d_it) (void)hipFree(d_it);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return rs;
}

void tdec_autotune_reset(tdec_ctx *ctx)
{
    if (!ctx) return;
    for (auto &v : ctx->tuned_nw) v = 0;
    ctx->lds_budget = kDefaultLdsBudget;
    ctx->item_order = TDEC_ORDER_K_DESC;
    ctx->grid_cap = 0;
    ++ctx->tune_gen;
}

void tdec_default_knobs(tdec_knobs *out)
{
    if (!out) return;
    out->lds_budget = kDefaultLdsBudget;
    out->order = TDEC_ORDER_K_DESC;
    out->win_target = 0;
    out->grid_cap = 0;
    out->us = 0.f;
}

}  // extern "C"

namespace {

bool knobs_ok(const tdec_knobs *k)
{
    return k && k->lds_budget >= 1 && k->lds_budget <= kLdsPerCu && k->order >= TDEC_ORDER_K_DESC &&
           k->order <= TDEC_ORDER_REQUEST &&
           (k->win_target == -1 || k->win_target == 0 || (k->win_target >= 8 && k->win_target <= 6144)) &&
           k->grid_cap >= 0;
}

// The most windows (at most 128, valid partitions only) whose length is at
// least `target` steps; one window for a block shorter than that.
int32_t windows_for_target(int32_t K, int32_t target)
{
    for (int32_t nw = std::min(128, K / 8); nw > 1; --nw)
        if (windows_ok(K, nw) && win_len(K, nw) >= target) return nw;
    return 1;
}

// Apply knobs; `keep` holds the per-size window counts win_target = -1 keeps.
void apply_knobs(tdec_ctx *ctx, const tdec_knobs &k, const int32_t *keep)
{
    ctx->lds_budget = k.lds_budget;
    ctx->item_order = k.order;
    ctx->grid_cap = k.grid_cap;
    if (k.win_target == 0) {
        for (auto &v : ctx->tuned_nw) v = 0;
    } else if (k.win_target > 0) {
        for (int i = 0; i < kNumK; ++i) ctx->tuned_nw[i] = windows_for_target(k_of_index(i), k.win_target);
    } else if (keep) {
        for (int i = 0; i < kNumK; ++i) ctx->tuned_nw[i] = keep[i];
    }
    ++ctx->tune_gen;
}

}  // namespace

extern "C" {

tdec_status tdec_set_knobs(tdec_ctx *ctx, const tdec_knobs *k)
{
    if (!ctx || !knobs_ok(k)) return TDEC_EINVAL;
    apply_knobs(ctx, *k, nullptr);
    return TDEC_OK;
}

tdec_status tdec_get_knobs(const tdec_ctx *ctx, tdec_knobs *out)
{
    if (!ctx || !out) return TDEC_EINVAL;
    out->lds_budget = ctx->lds_budget;
    out->order = ctx->item_order;
    out->win_target = -1;
    out->grid_cap = ctx->grid_cap;
    out->us = 0.f;
    return TDEC_OK;
}

tdec_status tdec_autotune_batch(tdec_ctx *ctx, int32_t n_tb, const int32_t *tbs,
                                const int64_t *llr_off, const int16_t *d_llr,
                                const tdec_params *params, int32_t min_W, tdec_knobs *out,
                                int32_t max_out, int32_t *n_out, tdec_knobs *best,
                                tdec_knobs *rule, void *stream)
{
    if (n_out) *n_out = 0;
    if (!ctx || n_tb <= 0 || !tbs || !llr_off || !d_llr || !params_ok(params) || min_W < 8 ||
        min_W > 6144 || max_out < 0 || (max_out > 0 && !out))
        return TDEC_EINVAL;
    for (int32_t i = 0; i < n_tb; ++i)
        if (tbs[i] < 1) return TDEC_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return TDEC_EDEVICE;
    hipStream_t st = (hipStream_t)stream;
    // what the context holds now: restored on failure, and the per-size
    // window counts that win_target = -1 keeps
    int32_t keep[kNumK];
    bool tuned = false;
    for (int i = 0; i < kNumK; ++i) {
        keep[i] = ctx->tuned_nw[i];
        tuned = tuned || keep[i] > 0;
    }
    const tdec_knobs saved = {ctx->lds_budget, ctx->item_order, -1, ctx->grid_cap, 0.f};
    std::vector<int64_t> bits_off((size_t)n_tb);
    int64_t nbytes = 0;
    for (int32_t i = 0; i < n_tb; ++i) {
        bits_off[i] = nbytes;
        nbytes += (tbs[i] + 7) / 8;
    }
    uint8_t *d_bits = nullptr;
    tdec_tb_result *d_res = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    tdec_status rs = TDEC_OK;
    if (hipMalloc(&d_bits, (size_t)nbytes) != hipSuccess ||
        hipMalloc(&d_res, (size_t)n_tb * sizeof(tdec_tb_result)) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        rs = TDEC_ENOMEM;
    // one untimed launch (plan build and upload), then `reps` between a pair
    // of events; <0: the knobs do not fit the workspace
    auto time_knobs = [&](const tdec_knobs &k, int reps, float *us) -> tdec_status {
        apply_knobs(ctx, k, keep);
        tdec_status s = tb_decode_batch(ctx, n_tb, tbs, llr_off, bits_off.data(), d_llr, params,
                                        d_bits, d_res, st);
        if (s == TDEC_ENOMEM) {
            *us = -1.f;
            return TDEC_OK;
        }
        if (s != TDEC_OK) return s;
        if (hipStreamSynchronize(st) != hipSuccess || hipEventRecord(e0, st) != hipSuccess)
            return TDEC_EDEVICE;
        for (int r = 0; r < reps; ++r) {
            s = tb_decode_batch(ctx, n_tb, tbs, llr_off, bits_off.data(), d_llr, params, d_bits,
                                d_res, st);
            if (s != TDEC_OK) return s;
        }
        float ms = 0.f;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            return TDEC_EDEVICE;
        *us = ms * 1000.f / (float)reps;
        return TDEC_OK;
    };
    std::vector<tdec_knobs> cand;
    {
        std::vector<int32_t> wins;
        if (tuned) wins.push_back(-1);
        wins.push_back(0);
        if (params->n_windows == 0)
            for (int f2 : {2, 3, 4, 6, 8}) wins.push_back(min_W * f2 / 2);
        for (int32_t w : wins)
            for (int32_t lb : {8192, 16384, kDefaultLdsBudget, 49152, 81920})
                for (int32_t o : {TDEC_ORDER_K_DESC, TDEC_ORDER_K_ASC, TDEC_ORDER_REQUEST})
                    cand.push_back({lb, o, std::min<int32_t>(w, 6144), 0, 0.f});
    }
    for (size_t c = 0; c < cand.size() && rs == TDEC_OK; ++c) rs = time_knobs(cand[c], 3, &cand[c].us);
    tdec_knobs def;
    tdec_default_knobs(&def);
    tdec_knobs pick = def;
    if (rs == TDEC_OK) {
        if (out)
            for (size_t c = 0; c < cand.size() && (int32_t)c < max_out; ++c) out[c] = cand[c];
        if (n_out) *n_out = (int32_t)std::min<size_t>(cand.size(), (size_t)max_out);
        // second pass: the five fastest and the built-in knobs, ten launches each
        std::vector<tdec_knobs> top;
        for (const tdec_knobs &k : cand)
            if (k.us > 0.f) top.push_back(k);
        std::stable_sort(top.begin(), top.end(),
                         [](const tdec_knobs &a, const tdec_knobs &b) { return a.us < b.us; });
        if (top.size() > 5) top.resize(5);
        rs = time_knobs(def, 10, &def.us);
        pick = def;
        for (size_t c = 0; c < top.size() && rs == TDEC_OK; ++c) {
            rs = time_knobs(top[c], 10, &top[c].us);
            if (rs == TDEC_OK && top[c].us > 0.f && (pick.us <= 0.f || top[c].us < pick.us))
                pick = top[c];
        }
    }
    if (rs == TDEC_OK) {
        apply_knobs(ctx, pick, keep);
        if (best) *best = pick;
        if (rule) *rule = def;
    } else {
        apply_knobs(ctx, saved, keep);
    }
    (void)hipStreamSynchronize(st);
    if (d_bits) (void)hipFree(d_bits);
    if (d_res) (void)hipFree(d_res);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return rs;
}


// ---------------------------------------------------------------- rate matching

static tdec_status rm_plan(tdec_ctx *ctx, int32_t n, const tdec_rm_desc *desc, char tag,
                           hipStream_t st, PlanSlot **out)
{
    std::string key(1, tag);
    key.append((const char *)desc, sizeof(tdec_rm_desc) * (size_t)n);
    bool hit;
    PlanSlot *ps = lookup(ctx, key, &hit);
    if (!hit) {
        if (sizeof(RmItem) * (size_t)n > kPlanSlotBytes) return TDEC_ENOMEM;
        std::vector<char> blob(sizeof(RmItem) * (size_t)n);
        RmItem *items = (RmItem *)blob.data();
        int max_k = 0;
        for (int32_t i = 0; i < n; ++i) {
            const tdec_rm_desc &d = desc[i];
            const int32_t kw = 3 * 32 * ((d.K + 4 + 31) / 32);
            if (k_index(d.K) < 0 || d.F < 0 || d.F >= d.K || d.rv < 0 || d.rv > 3 || d.E < 0 ||
                d.Ncb < 0 || d.Ncb > kw || d.e_off < 0 || d.soft_off < 0)
                return TDEC_EINVAL;
            const int32_t ncb = d.Ncb ? d.Ncb : kw;
            const tdec_ctx::RmTab *t = rm_get(ctx, d.K, d.F, ncb, st);
            if (!t) return TDEC_ENOMEM;
            items[i].e_off = d.e_off;
            items[i].soft_off = d.soft_off;
            items[i].tab_off = t->off;
            items[i].K = d.K;
            items[i].E = d.E;
            items[i].n_valid = t->n_valid;
            items[i].r0 = t->r0[d.rv];
            max_k = std::max(max_k, d.K);
        }
        ps->n_cb = n;
        ps->max_k = max_k;
        ps->off_items = 0;
        tdec_status s = upload(ctx, ps, key, blob, st);
        if (s != TDEC_OK) {
            ps->key.clear();
            return s;
        }
    }
    *out = ps;
    return TDEC_OK;
}

tdec_status tdec_derate_batch(tdec_ctx *ctx, int32_t n, const tdec_rm_desc *desc, const void *d_e,
                              int32_t e_bytes, int16_t *d_soft, int32_t combine, void *stream)
{
    if (!ctx || n < 0 || (e_bytes != 1 && e_bytes != 2) || (combine != 0 && combine != 1))
        return TDEC_EINVAL;
    if (n == 0) return TDEC_OK;
    if (!desc || !d_e || !d_soft) return TDEC_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    if (hipSetDevice(ctx->device) != hipSuccess) return TDEC_EDEVICE;
    PlanSlot *ps;
    tdec_status s = rm_plan(ctx, n, desc, 'D', st, &ps);
    if (s != TDEC_OK) return s;
    return launch_derate((const RmItem *)ps->d_buf, n, ps->max_k, d_e, e_bytes, d_soft,
                         ctx->d_rmtab, combine, st)
               ? TDEC_EDEVICE
               : TDEC_OK;
}

tdec_status tdec_rate_match_batch(tdec_ctx *ctx, int32_t n, const tdec_rm_desc *desc,
                                  const uint8_t *d_coded, uint8_t *d_e, void *stream)
{
    if (!ctx || n < 0) return TDEC_EINVAL;
    if (n == 0) return TDEC_OK;
    if (!desc || !d_coded || !d_e) return TDEC_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    if (hipSetDevice(ctx->device) != hipSuccess) return TDEC_EDEVICE;
    PlanSlot *ps;
    tdec_status s = rm_plan(ctx, n, desc, 'M', st, &ps);
    if (s != TDEC_OK) return s;
    return launch_rate_match((const RmItem *)ps->d_buf, n, ps->max_k, d_coded, d_e,
                             ctx->d_rmtab, st)
               ? TDEC_EDEVICE
               : TDEC_OK;
}

static tdec_status encode_list(tdec_ctx *ctx, std::vector<EncCb> &list, const std::string &key,
                               const uint8_t *src, uint8_t *d_coded, hipStream_t st)
{
    bool hit;
    PlanSlot *ps = lookup(ctx, key, &hit);
    if (!hit) {
        const size_t bytes = list.size() * sizeof(EncCb);
        if (bytes > kPlanSlotBytes) return TDEC_ENOMEM;
        std::vector<char> blob(bytes);
        memcpy(blob.data(), list.data(), bytes);
        ps->off_enc = 0;
        ps->n_cb = (int)list.size();
        tdec_status s = upload(ctx, ps, key, blob, st);
        if (s != TDEC_OK) {
            ps->key.clear();
            return s;
        }
    }
    if (launch_encode((const EncCb *)(ps->d_buf + ps->off_enc), ps->n_cb, src, d_coded,
                      ctx->d_crc_tab, st))
        return TDEC_EDEVICE;
    return TDEC_OK;
}

tdec_status cb_encode_batch(tdec_ctx *ctx, int32_t n_cb, const tdec_cb_desc *desc,
                            const uint8_t *d_payload, uint8_t *d_coded, void *stream)
{
    if (!ctx || n_cb < 0) return TDEC_EINVAL;
    if (n_cb == 0) return TDEC_OK;
    if (!desc || !d_payload || !d_coded) return TDEC_EINVAL;
    std::vector<EncCb> list((size_t)n_cb);
    for (int32_t i = 0; i < n_cb; ++i) {
        const tdec_cb_desc &d = desc[i];
        const int ki = k_index(d.K);
        if (ki < 0 || d.F < 0 || d.F >= d.K || d.crc < 0 || d.crc > 2 || d.llr_off < 0 ||
            d.bits_off < 0)
            return TDEC_EINVAL;
        if (d.crc && d.K - d.F < 24) return TDEC_EINVAL;
        EncCb &e = list[i];
        e.src_bit = 8 * d.bits_off;
        e.out_off = d.llr_off;
        e.K = d.K;
        qpp_coeffs(ki, &e.f1, &e.f2);
        e.F = d.F;
        e.crc = d.crc;
        e.rsv = 0;
    }
    if (hipSetDevice(ctx->device) != hipSuccess) return TDEC_EDEVICE;
    std::string key(1, 'E');
    key.append((const char *)desc, sizeof(tdec_cb_desc) * (size_t)n_cb);
    return encode_list(ctx, list, key, d_payload, d_coded, (hipStream_t)stream);
}

tdec_status tb_encode(tdec_ctx *ctx, const uint8_t *d_payload, int32_t tbs, uint8_t *d_coded,
                      void *stream)
{
    if (!ctx || !d_payload || !d_coded) return TDEC_EINVAL;
    int32_t s[8];
    if (segment(tbs, s)) return TDEC_ERANGE;
    if ((size_t)(s[0] + 7) / 8 > ctx->encbuf_bytes) return TDEC_ENOMEM;
    hipStream_t st = (hipStream_t)stream;
    if (hipSetDevice(ctx->device) != hipSuccess) return TDEC_EDEVICE;
    std::vector<EncCb> list((size_t)s[1]);
    int64_t bit = 0, out = 0;
    for (int r = 0; r < s[1]; ++r) {
        const int32_t K = r < s[6] ? s[4] : s[3];
        const int32_t F = r == 0 ? s[7] : 0;
        EncCb &e = list[r];
        e.src_bit = bit;
        e.out_off = out;
        e.K = K;
        qpp_coeffs(k_index(K), &e.f1, &e.f2);
        e.F = (int16_t)F;
        e.crc = (int8_t)(s[1] > 1 ? TDEC_CRC24B : TDEC_CRC_NONE);
        e.rsv = 0;
        bit += K - F - s[2];
        out += 3 * (int64_t)(K + 4);
    }
    if (launch_tb_crc_attach(d_payload, tbs, ctx->d_encbuf, ctx->d_crc_tab, st)) return TDEC_EDEVICE;
    std::string key(1, 'B');
    key.append((const char *)&tbs, sizeof tbs);
    return encode_list(ctx, list, key, ctx->d_encbuf, d_coded, st);
}

}  // extern "C"
