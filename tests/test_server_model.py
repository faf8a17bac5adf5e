"""Serving loop host logic (admission, batching, slot accounting, latency
statistics) with the modelled executor: no device is touched, every
"launch" lasts max(lat, ns_per_kbit * kbits)."""
import time

import numpy as np
import pytest

import paper_1905_01141_amd as T

MAX_TB = 75376  # 13 blocks of K = 5824
SLOT_MAX = ((3 * 13 * (5824 + 4) * 2) + 255) // 256 * 256  # one max-size TB slot


def _llr_buf(tbs):
    return np.zeros(T.tb_llr_count(tbs), np.int16)


def _submit(srv, tags, tbs, t=None):
    bufs = [_llr_buf(x) for x in tbs]
    k, st = srv.submit(tags, tbs, [b.ctypes.data for b in bufs], None, t, keep=bufs)
    return k, st


def _collect(srv, n, timeout=5.0):
    out, t0 = [], time.monotonic()
    while len(out) < n and time.monotonic() - t0 < timeout:
        out += srv.poll(4096, 20000)
    return out


def _nearest_rank(v, q):
    v = np.sort(np.asarray(v))
    r = int(np.ceil(q * len(v) - 1e-9))
    return int(v[min(max(r, 1), len(v)) - 1])


def test_continuous_batching_merges_waiting_blocks():
    # a launch lasts 30 ms; six arrivals 1 ms apart (even if the host is slow
    # to wake, well within 30 ms): the first launches alone, the other five
    # merge into the next launch
    cfg = T.server_cfg(T.params(8, 1, 0, 1), deadline_us=1_000_000, model_lat_ns=30_000_000)
    srv = T.Server.model(cfg, 30_000_000, 0)
    try:
        tags = []
        for tti in range(6):
            tg = list(range(tti * 20, tti * 20 + 20))
            k, st = _submit(srv, tg, [4000] * 20)
            assert k == 20 and (st == T.SERVE_DONE).all()
            tags += tg
            time.sleep(0.001)
        srv.drain(10000)
        res = _collect(srv, len(tags))
        s = srv.stats()
    finally:
        srv.close()
    assert sorted(r["tag"] for r in res) == tags
    assert all(r["status"] == T.SERVE_DONE and r["tb_ok"] == 1 for r in res)
    assert s["completed"] == 120 and s["admitted"] == 120
    assert s["batches"] < 120 and max(r["batch_tbs"] for r in res) > 20
    assert s["mean_batch_tbs"] == pytest.approx(120 / s["batches"])
    assert all(r["t_done_ns"] - r["t_arrive_ns"] >= 30_000_000 for r in res)
    assert s["slots_in_use_bytes"] == 0


def test_per_tb_mode_launches_each_block_alone():
    cfg = T.server_cfg(T.params(8, 1, 0, 1), deadline_us=100000, mode=T.SERVE_PER_TB)
    srv = T.Server.model(cfg, 200_000, 0)
    try:
        _submit(srv, list(range(15)), [3000] * 15)
        srv.drain(10000)
        res = _collect(srv, 15)
        s = srv.stats()
    finally:
        srv.close()
    assert s["batches"] == 15 and all(r["batch_tbs"] == 1 for r in res)
    # FIFO: completion order is arrival order
    assert [r["tag"] for r in res] == list(range(15))
    # the i-th block waits for the i launches before it
    lat = sorted(r["t_done_ns"] - r["t_arrive_ns"] for r in res)
    assert lat[-1] >= 15 * 200_000


def test_budget_admission_and_slot_release():
    # launches last 50 ms, so the slots are still held when the statistics
    # are read right after the submission
    cfg = T.server_cfg(T.params(8, 1, 0, 1), deadline_us=1_000_000,
                       slot_budget_bytes=2 * SLOT_MAX + 1000)
    srv = T.Server.model(cfg, 50_000_000, 0)
    try:
        k, st = _submit(srv, list(range(5)), [MAX_TB] * 5)
        assert k == 2
        assert list(st) == [T.SERVE_DONE] * 2 + [T.SERVE_REJ_BUDGET] * 3
        s = srv.stats()
        assert s["rej_budget"] == 3 and s["slots_in_use_bytes"] == 2 * SLOT_MAX
        srv.drain(10000)
        res = _collect(srv, 5)
        # slots come back: the same request fits again
        k2, _ = _submit(srv, [10, 11], [MAX_TB] * 2)
        assert k2 == 2
        srv.drain(10000)
        res += _collect(srv, 2)
        s = srv.stats()
    finally:
        srv.close()
    assert sorted(r["status"] for r in res) == [0, 0, 0, 0, 1, 1, 1]
    assert s["slots_in_use_bytes"] == 0 and s["slots_peak_bytes"] == 2 * SLOT_MAX


def test_deadline_admission_rejects_predicted_misses():
    # the model says a launch takes 5 ms; the deadline is 3 ms.  An idle
    # server admits the first block anyway (the model can only learn from
    # launches); everything behind it is predicted late and rejected.
    cfg = T.server_cfg(T.params(8, 1, 0, 1), deadline_us=3000,
                       admission=T.ADMIT_BUDGET | T.ADMIT_DEADLINE, model_lat_ns=5_000_000)
    srv = T.Server.model(cfg, 5_000_000, 0)
    try:
        k, st = _submit(srv, list(range(4)), [1000] * 4)
        srv.drain(10000)
        res = _collect(srv, 4)
        s = srv.stats()
    finally:
        srv.close()
    assert k == 1 and st[0] == T.SERVE_DONE and (st[1:] == T.SERVE_REJ_DEADLINE).all()
    assert s["rej_deadline"] == 3 and s["completed"] == 1 and s["deadline_miss"] == 1
    assert sorted(r["status"] for r in res) == [0, 2, 2, 2]


def test_deadline_admission_sheds_overload():
    # every arrival brings ~9 ms of decoding (20 blocks of 6144 bits at 75 us
    # per kbit) while arrivals come every ~5 ms: the predictor must shed load
    # so that admitted blocks keep (close to) their 15 ms deadline (all times
    # five times those of a real TTI, so that host scheduling noise of a few
    # ms cannot decide the outcome)
    cfg = T.server_cfg(T.params(8, 1, 0, 1), deadline_us=15000,
                       admission=T.ADMIT_BUDGET | T.ADMIT_DEADLINE,
                       model_lat_ns=1_000_000, model_ns_per_kbit=75_000, max_batch_cb=64)
    srv = T.Server.model(cfg, 1_000_000, 75_000)
    n = 0
    try:
        t0 = time.monotonic()
        while time.monotonic() - t0 < 0.4:
            _submit(srv, list(range(n, n + 20)), [6120] * 20)
            n += 20
            time.sleep(0.005)
        srv.drain(20000)
        res = _collect(srv, n)
        s = srv.stats()
    finally:
        srv.close()
    assert len(res) == n
    assert s["rej_deadline"] > 0 and s["completed"] > 0
    done = [r for r in res if r["status"] == T.SERVE_DONE]
    late = sum(r["t_done_ns"] - r["t_arrive_ns"] > 15_000_000 for r in done)
    assert late <= 0.2 * len(done)


def test_invalid_sizes_and_miss_counting():
    cfg = T.server_cfg(T.params(8, 1, 0, 1), deadline_us=1000)
    srv = T.Server.model(cfg, 1_500_000, 0)
    try:
        buf = _llr_buf(100)
        k, st = srv.submit([1, 2, 3], [100, 0, 400000], [buf.ctypes.data] * 3, keep=[buf] * 3)
        assert k == 1
        assert list(st) == [T.SERVE_DONE, T.SERVE_REJ_INVALID, T.SERVE_REJ_INVALID]
        srv.drain(10000)
        res = _collect(srv, 3)
        s = srv.stats()
    finally:
        srv.close()
    assert s["rej_invalid"] == 2 and s["completed"] == 1
    # a 1.5 ms launch against a 1 ms deadline: admitted (budget only) and late
    assert s["deadline_miss"] == 1
    assert {r["tag"]: r["status"] for r in res} == {1: 0, 2: 3, 3: 3}


def test_latency_percentiles_match_results():
    cfg = T.server_cfg(T.params(8, 1, 0, 1), deadline_us=100000)
    srv = T.Server.model(cfg, 100_000, 2_000)
    try:
        rng = np.random.default_rng(5)
        n = 0
        for _ in range(30):
            m = int(rng.integers(1, 8))
            _submit(srv, list(range(n, n + m)), rng.integers(100, 20000, m).tolist())
            n += m
            time.sleep(0.0005)
        srv.drain(10000)
        res = _collect(srv, n)
        s = srv.stats()
    finally:
        srv.close()
    lat = [r["t_done_ns"] - r["t_arrive_ns"] for r in res]
    assert s["completed"] == n == len(lat)
    assert s["lat_p50_ns"] == _nearest_rank(lat, 0.50)
    assert s["lat_p99_ns"] == _nearest_rank(lat, 0.99)
    assert s["lat_max_ns"] == max(lat)
    assert s["payload_bits"] == sum(r["tbs"] for r in res)


def test_per_tb_mode_deadline_admission_bounds_the_queue():
    # one launch per block of 300 us against 20 blocks per ~1 ms: the plain
    # per-TB form is overloaded 6x and must shed instead of queueing forever
    cfg = T.server_cfg(T.params(8, 1, 0, 1), deadline_us=3000, mode=T.SERVE_PER_TB,
                       admission=T.ADMIT_BUDGET | T.ADMIT_DEADLINE, model_lat_ns=300_000)
    srv = T.Server.model(cfg, 300_000, 0)
    n = 0
    try:
        t0 = time.monotonic()
        while time.monotonic() - t0 < 0.08:
            _submit(srv, list(range(n, n + 20)), [3000] * 20)
            n += 20
            time.sleep(0.001)
        srv.drain(20000)
        res = _collect(srv, n)
        s = srv.stats()
    finally:
        srv.close()
    assert len(res) == n and s["rej_deadline"] > 0.5 * n
    done = [r for r in res if r["status"] == T.SERVE_DONE]
    assert len(done) == s["completed"] > 0
    late = sum(r["t_done_ns"] - r["t_arrive_ns"] > 3_000_000 for r in done)
    assert late <= 0.2 * len(done)


def test_launch_records_account_for_every_block():
    """The per-launch record (the paper's performance captor, Sec. IV-D):
    launches in completion order, their TB and code block counts add up to
    what completed, each covers its coding delay, and a reset empties the
    ring."""
    cfg = T.server_cfg(T.params(8, 1, 0, 1), deadline_us=100000, model_lat_ns=500_000)
    srv = T.Server.model(cfg, 500_000, 0)
    try:
        tbs = [40, 6120, 6121, 20000, 75376]
        for tti in range(4):
            _submit(srv, list(range(tti * 5, tti * 5 + 5)), tbs)
            time.sleep(0.0007)
        srv.drain(10000)
        _collect(srv, 20)
        recs = srv.launches()
        s = srv.stats()
        srv.reset_stats()
        after = srv.launches()
    finally:
        srv.close()
    assert len(recs) == s["batches"] and after == []
    assert sum(r["n_tb"] for r in recs) == 20
    cbs = sum(T.segment(t)["C"] for t in tbs) * 4
    assert sum(r["n_cb"] for r in recs) == cbs
    bits = sum(T.segment(t)["Cplus"] * T.segment(t)["Kplus"] +
               T.segment(t)["Cminus"] * T.segment(t)["Kminus"] for t in tbs) * 4
    assert sum(r["cb_bits"] for r in recs) == bits
    for a, b in zip(recs, recs[1:]):
        assert b["t_end_ns"] >= a["t_end_ns"]
    for r in recs:
        assert r["t_end_ns"] - r["t_start_ns"] >= 500_000
        assert r["coding_ns"] == r["t_end_ns"] - r["t_start_ns"]
        assert r["oldest_wait_ns"] >= 0


def test_launch_ring_keeps_the_most_recent():
    cfg = T.server_cfg(T.params(8, 1, 0, 1), deadline_us=10_000_000, mode=T.SERVE_PER_TB)
    srv = T.Server.model(cfg, 1000, 0)
    try:
        n = 4200
        _submit(srv, list(range(n)), [40] * n)
        srv.drain(60000)
        recs = srv.launches(5000)
        last = srv.launches(3)
        s = srv.stats()
    finally:
        srv.close()
    assert s["batches"] == n and len(recs) == 4096
    assert all(r["n_tb"] == 1 and r["n_cb"] == 1 and r["cb_bits"] == 64 for r in recs)
    assert last == recs[-3:]
    assert all(b["t_start_ns"] >= a["t_end_ns"] for a, b in zip(recs, recs[1:]))


def test_slot_arena_coalesces_after_churn():
    """Many arrivals of mixed sizes, released batch by batch in completion
    order, fragment the slot arena; once everything has completed the free
    extents have merged back, so a request for the whole budget fits."""
    budget = 6 * SLOT_MAX
    cfg = T.server_cfg(T.params(8, 1, 0, 1), deadline_us=1_000_000, slot_budget_bytes=budget)
    srv = T.Server.model(cfg, 20_000, 0)
    g = np.random.default_rng(3)
    try:
        tag, n_rej = 0, 0
        for tti in range(60):
            tbs = [int(x) for x in np.exp(g.uniform(np.log(16), np.log(MAX_TB), 12))]
            k, st = _submit(srv, list(range(tag, tag + len(tbs))), tbs)
            n_rej += int((st == T.SERVE_REJ_BUDGET).sum())
            tag += len(tbs)
            if tti % 3 == 2:
                time.sleep(0.0005)
        srv.drain(20000)
        _collect(srv, tag, 20.0)
        s = srv.stats()
        assert s["slots_in_use_bytes"] == 0 and s["rej_budget"] == n_rej
        assert s["slots_peak_bytes"] <= budget
        k, st = _submit(srv, list(range(tag, tag + 6)), [MAX_TB] * 6)
        assert k == 6 and (st == T.SERVE_DONE).all()
        srv.drain(10000)
        _collect(srv, 6)
    finally:
        srv.close()


def test_creation_checks_every_decoder_parameter():
    """A bad stop rule, threshold, boundary mode or window count fails at
    creation, not later at every launch."""
    for p in (T.params(8, 8, 1, 0), T.params(8, T.STOP_MI, 1, 0, -1), T.params(8, T.STOP_MI, 1, 0, 32769),
              T.params(8, 1, 1, 3), T.params(8, 1, 129, 0), T.params(0, 1, 1, 0), T.params(17, 1, 1, 0)):
        with pytest.raises(T.TdecError):
            T.Server.model(T.server_cfg(p), 100_000, 0)
    srv = T.Server.model(T.server_cfg(T.params(8, T.STOP_MI | T.STOP_CRC, 0, 1, 1)), 100_000, 0)
    srv.close()


def test_arrivals_during_a_launch_go_out_on_another_lane():
    """Continuous batching across launches: a batch that arrives while a
    long launch runs is dispatched on a free lane shortly before that launch
    is predicted to end (its lead: a quarter of the launch, at most 200 us),
    so the two launches are in flight together and the hand-over is hidden;
    with one lane it waits for the first launch's results."""
    def run(max_inflight):
        cfg = T.server_cfg(T.params(8, 1, 0, 1), deadline_us=1_000_000,
                           model_lat_ns=20_000_000, max_inflight=max_inflight)
        srv = T.Server.model(cfg, 20_000_000, 0)
        try:
            _submit(srv, list(range(5)), [6000] * 5)
            time.sleep(0.004)
            _submit(srv, list(range(5, 8)), [3000] * 3)
            srv.drain(10000)
            res = {r["tag"]: r for r in _collect(srv, 8)}
            recs = srv.launches()
            s = srv.stats()
        finally:
            srv.close()
        return res, recs, s

    res, recs, s = run(0)
    assert s["batches"] == 2 and len(recs) == 2
    first = min(recs, key=lambda r: r["t_start_ns"])
    second = max(recs, key=lambda r: r["t_start_ns"])
    assert first["n_tb"] == 5 and second["n_tb"] == 3
    assert second["t_start_ns"] < first["t_end_ns"]                        # in flight together
    assert second["t_start_ns"] >= first["t_start_ns"] + 20_000_000 - 200_000 - 50_000  # the lead
    assert s["busy_ns"] < sum(r["t_end_ns"] - r["t_start_ns"] for r in recs)
    res1, recs1, s1 = run(1)
    a, b = sorted(recs1, key=lambda r: r["t_start_ns"])
    assert b["t_start_ns"] >= a["t_end_ns"]                                # one lane: one after the other


def test_max_inflight_range():
    for m in (-1, 9):
        with pytest.raises(T.TdecError):
            T.Server.model(T.server_cfg(T.params(8, 1, 0, 1), max_inflight=m), 100_000, 0)
    for m in (1, 8):
        T.Server.model(T.server_cfg(T.params(8, 1, 0, 1), max_inflight=m), 100_000, 0).close()


def test_replay_submits_each_tick_at_its_time():
    """The native load generator: counts[k] arrivals at tick k, stamped with
    the tick, tags in arrival order."""
    cfg = T.server_cfg(T.params(8, 1, 0, 1), deadline_us=1_000_000)
    srv = T.Server.model(cfg, 100_000, 0)
    bufs = [np.zeros(T.tb_llr_count(t), np.int16) for t in (40, 1000, 6121)]
    counts = [3, 0, 2, 4]
    tbs = [40, 1000, 6121, 40, 1000, 6121, 40, 1000, 6121]
    ptrs = [bufs[i % 3].ctypes.data for i in range(9)]
    try:
        t_first = T.now_ns() + 2_000_000
        late, smax = srv.replay(counts, tbs, ptrs, period_ns=2_000_000, t_first_ns=t_first,
                                tag_base=100)
        srv.drain(10000)
        res = _collect(srv, 9)
    finally:
        srv.close()
    assert late >= 0 and smax > 0
    by = {r["tag"]: r for r in res}
    assert sorted(by) == list(range(100, 109))
    ticks = [0, 0, 0, 2, 2, 3, 3, 3, 3]
    for i in range(9):
        r = by[100 + i]
        assert r["status"] == T.SERVE_DONE and r["tbs"] == tbs[i]
        assert r["t_arrive_ns"] == t_first + ticks[i] * 2_000_000
    with pytest.raises(T.TdecError):
        srv2 = T.Server.model(cfg, 100_000, 0)
        try:
            srv2.replay([1, -1], [], [])
        finally:
            srv2.close()


def test_ring_mode_takes_arrivals_at_once():
    """Ring mode (modelled): a batch that arrives while another is in flight
    is taken at once -- on the device its items join the running ring kernel
    -- rather than held until shortly before the first one's predicted end;
    four batches may be in flight by default, and the ring kernel's idle
    time is range-checked."""
    cfg = T.server_cfg(T.params(8, 1, 0, 1), deadline_us=1_000_000, model_lat_ns=20_000_000,
                       mode=T.SERVE_RING)
    srv = T.Server.model(cfg, 20_000_000, 0)
    try:
        _submit(srv, list(range(5)), [6000] * 5)
        time.sleep(0.004)
        _submit(srv, list(range(5, 8)), [3000] * 3)
        time.sleep(0.002)
        _submit(srv, [8], [3000])
        srv.drain(10000)
        res = _collect(srv, 9)
        recs = sorted(srv.launches(), key=lambda r: r["t_start_ns"])
    finally:
        srv.close()
    assert len(res) == 9 and [r["n_tb"] for r in recs] == [5, 3, 1]
    # taken within a few ms of arriving, long before the first batch's end
    assert recs[1]["t_start_ns"] < recs[0]["t_start_ns"] + 10_000_000
    assert recs[2]["t_start_ns"] < recs[0]["t_start_ns"] + 12_000_000
    for us in (-1, 10_000_001):
        with pytest.raises(T.TdecError):
            T.Server.model(T.server_cfg(T.params(8, 1, 0, 1), mode=T.SERVE_RING, ring_idle_us=us),
                           100_000, 0)
    T.Server.model(T.server_cfg(T.params(8, 1, 0, 1), mode=T.SERVE_RING, ring_idle_us=1),
                   100_000, 0).close()
