"""Ring mode of the serving loop on the GPU: one persistent decode kernel
takes the batches' work items from a ring that the host appends to while it
runs.  Results equal the oracle's and the same blocks decoded alone; blocks
that arrive while the kernel runs join it without a new launch; the kernel
leaves when it has had nothing to claim for its idle time (a limit the host
sets) and is launched again by the next batch."""
import sys
import time

import numpy as np
import pytest

import oracle as O
import workload as wl
from inputs import tb_batch

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    import torch
    import paper_1905_01141_amd as T
    if not torch.cuda.is_available():
        pytest.fail("a GPU is required for the gpu-marked tests")
    return T, T.Decoder(0), torch


def collect(srv, n, timeout=30.0):
    res, t0 = [], time.monotonic()
    while len(res) < n and time.monotonic() - t0 < timeout:
        res += srv.poll(4096, 100000)
    return {r["tag"]: r for r in res}


def check_oracle(T, D, llr, lo, tbs_list, out, res, op, idx=None):
    for i in (range(len(tbs_list)) if idx is None else idx):
        t = tbs_list[i]
        ob, ores = O.tb_decode_windows(llr[lo[i]:lo[i] + O.tb_llr_count(t)], t, op,
                                       [D.pick_windows(K) for K, _ in O.cb_sizes(t)])
        r = res[i]
        assert r["status"] == T.SERVE_DONE, i
        assert r["tb_ok"] == ores["tb_ok"] and r["max_iters_used"] == ores["max_iters_used"], (i, t)
        assert r["C"] == ores["C"]
        assert np.array_equal(out[i], ob), (i, t)


@pytest.mark.parametrize("device", [False, True])
def test_ring_matches_oracle(dev, device):
    """Mixed sizes (the size table's ends and both segmentation regimes) in
    four arrival batches, with the CRC stop: every block equals the oracle."""
    T, D, torch = dev
    g = wl.rng(21, 1)
    tbs_list = [min(int(x), 40000) for x in wl.tbs_log_uniform(g, 12)] + [40, 6120, 6121, 75376]
    esn0 = np.linspace(0.0, 6.0, len(tbs_list))
    say(f"[ring] oracle device={device} tbs={tbs_list}")
    llr, pays, lo, bo = tb_batch(tbs_list, "16qam", esn0, 21)
    pinned = torch.empty(llr.size, dtype=torch.int16, pin_memory=True)
    pinned.numpy()[:] = llr
    src = pinned.cuda() if device else pinned
    torch.cuda.synchronize()
    out = [np.zeros((t + 7) // 8, np.uint8) for t in tbs_list]
    p = T.params(6, 1, 0, 1)
    srv = T.Server(D, T.server_cfg(p, deadline_us=10_000_000, mode=T.SERVE_RING))
    try:
        for grp in np.array_split(np.arange(len(tbs_list)), 4):
            srv.submit(grp.tolist(), [tbs_list[i] for i in grp],
                       [src.data_ptr() + 2 * int(lo[i]) for i in grp],
                       [out[i].ctypes.data for i in grp], device=device)
            time.sleep(0.0003)
        srv.drain(60000)
        res = collect(srv, len(tbs_list))
        st = srv.stats()
        recs = srv.launches()
    finally:
        srv.close()
    assert st["completed"] == len(tbs_list) and st["rej_budget"] == 0
    assert st["ring_launches"] >= 1
    for r in recs:
        assert r["pre_ns"] > 0 and r["coding_ns"] > 0 and r["post_ns"] > 0
    check_oracle(T, D, llr, lo, tbs_list, out, res, O.params(6, 1, 0, 1))


def test_ring_takes_arrivals_into_the_running_kernel(dev):
    """A long batch (160 transport blocks of 75376 bits, 2080 code blocks at
    8 forced iterations) and, while it decodes, a batch of small blocks:
    both are decoded by the same kernel launch (the small batch's items are
    published while that kernel runs and claimed by its work groups as they
    free up), and every result equals its decode alone and the oracle's."""
    T, D, torch = dev
    big = [75376] * 160
    small = [40, 1000, 6121, 20000]
    tbs_list = big + small
    nbig = len(big)
    say(f"[ring] running kernel: {nbig} x 75376 then {small}")
    esn0 = [14.0] * nbig + [3.0] * len(small)
    llr, pays, lo, bo = tb_batch(tbs_list, "64qam", esn0, 22)
    x = torch.from_numpy(llr).cuda()
    torch.cuda.synchronize()
    p = T.params(8, 0, 0, 1)
    out = [np.zeros((t + 7) // 8, np.uint8) for t in tbs_list]
    srv = T.Server(D, T.server_cfg(p, deadline_us=10_000_000, mode=T.SERVE_RING,
                                   ring_idle_us=1_000_000))
    try:
        srv.submit(list(range(nbig)), big, [x.data_ptr() + 2 * int(lo[i]) for i in range(nbig)],
                   [out[i].ctypes.data for i in range(nbig)], device=True)
        time.sleep(0.0003)
        idx = list(range(nbig, len(tbs_list)))
        srv.submit(idx, small, [x.data_ptr() + 2 * int(lo[i]) for i in idx],
                   [out[i].ctypes.data for i in idx], device=True)
        srv.drain(60000)
        res = collect(srv, len(tbs_list))
        recs = sorted(srv.launches(), key=lambda r: r["t_start_ns"])
        st = srv.stats()
    finally:
        srv.close()
    assert [r["n_tb"] for r in recs] == [nbig, len(small)], recs
    a, b = recs
    # the small batch's items were published while the big batch decoded,
    # into the kernel that was already running
    assert b["t_start_ns"] + b["pre_ns"] < a["t_start_ns"] + a["pre_ns"] + a["coding_ns"], \
        "the small batch was published after the big one had finished"
    assert st["ring_launches"] == 1, st["ring_launches"]
    say(f"[ring] big batch {(a['t_end_ns'] - a['t_start_ns']) / 1e3:.0f} us (coding "
        f"{a['coding_ns'] / 1e3:.0f}), small one published "
        f"{(b['t_start_ns'] + b['pre_ns'] - a['t_start_ns']) / 1e3:.0f} us after the big one was "
        f"taken, done after {(b['t_end_ns'] - b['t_start_ns']) / 1e3:.0f} us")
    # alone: direct calls with the ring's window counts
    nb = int(bo[-1] + (tbs_list[-1] + 7) // 8)
    eb = torch.zeros(nb, dtype=torch.uint8, device="cuda")
    er = torch.zeros(len(tbs_list) * T.TB_RESULT_BYTES, dtype=torch.uint8, device="cuda")
    D.tb_decode_batch(big, lo[:nbig], bo[:nbig], x, p, eb, er[:nbig * T.TB_RESULT_BYTES])
    D.tb_decode_batch(small, lo[nbig:], bo[nbig:] - bo[nbig], x, p, eb[int(bo[nbig]):],
                      er[nbig * T.TB_RESULT_BYTES:])
    torch.cuda.synchronize()
    alone_b = eb.cpu().numpy()
    alone_r = T.parse_tb_results(er.cpu().numpy())
    for i, t in enumerate(tbs_list):
        r = res[i]
        assert r["status"] == T.SERVE_DONE
        assert r["tb_ok"] == alone_r[i]["tb_ok"], i
        assert r["max_iters_used"] == alone_r[i]["max_iters_used"] == 8, i
        assert np.array_equal(out[i], alone_b[bo[i]:bo[i] + (t + 7) // 8]), i
    check_oracle(T, D, llr, lo, tbs_list, out, res, O.params(8, 0, 0, 1),
                 [0, nbig // 2, nbig - 1] + idx)


def test_ring_kernel_leaves_when_idle_and_is_launched_again(dev):
    """With an idle time of 300 us set from the host, the ring kernel ends
    between two batches 30 ms apart (its work groups give up their bounded
    wait) and the second batch launches it again; results equal the
    oracle's, also with slots reused between the batches."""
    T, D, torch = dev
    tbs_list = [6120, 20000, 40, 75376, 3000, 6121]
    say(f"[ring] idle exit tbs={tbs_list}")
    llr, pays, lo, bo = tb_batch(tbs_list, "16qam", 4.0, 23)
    x = torch.from_numpy(llr).cuda()
    torch.cuda.synchronize()
    p = T.params(6, 1, 0, 1)
    out = [np.zeros((t + 7) // 8, np.uint8) for t in tbs_list]
    srv = T.Server(D, T.server_cfg(p, deadline_us=10_000_000, mode=T.SERVE_RING,
                                   ring_idle_us=300))
    try:
        for grp in (range(0, 3), range(3, 6)):
            grp = list(grp)
            srv.submit(grp, [tbs_list[i] for i in grp], [x.data_ptr() + 2 * int(lo[i]) for i in grp],
                       [out[i].ctypes.data for i in grp], device=True)
            srv.drain(60000)
            time.sleep(0.03)
        res = collect(srv, len(tbs_list))
        st = srv.stats()
    finally:
        srv.close()
    assert st["ring_launches"] >= 2, st["ring_launches"]
    check_oracle(T, D, llr, lo, tbs_list, out, res, O.params(6, 1, 0, 1))


def test_ring_mode_rejects_what_its_kernel_does_not_run(dev):
    """The ring kernel runs previous-iteration or no window boundaries,
    without the mutual-information stop, with at most 64 windows per block."""
    T, D, torch = dev
    for p in (T.params(6, 1, 0, 2), T.params(6, T.STOP_MI, 0, 1, 33), T.params(6, 1, 96, 1)):
        with pytest.raises(T.TdecError):
            T.Server(D, T.server_cfg(p, mode=T.SERVE_RING))


def test_ring_slot_churn_matches_oracle(dev):
    """Twenty batches one after another into one running ring kernel, each
    drained before the next, so every batch's LLRs land in the slots (and
    its plan in the buffers) that the batch before it used while the kernel
    has been reading them: every block still equals the oracle."""
    T, D, torch = dev
    g = wl.rng(24, 1)
    nb, per = 20, 6
    tbs_list = [min(int(x), 12000) for x in wl.tbs_log_uniform(g, nb * per)]
    say(f"[ring] slot churn {nb} batches of {per}")
    esn0 = np.linspace(1.0, 5.0, len(tbs_list))
    llr, pays, lo, bo = tb_batch(tbs_list, "16qam", esn0, 24)
    x = torch.from_numpy(llr).cuda()
    torch.cuda.synchronize()
    p = T.params(6, 1, 0, 1)
    out = [np.zeros((t + 7) // 8, np.uint8) for t in tbs_list]
    srv = T.Server(D, T.server_cfg(p, deadline_us=10_000_000, mode=T.SERVE_RING,
                                   ring_idle_us=1_000_000, slot_budget_bytes=1 << 20))
    try:
        for b in range(nb):
            grp = list(range(b * per, (b + 1) * per))
            k, st = srv.submit(grp, [tbs_list[i] for i in grp],
                               [x.data_ptr() + 2 * int(lo[i]) for i in grp],
                               [out[i].ctypes.data for i in grp], device=True)
            assert k == per, st
            srv.drain(60000)
        res = collect(srv, len(tbs_list))
        s = srv.stats()
    finally:
        srv.close()
    assert s["ring_launches"] == 1 and s["completed"] == len(tbs_list)
    check_oracle(T, D, llr, lo, tbs_list, out, res, O.params(6, 1, 0, 1))


def test_ring_every_block_size(dev):
    """All 188 code block sizes (one transport block of K - 24 bits each, so
    a single block of size K) in three arrival batches through one ring
    kernel: every QPP table, window count, LDS size and item packing of the
    size table, each block equal to the oracle."""
    T, D, torch = dev
    tbs_list = [k - 24 for k in T.k_table()]
    say(f"[ring] every block size: {len(tbs_list)} TBs")
    esn0 = np.linspace(0.5, 4.0, len(tbs_list))
    llr, pays, lo, bo = tb_batch(tbs_list, "qpsk", esn0, 25)
    x = torch.from_numpy(llr).cuda()
    torch.cuda.synchronize()
    p = T.params(5, 1, 0, 1)
    out = [np.zeros((t + 7) // 8, np.uint8) for t in tbs_list]
    srv = T.Server(D, T.server_cfg(p, deadline_us=10_000_000, mode=T.SERVE_RING,
                                   ring_idle_us=1_000_000))
    try:
        for grp in np.array_split(np.arange(len(tbs_list)), 3):
            srv.submit(grp.tolist(), [tbs_list[i] for i in grp],
                       [x.data_ptr() + 2 * int(lo[i]) for i in grp],
                       [out[i].ctypes.data for i in grp], device=True)
            time.sleep(0.0002)
        srv.drain(60000)
        res = collect(srv, len(tbs_list))
        s = srv.stats()
    finally:
        srv.close()
    assert s["completed"] == len(tbs_list)
    assert {T.segment(t)["C"] for t in tbs_list} == {1}
    check_oracle(T, D, llr, lo, tbs_list, out, res, O.params(5, 1, 0, 1))
