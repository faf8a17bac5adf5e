"""The serving loop on the GPU: transport blocks submitted over several
arrival batches come back with the oracle's bits and flags, in continuous
batching and in per-TB mode."""
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


def run_server(dev, mode, tbs_list, llr, lo, p, groups, device=False):
    T, D, torch = dev
    pinned = torch.empty(llr.size, dtype=torch.int16, pin_memory=True)
    pinned.numpy()[:] = llr
    src = pinned.cuda() if device else pinned
    torch.cuda.synchronize()
    base = src.data_ptr()
    out = [np.zeros((t + 7) // 8, np.uint8) for t in tbs_list]
    srv = T.Server(D, T.server_cfg(p, deadline_us=10_000_000, mode=mode))
    try:
        idx = np.array_split(np.arange(len(tbs_list)), groups)
        for g in idx:
            srv.submit(g.tolist(), [tbs_list[i] for i in g], [base + 2 * int(lo[i]) for i in g],
                       [out[i].ctypes.data for i in g], device=device)
            time.sleep(0.0005)
        srv.drain(60000)
        res, t0 = [], time.monotonic()
        while len(res) < len(tbs_list) and time.monotonic() - t0 < 30:
            res += srv.poll(4096, 100000)
        st = srv.stats()
    finally:
        srv.close()
    return out, {r["tag"]: r for r in res}, st


@pytest.mark.parametrize("mode,device", [(0, False), (1, False), (0, True)])
def test_server_matches_oracle(dev, mode, device):
    T = dev[0]
    g = wl.rng(7, 1)
    tbs_list = [int(x) for x in wl.tbs_log_uniform(g, 10)] + [40, 6120, 6121, 20000]
    tbs_list = [min(t, 30000) for t in tbs_list]
    esn0 = np.linspace(0.0, 5.0, len(tbs_list))
    say(f"[server] mode={mode} device={device} tbs={tbs_list}")
    llr, pays, lo, bo = tb_batch(tbs_list, "16qam", esn0, 7)
    out, res, st = run_server(dev, mode, tbs_list, llr, lo, T.params(6, 1, 1, 0), 3, device)
    assert st["completed"] == len(tbs_list) and st["rej_budget"] == 0
    if mode == 1:
        assert st["batches"] == len(tbs_list)
    assert st["mean_coding_ns"] > 0 and st["mean_pre_ns"] > 0
    p = O.params(6, 1, 1, 0)
    for i, tbs in enumerate(tbs_list):
        ob, ores = O.tb_decode(llr[lo[i]:lo[i] + O.tb_llr_count(tbs)], tbs, p)
        r = res[i]
        assert r["status"] == T.SERVE_DONE
        assert r["tb_ok"] == ores["tb_ok"] and r["max_iters_used"] == ores["max_iters_used"], i
        assert r["C"] == ores["C"]
        assert np.array_equal(out[i], ob), (i, tbs)
        assert r["t_done_ns"] > r["t_arrive_ns"]


def test_server_auto_windows_matches_direct_call(dev):
    """With the tuned window counts the server returns what one direct
    tb_decode_batch call returns (itself checked against the oracle)."""
    T, D, torch = dev
    g = wl.rng(8, 1)
    tbs_list = [int(x) for x in wl.tbs_log_uniform(g, 16)]
    say(f"[server] auto windows tbs={tbs_list}")
    llr, pays, lo, bo = tb_batch(tbs_list, "64qam", 14.0, 8)
    p = T.params(8, 1, 0, 1)
    out, res, st = run_server(dev, 0, tbs_list, llr, lo, p, 4)
    x = torch.from_numpy(llr).cuda()
    nb = int(bo[-1] + (tbs_list[-1] + 7) // 8)
    bits = torch.zeros(nb, dtype=torch.uint8, device="cuda")
    rr = torch.zeros(len(tbs_list) * T.TB_RESULT_BYTES, dtype=torch.uint8, device="cuda")
    D.tb_decode_batch(tbs_list, lo, bo, x, p, bits, rr)
    torch.cuda.synchronize()
    gb = bits.cpu().numpy()
    gr = T.parse_tb_results(rr.cpu().numpy())
    for i, tbs in enumerate(tbs_list):
        assert res[i]["tb_ok"] == gr[i]["tb_ok"]
        assert res[i]["max_iters_used"] == gr[i]["max_iters_used"]
        assert np.array_equal(out[i], gb[bo[i]:bo[i] + (tbs + 7) // 8])
        # at 14 dB 64QAM every TB decodes
        assert res[i]["tb_ok"] == 1
        assert np.array_equal(np.unpackbits(out[i])[:tbs], pays[i])


@pytest.mark.parametrize("shift", [0, 1, 2, 3, 8])
def test_device_submission_any_source_alignment(dev, shift):
    """Device submission copies each block's LLRs into the server's slots in
    16 KB chunks: sources 16-byte aligned, 4-byte aligned and 2-byte aligned
    (shift in int16 elements), blocks of one partial chunk and of many (the
    75376-bit maximum is 28 chunks and a tail) all decode like the oracle."""
    T, D, torch = dev
    tbs_list = [75376, 40, 6121, 20000, 8192 - 24]
    say(f"[server] device alignment shift={shift} tbs={tbs_list}")
    llr, pays, lo, bo = tb_batch(tbs_list, "16qam", 6.0, 9)
    buf = torch.zeros(llr.size + 16, dtype=torch.int16)
    buf[shift:shift + llr.size] = torch.from_numpy(llr)
    d = buf.cuda()
    torch.cuda.synchronize()
    base = d.data_ptr() + 2 * shift
    out = [np.zeros((t + 7) // 8, np.uint8) for t in tbs_list]
    srv = T.Server(D, T.server_cfg(T.params(6, 1, 1, 0), deadline_us=10_000_000, mode=0))
    try:
        srv.submit(list(range(len(tbs_list))), tbs_list, [base + 2 * int(o) for o in lo],
                   [o.ctypes.data for o in out], device=True)
        srv.drain(60000)
        res, t0 = [], time.monotonic()
        while len(res) < len(tbs_list) and time.monotonic() - t0 < 30:
            res += srv.poll(64, 100000)
    finally:
        srv.close()
    res = {r["tag"]: r for r in res}
    p = O.params(6, 1, 1, 0)
    for i, tbs in enumerate(tbs_list):
        ob, ores = O.tb_decode(llr[lo[i]:lo[i] + O.tb_llr_count(tbs)], tbs, p)
        assert res[i]["status"] == T.SERVE_DONE
        assert res[i]["tb_ok"] == ores["tb_ok"] == 1, i
        assert np.array_equal(out[i], ob), (i, tbs)


def test_launch_records_on_the_device(dev):
    """Launch records of a device server: one per launch, the TB and block
    counts add up, every delay is positive, the copies back are part of the
    post-processing, and launches do not overlap in time."""
    T, D, torch = dev
    tbs_list = [40, 6120, 6121, 20000, 75376, 1000]
    say(f"[server] launch records tbs={tbs_list}")
    llr, pays, lo, bo = tb_batch(tbs_list, "16qam", 6.0, 10)
    out, res, st = run_server(dev, 0, tbs_list, llr, lo, T.params(6, 1, 1, 0), 3)
    assert st["completed"] == len(tbs_list)
    srv = T.Server(D, T.server_cfg(T.params(6, 1, 1, 0), deadline_us=10_000_000))
    try:
        pinned = torch.empty(llr.size, dtype=torch.int16, pin_memory=True)
        pinned.numpy()[:] = llr
        outs = [np.zeros((t + 7) // 8, np.uint8) for t in tbs_list]
        for g in np.array_split(np.arange(len(tbs_list)), 2):
            srv.submit(g.tolist(), [tbs_list[i] for i in g],
                       [pinned.data_ptr() + 2 * int(lo[i]) for i in g], [outs[i].ctypes.data for i in g])
            srv.drain(60000)
        recs = srv.launches()
        s = srv.stats()
    finally:
        srv.close()
    assert len(recs) == s["batches"] >= 2
    assert sum(r["n_tb"] for r in recs) == len(tbs_list)
    assert sum(r["n_cb"] for r in recs) == sum(T.segment(t)["C"] for t in tbs_list)
    for r in recs:
        assert r["pre_ns"] > 0 and r["coding_ns"] > 0 and r["post_ns"] > 0
        assert 0 <= r["copy_ns"] <= r["post_ns"]
        assert r["t_end_ns"] - r["t_start_ns"] >= r["coding_ns"]
    for a, b in zip(recs, recs[1:]):
        assert b["t_start_ns"] >= a["t_end_ns"]
    for i, t in enumerate(tbs_list):
        assert np.array_equal(outs[i], out[i]), i


def test_arrivals_during_a_long_launch_overlap_on_the_device(dev):
    """Continuous batching: transport blocks submitted while a long launch
    runs are taken and enqueued on a second lane before the first launch has
    finished (their work groups take the compute units the first launch's
    leave, with no host round trip between); every result equals its decode
    alone (a direct call) and the oracle's."""
    T, D, torch = dev
    big = [75376] * 160          # 2080 code blocks, 8 forced iterations: a long launch
    small = [40, 1000, 6121, 20000]
    tbs_list = big + small
    say(f"[server] overlap: {len(big)} x 75376 then {small}")
    esn0 = [14.0] * len(big) + [3.0] * len(small)
    llr, pays, lo, bo = tb_batch(tbs_list, "64qam", esn0, 12)
    x = torch.from_numpy(llr).cuda()
    torch.cuda.synchronize()
    p = T.params(8, 0, 0, 1)
    # each group alone, direct calls
    nb = int(bo[-1] + (tbs_list[-1] + 7) // 8)
    eb = torch.zeros(nb, dtype=torch.uint8, device="cuda")
    er = torch.zeros(len(tbs_list) * T.TB_RESULT_BYTES, dtype=torch.uint8, device="cuda")
    nbig = len(big)
    D.tb_decode_batch(big, lo[:nbig], bo[:nbig], x, p, eb, er[:nbig * T.TB_RESULT_BYTES])
    D.tb_decode_batch(small, lo[nbig:], bo[nbig:] - bo[nbig], x, p, eb[int(bo[nbig]):],
                      er[nbig * T.TB_RESULT_BYTES:])
    torch.cuda.synchronize()
    alone_b = eb.cpu().numpy()
    alone_r = T.parse_tb_results(er.cpu().numpy())
    out = [np.zeros((t + 7) // 8, np.uint8) for t in tbs_list]
    srv = T.Server(D, T.server_cfg(p, deadline_us=10_000_000))
    try:
        srv.submit(list(range(nbig)), big, [x.data_ptr() + 2 * int(lo[i]) for i in range(nbig)],
                   [out[i].ctypes.data for i in range(nbig)], device=True)
        time.sleep(0.0002)
        idx = list(range(nbig, len(tbs_list)))
        srv.submit(idx, small, [x.data_ptr() + 2 * int(lo[i]) for i in idx],
                   [out[i].ctypes.data for i in idx], device=True)
        srv.drain(60000)
        res, t0 = [], time.monotonic()
        while len(res) < len(tbs_list) and time.monotonic() - t0 < 30:
            res += srv.poll(4096, 100000)
        recs = srv.launches()
    finally:
        srv.close()
    res = {r["tag"]: r for r in res}
    assert len(recs) == 2, recs
    a, b = sorted(recs, key=lambda r: r["t_start_ns"])
    assert a["n_tb"] == nbig and b["n_tb"] == len(small)
    # the second launch was enqueued while the first one's decode kernel ran
    assert b["t_start_ns"] + b["pre_ns"] < a["t_start_ns"] + a["pre_ns"] + a["coding_ns"], \
        "the second launch waited for the first"
    say(f"[server] big launch {(a['t_end_ns'] - a['t_start_ns']) / 1e3:.0f} us (coding "
        f"{a['coding_ns'] / 1e3:.0f}), small one taken {(b['t_start_ns'] - a['t_start_ns']) / 1e3:.0f}"
        f" us after it, {(b['t_end_ns'] - b['t_start_ns']) / 1e3:.0f} us (coding "
        f"{b['coding_ns'] / 1e3:.0f})")
    for i, t in enumerate(tbs_list):
        r = res[i]
        assert r["status"] == T.SERVE_DONE
        assert r["tb_ok"] == alone_r[i]["tb_ok"], i
        assert r["max_iters_used"] == alone_r[i]["max_iters_used"] == 8, i
        assert np.array_equal(out[i], alone_b[bo[i]:bo[i] + (t + 7) // 8]), i
    op = O.params(8, 0, 0, 1)
    for i in [0, nbig - 1] + idx:
        t = tbs_list[i]
        ob, ores = O.tb_decode_windows(llr[lo[i]:lo[i] + O.tb_llr_count(t)], t, op,
                                       [D.pick_windows(K) for K, _ in O.cb_sizes(t)])
        assert res[i]["tb_ok"] == ores["tb_ok"], i
        assert np.array_equal(out[i], ob), i
