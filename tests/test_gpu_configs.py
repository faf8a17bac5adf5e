"""The measured configurations' own decode shapes against the oracle:

* the worst-case stress shape: 75376-bit transport blocks (13 x K5824) in 56
  windows of 104 steps with previous-iteration boundaries, exactly 8
  iterations, 256QAM near its 30 % TB error point -- directly and through
  the serving loop;
* the mixed-TTI shape: one TTI of 64 transport blocks of log-uniform sizes,
  window counts autotuned with windows down to 32 steps (uneven partitions
  included), captured into a graph and replayed, every replay checked
  against the oracle run with the same per-block window counts;
* the same TTI under the launch knobs (packing, item order, window length
  target): the batch tuner's choice and a fixed non-default set, each
  checked against the oracle with the window counts it gives."""
import sys
import time

import numpy as np
import pytest

import oracle as O
import workload as wl
from inputs import tb_batch

pytestmark = pytest.mark.gpu

C5_TBS = 75376
C5_ESN0 = 10.65  # dB: TB error rate near 30 % at 8 iterations, 56 windows
C5_NW = 56


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


def oracle_tbs(llr, lo, tbs_list, p, nws):
    out = []
    for i, tbs in enumerate(tbs_list):
        out.append(O.tb_decode_windows(llr[lo[i]:lo[i] + O.tb_llr_count(tbs)], tbs, p, nws[i]))
    return out


def test_stress_shape_direct_and_served(dev):
    T, D, torch = dev
    n = 8
    say(f"[c5] {n} x {C5_TBS} bits, 256QAM {C5_ESN0} dB, {C5_NW} windows, 8 iterations forced")
    llr, pays, lo, bo = tb_batch([C5_TBS] * n, "256qam", C5_ESN0, 51)
    assert O.win_len(5824, C5_NW) == 104
    ref = oracle_tbs(llr, lo, [C5_TBS] * n, O.params(8, 0, C5_NW, 1), [[C5_NW] * 13] * n)
    n_fail = sum(1 - r[1]["tb_ok"] for r in ref)
    say(f"[c5] oracle: {n_fail} of {n} TBs fail CRC24A")
    # direct batch call
    x = torch.from_numpy(llr).cuda()
    nb = int(bo[-1]) + (C5_TBS + 7) // 8
    bits = torch.zeros(nb, dtype=torch.uint8, device="cuda")
    res = torch.zeros(n * T.TB_RESULT_BYTES, dtype=torch.uint8, device="cuda")
    p = T.params(8, 0, C5_NW, 1)
    D.tb_decode_batch([C5_TBS] * n, lo, bo, x, p, bits, res)
    torch.cuda.synchronize()
    gb = bits.cpu().numpy()
    gr = T.parse_tb_results(res.cpu().numpy())
    for i in range(n):
        ob, ores = ref[i]
        assert gr[i] == ores, i
        assert np.array_equal(gb[bo[i]:bo[i] + ob.size], ob), i
    # the serving loop, device-resident LLRs, the same parameters
    out = [np.zeros((C5_TBS + 7) // 8, np.uint8) for _ in range(n)]
    srv = T.Server(D, T.server_cfg(p, deadline_us=10_000_000))
    try:
        for g in np.array_split(np.arange(n), 2):
            srv.submit(g.tolist(), [C5_TBS] * len(g), [x.data_ptr() + 2 * int(lo[i]) for i in g],
                       [out[i].ctypes.data for i in g], device=True)
        srv.drain(60000)
        rr, t0 = [], time.monotonic()
        while len(rr) < n and time.monotonic() - t0 < 30:
            rr += srv.poll(64, 100000)
    finally:
        srv.close()
    rr = {r["tag"]: r for r in rr}
    for i in range(n):
        ob, ores = ref[i]
        assert rr[i]["status"] == T.SERVE_DONE
        assert rr[i]["tb_ok"] == ores["tb_ok"] and rr[i]["max_iters_used"] == 8, i
        assert np.array_equal(out[i], ob), i


def c3_shape():
    g = wl.rng(3, 77)
    tbs_list = [int(v) for v in wl.tbs_log_uniform(g, 64)]
    mods = [["qpsk", "16qam", "64qam"][i] for i in g.integers(0, 3, len(tbs_list))]
    esn0 = g.uniform(0.0, 18.0, len(tbs_list))
    return tbs_list, mods, esn0


def c3_tti(tbs_list, mods, esn0):
    """The TTI's LLRs, laid out as tb_batch lays them out."""
    parts, lo, bo, o, b = [], [], [], 0, 0
    gch = wl.rng(3, 78)
    for t, m, e in zip(tbs_list, mods, esn0):
        d, _ = O.tb_encode(wl.random_bits(gch, t))
        parts.append(wl.channel_blocks(d, O.cb_sizes(t), m, float(e), gch))
        lo.append(o)
        bo.append(b)
        o += parts[-1].size
        b += (t + 7) // 8
    return np.concatenate(parts), np.array(lo), np.array(bo), b


def test_mixed_tti_tuned_windows_graph_replays(dev):
    T, _, torch = dev
    tbs_list, mods, esn0 = c3_shape()
    Ks = sorted({K for t in tbs_list for K, _ in O.cb_sizes(t)})
    D2 = T.Decoder(0)
    try:
        say(f"[c3] autotune {len(Ks)} sizes, windows >= 32 steps")
        choice = D2.autotune(Ks, min_W=32, max_iters=8, batch_bits=0)
        uneven = [K for K in Ks if choice[K][0] > 1 and choice[K][0] * O.win_len(K, choice[K][0]) != K]
        say(f"[c3] sizes with uneven partitions: {uneven}")
        assert uneven, "no uneven partition chosen: the shape is not covered"
        for K in Ks:
            nw = choice[K][0]
            assert nw == 1 or O.win_len(K, nw) >= 32
        nws = [[choice[K][0] for K, _ in O.cb_sizes(t)] for t in tbs_list]
        p = T.params(8, 1, 0, 1)
        op = O.params(8, 1, 0, 1)
        llr, lo, bo, b = c3_tti(tbs_list, mods, esn0)
        x = torch.from_numpy(llr).cuda()
        gb = torch.zeros(b, dtype=torch.uint8, device="cuda")
        gr = torch.zeros(len(tbs_list) * T.TB_RESULT_BYTES, dtype=torch.uint8, device="cuda")
        graph = D2.graph_tb_decode(tbs_list, lo, bo, x, p, gb, gr)
        ref = oracle_tbs(llr, lo, tbs_list, op, nws)
        say(f"[c3] oracle: {sum(r[1]['tb_ok'] for r in ref)} of {len(ref)} TBs pass")
        try:
            for rep in range(3):
                gb.fill_(0xA5)
                gr.zero_()
                graph.launch()
                torch.cuda.synchronize()
                hb = gb.cpu().numpy()
                hr = T.parse_tb_results(gr.cpu().numpy())
                for i, t in enumerate(tbs_list):
                    ob, ores = ref[i]
                    assert hr[i] == ores, (rep, i, t)
                    assert np.array_equal(hb[bo[i]:bo[i] + ob.size], ob), (rep, i, t)
                # eager work of the program between replays
                torch.cuda.synchronize()
                _ = (x[:1024].float() * 2).sum().item()
        finally:
            graph.close()
    finally:
        D2.close()


def test_mixed_tti_launch_knobs(dev):
    T, _, torch = dev
    tbs_list, mods, esn0 = c3_shape()
    llr, lo, bo, b = c3_tti(tbs_list, mods, esn0)
    x = torch.from_numpy(llr).cuda()
    p = T.params(8, 1, 0, 1)
    op = O.params(8, 1, 0, 1)
    sizes = [[K for K, _ in O.cb_sizes(t)] for t in tbs_list]
    D2 = T.Decoder(0)
    try:
        say("[c3 knobs] batch tuner, windows >= 32 steps")
        r = D2.autotune_batch(tbs_list, lo, x, p, min_W=32)
        best, rule = r["best"], r["rule"]
        say(f"[c3 knobs] {len(r['candidates'])} candidates; best {best}; rule {rule}")
        assert len(r["candidates"]) == 5 * 3 * 6  # no per-size tuning: no -1 window choice
        assert rule["lds_budget"] == 30720 and rule["order"] == T.ORDER_K_DESC
        assert 0 < best["us"] <= rule["us"]
        k = D2.get_knobs()
        assert (k["lds_budget"], k["order"]) == (best["lds_budget"], best["order"])
        knob_sets = [("tuned", None), ("fixed", (8192, T.ORDER_REQUEST, 48)),
                     ("fixed", (81920, T.ORDER_K_ASC, 0))]
        for name, ks in knob_sets:
            if ks is not None:
                D2.set_knobs(*ks)
            nws = [[D2.pick_windows(K) for K in s] for s in sizes]
            for s, n in zip(sizes, nws):
                for K, nw in zip(s, n):
                    assert nw == 1 or O.win_len(K, nw) >= 32, (K, nw)
            say(f"[c3 knobs] {name} {ks}: decode and oracle")
            gb = torch.full((b,), 0xA5, dtype=torch.uint8, device="cuda")
            gr = torch.zeros(len(tbs_list) * T.TB_RESULT_BYTES, dtype=torch.uint8, device="cuda")
            D2.tb_decode_batch(tbs_list, lo, bo, x, p, gb, gr)
            torch.cuda.synchronize()
            hb = gb.cpu().numpy()
            hr = T.parse_tb_results(gr.cpu().numpy())
            ref = oracle_tbs(llr, lo, tbs_list, op, nws)
            for i, t in enumerate(tbs_list):
                ob, ores = ref[i]
                assert hr[i] == ores, (name, ks, i, t)
                assert np.array_equal(hb[bo[i]:bo[i] + ob.size], ob), (name, ks, i, t)
    finally:
        D2.close()
