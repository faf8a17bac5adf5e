"""Batched launch forms on the GPU: captured graphs replayed over changing
LLRs (every replay checked against a direct call and the oracle), and the
autotuner's window choice (decoding with it matches the oracle run with the
same window counts)."""
import sys

import numpy as np
import pytest

import oracle as O
import workload as wl
from inputs import cb_batch, oracle_cb_batch, tb_batch

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


def tdesc(T, od):
    d = (T.CbDesc * len(od))()
    for i, o in enumerate(od):
        d[i].llr_off, d[i].bits_off, d[i].K, d[i].F, d[i].crc = o.llr_off, o.bits_off, o.K, o.F, o.crc
    return d


MIXED = [(6144, 0, O.CRC24B), (40, 8, O.CRC24B), (1056, 0, O.CRC24B), (5824, 0, O.CRC24B),
         (512, 0, O.CRC24A), (3136, 15, O.CRC24B), (6144, 0, O.CRC24B), (2112, 0, O.CRC24B)]


def test_graph_cb_replays_follow_the_inputs(dev):
    T, D, torch = dev
    say("[graph] code block batch, 4 replays")
    llr0, _, od, n_llr, n_bytes = cb_batch(MIXED, "16qam", 3.0, 301)
    td = tdesc(T, od)
    x = torch.from_numpy(llr0).cuda()
    gb = torch.zeros(n_bytes, dtype=torch.uint8, device="cuda")
    gok = torch.zeros(len(td), dtype=torch.uint8, device="cuda")
    git = torch.zeros(len(td), dtype=torch.uint8, device="cuda")
    p = T.params(6, 1, 1, 1)  # full length: one window count that suits every size
    g = D.graph_cb_decode(td, x, p, gb, gok, git)
    eb = torch.zeros_like(gb)
    eok = torch.zeros_like(gok)
    eit = torch.zeros_like(git)
    try:
        for r in range(4):
            llr, _, _, _, _ = cb_batch(MIXED, "16qam", 1.0 + r, 301 + r)
            x.copy_(torch.from_numpy(llr))
            D.cb_decode_batch(td, x, p, eb, eok, eit)       # direct call, same inputs
            torch.cuda.synchronize()
            gb.zero_()
            g.launch()
            torch.cuda.synchronize()
            assert torch.equal(gb, eb) and torch.equal(gok, eok) and torch.equal(git, eit), r
            if r < 2:
                ob, ook, oit = oracle_cb_batch(od, llr, O.params(6, 1, 1, 1))
                assert np.array_equal(gb.cpu().numpy(), ob)
                assert np.array_equal(gok.cpu().numpy(), ook)
                assert np.array_equal(git.cpu().numpy(), oit)
    finally:
        g.close()


def test_graph_tb_replays_follow_the_inputs(dev):
    T, D, torch = dev
    tbs_list = [75376, 16, 6121, 30000, 2000]
    say(f"[graph] transport block batch {tbs_list}, 3 replays")
    llr0, _, lo, bo = tb_batch(tbs_list, "qpsk", 1.0, 311)
    nb = int(bo[-1] + (tbs_list[-1] + 7) // 8)
    p = T.params(6, 1, 0, 1)
    x = torch.from_numpy(llr0).cuda()
    gb = torch.zeros(nb, dtype=torch.uint8, device="cuda")
    gr = torch.zeros(len(tbs_list) * T.TB_RESULT_BYTES, dtype=torch.uint8, device="cuda")
    g = D.graph_tb_decode(tbs_list, lo, bo, x, p, gb, gr)
    eb, er = torch.zeros_like(gb), torch.zeros_like(gr)
    try:
        for r in range(3):
            llr, pays, _, _ = tb_batch(tbs_list, "qpsk", 0.5 + r, 311 + r)
            x.copy_(torch.from_numpy(llr))
            D.tb_decode_batch(tbs_list, lo, bo, x, p, eb, er)
            torch.cuda.synchronize()
            gb.zero_()
            gr.zero_()
            g.launch()
            torch.cuda.synchronize()
            assert torch.equal(gb, eb) and torch.equal(gr, er), r
            res = T.parse_tb_results(gr.cpu().numpy())
            if r == 0:
                for i, tbs in enumerate(tbs_list):
                    ob, ores = O.tb_decode_windows(llr[lo[i]:lo[i] + O.tb_llr_count(tbs)], tbs,
                                                   O.params(6, 1, 0, 1),
                                                   [D.pick_windows(K) for K, _ in O.cb_sizes(tbs)])
                    assert res[i] == ores, i
                    assert np.array_equal(gb.cpu().numpy()[bo[i]:bo[i] + ob.size], ob)
    finally:
        g.close()


def test_autotuned_windows_decode_like_the_oracle(dev):
    T, _, torch = dev
    D2 = T.Decoder(0)
    try:
        Ks = [40, 488, 1056, 3136, 6144]  # 488: only uneven windows reach W >= 64
        say(f"[autotune] {Ks}")
        choice = D2.autotune(Ks, min_W=64, max_iters=2, batch_bits=2_000_000)
        say(f"[autotune] choice {choice}")
        for K in Ks:
            nw, ns = choice[K]
            W = O.win_len(K, nw)  # the oracle's partition rule
            assert W > 0 and W % 8 == 0 and (nw == 1 or W >= 64)
            assert ns > 0
            assert D2.pick_windows(K) == nw
        cbs = [(K, 0, O.CRC24B) for K in Ks] * 2
        llr, _, od, n_llr, n_bytes = cb_batch(cbs, "16qam", 2.0, 321)
        td = tdesc(T, od)
        x = torch.from_numpy(llr).cuda()
        b = torch.zeros(n_bytes, dtype=torch.uint8, device="cuda")
        ok = torch.zeros(len(td), dtype=torch.uint8, device="cuda")
        it = torch.zeros(len(td), dtype=torch.uint8, device="cuda")
        D2.cb_decode_batch(td, x, T.params(6, 1, 0, 1), b, ok, it)
        torch.cuda.synchronize()
        gb, gok, git = b.cpu().numpy(), ok.cpu().numpy(), it.cpu().numpy()
        for i, (K, F, crc) in enumerate(cbs):
            sub, _, nb = O.make_descs([(K, F, crc)])
            d = od[i]
            ob, ook, oit = O.cb_decode_batch(sub, llr[d.llr_off:d.llr_off + 3 * (K + 4)],
                                             O.params(6, 1, choice[K][0], 1), nb)
            assert gok[i] == ook[0] and git[i] == oit[0]
            assert np.array_equal(gb[d.bits_off:d.bits_off + nb], ob)
        D2.autotune_reset()
        assert D2.pick_windows(6144) == dev[1].pick_windows(6144)
    finally:
        D2.close()
