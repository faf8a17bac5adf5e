"""The mutual-information stop on the GPU (paper Sec. IV-B, decoding
function): the kernel sums the entropy of decoder 2's hard decisions per
block and stops a block when the sum has converged.  Bits, CRC flags and
iteration counts equal the oracle's, bit for bit, alone and combined with the
CRC stop, over windowed, exact-boundary, transport-block and captured-graph
launches, and at the full 4096 x K6144 batch on sampled blocks.  With the
purge of Algorithm 2 on, transport blocks follow the oracle's model of the
rule (test_purge_follows_the_model)."""
import sys

import numpy as np
import pytest

import oracle as O
from inputs import cb_batch, oracle_cb_batch, tb_batch

pytestmark = pytest.mark.gpu

MI, CRC = O.STOP_MI, O.STOP_CRC


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


def gpu_cbs(dev, od, llr, tp, n_bytes):
    T, D, torch = dev
    x = torch.from_numpy(llr).cuda()
    bits = torch.zeros(max(n_bytes, 1), dtype=torch.uint8, device="cuda")
    ok = torch.zeros(len(od), dtype=torch.uint8, device="cuda")
    it = torch.zeros(len(od), dtype=torch.uint8, device="cuda")
    D.cb_decode_batch(tdesc(T, od), x, tp, bits, ok, it)
    torch.cuda.synchronize()
    return bits.cpu().numpy()[:n_bytes], ok.cpu().numpy(), it.cpu().numpy()


@pytest.mark.parametrize("K,F,crc,nw,wi,mode,eps", [
    (40, 8, O.CRC24B, 3, 1, MI, 33),          # uneven windows with filler
    (512, 0, O.CRC_NONE, 8, 1, MI, 33),       # no CRC: only the MI rule can stop
    (1056, 13, O.CRC24A, 4, 0, MI | CRC, 33),
    (2048, 0, O.CRC24B, 16, 1, MI, 0),        # eps 0: exact plateau or S = 0 only
    (6144, 0, O.CRC24B, 32, 1, MI | CRC, 33),
    (6144, 0, O.CRC24B, 96, 1, MI, 300),      # 256-thread work groups
    (5824, 0, O.CRC24B, 56, 1, MI, 16),
    (488, 0, O.CRC24B, 8, 1, MI | CRC, 33),   # uneven: 7 of 64, the last of 40
    (40, 0, O.CRC_NONE, 5, 0, MI, 32768),     # several blocks per work group; stop at once
])
def test_mi_stop_matches_oracle(dev, K, F, crc, nw, wi, mode, eps):
    T = dev[0]
    n = 16 if K <= 512 else 8
    esn0 = list(np.linspace(0.0, 6.0, n))
    say(f"[mi] K={K} F={F} crc={crc} nw={nw} win_init={wi} mode={mode} eps={eps} n={n}")
    llr, _, od, _, n_bytes = cb_batch([(K, F, crc)] * n, "16qam", esn0, 401, K + nw + mode)
    gb, gok, git = gpu_cbs(dev, od, llr, T.params(8, mode, nw, wi, eps), n_bytes)
    ob, ook, oit = oracle_cb_batch(od, llr, O.params(8, mode, nw, wi, eps))
    assert np.array_equal(git, oit), (git, oit)
    assert np.array_equal(gok, ook), (gok, ook)
    assert np.array_equal(gb, ob)


def test_mi_stop_mixed_sizes_one_launch(dev):
    """Every size class and crc kind in one launch (items of different sizes
    share the launch's LDS layout)."""
    T = dev[0]
    cbs = [(6144, 0, O.CRC24B), (40, 8, O.CRC24B), (1056, 0, O.CRC_NONE), (5824, 0, O.CRC24B),
           (512, 0, O.CRC24A), (3136, 15, O.CRC24B), (6144, 0, O.CRC24B), (2112, 0, O.CRC_NONE)] * 3
    esn0 = list(np.linspace(1.0, 5.0, len(cbs)))
    say(f"[mi] mixed sizes, {len(cbs)} blocks")
    llr, _, od, _, n_bytes = cb_batch(cbs, "16qam", esn0, 402)
    gb, gok, git = gpu_cbs(dev, od, llr, T.params(8, MI | CRC, 0, 1, 33), n_bytes)
    D = dev[1]
    nws = [D.pick_windows(o.K) for o in od]
    for i, o in enumerate(od):
        L = 0 if o.crc == O.CRC_NONE else 24
        r = O.cb_decode(llr[o.llr_off:o.llr_off + 3 * (o.K + 4)], o.K, o.F, o.crc,
                        O.params(8, MI | CRC, nws[i], 1, 33))
        nb = (o.K - o.F - L + 7) // 8
        want = np.packbits(r["bits"][o.F:o.K - L])
        assert git[i] == r["iters"] and gok[i] == r["ok"], i
        assert np.array_equal(gb[o.bits_off:o.bits_off + nb], want[:nb]), i


@pytest.mark.parametrize("K,nw", [(6144, 32), (1024, 16), (40, 5),
                                  (5824, 122),   # uneven: 121 of 48, the last of 16
                                  (488, 8)])     # uneven: 7 of 64, the last of 40
def test_mi_stop_exact_windows_equal_full_length(dev, K, nw):
    T = dev[0]
    n = 8
    say(f"[mi] exact boundaries K={K} nw={nw}")
    llr, _, od, _, n_bytes = cb_batch([(K, 0, O.CRC24B)] * n, "qpsk", list(np.linspace(-1, 4, n)),
                                      403, K + nw)
    gb, gok, git = gpu_cbs(dev, od, llr, T.params(8, MI, nw, 2, 33), n_bytes)
    ob, ook, oit = oracle_cb_batch(od, llr, O.params(8, MI, 1, 0, 33))
    assert np.array_equal(git, oit) and np.array_equal(gok, ook)
    assert np.array_equal(gb, ob)


def test_mi_stop_transport_blocks_and_graph(dev):
    T, D, torch = dev
    tbs_list = [75376, 16, 6121, 30000, 2000]
    say(f"[mi] transport blocks {tbs_list}: direct call, graph, oracle")
    llr, _, lo, bo = tb_batch(tbs_list, "qpsk", [0.5, 2.0, 1.0, 1.5, 3.0], 404)
    nb = int(bo[-1] + (tbs_list[-1] + 7) // 8)
    p = T.params(8, MI | CRC, 0, 1, 33)
    x = torch.from_numpy(llr).cuda()
    eb = torch.zeros(nb, dtype=torch.uint8, device="cuda")
    er = torch.zeros(len(tbs_list) * T.TB_RESULT_BYTES, dtype=torch.uint8, device="cuda")
    D.tb_decode_batch(tbs_list, lo, bo, x, p, eb, er)
    torch.cuda.synchronize()
    res = T.parse_tb_results(er.cpu().numpy())
    for i, tbs in enumerate(tbs_list):
        ob, ores = O.tb_decode_windows(llr[lo[i]:lo[i] + O.tb_llr_count(tbs)], tbs,
                                       O.params(8, MI | CRC, 0, 1, 33),
                                       [D.pick_windows(K) for K, _ in O.cb_sizes(tbs)])
        assert res[i] == ores, i
        assert np.array_equal(eb.cpu().numpy()[bo[i]:bo[i] + ob.size], ob)
    gb, gr = torch.zeros_like(eb), torch.zeros_like(er)
    g = D.graph_tb_decode(tbs_list, lo, bo, x, p, gb, gr)
    try:
        for r in range(3):
            gb.zero_()
            gr.zero_()
            g.launch()
            torch.cuda.synchronize()
            assert torch.equal(gb, eb) and torch.equal(gr, er), r
    finally:
        g.close()


def test_mi_stop_full_batch_sampled(dev):
    """4096 blocks of K = 6144 in 32 windows, Es/N0 spread over the
    waterfall: every block's iteration count is in range, and 48 sampled
    blocks equal the oracle."""
    T, D, torch = dev
    n, K = 4096, 6144
    esn0 = np.linspace(2.0, 8.0, n)
    say(f"[mi] full batch {n} x K{K}")
    llr, _, od, _, n_bytes = cb_batch([(K, 0, O.CRC24B)] * n, "16qam", esn0, 405)
    gb, gok, git = gpu_cbs(dev, od, llr, T.params(8, MI | CRC, 32, 1, 33), n_bytes)
    assert git.min() >= 1 and git.max() <= 8
    pick = np.random.default_rng(7).choice(n, 48, replace=False)
    for i in pick:
        o = od[i]
        r = O.cb_decode(llr[o.llr_off:o.llr_off + 3 * (K + 4)], K, 0, O.CRC24B,
                        O.params(8, MI | CRC, 32, 1, 33))
        nb = (K - 24) // 8
        assert git[i] == r["iters"] and gok[i] == r["ok"], i
        assert np.array_equal(gb[o.bits_off:o.bits_off + nb], np.packbits(r["bits"][:K - 24])), i


def test_mi_params_rejected(dev):
    T = dev[0]
    llr, _, od, _, n_bytes = cb_batch([(40, 0, O.CRC24B)], "qpsk", 3.0, 406)
    for p in (T.params(8, 8, 1, 0), T.params(8, MI, 1, 0, -1), T.params(8, MI, 1, 0, 32769)):
        with pytest.raises(T.TdecError):
            gpu_cbs(dev, od, llr, p, n_bytes)


def test_mi_stop_through_the_serving_loop(dev):
    """The serving loop hands its parameters to every launch: with the MI
    and CRC stops set, each TB comes back with the oracle's bits, pass flag and
    iteration count."""
    import time
    T, D, torch = dev
    tbs_list = [75376, 40, 6120, 6121, 20000, 3000, 12000, 500]
    esn0 = np.linspace(0.5, 4.0, len(tbs_list))
    say(f"[mi] serving loop, tbs={tbs_list}")
    llr, _, lo, _ = tb_batch(tbs_list, "16qam", esn0, 407)
    pinned = torch.empty(llr.size, dtype=torch.int16, pin_memory=True)
    pinned.numpy()[:] = llr
    out = [np.zeros((t + 7) // 8, np.uint8) for t in tbs_list]
    p = T.params(8, MI | CRC, 1, 0, 1)
    srv = T.Server(D, T.server_cfg(p, deadline_us=10_000_000, mode=0))
    try:
        base = pinned.data_ptr()
        for g in np.array_split(np.arange(len(tbs_list)), 2):
            srv.submit(g.tolist(), [tbs_list[i] for i in g], [base + 2 * int(lo[i]) for i in g],
                       [out[i].ctypes.data for i in g])
            time.sleep(0.0005)
        srv.drain(60000)
        res, t0 = [], time.monotonic()
        while len(res) < len(tbs_list) and time.monotonic() - t0 < 30:
            res += srv.poll(4096, 100000)
    finally:
        srv.close()
    res = {r["tag"]: r for r in res}
    op = O.params(8, MI | CRC, 1, 0, 1)
    for i, tbs in enumerate(tbs_list):
        ob, ores = O.tb_decode(llr[lo[i]:lo[i] + O.tb_llr_count(tbs)], tbs, op)
        r = res[i]
        assert r["status"] == T.SERVE_DONE
        assert r["tb_ok"] == ores["tb_ok"] and r["max_iters_used"] == ores["max_iters_used"], i
        assert np.array_equal(out[i], ob), (i, tbs)



def test_purge_follows_the_model(dev):
    """Purge (Algorithm 2): transport blocks of 13 blocks at low Es/N0, some
    with one block that carries noise only, MI stop with eps 300.  A block
    that stops failed marks its transport block; its siblings still running
    are purged (iters 0, ok 0).  Per the oracle's model: an unmarked
    transport block equals the oracle in everything; a marked one has
    tb_ok = 0 and each block either equals the oracle or was purged.  The
    same launch without the purge equals the oracle throughout."""
    T, D, torch = dev
    tbs = 75376
    n = 24
    g = np.random.default_rng(1905)
    esn0 = np.linspace(2.6, 3.6, n)
    llr, _, lo, bo = tb_batch([tbs] * n, "16qam", esn0, 407)
    sizes = O.cb_sizes(tbs)
    noisy = [i for i in range(n) if i % 3 == 0]
    for i in noisy:  # block 5 of these transport blocks: noise only
        o = int(lo[i]) + sum(3 * (K + 4) for K, _ in sizes[:5])
        llr[o:o + 3 * (sizes[5][0] + 4)] = g.integers(-40, 41, 3 * (sizes[5][0] + 4))
    x = torch.from_numpy(llr).cuda()
    nb = int(bo[-1]) + (tbs + 7) // 8
    nws = [D.pick_windows(K) for K, _ in sizes]
    op = O.params(8, MI, 0, 1, 300)
    model = [O.tb_purge_marked(llr[lo[i]:lo[i] + O.tb_llr_count(tbs)], tbs, op, nws)
             for i in range(n)]
    n_marked = sum(m[2] for m in model)
    say(f"[purge] {n} x {tbs}: {n_marked} transport blocks marked by the model")
    assert n_marked >= len(noisy)
    for purge in (False, True):
        p = T.params(8, MI | (T.STOP_PURGE if purge else 0), 0, 1, 300)
        eb = torch.zeros(nb, dtype=torch.uint8, device="cuda")
        er = torch.zeros(n * T.TB_RESULT_BYTES, dtype=torch.uint8, device="cuda")
        D.tb_decode_batch([tbs] * n, lo, bo, x, p, eb, er)
        torch.cuda.synchronize()
        res, hb = T.parse_tb_results(er.cpu().numpy()), eb.cpu().numpy()
        purged = 0
        for i, (ob, ores, marked) in enumerate(model):
            if not purge or not marked:
                assert res[i] == ores, (purge, i)
                assert np.array_equal(hb[bo[i]:bo[i] + ob.size], ob), (purge, i)
                continue
            assert res[i]["tb_ok"] == 0, i
            for r in range(len(sizes)):
                got = (res[i]["cb_ok"][r], res[i]["cb_iters"][r])
                want = (ores["cb_ok"][r], ores["cb_iters"][r])
                assert got == want or got == (0, 0), (i, r, got, want)
                purged += got == (0, 0) and want != (0, 0)
        if purge:
            say(f"[purge] blocks purged: {purged}")
            assert purged >= 1
