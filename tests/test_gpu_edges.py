"""Edge cases on the GPU: empty batches, the largest transport block (64
code blocks), the most filler a block can carry, degenerate all-zero and
out-of-range LLRs, one and sixteen iterations -- each against the oracle."""
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


def gpu_cb(dev, od, llr, p, nb):
    T, D, torch = dev
    td = tdesc(T, od)
    b = torch.zeros(max(nb, 1), dtype=torch.uint8, device="cuda")
    ok = torch.zeros(len(td), dtype=torch.uint8, device="cuda")
    it = torch.zeros(len(td), dtype=torch.uint8, device="cuda")
    D.cb_decode_batch(td, torch.from_numpy(llr).cuda(), p, b, ok, it)
    torch.cuda.synchronize()
    return b.cpu().numpy()[:nb], ok.cpu().numpy(), it.cpu().numpy()


def test_empty_batches_are_no_ops(dev):
    T, D, torch = dev
    say("[edge] empty batches")
    x = torch.zeros(4, dtype=torch.int16, device="cuda")
    b = torch.full((4,), 7, dtype=torch.uint8, device="cuda")
    D.cb_decode_batch((T.CbDesc * 0)(), x, T.params(4, 0, 1, 0), b,
                      torch.zeros(1, dtype=torch.uint8, device="cuda"),
                      torch.zeros(1, dtype=torch.uint8, device="cuda"))
    D.tb_decode_batch([], [], [], x, T.params(4, 0, 1, 0), b,
                      torch.zeros(1, dtype=torch.uint8, device="cuda"))
    D.derate_batch((T.RmDesc * 0)(), torch.zeros(1, dtype=torch.int16, device="cuda"),
                   torch.zeros(1, dtype=torch.int16, device="cuda"), combine=0)
    torch.cuda.synchronize()
    assert (b.cpu().numpy() == 7).all()


def test_largest_transport_block(dev):
    """tbs = 391656: 64 code blocks of K = 6144, the most a result holds."""
    T, D, torch = dev
    tbs = 391656
    assert O.segment(tbs)["C"] == 64
    say("[edge] largest TB, 64 blocks")
    llr, pays, lo, bo = tb_batch([tbs], "16qam", 6.0, 501)
    x = torch.from_numpy(llr).cuda()
    bits = torch.zeros((tbs + 7) // 8, dtype=torch.uint8, device="cuda")
    res = torch.zeros(T.TB_RESULT_BYTES, dtype=torch.uint8, device="cuda")
    D.tb_decode_batch([tbs], lo, bo, x, T.params(6, 1, 0, 1), bits, res)
    torch.cuda.synchronize()
    gres = T.parse_tb_results(res.cpu().numpy())[0]
    nws = [D.pick_windows(K) for K, _ in O.cb_sizes(tbs)]
    ob, ores = O.tb_decode_windows(llr, tbs, O.params(6, 1, 0, 1), nws)
    assert gres == ores and gres["C"] == 64
    assert np.array_equal(bits.cpu().numpy(), ob)
    with pytest.raises(T.TdecError):  # 65 blocks do not fit a result
        D.tb_decode_batch([tbs + 6200], lo, bo,
                          torch.zeros(T.tb_llr_count(tbs + 6200), dtype=torch.int16,
                                      device="cuda"),
                          T.params(6, 1, 0, 1),
                          torch.zeros((tbs + 6200 + 7) // 8, dtype=torch.uint8, device="cuda"),
                          res)


@pytest.mark.parametrize("K,F,crc,nw", [(40, 16, O.CRC24A, 1), (6144, 6119, O.CRC_NONE, 32),
                                        (1056, 1031, O.CRC24B, 4)])
def test_maximum_filler(dev, K, F, crc, nw):
    T = dev[0]
    cbs = [(K, F, crc)] * 3
    say(f"[edge] K={K} F={F} nw={nw}")
    llr, pays, od, n_llr, nb = cb_batch(cbs, "qpsk", [0.0, 2.0, 5.0], 502)
    p = O.params(6, 1, nw, 1)
    gb, gok, git = gpu_cb(dev, od, llr, T.params(6, 1, nw, 1), nb)
    ob, ook, oit = oracle_cb_batch(od, llr, p)
    assert np.array_equal(gok, ook) and np.array_equal(git, oit) and np.array_equal(gb, ob)


@pytest.mark.parametrize("fill", ["zeros", "huge"])
def test_degenerate_llrs(dev, fill):
    """All-zero LLRs (every hard decision 0, which a CRC of zeros accepts)
    and values far outside +-2047 (clamped, not rejected)."""
    T = dev[0]
    cbs = [(6144, 0, O.CRC24B), (40, 0, O.CRC24A), (512, 8, O.CRC_NONE)]
    od, n_llr, nb = O.make_descs(cbs)
    if fill == "zeros":
        llr = np.zeros(n_llr, np.int16)
    else:
        llr = np.random.default_rng(503).choice([-32768, 32767, -5000, 5000], n_llr).astype(np.int16)
    say(f"[edge] {fill} LLRs")
    for p in (O.params(1, 0, 1, 0), O.params(16, 1, 8, 1), O.params(16, 0, 1, 1)):
        if any(K % 8 or (p.n_windows > 1 and O.win_len(K, p.n_windows) == 0) for K, _, _ in cbs):
            continue
        gb, gok, git = gpu_cb(dev, od, llr, T.params(p.max_iters, p.early_stop, p.n_windows,
                                                     p.win_init), nb)
        ob, ook, oit = oracle_cb_batch(od, llr, p)
        assert np.array_equal(gok, ook) and np.array_equal(git, oit) and np.array_equal(gb, ob)
    if fill == "zeros":
        assert gok.tolist() == [1, 1, 1]  # the all-zero word passes any CRC24


@pytest.mark.parametrize("shift", [1, 2, 3])
def test_llr_buffer_at_any_alignment(dev, shift):
    """The LLR buffer may start at any int16 address: a view 1 to 3 elements
    into an allocation (2-, 4- and 2-byte aligned) decodes like the oracle,
    through both the tiled restage (large blocks) and the direct one (40-bit
    blocks, many per item)."""
    T, D, torch = dev
    cbs = [(6144, 0, O.CRC24B), (40, 8, O.CRC24A), (1056, 0, O.CRC24B), (40, 0, O.CRC_NONE),
           (5824, 0, O.CRC24B), (512, 3, O.CRC24A)] * 2
    llr, _, od, _, nb = cb_batch(cbs, "16qam", list(np.linspace(1.0, 5.0, len(cbs))), 504 + shift)
    base = torch.zeros(llr.size + 8, dtype=torch.int16, device="cuda")
    x = base[shift:shift + llr.size]
    x.copy_(torch.from_numpy(llr))
    say(f"[edge] LLR buffer shifted by {shift} elements (address mod 8 = {x.data_ptr() % 8})")
    td = tdesc(T, od)
    b = torch.zeros(nb, dtype=torch.uint8, device="cuda")
    ok = torch.zeros(len(td), dtype=torch.uint8, device="cuda")
    it = torch.zeros(len(td), dtype=torch.uint8, device="cuda")
    D.cb_decode_batch(td, x, T.params(6, 1, 0, 1), b, ok, it)
    torch.cuda.synchronize()
    nws = [D.pick_windows(o.K) for o in od]
    for i, o in enumerate(od):
        L = 0 if o.crc == O.CRC_NONE else 24
        r = O.cb_decode(llr[o.llr_off:o.llr_off + 3 * (o.K + 4)], o.K, o.F, o.crc,
                        O.params(6, 1, nws[i], 1))
        n = (o.K - o.F - L + 7) // 8
        assert ok[i].item() == r["ok"] and it[i].item() == r["iters"], i
        assert np.array_equal(b.cpu().numpy()[o.bits_off:o.bits_off + n],
                              np.packbits(r["bits"][o.F:o.K - L])[:n]), i


def test_invalid_requests_are_refused(dev):
    T, D, torch = dev
    x = torch.zeros(3 * (6144 + 4), dtype=torch.int16, device="cuda")
    ok = torch.zeros(1, dtype=torch.uint8, device="cuda")
    bad = [((6144, 0, T.CRC24B), T.params(6, 0, 129, 1)),   # too many windows
           ((6144, 0, T.CRC24B), T.params(0, 0, 32, 1)),    # no iterations
           ((6144, 0, T.CRC24B), T.params(17, 0, 32, 1)),   # too many iterations
           ((6000, 0, T.CRC24B), T.params(6, 0, 1, 1)),     # not a table size
           ((40, 17, T.CRC24A), T.params(6, 0, 1, 1))]      # CRC does not fit behind the filler
    for (K, F, crc), p in bad:
        d = (T.CbDesc * 1)()
        d[0].llr_off, d[0].bits_off, d[0].K, d[0].F, d[0].crc = 0, 0, K, F, crc
        rc = T.lib().cb_decode_batch(D._h, 1, d, T._dptr(x), p, None, T._dptr(ok), T._dptr(ok),
                                     T._stream(None))
        assert rc == -1, (K, F, crc, rc)  # EINVAL, checked on the host before any launch
    torch.cuda.synchronize()
