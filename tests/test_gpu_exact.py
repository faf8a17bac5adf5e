"""Exact window boundaries (win_init = 2) on the GPU: windowed decoding whose
boundary metrics come from max-plus transfer matrices and a scan along the
windows returns exactly what the oracle's full-length decoder (one window)
returns: bits, CRC flags and iteration counts, bit for bit."""
import sys

import numpy as np
import pytest

import oracle as O
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


def gpu_cbs(dev, od, llr, tp, n_bytes):
    T, D, torch = dev
    td = (T.CbDesc * len(od))()
    for i, o in enumerate(od):
        td[i].llr_off, td[i].bits_off, td[i].K, td[i].F, td[i].crc = o.llr_off, o.bits_off, o.K, o.F, o.crc
    x = torch.from_numpy(llr).cuda()
    bits = torch.zeros(max(n_bytes, 1), dtype=torch.uint8, device="cuda")
    ok = torch.zeros(len(td), dtype=torch.uint8, device="cuda")
    it = torch.zeros(len(td), dtype=torch.uint8, device="cuda")
    D.cb_decode_batch(td, x, tp, bits, ok, it)
    torch.cuda.synchronize()
    return bits.cpu().numpy()[:n_bytes], ok.cpu().numpy(), it.cpu().numpy()


@pytest.mark.parametrize("K,F,crc,nw,es,iters", [
    (40, 8, O.CRC24B, 3, 1, 8),        # uneven windows with filler: 16, 16, 8
    (512, 0, O.CRC_NONE, 8, 0, 4),
    (1056, 13, O.CRC24A, 4, 1, 6),
    (5824, 0, O.CRC24B, 91, 0, 6),     # the single-TB blocks in 64-step windows
    (5824, 0, O.CRC24B, 122, 0, 6),    # uneven: 121 of 48, the last of 16
    (6144, 0, O.CRC24B, 32, 1, 8),
    (6144, 0, O.CRC24B, 96, 1, 6),     # 256-thread work groups
    (488, 0, O.CRC24B, 8, 1, 8),       # uneven: 7 of 64, the last of 40
    (6144, 0, O.CRC24B, 70, 0, 6),     # uneven, 256-thread work groups
    (1024, 0, O.CRC24B, 128, 0, 4),    # 128 windows of 8 steps
    (40, 0, O.CRC24B, 5, 0, 3),        # several blocks per work group
])
def test_exact_windows_equal_full_length(dev, K, F, crc, nw, es, iters):
    T = dev[0]
    n = 12 if K <= 512 else 6
    cbs = [(K, F, crc)] * n
    esn0 = list(np.linspace(-1.0, 4.0, n))
    say(f"[exact] K={K} F={F} nw={nw} es={es} iters={iters} n={n}")
    llr, pays, od, n_llr, n_bytes = cb_batch(cbs, "qpsk", esn0, 301, K + nw)
    gb, gok, git = gpu_cbs(dev, od, llr, T.params(iters, es, nw, 2), n_bytes)
    ob, ook, oit = oracle_cb_batch(od, llr, O.params(iters, es, 1, 0))
    assert np.array_equal(gok, ook), (gok, ook)
    assert np.array_equal(git, oit), (git, oit)
    assert np.array_equal(gb, ob)


def test_exact_windows_adversarial_llrs(dev):
    """Saturated extremes and random full-range values: the int16 bounds of
    the transfer runs and of the windows hold."""
    T = dev[0]
    g = np.random.default_rng(12)
    for K, nw in ((2048, 16), (6144, 48)):
        cbs = [(K, 0, O.CRC24B)] * 3
        od, n_llr, n_bytes = O.make_descs(cbs)
        for s_i, v in enumerate((g.choice([-2047, 2047], n_llr),
                                 g.integers(-32768, 32768, n_llr))):
            llr = np.asarray(v, np.int16)
            say(f"[exact adversarial] K={K} nw={nw} set={s_i}")
            gb, gok, git = gpu_cbs(dev, od, llr, T.params(5, 0, nw, 2), n_bytes)
            ob, ook, oit = oracle_cb_batch(od, llr, O.params(5, 0, 1, 0))
            assert np.array_equal(gok, ook) and np.array_equal(git, oit)
            assert np.array_equal(gb, ob)


def test_exact_windows_single_tb(dev):
    """The 75376-bit transport block (13 blocks of K=5824) in 91 windows per
    block with exact boundaries equals the oracle's full-length decode."""
    T, D, torch = dev
    tbs = 75376
    say(f"[exact] tb {tbs}")
    llr, pays, lo, bo = tb_batch([tbs], "qpsk", 2.0, 302)
    x = torch.from_numpy(llr).cuda()
    bits = torch.zeros((tbs + 7) // 8, dtype=torch.uint8, device="cuda")
    res = torch.zeros(T.TB_RESULT_BYTES, dtype=torch.uint8, device="cuda")
    D.tb_decode(x, tbs, T.params(6, 0, 91, 2), bits, res)
    torch.cuda.synchronize()
    r = T.parse_tb_results(res.cpu().numpy())[0]
    ob, ores = O.tb_decode(llr, tbs, O.params(6, 0, 1, 0))
    assert r["tb_ok"] == ores["tb_ok"] and r["max_iters_used"] == ores["max_iters_used"]
    assert np.array_equal(bits.cpu().numpy(), ob)
