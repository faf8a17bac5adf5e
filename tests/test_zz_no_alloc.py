"""The allocation-free decode entry point (cb_decode_batch_fixed): its decode
kernel's scratch is the library's fixed device array.  Two calls in a row
through the C ABI -- a large batch whose work groups the fixed array caps,
then a smaller mixed one -- each equal bit for bit to cb_decode_batch on the
same inputs and to the oracle."""
import sys

import numpy as np
import pytest

import oracle as O
from inputs import cb_batch, oracle_cb_batch

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


def both(T, D, torch, od, llr, p, n_bytes):
    """(fixed-scratch outputs, cb_decode_batch outputs) as numpy arrays."""
    td = tdesc(T, od)
    x = torch.from_numpy(llr).cuda()
    out = []
    for fn in (D.cb_decode_batch_fixed, D.cb_decode_batch):
        b = torch.full((n_bytes,), 0x5A, dtype=torch.uint8, device="cuda")
        ok = torch.full((len(td),), 7, dtype=torch.uint8, device="cuda")
        it = torch.full((len(td),), 99, dtype=torch.uint8, device="cuda")
        fn(td, x, p, b, ok, it)
        torch.cuda.synchronize()
        out.append((b.cpu().numpy(), ok.cpu().numpy(), it.cpu().numpy()))
    return out


def test_fixed_scratch_two_calls(dev):
    T, D, torch = dev
    # call 1: 2048 K6144 blocks at 32 windows (one work group's scratch is about
    # 127 KB, so the 64 MiB array runs about 500 work groups at once and each
    # claims several items); 256 distinct blocks tiled 8 times
    n_dist, reps = 256, 8
    say(f"[fixed] call 1: {n_dist * reps} x K6144, 32 windows, win_init 1, 6 iterations")
    llr1, _, od1, n_llr1, nb1 = cb_batch([(6144, 0, O.CRC24B)] * n_dist, "16qam", 3.5, 901)
    big = [(6144, 0, O.CRC24B)] * (n_dist * reps)
    odb, n_llrb, nbb = O.make_descs(big)
    llrb = np.tile(llr1, reps)
    p = T.params(6, 0, 32, 1)
    (fb, fok, fit), (eb, eok, eit) = both(T, D, torch, odb, llrb, p, nbb)
    assert np.array_equal(fb, eb) and np.array_equal(fok, eok) and np.array_equal(fit, eit)
    ob, ook, oit = oracle_cb_batch(od1, llr1, O.params(6, 0, 32, 1))
    per = nb1 // n_dist
    for r in range(reps):
        assert np.array_equal(fb[r * nb1:(r + 1) * nb1], ob), r
        assert np.array_equal(fok[r * n_dist:(r + 1) * n_dist], ook), r
        assert np.array_equal(fit[r * n_dist:(r + 1) * n_dist], oit), r
    assert per * n_dist == nb1
    say(f"[fixed] call 1 ok: CRC pass {int(fok.sum())}/{fok.size}")

    # call 2: a smaller batch of mixed sizes, filler and CRC kinds, early stop
    mixed = [(6144, 0, O.CRC24B), (40, 8, O.CRC24B), (1056, 0, O.CRC24A), (5824, 0, O.CRC24B),
             (512, 0, O.CRC_NONE), (3136, 15, O.CRC24B), (2112, 0, O.CRC24B)] * 3
    say(f"[fixed] call 2: {len(mixed)} mixed blocks, 8 windows of the library's rule, CRC stop")
    llr2, _, od2, n_llr2, nb2 = cb_batch(mixed, "qpsk", 1.0, 902)
    p2 = T.params(8, 1, 0, 1)
    (fb, fok, fit), (eb, eok, eit) = both(T, D, torch, od2, llr2, p2, nb2)
    assert np.array_equal(fb, eb) and np.array_equal(fok, eok) and np.array_equal(fit, eit)
    nws = [D.pick_windows(K) for K, _, _ in mixed]
    # the oracle with the same per-block window counts
    ob = np.zeros(nb2, np.uint8)
    ook = np.zeros(len(mixed), np.uint8)
    oit = np.zeros(len(mixed), np.uint8)
    for i, (K, F, crc) in enumerate(mixed):
        d1, _, n1 = O.make_descs([(K, F, crc)])
        o = od2[i].llr_off
        b1, k1, t1 = O.cb_decode_batch(d1, llr2[o:o + 3 * (K + 4)], O.params(8, 1, nws[i], 1), n1)
        ob[od2[i].bits_off:od2[i].bits_off + n1] = b1
        ook[i], oit[i] = k1[0], t1[0]
    assert np.array_equal(fb, ob) and np.array_equal(fok, ook) and np.array_equal(fit, oit)
    say(f"[fixed] call 2 ok: iterations {fit.tolist()}")
