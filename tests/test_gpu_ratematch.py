"""Rate matching on the GPU against the oracle, bit for bit: the receiver's
soft combining (int8 and int16 inputs, first transmission and HARQ
retransmissions, puncturing and repetition, filler) and the transmitter's
bit selection; and decoding straight from the combined soft buffers."""
import sys

import numpy as np
import pytest

import oracle as O
import workload as wl

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


BLOCKS = [(40, 0, 0, 100), (40, 8, 1, 333), (488, 0, 2, 700), (1056, 13, 3, 5000),
          (6144, 0, 0, 12000), (6144, 0, 2, 30000), (5824, 0, 1, 17484), (512, 0, 3, 1)]


def _coded(K, F, g):
    c = np.zeros(K, np.uint8)
    c[F:] = wl.random_bits(g, K - F)
    return O.turbo_encode_cb(c).reshape(-1)


def test_rate_match_equals_oracle(dev):
    T, D, torch = dev
    g = wl.rng(401, 0)
    descs, ne, ns = T.make_rm_descs(BLOCKS)
    coded = np.concatenate([_coded(K, F, g) for K, F, _, _ in BLOCKS])
    say(f"[rm] transmitter {len(BLOCKS)} blocks, {ne} bits")
    dc = torch.from_numpy(coded).cuda()
    de = torch.zeros(ne, dtype=torch.uint8, device="cuda")
    D.rate_match_batch(descs, dc, de)
    torch.cuda.synchronize()
    got = de.cpu().numpy()
    for d, (K, F, rv, E) in zip(descs, BLOCKS):
        want = O.rate_match(coded[d.soft_off:d.soft_off + 3 * (K + 4)], K, F, E, rv)
        assert np.array_equal(got[d.e_off:d.e_off + E], want), (K, F, rv, E)


def test_unaligned_buffers_equal_oracle(dev):
    """Blocks placed 1 to 3 elements apart, so that the coded bits are not
    4-byte aligned and the soft buffers not 8-byte aligned for some of them:
    the kernels' element-wise staging paths give the oracle's results too, and
    nothing outside the blocks is written."""
    T, D, torch = dev
    g = wl.rng(405, 0)
    descs, ne, _ = T.make_rm_descs(BLOCKS)
    so = 0
    for i, (K, F, rv, E) in enumerate(BLOCKS):
        so += 1 + i % 3
        descs[i].soft_off = so
        so += 3 * (K + 4)
    ns = so + 4
    coded = np.full(ns, 1, np.uint8)
    for d, (K, F, _, _) in zip(descs, BLOCKS):
        coded[d.soft_off:d.soft_off + 3 * (K + 4)] = _coded(K, F, g)
    say(f"[rm] unaligned offsets {[d.soft_off % 8 for d in descs]}")
    de = torch.zeros(ne, dtype=torch.uint8, device="cuda")
    D.rate_match_batch(descs, torch.from_numpy(coded).cuda(), de)
    e = g.integers(-127, 128, ne).astype(np.int8)
    soft = torch.full((ns,), 777, dtype=torch.int16, device="cuda")
    D.derate_batch(descs, torch.from_numpy(e).cuda(), soft, combine=0)
    D.derate_batch(descs, torch.from_numpy(e).cuda(), soft, combine=1)
    torch.cuda.synchronize()
    got_e, got_s = de.cpu().numpy(), soft.cpu().numpy()
    inside = np.zeros(ns, bool)
    for d, (K, F, rv, E) in zip(descs, BLOCKS):
        sl = slice(d.soft_off, d.soft_off + 3 * (K + 4))
        inside[sl] = True
        assert np.array_equal(got_e[d.e_off:d.e_off + E], O.rate_match(coded[sl], K, F, E, rv)), K
        ee = e[d.e_off:d.e_off + E].astype(np.int16)
        want = O.derate_match(ee, K, F, rv, O.derate_match(ee, K, F, rv, None))
        assert np.array_equal(got_s[sl], want), (K, d.soft_off % 4)
    assert (got_s[~inside] == 777).all()


@pytest.mark.parametrize("ebits", [8, 16])
def test_soft_combining_equals_oracle(dev, ebits):
    T, D, torch = dev
    g = np.random.default_rng(402 + ebits)
    descs, ne, ns = T.make_rm_descs(BLOCKS)
    say(f"[rm] receiver int{ebits}, 3 transmissions")
    lim = 127 if ebits == 8 else 20000   # int16 inputs large enough to saturate on repeats
    dt = np.int8 if ebits == 8 else np.int16
    soft_gpu = torch.zeros(ns, dtype=torch.int16, device="cuda")
    soft_ref = np.full(ns, 1234, np.int16)  # garbage: the first pass must clear it
    soft_gpu.copy_(torch.from_numpy(soft_ref))
    for tx in range(3):
        e = g.integers(-lim, lim + 1, ne).astype(dt)
        for i, (K, F, _, E) in enumerate(BLOCKS):
            descs[i].rv = (tx * 2 + i) % 4
        D.derate_batch(descs, torch.from_numpy(e).cuda(), soft_gpu, combine=1 if tx else 0)
        for d, (K, F, _, E) in zip(descs, BLOCKS):
            sl = slice(d.soft_off, d.soft_off + 3 * (K + 4))
            base = None if tx == 0 else soft_ref[sl]
            soft_ref[sl] = O.derate_match(e[d.e_off:d.e_off + E].astype(np.int16), K, F,
                                          int(d.rv), base)
        torch.cuda.synchronize()
        assert np.array_equal(soft_gpu.cpu().numpy(), soft_ref), tx


def test_harq_decode_from_combined_buffers(dev):
    """Rate-3/4 transmissions over 16QAM at 7 dB: GPU de-rate-matching plus
    GPU decoding of the combined buffers equals the oracle's chain after each
    redundancy version."""
    T, D, torch = dev
    g = wl.rng(403, 0)
    Ks = [2048, 1056, 6144, 512]
    cbs = [(K, 0, O.CRC24A) for K in Ks]
    cw = []
    for K in Ks:
        c = np.zeros(K, np.uint8)
        c[:K - 24] = wl.random_bits(g, K - 24)
        p = O.crc24(c[:K - 24], O.CRC24A)
        c[K - 24:] = [(p >> (23 - i)) & 1 for i in range(24)]
        cw.append(O.turbo_encode_cb(c).reshape(-1))
    blocks = [(K, 0, 0, (4 * K) // 3) for K in Ks]
    descs, ne, ns = T.make_rm_descs(blocks)
    soft = torch.zeros(ns, dtype=torch.int16, device="cuda")
    soft_ref = np.zeros(ns, np.int16)
    od, _, nb = O.make_descs(cbs)
    td = (T.CbDesc * len(od))()
    for i, o in enumerate(od):
        td[i].llr_off, td[i].bits_off, td[i].K, td[i].F, td[i].crc = o.llr_off, o.bits_off, o.K, o.F, o.crc
    for tx, rv in enumerate((0, 2, 3)):
        e = np.zeros(ne, np.int16)
        for i, d in enumerate(descs):
            d.rv = rv
            bits = O.rate_match(cw[i], Ks[i], 0, d.E, rv)
            e[d.e_off:d.e_off + d.E] = wl.awgn_llr(bits, "16qam", 7.0, g)
            sl = slice(d.soft_off, d.soft_off + 3 * (Ks[i] + 4))
            soft_ref[sl] = O.derate_match(e[d.e_off:d.e_off + d.E], Ks[i], 0, rv,
                                          None if tx == 0 else soft_ref[sl])
        D.derate_batch(descs, torch.from_numpy(e).cuda(), soft, combine=1 if tx else 0)
        b = torch.zeros(nb, dtype=torch.uint8, device="cuda")
        ok = torch.zeros(len(td), dtype=torch.uint8, device="cuda")
        it = torch.zeros(len(td), dtype=torch.uint8, device="cuda")
        D.cb_decode_batch(td, soft, T.params(8, 1, 1, 0), b, ok, it)
        torch.cuda.synchronize()
        assert np.array_equal(soft.cpu().numpy(), soft_ref)
        ob, ook, oit = O.cb_decode_batch(od, soft_ref, O.params(8, 1, 1, 0), nb)
        assert np.array_equal(ok.cpu().numpy(), ook) and np.array_equal(it.cpu().numpy(), oit)
        assert np.array_equal(b.cpu().numpy(), ob)
        say(f"[rm] after rv {rv}: crc ok {ook.tolist()}")
