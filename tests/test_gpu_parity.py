"""GPU parity: libtdec's HIP decoder against the CPU oracle, bit for bit.

Every comparison is exact: packed payload bits, CRC flags and iteration
counts (the decoder's arithmetic is integer and fully specified, so there is
exactly one correct output).  Inputs come from the oracle's encoder and the
seeded workload channel.
"""
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


def to_tdesc(T, odescs):
    d = (T.CbDesc * len(odescs))()
    for i, o in enumerate(odescs):
        d[i].llr_off, d[i].bits_off, d[i].K, d[i].F, d[i].crc = o.llr_off, o.bits_off, o.K, o.F, o.crc
    return d


def gpu_cb_batch(dev, odescs, llr, p, n_bytes):
    T, D, torch = dev
    td = to_tdesc(T, odescs)
    x = torch.from_numpy(llr).cuda()
    bits = torch.zeros(max(n_bytes, 1), dtype=torch.uint8, device="cuda")
    ok = torch.zeros(len(td), dtype=torch.uint8, device="cuda")
    it = torch.zeros(len(td), dtype=torch.uint8, device="cuda")
    D.cb_decode_batch(td, x, p, bits, ok, it)
    torch.cuda.synchronize()
    return bits.cpu().numpy()[:n_bytes], ok.cpu().numpy(), it.cpu().numpy()


def check_cb_parity(dev, cbs, mod, esn0, p, cfg, stream=0, tag=""):
    say(f"[parity] {tag} n={len(cbs)} K={sorted(set(c[0] for c in cbs))} mod={mod} "
        f"esn0={esn0} p=({p.max_iters},{p.early_stop},{p.n_windows},{p.win_init})")
    llr, pays, od, n_llr, n_bytes = cb_batch(cbs, mod, esn0, cfg, stream)
    T = dev[0]
    tp = T.params(p.max_iters, p.early_stop, p.n_windows, p.win_init)
    gb, gok, git = gpu_cb_batch(dev, od, llr, tp, n_bytes)
    ob, ook, oit = oracle_cb_batch(od, llr, p)
    assert np.array_equal(gok, ook), (gok, ook)
    assert np.array_equal(git, oit), (git, oit)
    assert np.array_equal(gb, ob)
    return gok, git


@pytest.mark.parametrize("K,F,crc,nw,win_init,es,iters", [
    (40, 0, O.CRC24B, 1, 0, 0, 3),
    (40, 8, O.CRC24B, 5, 1, 1, 8),
    (512, 0, O.CRC_NONE, 1, 0, 0, 4),
    (1056, 13, O.CRC24A, 4, 1, 1, 6),
    (6144, 0, O.CRC24B, 32, 1, 1, 8),
    (6144, 0, O.CRC24B, 32, 0, 0, 6),
    (5824, 0, O.CRC24B, 1, 0, 0, 2),
    (3136, 15, O.CRC24B, 14, 1, 1, 8),
    (6144, 0, O.CRC24B, 96, 1, 1, 6),    # 256-thread work groups (more than 64 windows)
    (1024, 0, O.CRC24B, 128, 1, 0, 4),   # 128 windows of 8 steps
    (488, 0, O.CRC24B, 8, 1, 1, 8),      # uneven: 7 windows of 64, the last of 40
    (6144, 0, O.CRC24B, 31, 1, 0, 6),    # uneven: 30 of 200, the last of 144
    (200, 0, O.CRC_NONE, 3, 0, 0, 4),    # uneven: 72, 72, 56
    (40, 8, O.CRC24B, 3, 1, 1, 8),       # uneven with filler: 16, 16, 8
    (6144, 0, O.CRC24B, 70, 1, 1, 6),    # uneven, 256-thread groups: 69 of 88, the last of 72
])
def test_cb_parity_noisy(dev, K, F, crc, nw, win_init, es, iters):
    cbs = [(K, F, crc)] * 6
    p = O.params(iters, es, nw, win_init)
    check_cb_parity(dev, cbs, "qpsk", [-1.0, 0.0, 0.5, 1.0, 2.0, 4.0], p, 201, K + nw,
                    tag=f"K{K}")


def test_adversarial_llrs(dev):
    """Saturated and alternating extremes, random signs: every range bound."""
    T, D, torch = dev
    g = np.random.default_rng(7)
    for K, nw in ((40, 1), (6144, 32), (2048, 16)):
        cbs = [(K, 0, O.CRC24B)] * 4
        od, n_llr, n_bytes = O.make_descs(cbs)
        sets = [
            g.choice([-2047, 2047], n_llr),
            np.where(np.arange(n_llr) % 2 == 0, 2047, -2047),
            g.integers(-32768, 32768, n_llr),
            np.zeros(n_llr),
        ]
        for s_i, v in enumerate(sets):
            llr = np.asarray(v, np.int16)
            for p in (O.params(5, 0, nw, 1), O.params(4, 1, nw, 0)):
                say(f"[adversarial] K={K} nw={nw} set={s_i} p=({p.max_iters},{p.early_stop})")
                tp = T.params(p.max_iters, p.early_stop, p.n_windows, p.win_init)
                gb, gok, git = gpu_cb_batch(dev, od, llr, tp, n_bytes)
                ob, ook, oit = oracle_cb_batch(od, llr, p)
                assert np.array_equal(gok, ook) and np.array_equal(git, oit)
                assert np.array_equal(gb, ob)


def test_mixed_sizes_one_launch(dev):
    """A batch of uneven K (filler, no CRC, both CRCs) in one launch equals the
    oracle, and each block equals itself decoded alone."""
    T = dev[0]
    g = np.random.default_rng(11)
    ks = O.k_table()
    cbs = []
    for _ in range(40):
        K = int(g.choice(ks))
        F = int(g.integers(0, 16)) if K >= 64 else 0
        crc = int(g.choice([O.CRC24A, O.CRC24B, O.CRC_NONE]))
        cbs.append((K, F, crc))
    p = O.params(8, 1, 1, 0)
    gok, git = check_cb_parity(dev, cbs, "16qam", 4.0, p, 202, tag="mixed")
    llr, pays, od, n_llr, n_bytes = cb_batch(cbs, "16qam", 4.0, 202)
    tp = T.params(8, 1, 1, 0)
    gb_all, _, _ = gpu_cb_batch(dev, od, llr, tp, n_bytes)
    for i in (0, 7, 23, 39):
        d = od[i]
        sub, _, nb = O.make_descs([cbs[i]])
        one = llr[d.llr_off:d.llr_off + 3 * (d.K + 4)]
        b1, ok1, it1 = gpu_cb_batch(dev, sub, one, tp, nb)
        assert np.array_equal(b1, gb_all[d.bits_off:d.bits_off + nb])
        assert ok1[0] == gok[i] and it1[0] == git[i]


def test_auto_windows_match_oracle(dev):
    T, D, torch = dev
    cbs = [(6144, 0, O.CRC24B), (5824, 0, O.CRC24B), (1024, 0, O.CRC24B), (40, 0, O.CRC24B)]
    llr, pays, od, n_llr, n_bytes = cb_batch(cbs, "qpsk", 1.0, 203)
    tp = T.params(6, 1, 0, 1)
    gb, gok, git = gpu_cb_batch(dev, od, llr, tp, n_bytes)
    for i, (K, F, crc) in enumerate(cbs):
        nw = D.pick_windows(K)
        assert nw >= 1 and K % nw == 0
        sub, _, nb = O.make_descs([(K, F, crc)])
        d = od[i]
        ob, ook, oit = O.cb_decode_batch(sub, llr[d.llr_off:d.llr_off + 3 * (K + 4)],
                                         O.params(6, 1, nw, 1), nb)
        assert gok[i] == ook[0] and git[i] == oit[0]
        assert np.array_equal(gb[d.bits_off:d.bits_off + nb], ob)


# ------------------------------------------------------------------ transport blocks


def gpu_tb_batch(dev, tbs_list, llr, llr_off, bits_off, p):
    T, D, torch = dev
    x = torch.from_numpy(llr).cuda()
    nb = int(bits_off[-1] + (tbs_list[-1] + 7) // 8)
    bits = torch.zeros(nb, dtype=torch.uint8, device="cuda")
    res = torch.zeros(len(tbs_list) * T.TB_RESULT_BYTES, dtype=torch.uint8, device="cuda")
    D.tb_decode_batch(tbs_list, llr_off, bits_off, x, p, bits, res)
    torch.cuda.synchronize()
    return bits.cpu().numpy(), T.parse_tb_results(res.cpu().numpy())


def test_single_tb_full_length(dev):
    """One 75376-bit TB (13 x K5824), QPSK at Es/N0 2 dB, full-length
    max-log-MAP, exactly 6 iterations, no early stop."""
    T = dev[0]
    tbs = 75376
    say("[tb] single TB 75376 full length 6 iterations")
    llr, pays, lo, bo = tb_batch([tbs], "qpsk", 2.0, 1)
    p = O.params(6, 0, 1, 0)
    gb, gres = gpu_tb_batch(dev, [tbs], llr, lo, bo, T.params(6, 0, 1, 0))
    ob, ores = O.tb_decode(llr, tbs, p)
    assert gres[0] == ores
    assert np.array_equal(gb, ob)
    assert gres[0]["C"] == 13


def test_tb_batch_mixed(dev):
    T = dev[0]
    g = wl.rng(3, 9)
    tbs_list = [int(x) for x in wl.tbs_log_uniform(g, 12)] + [16, 6120, 6121, 75376]
    esn0 = np.linspace(-1.0, 6.0, len(tbs_list))
    say(f"[tb] mixed batch {tbs_list}")
    llr, pays, lo, bo = tb_batch(tbs_list, "16qam", esn0, 3)
    p = O.params(8, 1, 1, 0)
    gb, gres = gpu_tb_batch(dev, tbs_list, llr, lo, bo, T.params(8, 1, 1, 0))
    for i, tbs in enumerate(tbs_list):
        ob, ores = O.tb_decode(llr[lo[i]:lo[i] + O.tb_llr_count(tbs)], tbs, p)
        assert gres[i] == ores, (i, tbs)
        assert np.array_equal(gb[bo[i]:bo[i] + ob.size], ob), (i, tbs)


# ------------------------------------------------------------------ encoder


def test_encoder_parity_every_size(dev):
    """Every one of the 188 block sizes (the chunked parallel encoder splits a
    block into 64 chunks of ceil(K/64) steps, so chunk lengths cover every
    residue mod 7 and the short last chunk every length), with filler and
    each CRC type, equals the oracle's serial encoder."""
    T, D, torch = dev
    g = np.random.default_rng(6)
    Ks = [int(k) for k in O.k_table()]
    crcs = (O.CRC24B, O.CRC24A, O.CRC_NONE)
    cbs = [(int(K), int(g.integers(0, 16)) if K >= 64 else 0, crcs[i % 3]) for i, K in enumerate(Ks)]
    td, n_llr, n_bytes = T.make_descs(cbs)
    pay = g.integers(0, 256, n_bytes).astype(np.uint8)
    # every output byte must be written: start from a pattern that no coded bit has
    coded = torch.full((n_llr,), 0xAA, dtype=torch.uint8, device="cuda")
    say(f"[enc] cb_encode_batch of {len(cbs)} sizes")
    D.cb_encode_batch(td, torch.from_numpy(pay).cuda(), coded)
    torch.cuda.synchronize()
    got = coded.cpu().numpy()
    for i, (K, F, crc) in enumerate(cbs):
        L = 0 if crc == O.CRC_NONE else 24
        bits = np.unpackbits(pay[td[i].bits_off:])[:K - F - L]
        c = np.zeros(K, np.uint8)
        c[F:K - L] = bits
        if L:
            p = O.crc24(c[:K - L], crc)
            c[K - L:] = [(p >> (23 - j)) & 1 for j in range(24)]
        ref = O.turbo_encode_cb(c).reshape(3, K + 4)
        g3 = got[td[i].llr_off:td[i].llr_off + 3 * (K + 4)].reshape(3, K + 4)
        ref[:2, :F] = 0
        assert np.array_equal(g3, ref), (K, F, crc)


def test_encoder_parity(dev):
    T, D, torch = dev
    g = np.random.default_rng(5)
    cbs = [(40, 0, O.CRC24B), (6144, 0, O.CRC24B), (1056, 9, O.CRC24A), (512, 3, O.CRC_NONE)]
    td, n_llr, n_bytes = T.make_descs(cbs)
    pay = g.integers(0, 256, n_bytes).astype(np.uint8)
    coded = torch.full((n_llr,), 0xAA, dtype=torch.uint8, device="cuda")
    say("[enc] cb_encode_batch")
    D.cb_encode_batch(td, torch.from_numpy(pay).cuda(), coded)
    torch.cuda.synchronize()
    got = coded.cpu().numpy()
    for i, (K, F, crc) in enumerate(cbs):
        L = 0 if crc == O.CRC_NONE else 24
        bits = np.unpackbits(pay[td[i].bits_off:])[:K - F - L]
        c = np.zeros(K, np.uint8)
        c[F:K - L] = bits
        if L:
            p = O.crc24(c[:K - L], crc)
            c[K - L:] = [(p >> (23 - j)) & 1 for j in range(24)]
        ref = O.turbo_encode_cb(c).reshape(3, K + 4)
        g3 = got[td[i].llr_off:td[i].llr_off + 3 * (K + 4)].reshape(3, K + 4)
        ref[:2, :F] = 0
        assert np.array_equal(g3, ref), (K, F, crc)
    # 6121..6128: block 1's payload starts at bit offsets of every residue mod 8
    for tbs in (1, 16, 6121, 6122, 6123, 6124, 6125, 6126, 6127, 6128, 12345, 30001, 75376):
        pay_bits = g.integers(0, 2, tbs).astype(np.uint8)
        packed = np.packbits(pay_bits)
        out = torch.full((T.tb_llr_count(tbs),), 0xAA, dtype=torch.uint8, device="cuda")
        say(f"[enc] tb_encode {tbs}")
        D.tb_encode(torch.from_numpy(packed).cuda(), tbs, out)
        torch.cuda.synchronize()
        ref, _ = O.tb_encode(pay_bits)
        got = out.cpu().numpy()
        # filler positions of d0/d1 in block 0 are not transmitted; compare the rest
        K0, F0 = O.cb_sizes(tbs)[0]
        mask = np.ones_like(ref, bool)
        mask[:F0] = False
        mask[K0 + 4:K0 + 4 + F0] = False
        assert np.array_equal(got[mask], ref[mask]), tbs


def _oracle_coded(pay, bits_off, K, F, crc):
    L = 0 if crc == O.CRC_NONE else 24
    bits = np.unpackbits(pay[bits_off:])[:K - F - L]
    c = np.zeros(K, np.uint8)
    c[F:K - L] = bits
    if L:
        p = O.crc24(c[:K - L], crc)
        c[K - L:] = [(p >> (23 - j)) & 1 for j in range(24)]
    ref = O.turbo_encode_cb(c).reshape(3, K + 4)
    ref[:2, :F] = 0
    return ref


def test_encoder_unaligned_destinations(dev):
    """Output blocks 1 to 7 bytes apart, so the three streams of a block start
    at every address residue mod 8 (the kernel stores 8 bytes at a time after
    a byte-wise head): every block equals the oracle and the gap bytes keep
    their pattern."""
    T, D, torch = dev
    g = np.random.default_rng(9)
    Ks = [40, 48, 56, 64, 72, 512, 1056, 2048, 3136, 6144, 6080, 4032]
    crcs = (O.CRC24B, O.CRC24A, O.CRC_NONE)
    cbs, offs, pays_off, o, b = [], [], [], 0, 0
    for i, K in enumerate(Ks * 2):
        crc = crcs[i % 3]
        F = int(g.integers(0, 16)) if K >= 64 else 0
        o += 1 + i % 7                      # gap of 1..7 bytes before the block
        cbs.append((K, F, crc))
        offs.append(o)
        pays_off.append(b)
        L = 0 if crc == O.CRC_NONE else 24
        o += 3 * (K + 4)
        b += (K - F - L + 7) // 8 + 3
    d = (T.CbDesc * len(cbs))()
    for i, (K, F, crc) in enumerate(cbs):
        d[i].llr_off, d[i].bits_off, d[i].K, d[i].F, d[i].crc = offs[i], pays_off[i], K, F, crc
    pay = g.integers(0, 256, b).astype(np.uint8)
    coded = torch.full((o + 5,), 0xAA, dtype=torch.uint8, device="cuda")
    say(f"[enc] unaligned destinations, {len(cbs)} blocks")
    D.cb_encode_batch(d, torch.from_numpy(pay).cuda(), coded)
    torch.cuda.synchronize()
    got = coded.cpu().numpy()
    written = np.zeros(got.size, bool)
    for i, (K, F, crc) in enumerate(cbs):
        g3 = got[offs[i]:offs[i] + 3 * (K + 4)].reshape(3, K + 4)
        assert np.array_equal(g3, _oracle_coded(pay, pays_off[i], K, F, crc)), (i, K, offs[i] % 8)
        written[offs[i]:offs[i] + 3 * (K + 4)] = True
    assert (got[~written] == 0xAA).all()


def test_encoder_full_batch_sampled(dev):
    """The 4096 x K6144 CRC24B launch the encoder benchmark times: 48 sampled
    blocks equal the oracle's encoder, and every output byte is a bit."""
    T, D, torch = dev
    n, K = 4096, 6144
    g = np.random.default_rng(10)
    td, n_llr, n_bytes = T.make_descs([(K, 0, T.CRC24B)] * n)
    pay = g.integers(0, 256, n_bytes).astype(np.uint8)
    coded = torch.full((n_llr,), 0xAA, dtype=torch.uint8, device="cuda")
    say(f"[enc] full batch {n} x K{K}")
    D.cb_encode_batch(td, torch.from_numpy(pay).cuda(), coded)
    torch.cuda.synchronize()
    got = coded.cpu().numpy()
    assert got.max() <= 1
    for i in g.choice(n, 48, replace=False):
        g3 = got[td[i].llr_off:td[i].llr_off + 3 * (K + 4)].reshape(3, K + 4)
        assert np.array_equal(g3, _oracle_coded(pay, td[i].bits_off, K, 0, O.CRC24B)), i


# ------------------------------------------------------------------ full-size workload


def test_uniform_batch_full_size_sampled(dev):
    """4096 x K6144 (16QAM, Es/N0 8 dB, 32 windows of 192, boundary init), the
    shape the benchmark times, decoded in one launch; a sample of blocks is
    re-decoded by the oracle, the rest checked for internal consistency."""
    T, D, torch = dev
    n = 4096
    K = 6144
    g = wl.rng(2, 0)
    say("[c2] building 4096 x K6144 inputs (sampled oracle encodes)")
    # encode a pool of 64 distinct blocks with the oracle; tile them
    cbs = [(K, 0, O.CRC24B)] * 64
    llr_pool, pays, od, n_llr, n_bytes = cb_batch(cbs, "16qam", 8.0, 2)
    blk = 3 * (K + 4)
    reps = n // 64
    llr = np.tile(llr_pool, reps)
    descs, tot, nbytes = T.make_descs([(K, 0, T.CRC24B)] * n)
    x = torch.from_numpy(llr).cuda()
    for es, iters in ((1, 8), (0, 6)):
        bits = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
        ok = torch.zeros(n, dtype=torch.uint8, device="cuda")
        it = torch.zeros(n, dtype=torch.uint8, device="cuda")
        say(f"[c2] decode es={es} iters={iters}")
        D.cb_decode_batch(descs, x, T.params(iters, es, 32, 1), bits, ok, it)
        torch.cuda.synchronize()
        gb = bits.cpu().numpy().reshape(n, -1)
        gok, git = ok.cpu().numpy(), it.cpu().numpy()
        # identical inputs give identical outputs wherever they sit in the batch
        for r in range(1, reps):
            assert np.array_equal(gb[r * 64:(r + 1) * 64], gb[:64])
            assert np.array_equal(git[r * 64:(r + 1) * 64], git[:64])
        sample = list(range(0, 64, 4))
        for i in sample:
            sub, _, nb = O.make_descs([(K, 0, O.CRC24B)])
            ob, ook, oit = O.cb_decode_batch(sub, llr_pool[i * blk:(i + 1) * blk],
                                             O.params(iters, es, 32, 1), nb)
            assert gok[i] == ook[0] and git[i] == oit[0], i
            assert np.array_equal(gb[i], ob), i


@pytest.mark.parametrize("cbs,p", [
    ([(6144, 0, O.CRC24B)] * 24, O.params(6, 0, 32, 1)),
    ([(6144, 0, O.CRC24B)] * 9, O.params(4, 1, 31, 1)),     # uneven windows
    ([(1056, 13, O.CRC24A)] * 30, O.params(5, 1, 4, 2)),    # exact boundaries
    ([(512, 0, O.CRC_NONE)] * 80 + [(40, 8, O.CRC24B)] * 70, O.params(8, 1, 1, 0)),
])
def test_small_grid(dev, cbs, p):
    """A grid capped far below the item count: every work group restages and
    decodes many items in turn (claims, scratch and LDS reuse); the outputs
    equal the oracle's."""
    T, _, torch = dev
    D2 = T.Decoder(0)
    try:
        D2.set_knobs(grid_cap=3)
        say(f"[small grid] n={len(cbs)} K={sorted(set(c[0] for c in cbs))} "
            f"p=({p.max_iters},{p.early_stop},{p.n_windows},{p.win_init}) grid_cap=3")
        llr, pays, od, n_llr, n_bytes = cb_batch(cbs, "qpsk", [(0.0, 1.0, 2.0)[i % 3]
                                                               for i in range(len(cbs))], 204)
        gb, gok, git = gpu_cb_batch((T, D2, torch), od, llr,
                                    T.params(p.max_iters, p.early_stop, p.n_windows, p.win_init),
                                    n_bytes)
        # exact boundaries equal full-length decoding (one window)
        op = O.params(p.max_iters, p.early_stop, 1, 0) if p.win_init == 2 else p
        ob, ook, oit = oracle_cb_batch(od, llr, op)
        assert np.array_equal(gok, ook) and np.array_equal(git, oit)
        assert np.array_equal(gb, ob)
    finally:
        D2.close()
