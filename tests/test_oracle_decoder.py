"""Pins for the oracle's max-log-MAP constituent decoder and turbo iteration.

* A full-length constituent pass must equal the plain definition of the
  max-log extrinsic: a difference of maxima over every terminated codeword
  (brute force over all 2^K inputs, K <= 11).
* Window plumbing: feeding the boundary outputs of one pass into the next
  makes the boundaries exact after nw passes, and then the windowed
  extrinsic equals the full-length one.
* The int16 twin (saturating int16 metrics with renormalisation) equals the
  exact int64 core on random and adversarial inputs, with no saturated
  decision.
* Turbo decoder: noiseless round trip, codeword-translation symmetry,
  iteration-count semantics, CRC false pass on all-zero input, TB rule.
"""
import numpy as np
import pytest

import workload as wl

# ------------------------------------------------------------------ brute force


def _code_paths(K):
    """All 2^K terminated paths of the RSC code: returns (U, Z, TX, TZ)."""
    n = 1 << K
    U = ((np.arange(n)[:, None] >> np.arange(K - 1, -1, -1)[None, :]) & 1).astype(np.int64)
    a1 = np.zeros(n, np.int64)
    a2 = np.zeros(n, np.int64)
    a3 = np.zeros(n, np.int64)
    Z = np.zeros((n, K), np.int64)
    for k in range(K):
        a = U[:, k] ^ a2 ^ a3          # feedback g0 = 1 + D^2 + D^3
        Z[:, k] = a ^ a1 ^ a3           # parity   g1 = 1 + D + D^3
        a1, a2, a3 = a, a1, a2
    TX = np.zeros((n, 3), np.int64)
    TZ = np.zeros((n, 3), np.int64)
    for j in range(3):
        u = a2 ^ a3                      # input equal to the feedback: a = 0
        TX[:, j] = u
        TZ[:, j] = 0 ^ a1 ^ a3
        a1, a2, a3 = 0 * a1, a1, a2
    assert not (a1 | a2 | a3).any()
    return U, Z, TX, TZ


def brute_extrinsic(lsa, lp, tail):
    K = len(lsa)
    U, Z, TX, TZ = _code_paths(K)
    tail = np.asarray(tail, np.int64)
    phi = U @ lsa + Z @ lp + TX @ tail[0::2] + TZ @ tail[1::2]
    le = np.zeros(K, np.int64)
    for k in range(K):
        one = U[:, k] == 1
        le[k] = (phi[one] - lsa[k]).max() - phi[~one].max()
    return le


@pytest.mark.parametrize("seed", range(30))
def test_constituent_equals_max_over_codewords(orc, seed):
    rng = np.random.default_rng(100 + seed)
    K = int(rng.integers(1, 12))
    lsa = rng.integers(-4094, 4095, K)
    lp = rng.integers(-2047, 2048, K)
    tail = rng.integers(-2047, 2048, 6)
    le, _, _ = orc.constituent(lsa, lp, tail)
    assert np.array_equal(le, brute_extrinsic(lsa, lp, tail))


def test_constituent_bruteforce_extremes(orc):
    rng = np.random.default_rng(5)
    for _ in range(10):
        K = 11
        lsa = rng.choice([-4094, 4094], K)
        lp = rng.choice([-2047, 2047], K)
        tail = rng.choice([-2047, 2047], 6)
        le, _, _ = orc.constituent(lsa, lp, tail)
        assert np.array_equal(le, brute_extrinsic(lsa, lp, tail))
        le16, _, _, sat = orc.constituent(lsa, lp, tail, use16=True)
        assert sat == 0 and np.array_equal(le16, le)


# ------------------------------------------------------------------ windows


@pytest.mark.parametrize("K,nw", [(64, 4), (192, 8), (6144, 32), (40, 5),
                                  (488, 8), (6144, 31), (200, 3)])  # uneven: last window shorter
def test_window_boundaries_converge_to_full_length(orc, K, nw):
    rng = np.random.default_rng(K + nw)
    lsa = rng.integers(-4094, 4095, K)
    lp = rng.integers(-2047, 2048, K)
    tail = rng.integers(-2047, 2048, 6)
    full, _, _ = orc.constituent(lsa, lp, tail, n_windows=1)
    a = np.zeros(nw * 8, np.int64)
    b = np.zeros(nw * 8, np.int64)
    first = None
    for p in range(nw):
        le, a, b = orc.constituent(lsa, lp, tail, n_windows=nw, a_in=a, b_in=b)
        if first is None:
            first = le
    le, _, _ = orc.constituent(lsa, lp, tail, n_windows=nw, a_in=a, b_in=b)
    assert np.array_equal(le, full)
    # with zero boundaries the windows really are cut
    assert nw == 1 or not np.array_equal(first, full) or K < 64


def test_window_partition_rule(orc):
    """Windows of W = 8*ceil(K/(8n)) steps, only the last one shorter; the
    even partition W = K/n whenever 8n divides K; a count that would leave a
    window empty is refused."""
    assert orc.win_len(6144, 32) == 192 and orc.win_len(40, 5) == 8
    assert orc.win_len(488, 8) == 64          # 7 windows of 64, the last of 40
    assert orc.win_len(6144, 31) == 200       # 30 of 200, the last of 144
    assert orc.win_len(200, 3) == 72          # 72, 72, 56
    assert orc.win_len(16, 3) == 0            # 8, 8 and an empty third
    assert orc.win_len(11, 1) == 11
    for K in (40, 488, 1000, 6144):
        for n in range(2, 129):
            W = orc.win_len(K, n)
            if W:
                last = K - (n - 1) * W
                assert 0 < last <= W and W % 8 == 0
                if K % (8 * n) == 0:
                    assert W == K // n and last == W


def test_single_window_is_full_length(orc):
    rng = np.random.default_rng(3)
    K = 528
    llr = rng.integers(-700, 700, 3 * (K + 4)).astype(np.int16)
    for crc in (orc.CRC_NONE, orc.CRC24B):
        r1 = orc.cb_decode(llr, K, 0, crc, orc.params(4, 0, 1, 0))
        r2 = orc.cb_decode(llr, K, 0, crc, orc.params(4, 0, 1, 1))
        assert np.array_equal(r1["lapp"], r2["lapp"])


# ------------------------------------------------------------------ int16 twin


def _adversarial_sets(rng, K):
    yield rng.integers(-4094, 4095, K), rng.integers(-2047, 2048, K), rng.integers(-2047, 2048, 6)
    yield rng.choice([-4094, 4094], K), rng.choice([-2047, 2047], K), rng.choice([-2047, 2047], 6)
    alt = np.where(np.arange(K) % 2 == 0, 4094, -4094)
    yield alt, -alt // 2, np.array([2047, -2047] * 3)
    yield np.full(K, 4094), np.full(K, -2047), np.full(6, 2047)
    yield np.full(K, -4094), np.full(K, 2047), np.full(6, -2047)
    yield rng.integers(-60, 61, K), rng.integers(-60, 61, K), rng.integers(-60, 61, 6)


@pytest.mark.parametrize("periods", [(4, 2), (2, 4), (2, 2)])
@pytest.mark.parametrize("K,nw", [(40, 1), (192, 1), (192, 8), (6144, 32), (1056, 11),
                                  (488, 8), (6144, 31)])
def test_int16_twin_equals_exact_constituent(orc, K, nw, periods):
    """Every shift schedule the GPU kernel uses (the recomputed recursion
    every 4 steps, the one beside the extrinsic every 2; either direction)."""
    rng = np.random.default_rng(K * 7 + nw)
    for lsa, lp, tail in _adversarial_sets(rng, K):
        a64 = b64 = a16 = b16 = None
        for it in range(3):  # boundary metrics carried across passes
            le, a64, b64 = orc.constituent(lsa, lp, tail, nw, a64, b64)
            le16, a16, b16, sat = orc.constituent(lsa, lp, tail, nw, a16, b16, use16=True,
                                                  periods=periods)
            assert sat == 0
            assert np.array_equal(le, le16)
            lsa = np.clip(lsa + rng.integers(-300, 301, K), -4094, 4094)


@pytest.mark.parametrize("periods", [(8, 2), (2, 8)])
def test_int16_twin_counts_saturation_of_sparser_schedules(orc, periods):
    """Shifting less often than the GPU kernel does lets winning sums leave
    int16 on extreme inputs, and the twin counts it: the bound is tight
    enough to matter (a control for the test above)."""
    rng = np.random.default_rng(99)
    K = 192
    hits = 0
    for _ in range(40):
        lsa = rng.choice([-4094, 4094], K)
        lp = rng.choice([-2047, 2047], K)
        tail = rng.choice([-2047, 2047], 6)
        hits += orc.constituent(lsa, lp, tail, 1, use16=True, periods=periods)[3]
        hits += orc.constituent(np.full(K, 4094), np.full(K, 2047), np.full(6, 2047), 1,
                                use16=True, periods=periods)[3]
    assert hits > 0


def test_int16_twin_worst_case_boundary_inits(orc):
    """Boundary vectors with the largest spread a normalised metric can have
    (3 * 6141 = 18423) next to the strongest possible branch metrics."""
    rng = np.random.default_rng(21)
    K, nw = 192, 8
    for _ in range(20):
        lsa = rng.choice([-4094, 4094], K)
        lp = rng.choice([-2047, 2047], K)
        tail = rng.choice([-2047, 2047], 6)
        a = -rng.choice([0, 18423], nw * 8) * rng.integers(0, 2, nw * 8)
        b = -rng.choice([0, 18423], nw * 8) * rng.integers(0, 2, nw * 8)
        a.reshape(nw, 8)[:, 0] = 0
        b.reshape(nw, 8)[:, 3] = 0
        le, _, _ = orc.constituent(lsa, lp, tail, nw, a, b)
        for periods in ((4, 2), (2, 4)):
            le16, _, _, sat = orc.constituent(lsa, lp, tail, nw, a, b, use16=True,
                                              periods=periods)
            assert sat == 0 and np.array_equal(le, le16)


# ------------------------------------------------------------------ turbo


def _encode(orc, K, F, rng, crc):
    c = np.zeros(K, np.uint8)
    L = 0 if crc == orc.CRC_NONE else 24
    c[F:K - L] = rng.integers(0, 2, K - F - L)
    if L:
        p = orc.crc24(c[:K - L], crc)
        c[K - 24:] = [(p >> (23 - i)) & 1 for i in range(24)]
    return c, orc.turbo_encode_cb(c).reshape(-1)


@pytest.mark.parametrize("K,F,nw", [(40, 0, 1), (40, 8, 5), (6144, 0, 32), (3136, 15, 1),
                                    (488, 0, 8)])
def test_noiseless_round_trip(orc, K, F, nw):
    rng = np.random.default_rng(K + F)
    c, d = _encode(orc, K, F, rng, orc.CRC24B)
    llr = wl.noiseless_llr(d)
    for use16 in (False, True):
        r = orc.cb_decode(llr, K, F, orc.CRC24B, orc.params(8, 1, nw, 1), use16=use16)
        assert r["ok"] == 1 and r["iters"] == 1
        assert np.array_equal(r["bits"][F:], c[F:])


@pytest.mark.parametrize("K,F,nw,win_init", [(104, 0, 1, 0), (512, 9, 4, 1), (6144, 0, 32, 1),
                                             (488, 5, 8, 1)])
def test_codeword_translation_symmetry(orc, K, F, nw, win_init):
    """Flipping the LLR signs on the 1-positions of any codeword flips the
    decoder's a-posteriori values exactly on that codeword's 1-positions."""
    rng = np.random.default_rng(K * 3 + nw)
    y = rng.integers(-900, 900, 3 * (K + 4)).astype(np.int16)
    y.reshape(3, K + 4)[:2, :F] = 0
    cw, d = _encode(orc, K, F, rng, orc.CRC_NONE)
    y2 = np.where(d > 0, -y, y).astype(np.int16)
    p = orc.params(5, 0, nw, win_init)
    r1 = orc.cb_decode(y, K, F, orc.CRC_NONE, p)
    r2 = orc.cb_decode(y2, K, F, orc.CRC_NONE, p)
    sign = np.where(cw > 0, -1, 1)
    assert np.array_equal(r2["lapp"], sign * r1["lapp"])


def test_iteration_semantics(orc):
    rng = np.random.default_rng(31)
    K = 1024
    y = rng.integers(-2047, 2048, 3 * (K + 4)).astype(np.int16)  # random signs: no codeword
    r = orc.cb_decode(y, K, 0, orc.CRC24B, orc.params(7, 1, 1, 0))
    assert r["ok"] == 0 and r["iters"] == 7
    r = orc.cb_decode(y, K, 0, orc.CRC24B, orc.params(5, 0, 4, 1))
    assert r["ok"] == 0 and r["iters"] == 5
    # all-zero LLRs decode to all-zero bits, which pass a zero-init CRC
    z = np.zeros(3 * (K + 4), np.int16)
    r = orc.cb_decode(z, K, 0, orc.CRC24B, orc.params(3, 1, 1, 0))
    assert r["ok"] == 1 and r["iters"] == 1 and not r["bits"].any()
    # crc none: ok is 1, and no early stop
    r = orc.cb_decode(y, K, 0, orc.CRC_NONE, orc.params(3, 1, 1, 0))
    assert r["ok"] == 1 and r["iters"] == 3


def test_inputs_are_clamped_and_filler_ignored(orc):
    rng = np.random.default_rng(32)
    K, F = 6144, 37
    y = rng.integers(-30000, 30000, 3 * (K + 4)).astype(np.int16)
    yc = np.clip(y, -2047, 2047).astype(np.int16)
    yf = yc.copy()
    yf.reshape(3, K + 4)[:2, :F] = rng.integers(-2047, 2048, (2, F))
    p = orc.params(2, 0, 32, 1)
    a = orc.cb_decode(y, K, F, orc.CRC24B, p)
    b = orc.cb_decode(yc, K, F, orc.CRC24B, p)
    c = orc.cb_decode(yf, K, F, orc.CRC24B, p)
    assert np.array_equal(a["lapp"], b["lapp"]) and np.array_equal(a["lapp"], c["lapp"])


@pytest.mark.parametrize("mod,esn0,nw", [("qpsk", 0.0, 1), ("16qam", 5.0, 8), ("qpsk", -1.0, 4)])
def test_int16_twin_equals_exact_turbo(orc, mod, esn0, nw):
    g = wl.rng(99, int(esn0 * 10) + 100 + nw)
    K = 1024
    c, d = _encode(orc, K, 0, g, orc.CRC24B)
    y = wl.channel_blocks(d, [(K, 0)], mod, esn0, g)
    p = orc.params(8, 1, nw, 1)
    a = orc.cb_decode(y, K, 0, orc.CRC24B, p)
    b = orc.cb_decode(y, K, 0, orc.CRC24B, p, use16=True)
    assert b["sat"] == 0
    assert a["ok"] == b["ok"] and a["iters"] == b["iters"]
    assert np.array_equal(a["bits"], b["bits"]) and np.array_equal(a["lapp"], b["lapp"])


def test_decoding_improves_with_snr(orc):
    """Sanity, not a pin: block errors fall as Es/N0 rises."""
    K = 512
    errs = []
    for esn0 in (-5.0, 3.0):
        g = wl.rng(98, int(esn0 + 10))
        bad = 0
        for _ in range(6):
            c, d = _encode(orc, K, 0, g, orc.CRC24B)
            y = wl.channel_blocks(d, [(K, 0)], "qpsk", esn0, g)
            r = orc.cb_decode(y, K, 0, orc.CRC24B, orc.params(6, 1, 1, 0))
            bad += int(not np.array_equal(r["bits"], c))
        errs.append(bad)
    assert errs[0] > errs[1]


def test_tb_rule_and_reassembly(orc):
    g = wl.rng(97, 0)
    tbs = 20000
    pay = wl.random_bits(g, tbs)
    d, _ = orc.tb_encode(pay)
    llr = wl.noiseless_llr(d)
    bits, res = orc.tb_decode(llr, tbs, orc.params(4, 1, 1, 0))
    assert res["tb_ok"] == 1 and res["C"] == 4 and all(res["cb_ok"])
    assert np.array_equal(np.unpackbits(bits)[:tbs], pay)
    # spoil one block: that block and the TB fail, the others still pass
    sizes = orc.cb_sizes(tbs)
    off = 3 * (sizes[0][0] + 4)
    llr2 = llr.copy()
    llr2[off:off + 3 * (sizes[1][0] + 4)] = g.integers(-2047, 2048, 3 * (sizes[1][0] + 4))
    bits2, res2 = orc.tb_decode(llr2, tbs, orc.params(4, 1, 1, 0))
    assert res2["tb_ok"] == 0 and res2["cb_ok"] == [1, 0, 1, 1]
    assert res2["cb_iters"][1] == 4 and res2["max_iters_used"] == 4


@pytest.mark.parametrize("K,F,nw,win_init", [(256, 0, 1, 0), (1056, 13, 8, 1)])
def test_iteration_dataflow(orc, K, F, nw, win_init):
    """Two full iterations composed by hand from the (brute-force pinned)
    constituent pass and the paper's dataflow: decoder 2 takes decoder 1's
    scaled extrinsic interleaved, the interleaved systematic LLRs and parity 2;
    its extrinsic goes back de-interleaved.  Scale 0.75 truncated toward
    zero, then clamped to +-2047 (written here in floating point)."""
    rng = np.random.default_rng(K + nw)
    y = rng.integers(-2500, 2500, 3 * (K + 4)).astype(np.int64)
    d = np.clip(y, -2047, 2047).reshape(3, K + 4)
    Ls, Lp1, Lp2 = d[0, :K].copy(), d[1, :K].copy(), d[2, :K].copy()
    Ls[:F] = Lp1[:F] = -2047
    t1 = [d[0, K], d[1, K], d[2, K], d[0, K + 1], d[1, K + 1], d[2, K + 1]]
    t2 = [d[0, K + 2], d[1, K + 2], d[2, K + 2], d[0, K + 3], d[1, K + 3], d[2, K + 3]]
    pi = orc.qpp(K)

    def scale(e):
        return np.clip(np.trunc(0.75 * e.astype(np.float64)), -2047, 2047).astype(np.int64)

    La1 = np.zeros(K, np.int64)
    bnd = [[None, None], [None, None]]
    for _ in range(2):
        le1, a, b = orc.constituent(Ls + La1, Lp1, t1, nw, *bnd[0])
        if win_init:
            bnd[0] = [a, b]
        La2 = scale(le1[pi])
        lsa2 = Ls[pi] + La2
        le2, a, b = orc.constituent(lsa2, Lp2, t2, nw, *bnd[1])
        if win_init:
            bnd[1] = [a, b]
        La1 = np.zeros(K, np.int64)
        La1[pi] = scale(le2)
        lapp = np.zeros(K, np.int64)
        lapp[pi] = lsa2 + le2
    r = orc.cb_decode(y.astype(np.int16), K, F, orc.CRC_NONE, orc.params(2, 0, nw, win_init))
    assert np.array_equal(r["lapp"], lapp)
    assert np.array_equal(r["bits"], (lapp > 0).astype(np.uint8))


def test_tb_decode_per_block_windows_reduces_to_common_count(orc):
    """Per-block window counts equal to the common count give the same TB
    result, and each block of a per-block run equals that block decoded alone
    with its own count (reassembly does not depend on the counts)."""
    import workload as wl
    tbs = 6121 + 6144  # 3 blocks: K 4096 (55 filler bits), 4160, 4160
    sizes = orc.cb_sizes(tbs)
    g = wl.rng(41, 0)
    pay = wl.random_bits(g, tbs)
    d, _ = orc.tb_encode(pay)
    llr = wl.channel_blocks(d, sizes, "qpsk", 1.5, g)
    p = orc.params(4, 0, 8, 1)
    b0, r0 = orc.tb_decode(llr, tbs, p)
    b1, r1 = orc.tb_decode_windows(llr, tbs, p, [8] * len(sizes))
    assert r0 == r1 and np.array_equal(b0, b1)
    nws = [1 if k % 16 else 2 for k, _ in sizes]
    b2, r2 = orc.tb_decode_windows(llr, tbs, p, nws)
    off = 0
    for r, (K, F) in enumerate(sizes):
        crc = orc.CRC24B if len(sizes) > 1 else orc.CRC24A
        res = orc.cb_decode(llr[off:off + 3 * (K + 4)], K, F, crc, orc.params(4, 0, nws[r], 1))
        assert res["ok"] == r2["cb_ok"][r] and res["iters"] == r2["cb_iters"][r]
        off += 3 * (K + 4)
