"""Pins of the oracle's rate matching and de-rate-matching (TS 36.212
5.1.4.1; the paper's puncturing, Sec. IV-B "Encoding function", and
retransmission, Sec. V).

What the standard fixes and these tests check without a copy of it: the
inter-column permutation is the 5-bit bit reversal; the redundancy version
start k0 = R (2 ceil(Ncb / 8R) rv + 2) (hand values below); a full-length
first transmission sends every non-<NULL> bit exactly once; receiver and
transmitter are adjoint (the receiver adds each soft value where the
transmitter took its bit); repetition adds, puncturing leaves zeros; and a
rate-matched block decodes through the turbo decoder.  The exact column
order and the <NULL> placement follow the standard as recalled (parity
unpinned beyond these properties).
"""
import numpy as np
import pytest

import workload as wl


def bitrev5(i):
    return int(f"{i:05b}"[::-1], 2)


def test_subblock_permutation_is_bit_reversal(orc):
    assert orc.subblock_perm().tolist() == [bitrev5(i) for i in range(32)]


@pytest.mark.parametrize("K,kw,k0s", [
    (40, 192, [4, 52, 100, 148]),            # R = 2: 2 * (2*12*rv + 2)
    (6144, 18528, [386, 5018, 9650, 14282]),  # R = 193: 193 * (2*12*rv + 2)
])
def test_buffer_length_and_rv_starts(orc, K, kw, k0s):
    assert orc.rm_kw(K) == kw
    assert [orc.rm_k0(K, kw, rv) for rv in range(4)] == k0s


def _positions(orc, K, F, E, rv, ncb=None):
    """Where each transmitted value lands: de-rate e_k = k + 1 into zeros."""
    e = np.arange(1, E + 1, dtype=np.int16)
    return orc.derate_match(e, K, F, rv, None, ncb)


@pytest.mark.parametrize("K,F", [(40, 0), (40, 8), (512, 5), (6144, 0)])
def test_full_first_transmission_sends_every_bit_once(orc, K, F):
    n = 3 * (K + 4) - 2 * F  # every bit but the filler of streams 0 and 1
    for rv in range(4):
        soft = _positions(orc, K, F, n, rv)
        s = soft.reshape(3, K + 4)
        assert (s[:2, :F] == 0).all()            # filler positions never sent
        assert sorted(soft[soft != 0].tolist()) == list(range(1, n + 1))


@pytest.mark.parametrize("K,F,E,rv", [(40, 0, 100, 0), (40, 8, 333, 2), (1056, 13, 2000, 1),
                                      (6144, 0, 12000, 3), (512, 0, 4000, 0)])
def test_receiver_is_adjoint_of_transmitter(orc, K, F, E, rv):
    """sum_k e_k * x(sel_k) == sum_i soft_i * x_i for the +-1 image x of any d."""
    rng = np.random.default_rng(K + E + rv)
    d = rng.integers(0, 2, 3 * (K + 4)).astype(np.uint8)
    d.reshape(3, K + 4)[:2, :F] = 0
    e = rng.integers(-40, 41, E).astype(np.int16)
    tx = orc.rate_match(d, K, F, E, rv).astype(np.int64) * 2 - 1
    soft = orc.derate_match(e, K, F, rv)
    x = d.astype(np.int64) * 2 - 1
    assert int((e.astype(np.int64) * tx).sum()) == int((soft.astype(np.int64) * x).sum())


def test_repetition_adds_and_puncturing_leaves_zeros(orc):
    K, F = 512, 0
    n = 3 * (K + 4)
    ones = np.ones(2 * n + 5, np.int16)
    soft = orc.derate_match(ones, K, F, 0)
    assert sorted(set(soft.tolist())) == [2, 3] and int(soft.sum()) == 2 * n + 5
    half = orc.derate_match(np.ones(n // 2, np.int16), K, F, 0)
    assert int((half != 0).sum()) == n // 2


def test_combining_saturates(orc):
    K = 40
    n = 3 * (K + 4)
    e = np.full(n, 30000, np.int16)
    soft = orc.derate_match(e, K, 0, 0)
    soft = orc.derate_match(e, K, 0, 0, soft)
    assert (soft == 32767).all()


def test_rate_matched_block_decodes(orc):
    """Encode, send rate 1/2 (E = 2K) at rv 0 noiselessly, de-rate-match,
    decode: CRC passes in one iteration and the bits come back."""
    K, F = 1056, 0
    rng = np.random.default_rng(5)
    c = np.zeros(K, np.uint8)
    c[:K - 24] = rng.integers(0, 2, K - 24)
    p = orc.crc24(c[:K - 24], orc.CRC24A)
    c[K - 24:] = [(p >> (23 - i)) & 1 for i in range(24)]
    d = orc.turbo_encode_cb(c).reshape(-1)
    e = orc.rate_match(d, K, F, 2 * K, 0)
    llr = np.where(e > 0, 600, -600).astype(np.int16)
    soft = orc.derate_match(llr, K, F, 0)
    r = orc.cb_decode(soft, K, F, orc.CRC24A, orc.params(8, 1, 1, 0))
    assert r["ok"] == 1 and np.array_equal(r["bits"], c)


def test_second_redundancy_version_rescues_a_failed_block(orc):
    """HARQ: a rate-3/4 first transmission that fails at this noise level
    decodes once a second redundancy version is combined into the soft
    buffer (seeded; checked for the oracle's own outputs)."""
    K, F = 2048, 0
    g = wl.rng(77, 0)
    c = np.zeros(K, np.uint8)
    c[:K - 24] = wl.random_bits(g, K - 24)
    p = orc.crc24(c[:K - 24], orc.CRC24A)
    c[K - 24:] = [(p >> (23 - i)) & 1 for i in range(24)]
    d = orc.turbo_encode_cb(c).reshape(-1)
    E = (4 * K) // 3
    soft = None
    oks = []
    for rv in (0, 2):
        e = orc.rate_match(d, K, F, E, rv)
        llr = wl.awgn_llr(e, "16qam", 7.0, g)
        soft = orc.derate_match(llr, K, F, rv, soft)
        oks.append(orc.cb_decode(soft, K, F, orc.CRC24A, orc.params(8, 1, 1, 0))["ok"])
    assert oks == [0, 1]
