"""Pins for the oracle's turbo encoder (support code that builds test inputs).

The RSC code is fixed by g0 = 1 + D^2 + D^3 and g1 = 1 + D + D^3; these tests
check the encoder against polynomial identities over GF(2) that a shift
register realisation must satisfy, not against another shift register.
"""
import numpy as np

G0 = np.array([1, 0, 1, 1], np.uint8)  # 1 + D^2 + D^3
G1 = np.array([1, 1, 0, 1], np.uint8)  # 1 + D + D^3


def gf2_mul(a, b):
    return (np.convolve(np.asarray(a, np.int64), np.asarray(b, np.int64)) & 1).astype(np.uint8)


def _streams(d, K):
    d = d.reshape(3, K + 4)
    x, z1, z2 = d[0, :K], d[1, :K], d[2, :K]
    t1x = [d[0, K], d[2, K], d[1, K + 1]]
    t1z = [d[1, K], d[0, K + 1], d[2, K + 1]]
    t2x = [d[0, K + 2], d[2, K + 2], d[1, K + 3]]
    t2z = [d[1, K + 2], d[0, K + 3], d[2, K + 3]]
    return x, z1, z2, t1x, t1z, t2x, t2z


def test_impulse_response(orc):
    """A single 1 gives the parity g1/g0 = 1111001 (0111001)^* (g0 primitive, period 7)."""
    K = 64
    c = np.zeros(K, np.uint8)
    c[0] = 1
    d = orc.turbo_encode_cb(c)
    z = d.reshape(3, K + 4)[1, :K]
    expect = [1, 1, 1, 1, 0, 0, 1] + [0, 1, 1, 1, 0, 0, 1] * 10
    assert z.tolist() == expect[:K]


def test_terminated_words_satisfy_the_parity_identity(orc):
    """For each terminated constituent word (u = info + 3 tail inputs):
    g0 divides u, and u * g1 = z * g0 exactly (z = parity incl. tail)."""
    rng = np.random.default_rng(11)
    for K in (40, 112, 1056, 6144):
        c = rng.integers(0, 2, K).astype(np.uint8)
        d = orc.turbo_encode_cb(c)
        x, z1, z2, t1x, t1z, t2x, t2z = _streams(d, K)
        pi = orc.qpp(K)
        for info, par, tx, tz in ((c, z1, t1x, t1z), (c[pi], z2, t2x, t2z)):
            # polynomials with the first transmitted bit as the constant term
            u = np.concatenate([info, tx]).astype(np.uint8)
            z = np.concatenate([par, tz]).astype(np.uint8)
            lhs = gf2_mul(u, G1)
            rhs = gf2_mul(z, G0)
            assert np.array_equal(lhs, rhs)
            # the register ends at zero <=> u(D) is a multiple of g0(D): the
            # quotient a(D) = u/g0 has degree < K + 3 and remainder 0
            rem = list(u[::-1].astype(int))  # highest degree first
            g0 = [1, 1, 0, 1]  # D^3 + D^2 + 1, highest degree first
            for i in range(len(rem) - 3):
                if rem[i]:
                    for j in range(4):
                        rem[i + j] ^= g0[j]
            assert not any(rem[-3:])


def test_systematic_stream_and_lengths(orc):
    rng = np.random.default_rng(12)
    for K in (40, 6144):
        c = rng.integers(0, 2, K).astype(np.uint8)
        d = orc.turbo_encode_cb(c)
        assert d.size == 3 * K + 12
        assert np.array_equal(d.reshape(3, K + 4)[0, :K], c)


def test_zero_in_zero_out_and_linearity(orc):
    rng = np.random.default_rng(13)
    K = 528
    assert not orc.turbo_encode_cb(np.zeros(K, np.uint8)).any()
    a = rng.integers(0, 2, K).astype(np.uint8)
    b = rng.integers(0, 2, K).astype(np.uint8)
    assert np.array_equal(orc.turbo_encode_cb(a ^ b),
                          orc.turbo_encode_cb(a) ^ orc.turbo_encode_cb(b))


def test_tb_encode_structure(orc):
    """CRC24A over the payload, CRC24B per block, filler zeros leading block 0."""
    rng = np.random.default_rng(14)
    for tbs in (8, 6121, 20000):
        pay = rng.integers(0, 2, tbs).astype(np.uint8)
        d, cb = orc.tb_encode(pay)
        sizes = orc.cb_sizes(tbs)
        s = orc.segment(tbs)
        off = 0
        b = []
        for r, (K, F) in enumerate(sizes):
            blk = cb[off:off + K]
            assert not blk[:F].any()
            if s["C"] > 1:
                assert orc.crc24(blk, orc.CRC24B) == 0
                b.append(blk[F:K - 24])
            else:
                b.append(blk[F:])
            off += K
        b = np.concatenate(b)
        assert b.size == tbs + 24
        assert np.array_equal(b[:tbs], pay)
        assert orc.crc24(b, orc.CRC24A) == 0
