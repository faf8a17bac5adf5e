"""Pins for the oracle's CRC, block-size table, segmentation and QPP.

Each value here comes from outside the oracle: the public CRC catalogue, the
segmentation formula worked by hand, the table's step rule, and properties
(bijection, contention freedom, linearity) that any correct realisation has.
"""
import numpy as np
import pytest

from conftest import golden

# ------------------------------------------------------------------ CRC


def _bits_of(data: bytes) -> np.ndarray:
    return np.unpackbits(np.frombuffer(data, np.uint8))


def test_crc_catalogue_check_values(orc):
    g = golden("crc24_check_values.json")
    b = _bits_of(g["message_ascii"].encode())
    assert orc.crc24(b, orc.CRC24A) == int(g["crc24a"], 16)
    assert orc.crc24(b, orc.CRC24B) == int(g["crc24b"], 16)


def test_crc_of_single_one_is_the_polynomial(orc):
    g = golden("crc24_check_values.json")
    # "1" * D^24 mod g(D) = g(D) - D^24: the low 24 bits of the polynomial
    assert orc.crc24([1], orc.CRC24A) == int(g["poly24a"], 16)
    assert orc.crc24([1], orc.CRC24B) == int(g["poly24b"], 16)


def test_crc_zero_message_and_leading_zeros(orc):
    rng = np.random.default_rng(7)
    assert orc.crc24(np.zeros(1000, np.uint8), orc.CRC24A) == 0
    m = rng.integers(0, 2, 333).astype(np.uint8)
    for which in (orc.CRC24A, orc.CRC24B):
        assert orc.crc24(np.concatenate([np.zeros(57, np.uint8), m]), which) == orc.crc24(m, which)


def test_crc_linearity_and_append_check(orc):
    rng = np.random.default_rng(8)
    for which in (orc.CRC24A, orc.CRC24B):
        for n in (1, 24, 100, 6120):
            a = rng.integers(0, 2, n).astype(np.uint8)
            b = rng.integers(0, 2, n).astype(np.uint8)
            assert orc.crc24(a ^ b, which) == orc.crc24(a, which) ^ orc.crc24(b, which)
            p = orc.crc24(a, which)
            parity = np.array([(p >> (23 - i)) & 1 for i in range(24)], np.uint8)
            assert orc.crc24(np.concatenate([a, parity]), which) == 0


def test_crc_matches_polynomial_long_division(orc):
    """Remainder of M(D) * D^24 by g(D) computed with integer polynomials."""
    rng = np.random.default_rng(9)
    polys = {orc.CRC24A: 0x1864CFB, orc.CRC24B: 0x1800063}
    for which, g in polys.items():
        for n in (5, 40, 129):
            m = rng.integers(0, 2, n).astype(np.uint8)
            v = int("".join(map(str, m)), 2) << 24
            while v.bit_length() > 24:
                v ^= g << (v.bit_length() - 25)
            assert orc.crc24(m, which) == v


# ------------------------------------------------------------------ K table


def test_k_table_step_rule(orc):
    expect = (list(range(40, 513, 8)) + list(range(528, 1025, 16)) +
              list(range(1056, 2049, 32)) + list(range(2112, 6145, 64)))
    assert len(expect) == 188
    assert orc.k_table().tolist() == expect


# ------------------------------------------------------------------ segmentation


def test_segmentation_worked_examples(orc):
    g = golden("segmentation_examples.json")
    for ex in g["examples"]:
        s = orc.segment(ex["tbs"])
        for key in ("B", "C", "Kminus", "Cminus", "Kplus", "Cplus", "F"):
            assert s[key] == ex[key], (ex["tbs"], key)
    cmax = g["cb_max_size"]
    assert orc.segment(cmax)["C"] == 1 and orc.segment(cmax + 1)["C"] == 2


def _check_segmentation(orc, tbs, ktab):
    s = orc.segment(tbs)
    B, C, L, F = s["B"], s["C"], s["L"], s["F"]
    assert B == tbs + 24
    Bp = B + C * L
    Ks = [K for K, _ in orc.cb_sizes(tbs)]
    assert len(Ks) == C
    assert all(K in ktab for K in Ks)
    assert sum(Ks) == Bp + F
    assert 0 <= F < 6144
    if B <= 6144:
        assert C == 1 and L == 0
    else:
        assert L == 24 and C == -(-B // 6120)
    # K+ is the smallest table size with C * K+ >= B'
    assert s["Kplus"] == min(K for K in ktab if C * K >= Bp)
    # K- blocks first; sizes differ by one table step at most
    assert Ks == sorted(Ks)
    # payload bits reassemble to B
    assert sum(K - L for K in Ks) - F == B


def test_segmentation_invariants(orc):
    ktab = set(orc.k_table().tolist())
    rng = np.random.default_rng(10)
    sizes = list(range(1, 400)) + [6096, 6119, 6120, 6121, 6122, 12240, 12241, 75376, 391656]
    sizes += rng.integers(1, 400000, 300).tolist()
    for tbs in sizes:
        _check_segmentation(orc, int(tbs), ktab)


def test_segmentation_rejects_out_of_range(orc):
    with pytest.raises(ValueError):
        orc.segment(0)
    with pytest.raises(ValueError):
        orc.segment((1 << 20) + 1)


# ------------------------------------------------------------------ QPP


def test_qpp_spot_values(orc):
    for row in golden("qpp_spot_values.json")["rows"]:
        assert orc.qpp_params(row["K"]) == (row["f1"], row["f2"])


def test_qpp_is_a_permutation_for_every_K(orc):
    for K in orc.k_table().tolist():
        pi = orc.qpp(K)
        assert pi[0] == 0
        assert np.array_equal(np.sort(pi), np.arange(K)), K


def test_qpp_recurrence_form(orc):
    """pi(i+1) = pi(i) + g(i), g(i+1) = g(i) + 2 f2 (mod K), g(0) = f1 + f2."""
    for K in (40, 512, 1056, 5824, 6144):
        f1, f2 = orc.qpp_params(K)
        pi = orc.qpp(K)
        p, g = 0, (f1 + f2) % K
        for i in range(K):
            assert pi[i] == p
            p, g = (p + g) % K, (g + 2 * f2) % K


@pytest.mark.parametrize("K,nw", [(6144, 32), (5824, 13), (6144, 16), (4096, 64), (40, 5)])
def test_qpp_contention_free_windows(orc, K, nw):
    """At every step t, the nw windows of decoder 2 touch nw distinct windows
    of the natural order (a property of QPP interleavers)."""
    W = K // nw
    pi = orc.qpp(K).reshape(nw, W)
    for t in range(W):
        assert len(set((pi[:, t] // W).tolist())) == nw
