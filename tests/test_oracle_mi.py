"""Pins of the oracle's mutual-information stop (paper Sec. IV-B, "Decoding
function": the iterations stop once the average mutual information of the
LLRs converges).

The estimate is 1 - I = mean_k h(1 / (1 + e^|L_k|)) (Land, Hoeher et al.,
consistent LLRs, no reference bits), tabulated in units of 2^-15 bit for L
in 1/8 nat.  What fixes it here, without retyping the formula:
  * h(1/2) = 1 at L = 0, and the closed-form tail bound
    h(p) <= (1 + x) e^-x / ln 2 for p = 1/(1 + e^x);
  * on consistent Gaussian LLRs the estimate equals the binary-input AWGN
    mutual information J(sigma), computed here by numerical integration of
    the reference-bit form 1 - E[log2(1 + e^-L)];
  * the stop rule's special cases (eps at its maximum, a channel that carries
    nothing, a noiseless block) and the invariance of the decoding trajectory
    under the stop.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import inputs
import workload as wl


def test_table_endpoints_and_tail(orc):
    T = orc.mi_table()
    assert T.size == orc.MI_TAB_N
    assert T[0] == 32768                         # L = 0: a coin flip, one bit of entropy
    assert (np.diff(T) <= 0).all() and T[-1] == 0
    for m in range(T.size):
        x = m / 8.0
        bound = 32768 * (1 + x) * math.exp(-x) / math.log(2)
        assert T[m] <= bound + 0.5


@pytest.mark.parametrize("sigma", [0.8, 1.6, 2.5, 4.0])
def test_estimator_matches_bi_awgn_mutual_information(orc, sigma):
    """Consistent LLRs L ~ N(s sigma^2/2, sigma^2) for s = +-1 (nats): the
    blind estimate from |L| alone equals J(sigma)."""
    def f(l):
        return math.exp(-(l - sigma * sigma / 2) ** 2 / (2 * sigma * sigma)) / \
            (sigma * math.sqrt(2 * math.pi)) * math.log2(1 + math.exp(-l))
    J = 1 - integrate.quad(f, -60, 60, limit=400)[0]
    g = np.random.default_rng(int(sigma * 100))
    n = 400_000
    s = np.where(g.integers(0, 2, n) == 1, 1.0, -1.0)
    L = s * sigma * sigma / 2 + sigma * g.standard_normal(n)
    Lq = np.round(8 * L).astype(np.int64)     # decoder units: 1/8 nat
    est = 1 - orc.mi_sum(Lq) / (32768 * n)
    assert abs(est - J) < 6e-3, (est, J)


def test_mi_sum_clips_large_magnitudes(orc):
    L = np.array([0, 5, -5, 127, -128, 3000, -30000], np.int64)
    T = orc.mi_table()
    want = T[0] + 2 * T[5] + 4 * T[127]
    assert orc.mi_sum(L) == want


def test_converged_rule(orc):
    K = 1000
    assert orc.mi_converged(100, 0, 1, K, 1)            # 1 - I <= eps at once
    assert not orc.mi_converged(1001, 0, 1, K, 1)        # iteration 1: no previous sum
    assert orc.mi_converged(50_000, 49_000, 2, K, 1)     # change 1000 <= K eps
    assert not orc.mi_converged(50_000, 48_999, 2, K, 1)
    assert orc.mi_converged(49_000, 50_000, 3, K, 1)     # either direction


def _noisy_cb(orc, K, esn0, seed, crc=None):
    crc = orc.CRC24B if crc is None else crc
    llr, pays, descs, _, _ = inputs.cb_batch([(K, 0, crc)], "16qam", esn0, 1905, seed)
    return llr


def test_max_eps_stops_after_one_iteration(orc):
    llr = _noisy_cb(orc, 512, 3.0, 1)
    r = orc.cb_decode(llr, 512, 0, orc.CRC24B, orc.params(8, orc.STOP_MI, 1, 0, 32768))
    assert r["iters"] == 1


def test_zero_llrs_stop_at_the_second_iteration(orc):
    """No channel information: every a-posteriori value stays 0, so the sum
    is K 2^15 each iteration and the change 0 stops the second one."""
    K = 256
    llr = np.zeros(3 * (K + 4), np.int16)
    r = orc.cb_decode(llr, K, 0, orc.CRC24A, orc.params(8, orc.STOP_MI, 1, 0, 0))
    assert r["iters"] == 2 and orc.mi_sum(r["lapp"]) == K * 32768


def test_noiseless_block_stops_at_once(orc):
    K = 1024
    g = wl.rng(1905, 7)
    _, d = inputs.encode_cb(K, 0, orc.CRC24A, g)
    llr = wl.noiseless_llr(d)
    r = orc.cb_decode(llr, K, 0, orc.CRC24A, orc.params(8, orc.STOP_MI, 1, 0, 0))
    assert r["iters"] == 1 and r["ok"] == 1 and orc.mi_sum(r["lapp"]) == 0


@pytest.mark.parametrize("K,esn0,nw,win_init,eps", [
    (1024, 1.2, 1, 0, 33), (2048, 0.6, 8, 1, 33), (512, 2.0, 4, 1, 300), (6144, 0.9, 32, 1, 16)])
def test_stop_leaves_the_trajectory_unchanged(orc, K, esn0, nw, win_init, eps):
    """The stopped decode equals the unstopped one cut at the same iteration,
    and that iteration is the first whose sums meet the rule."""
    llr = _noisy_cb(orc, K, esn0, K + nw)
    sums, runs = [], []
    for it in range(1, 9):
        r = orc.cb_decode(llr, K, 0, orc.CRC24B, orc.params(it, 0, nw, win_init))
        runs.append(r)
        sums.append(orc.mi_sum(r["lapp"]))
    want = next((i + 1 for i in range(8)
                 if orc.mi_converged(sums[i], sums[i - 1] if i else 0, i + 1, K, eps)), 8)
    for mode in (orc.STOP_MI, orc.STOP_MI | orc.STOP_CRC):
        r = orc.cb_decode(llr, K, 0, orc.CRC24B, orc.params(8, mode, nw, win_init, eps))
        crc_it = next((i + 1 for i in range(8) if runs[i]["ok"]), 99)
        it = min(want, crc_it) if mode & orc.STOP_CRC else want
        it = min(it, 8)
        assert r["iters"] == it
        assert np.array_equal(r["bits"], runs[it - 1]["bits"])
        assert np.array_equal(r["lapp"], runs[it - 1]["lapp"])
        assert r["ok"] == runs[it - 1]["ok"]


def test_mi_stop_ends_blocks_without_crc(orc):
    """What the rule adds: a block without a CRC, which the CRC stop can only
    run to the maximum, stops once its information has reached 1, with its
    payload decoded."""
    K = 1024
    for seed in range(3):
        g = wl.rng(1905, 40 + seed)
        pay, d = inputs.encode_cb(K, 0, orc.CRC_NONE, g)
        llr = wl.channel_blocks(d, [(K, 0)], "16qam", 5.0, g)
        crc = orc.cb_decode(llr, K, 0, orc.CRC_NONE, orc.params(8, orc.STOP_CRC, 1, 0))
        mi = orc.cb_decode(llr, K, 0, orc.CRC_NONE, orc.params(8, orc.STOP_MI, 1, 0, 1))
        assert crc["iters"] == 8 and mi["iters"] <= 3
        assert np.array_equal(mi["bits"], pay) and mi["ok"] == 1
        assert orc.mi_sum(mi["lapp"]) <= 2 * K


def test_bad_params_rejected(orc):
    llr = np.zeros(3 * 44, np.int16)
    for p in (orc.params(8, 4, 1, 0), orc.params(8, 2, 1, 0, -1), orc.params(8, 2, 1, 0, 32769)):
        with pytest.raises(Exception):
            orc.cb_decode(llr, 40, 0, orc.CRC_NONE, p)


def test_purge_model(orc):
    """Algorithm 2's rule on top of block decoding: a transport block is
    marked failed when one of its blocks stops on the MI rule with a failed
    CRC; blocks that decode, or blocks that fail without the rule firing,
    leave it unmarked."""
    tbs = 9000                       # two code blocks
    sizes = orc.cb_sizes(tbs)
    assert len(sizes) == 2
    g = wl.rng(1905, 11)
    d, _ = orc.tb_encode(wl.random_bits(g, tbs))
    clean = wl.channel_blocks(d, sizes, "qpsk", 6.0, g)
    p = orc.params(8, orc.STOP_MI, 1, 0, 300)
    _, res, marked = orc.tb_purge_marked(clean, tbs, p)
    assert res["tb_ok"] == 1 and not marked
    # the second block carries noise only: it fails, and with eps 300 its
    # a-posteriori sum settles well before the last iteration
    bad = clean.copy()
    n0 = 3 * (sizes[0][0] + 4)
    bad[n0:] = g.integers(-40, 41, bad.size - n0).astype(np.int16)
    _, res, marked = orc.tb_purge_marked(bad, tbs, p)
    assert res["cb_ok"][1] == 0 and res["cb_iters"][1] < 8 and marked
    assert res["tb_ok"] == 0
    # no stopping rule: nothing stops early, nothing is marked
    _, res, marked = orc.tb_purge_marked(bad, tbs, orc.params(8, 0, 1, 0, 0))
    assert res["cb_iters"] == [8, 8] and not marked
    # a block that fails at the last iteration is marked only if the rule
    # fired there: eps 0 with a noise block that never settles
    _, res, marked = orc.tb_purge_marked(bad, tbs, orc.params(2, orc.STOP_MI, 1, 0, 0))
    _, r3 = orc.tb_decode(bad, tbs, orc.params(3, orc.STOP_MI, 1, 0, 0))
    assert marked == (res["cb_ok"][1] == 0 and r3["cb_iters"][1] == 2 or res["cb_iters"][1] < 2)
