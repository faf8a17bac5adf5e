"""Seeded synthetic workloads: payload bits, channel, LLR quantisation.

This module holds none of the decoder's arithmetic.  It draws random payload
bits and passes already-encoded bits through a QAM/AWGN channel with an exact
max-log demapper and the int16 quantiser of the decoder's input format.  The
same generator feeds the oracle and the GPU path; which encoder produced the
coded bits is the caller's business.

The paper's traffic (live file transfers from commercial phones over a USRP
front end, Sec. V) cannot be reproduced, so every workload here is synthetic
AWGN traffic with the shapes of the decoder's configurations.

Channel recipe:
  * bits of one code block are sent as d0[F:] + d1[F:] + d2 (the filler
    positions of d0 and d1 are not transmitted), blocks in order, the last
    symbol padded with zeros;
  * square QAM with 2^(m/2) levels per axis, binary-reflected Gray labels per
    axis (first m/2 bits of a symbol on I, the rest on Q), unit average
    symbol energy;
  * complex AWGN with variance N0 = 10^(-EsN0/10);
  * exact max-log LLR in nats, positive meaning bit 1:
      L = (min_{x: b=0} (y-x)^2 - min_{x: b=1} (y-x)^2) / N0 per axis;
  * int16 quantisation q = clamp(round_half_away(8 * L), -2047, 2047).
"""
from __future__ import annotations

import numpy as np

SEED_BASE = (1905, 1141)
LLR_SCALE = 8.0
LLR_MAX = 2047
MOD_BITS = {"qpsk": 2, "16qam": 4, "64qam": 6, "256qam": 8}


def rng(cfg: int, stream: int = 0) -> np.random.Generator:
    """The generator for configuration `cfg`, sub-stream `stream`."""
    return np.random.default_rng([*SEED_BASE, int(cfg), int(stream)])


def random_bits(g: np.random.Generator, n: int) -> np.ndarray:
    """Bernoulli(0.5) bits, one per byte."""
    return g.integers(0, 2, size=int(n), dtype=np.uint8)


def _axis_constellation(m_axis: int):
    """Levels (ascending) and the Gray label of each level for one axis."""
    M = 1 << m_axis
    idx = np.arange(M)
    labels = idx ^ (idx >> 1)  # binary-reflected Gray code of the level index
    scale = np.sqrt(3.0 / (2.0 * (M * M - 1)))  # unit average energy over I and Q
    levels = (2.0 * idx - (M - 1)) * scale
    return levels, labels


def _bits_to_axis(bits: np.ndarray, m_axis: int) -> np.ndarray:
    """Map groups of m_axis bits (MSB first) to level values."""
    levels, labels = _axis_constellation(m_axis)
    inv = np.empty_like(labels)
    inv[labels] = np.arange(labels.size)
    b = bits.reshape(-1, m_axis).astype(np.int64)
    v = np.zeros(b.shape[0], np.int64)
    for j in range(m_axis):
        v = (v << 1) | b[:, j]
    return levels[inv[v]]


def _axis_llr(y: np.ndarray, m_axis: int, n0: float) -> np.ndarray:
    """Exact max-log LLRs (nats) of the m_axis bits carried on one axis."""
    levels, labels = _axis_constellation(m_axis)
    d2 = (y[:, None] - levels[None, :]) ** 2
    out = np.empty((y.size, m_axis), np.float64)
    for j in range(m_axis):
        bit = (labels >> (m_axis - 1 - j)) & 1
        out[:, j] = (d2[:, bit == 0].min(axis=1) - d2[:, bit == 1].min(axis=1)) / n0
    return out.reshape(-1)


def quantise(llr_nats: np.ndarray) -> np.ndarray:
    v = LLR_SCALE * llr_nats
    q = np.sign(v) * np.floor(np.abs(v) + 0.5)
    return np.clip(q, -LLR_MAX, LLR_MAX).astype(np.int16)


def awgn_llr(bits: np.ndarray, mod: str, esn0_db: float, g: np.random.Generator,
             chunk: int = 1 << 22) -> np.ndarray:
    """int16 LLRs for a bit stream sent over QAM + AWGN (see module doc)."""
    m = MOD_BITS[mod]
    ma = m // 2
    n = bits.size
    pad = (-n) % m
    b = np.concatenate([bits.astype(np.uint8), np.zeros(pad, np.uint8)]) if pad else bits
    n0 = 10.0 ** (-esn0_db / 10.0)
    sigma = np.sqrt(n0 / 2.0)
    out = np.empty(b.size, np.int16)
    step = (chunk // m) * m
    for s in range(0, b.size, step):
        bb = b[s:s + step].reshape(-1, m)
        yi = _bits_to_axis(bb[:, :ma].reshape(-1), ma) + sigma * g.standard_normal(bb.shape[0])
        yq = _bits_to_axis(bb[:, ma:].reshape(-1), ma) + sigma * g.standard_normal(bb.shape[0])
        li = _axis_llr(yi, ma, n0).reshape(-1, ma)
        lq = _axis_llr(yq, ma, n0).reshape(-1, ma)
        out[s:s + bb.size] = quantise(np.concatenate([li, lq], axis=1).reshape(-1))
    return out[:n]


def tx_bits(d: np.ndarray, K: int, F: int) -> np.ndarray:
    """The transmitted bits of one code block's [3][K+4] coded array."""
    d = d.reshape(3, K + 4)
    return np.concatenate([d[0, F:], d[1, F:], d[2]])


def rx_llr(llr_tx: np.ndarray, K: int, F: int) -> np.ndarray:
    """Put received LLRs back into the [3][K+4] layout (filler positions 0)."""
    out = np.zeros((3, K + 4), np.int16)
    n01 = K + 4 - F
    out[0, F:] = llr_tx[:n01]
    out[1, F:] = llr_tx[n01:2 * n01]
    out[2] = llr_tx[2 * n01:2 * n01 + K + 4]
    return out


def channel_blocks(d_flat: np.ndarray, blocks, mod: str, esn0_db: float,
                   g: np.random.Generator) -> np.ndarray:
    """Send the code blocks of d_flat ([3][K+4] arrays back to back, sizes
    `blocks` = [(K, F), ...]) over one channel realisation; returns the int16
    LLRs in the same layout."""
    parts, offs = [], []
    off = 0
    for K, F in blocks:
        parts.append(tx_bits(d_flat[off:off + 3 * (K + 4)], K, F))
        offs.append(off)
        off += 3 * (K + 4)
    stream = np.concatenate(parts) if parts else np.zeros(0, np.uint8)
    llr = awgn_llr(stream, mod, esn0_db, g)
    out = np.zeros(off, np.int16)
    pos = 0
    for (K, F), o in zip(blocks, offs):
        n = 3 * (K + 4) - 2 * F
        out[o:o + 3 * (K + 4)] = rx_llr(llr[pos:pos + n], K, F).reshape(-1)
        pos += n
    return out


def noiseless_llr(d_flat: np.ndarray, amp: int = LLR_MAX) -> np.ndarray:
    """+amp for a 1, -amp for a 0."""
    return np.where(np.asarray(d_flat) > 0, amp, -amp).astype(np.int16)


def tbs_log_uniform(g: np.random.Generator, n: int, lo: int = 16, hi: int = 75376) -> np.ndarray:
    """Transport block sizes drawn log-uniform in [lo, hi], rounded to whole bytes."""
    v = np.exp(g.uniform(np.log(lo), np.log(hi), size=n))
    return np.clip(np.round(v / 8.0) * 8, lo, hi).astype(np.int64)
