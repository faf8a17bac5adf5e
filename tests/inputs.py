"""Seeded test inputs built with the oracle's encoder and the workload channel.

Used by the GPU parity tests: the LLRs handed to both the GPU decoder and
the oracle come from here, never from the GPU path.
"""
from __future__ import annotations

import numpy as np

import oracle as O
import workload as wl


def encode_cb(K: int, F: int, crc: int, g: np.random.Generator):
    """Random payload + CRC in one code block; returns (payload bits, coded d)."""
    L = 0 if crc == O.CRC_NONE else 24
    c = np.zeros(K, np.uint8)
    pay = wl.random_bits(g, K - F - L)
    c[F:K - L] = pay
    if L:
        p = O.crc24(c[:K - L], crc)
        c[K - L:] = [(p >> (23 - i)) & 1 for i in range(24)]
    return pay, O.turbo_encode_cb(c).reshape(-1)


def cb_batch(cbs, mod: str, esn0, cfg: int, stream: int = 0):
    """cbs: [(K, F, crc)]; esn0: a number or one per block.  Returns
    (llr int16 flat, payloads list, oracle descs, llr elements, payload bytes)."""
    g = wl.rng(cfg, stream)
    descs, n_llr, n_bytes = O.make_descs(cbs)
    llr = np.zeros(n_llr, np.int16)
    pays = []
    esn0s = np.broadcast_to(np.asarray(esn0, np.float64), (len(cbs),))
    for i, (K, F, crc) in enumerate(cbs):
        pay, d = encode_cb(K, F, crc, g)
        o = descs[i].llr_off
        llr[o:o + 3 * (K + 4)] = wl.channel_blocks(d, [(K, F)], mod, float(esn0s[i]), g)
        pays.append(pay)
    return llr, pays, descs, n_llr, n_bytes


def tb_batch(tbs_list, mod: str, esn0, cfg: int, stream: int = 0):
    """Transport blocks back to back; returns (llr, payloads, llr_off, bits_off)."""
    g = wl.rng(cfg, stream)
    esn0s = np.broadcast_to(np.asarray(esn0, np.float64), (len(tbs_list),))
    parts, pays, llr_off, bits_off = [], [], [], []
    lo = bo = 0
    for i, tbs in enumerate(tbs_list):
        pay = wl.random_bits(g, tbs)
        d, _ = O.tb_encode(pay)
        parts.append(wl.channel_blocks(d, O.cb_sizes(tbs), mod, float(esn0s[i]), g))
        pays.append(pay)
        llr_off.append(lo)
        bits_off.append(bo)
        lo += parts[-1].size
        bo += (tbs + 7) // 8
    return np.concatenate(parts), pays, np.array(llr_off), np.array(bits_off)


def oracle_cb_batch(descs, llr, p):
    n_bytes = 0
    for d in descs:
        L = 0 if d.crc == O.CRC_NONE else 24
        n_bytes = max(n_bytes, d.bits_off + (d.K - d.F - L + 7) // 8)
    return O.cb_decode_batch(descs, llr, p, n_bytes)
