"""Python access to the CPU oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY: the oracle is the reference the GPU decoder is
checked against.  Only ``tests/``, the smoke check and the benchmark's CPU
baseline leg may import this package; the product path never does.

The C library follows the paper's decoding function (Sec. IV-B, Fig. 4) and
TS 36.212 for the constants the paper does not print; see ``oracle.h``.
This module only marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

CRC_NONE, CRC24A, CRC24B = 0, 1, 2
LLR_MAX = 2047
NUM_K = 188


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain C99, -O2, no intrinsics)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.run(
            ["gcc", "-O2", "-std=c99", "-Wall", "-shared", "-fPIC",
             os.path.join(HERE, "oracle.c"), "-o", tmp, "-lm"],
            check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Seg(ct.Structure):
    _fields_ = [(n, ct.c_int32) for n in
                ("B", "C", "L", "Kplus", "Kminus", "Cplus", "Cminus", "F")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class Params(ct.Structure):
    _fields_ = [("max_iters", ct.c_int32), ("early_stop", ct.c_int32),
                ("n_windows", ct.c_int32), ("win_init", ct.c_int32),
                ("mi_eps", ct.c_int32)]


class CbDesc(ct.Structure):
    _fields_ = [("llr_off", ct.c_int64), ("bits_off", ct.c_int64),
                ("K", ct.c_int32), ("F", ct.c_int16), ("crc", ct.c_int8),
                ("rsv", ct.c_int8)]


class TbResult(ct.Structure):
    _fields_ = [("tb_ok", ct.c_int32), ("max_iters_used", ct.c_int32),
                ("C", ct.c_int32), ("rsv", ct.c_int32),
                ("cb_ok", ct.c_uint8 * 64), ("cb_iters", ct.c_uint8 * 64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        L = ct.CDLL(LIB_PATH)
        P = ct.POINTER
        L.or_crc24.restype = ct.c_uint32
        L.or_crc24.argtypes = [ct.c_void_p, ct.c_int64, ct.c_int]
        L.or_k_table.argtypes = [ct.c_void_p]
        L.or_k_index.argtypes = [ct.c_int32]
        L.or_qpp_params.argtypes = [ct.c_int32, P(ct.c_int32), P(ct.c_int32)]
        L.or_qpp.argtypes = [ct.c_int32, ct.c_void_p]
        L.or_segment.argtypes = [ct.c_int32, P(Seg)]
        L.or_seg_k.argtypes = [P(Seg), ct.c_int32]
        L.or_turbo_encode_cb.argtypes = [ct.c_void_p, ct.c_int32, ct.c_void_p]
        L.or_tb_encode.argtypes = [ct.c_void_p, ct.c_int32, ct.c_void_p, ct.c_void_p]
        for fn in (L.or_constituent, L.or16_constituent):
            fn.argtypes = [ct.c_int32, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int32,
                           ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p] + \
                          ([ct.c_void_p] if fn is L.or16_constituent else [])
        L.or16_constituent_sched.argtypes = [ct.c_int32, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                             ct.c_int32, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                             ct.c_void_p, ct.c_void_p, ct.c_int32, ct.c_int32,
                                             ct.c_void_p]
        L.or_cb_decode_ex.argtypes = [ct.c_void_p, ct.c_int32, ct.c_int32, ct.c_int32, P(Params),
                                      ct.c_void_p, ct.c_void_p, P(ct.c_int32), P(ct.c_int32),
                                      ct.c_int32, ct.c_void_p]
        L.or_cb_decode_batch.argtypes = [ct.c_int32, ct.c_void_p, ct.c_void_p, P(Params),
                                         ct.c_void_p, ct.c_void_p, ct.c_void_p]
        L.or_tb_decode.argtypes = [ct.c_void_p, ct.c_int32, P(Params), ct.c_void_p, P(TbResult)]
        L.or_subblock_perm.argtypes = [ct.c_void_p]
        L.or_subblock_perm.restype = None
        L.or_rm_kw.argtypes = [ct.c_int32]
        L.or_rm_kw.restype = ct.c_int32
        L.or_rm_k0.argtypes = [ct.c_int32, ct.c_int32, ct.c_int32]
        L.or_rm_k0.restype = ct.c_int32
        L.or_rate_match.argtypes = [ct.c_void_p, ct.c_int32, ct.c_int32, ct.c_int32, ct.c_int32,
                                    ct.c_int32, ct.c_void_p]
        L.or_derate_match.argtypes = [ct.c_void_p, ct.c_int32, ct.c_int32, ct.c_int32,
                                      ct.c_int32, ct.c_int32, ct.c_void_p]
        L.or_win_len.argtypes = [ct.c_int32, ct.c_int32]
        L.or_win_len.restype = ct.c_int32
        L.or_tb_decode_w.argtypes = [ct.c_void_p, ct.c_int32, P(Params), ct.c_void_p,
                                     ct.c_void_p, P(TbResult)]
        L.or_mi_table.argtypes = [ct.c_void_p]
        L.or_mi_table.restype = None
        L.or_mi_sum.argtypes = [ct.c_void_p, ct.c_int32]
        L.or_mi_sum.restype = ct.c_int64
        L.or_mi_converged.argtypes = [ct.c_int64, ct.c_int64, ct.c_int32, ct.c_int32, ct.c_int32]
        L.or_mi_converged.restype = ct.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ct.c_void_p)


def _bits(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint8))


# --------------------------------------------------------------------------- CRC
def crc24(bits, which: int) -> int:
    b = _bits(bits)
    return int(lib().or_crc24(_ptr(b), b.size, which))


# --------------------------------------------------------------------------- tables
def k_table() -> np.ndarray:
    out = np.zeros(NUM_K, np.int32)
    lib().or_k_table(_ptr(out))
    return out


def qpp_params(K: int) -> tuple[int, int]:
    f1, f2 = ct.c_int32(), ct.c_int32()
    if lib().or_qpp_params(K, ct.byref(f1), ct.byref(f2)):
        raise ValueError(f"K={K} is not a code block size")
    return f1.value, f2.value


def qpp(K: int) -> np.ndarray:
    out = np.zeros(K, np.int32)
    if lib().or_qpp(K, _ptr(out)):
        raise ValueError(f"K={K} is not a code block size")
    return out


def segment(tbs: int) -> dict:
    s = Seg()
    if lib().or_segment(tbs, ct.byref(s)):
        raise ValueError(f"tbs={tbs} out of range")
    return s.as_dict()


def cb_sizes(tbs: int) -> list[tuple[int, int]]:
    """(K_r, F_r) for every code block of a transport block."""
    s = segment(tbs)
    return [(s["Kminus"] if r < s["Cminus"] else s["Kplus"], s["F"] if r == 0 else 0)
            for r in range(s["C"])]


def tb_llr_count(tbs: int) -> int:
    return sum(3 * (K + 4) for K, _ in cb_sizes(tbs))


# --------------------------------------------------------------------------- encoder
def turbo_encode_cb(c) -> np.ndarray:
    c = _bits(c)
    K = c.size
    d = np.zeros((3, K + 4), np.uint8)
    if lib().or_turbo_encode_cb(_ptr(c), K, _ptr(d)):
        raise ValueError(f"K={K} is not a code block size")
    return d


def tb_encode(payload) -> tuple[np.ndarray, np.ndarray]:
    """Returns (d, cb_bits): concatenated [3][K_r+4] coded bits (flat) and the
    concatenated code block input bits."""
    p = _bits(payload)
    tbs = p.size
    n_d = tb_llr_count(tbs)
    n_c = sum(K for K, _ in cb_sizes(tbs))
    d = np.zeros(n_d, np.uint8)
    cb = np.zeros(n_c, np.uint8)
    if lib().or_tb_encode(_ptr(p), tbs, _ptr(d), _ptr(cb)) < 0:
        raise ValueError("tb_encode failed")
    return d, cb


# --------------------------------------------------------------------------- decoder
MI_TAB_N = 128
STOP_CRC, STOP_MI = 1, 2  # early_stop bits


def params(max_iters=6, early_stop=0, n_windows=1, win_init=0, mi_eps=0) -> Params:
    return Params(max_iters, early_stop, n_windows, win_init, mi_eps)


def mi_table() -> np.ndarray:
    """T[m] = round(2^15 h(1 / (1 + e^(m/8)))), h the binary entropy, m <
    MI_TAB_N (paper Sec. IV-B mutual-information stop; the estimator of Land,
    Hoeher et al. for consistent LLRs without reference bits)."""
    out = np.zeros(MI_TAB_N, np.int32)
    lib().or_mi_table(_ptr(out))
    return out


def mi_sum(L) -> int:
    """Sum of T[min(|L_k|, MI_TAB_N - 1)]: 1 - I = mi_sum / (2^15 K)."""
    L = np.ascontiguousarray(L, np.int64)
    return int(lib().or_mi_sum(_ptr(L), L.size))


def mi_converged(s, s_prev, it, K, eps) -> bool:
    return bool(lib().or_mi_converged(s, s_prev, it, K, eps))


def constituent(lsa, lp, tail, n_windows=1, a_in=None, b_in=None, use16=False, periods=(4, 2)):
    """One max-log-MAP pass; returns (le, a_out, b_out[, sat]).  use16: the
    int16 twin, shifting the forward / backward metrics every periods[0] /
    periods[1] steps."""
    lsa = np.ascontiguousarray(lsa, np.int64)
    lp = np.ascontiguousarray(lp, np.int64)
    tail = np.ascontiguousarray(tail, np.int64)
    K = lsa.size
    nw = n_windows
    a_in = np.zeros(nw * 8, np.int64) if a_in is None else np.ascontiguousarray(a_in, np.int64)
    b_in = np.zeros(nw * 8, np.int64) if b_in is None else np.ascontiguousarray(b_in, np.int64)
    a_out = np.zeros(nw * 8, np.int64)
    b_out = np.zeros(nw * 8, np.int64)
    le = np.zeros(K, np.int64)
    if use16:
        sat = np.zeros(1, np.int64)
        rc = lib().or16_constituent_sched(K, _ptr(lsa), _ptr(lp), _ptr(tail), nw, _ptr(a_in),
                                          _ptr(b_in), _ptr(a_out), _ptr(b_out), _ptr(le),
                                          int(periods[0]), int(periods[1]), _ptr(sat))
    else:
        rc = lib().or_constituent(K, _ptr(lsa), _ptr(lp), _ptr(tail), nw, _ptr(a_in),
                                  _ptr(b_in), _ptr(a_out), _ptr(b_out), _ptr(le))
    if rc:
        raise ValueError("bad constituent arguments")
    return (le, a_out, b_out, int(sat[0])) if use16 else (le, a_out, b_out)


def cb_decode(llr, K: int, F: int = 0, crc: int = CRC24B, p: Params | None = None,
              use16: bool = False):
    """Decode one code block; returns dict(bits, lapp, ok, iters, sat)."""
    llr = np.ascontiguousarray(llr, np.int16).reshape(-1)
    assert llr.size == 3 * (K + 4)
    p = p or params()
    bits = np.zeros(K, np.uint8)
    lapp = np.zeros(K, np.int64)
    ok, it = ct.c_int32(), ct.c_int32()
    sat = np.zeros(1, np.int64)
    if lib().or_cb_decode_ex(_ptr(llr), K, F, crc, ct.byref(p), _ptr(bits), _ptr(lapp),
                             ct.byref(ok), ct.byref(it), int(use16), _ptr(sat)):
        raise ValueError("bad cb_decode arguments")
    return {"bits": bits, "lapp": lapp, "ok": ok.value, "iters": it.value, "sat": int(sat[0])}


def make_descs(cbs, payload_bits: bool = True):
    """Descriptor array for (K, F, crc) tuples laid out back to back."""
    descs = (CbDesc * len(cbs))()
    llr_off = bits_off = 0
    for i, (K, F, crc) in enumerate(cbs):
        descs[i].llr_off, descs[i].bits_off = llr_off, bits_off
        descs[i].K, descs[i].F, descs[i].crc = K, F, crc
        llr_off += 3 * (K + 4)
        L = 0 if crc == CRC_NONE else 24
        bits_off += (K - F - L + 7) // 8
    return descs, llr_off, bits_off


def cb_decode_batch(descs, llr, p: Params, n_bits_bytes: int):
    n = len(descs)
    llr = np.ascontiguousarray(llr, np.int16)
    bits = np.zeros(max(n_bits_bytes, 1), np.uint8)
    ok = np.zeros(max(n, 1), np.uint8)
    it = np.zeros(max(n, 1), np.uint8)
    if lib().or_cb_decode_batch(n, ct.cast(descs, ct.c_void_p), _ptr(llr), ct.byref(p),
                                _ptr(bits), _ptr(ok), _ptr(it)):
        raise ValueError("bad batch arguments")
    return bits[:n_bits_bytes], ok[:n], it[:n]


def subblock_perm() -> np.ndarray:
    out = np.zeros(32, np.int32)
    lib().or_subblock_perm(_ptr(out))
    return out


def rm_kw(K: int) -> int:
    return int(lib().or_rm_kw(int(K)))


def rm_k0(K: int, ncb: int, rv: int) -> int:
    return int(lib().or_rm_k0(int(K), int(ncb), int(rv)))


def rate_match(d, K: int, F: int, E: int, rv: int, ncb: int | None = None) -> np.ndarray:
    """The E coded bits that redundancy version rv sends (one per byte)."""
    d = np.ascontiguousarray(d, np.uint8)
    e = np.zeros(max(E, 1), np.uint8)
    if lib().or_rate_match(_ptr(d), K, F, E, rv, rm_kw(K) if ncb is None else ncb, _ptr(e)):
        raise ValueError("bad rate matching arguments")
    return e[:E]


def derate_match(e, K: int, F: int, rv: int, soft=None, ncb: int | None = None) -> np.ndarray:
    """Add soft values e into a [3][K+4] int16 soft buffer (new if None)."""
    e = np.ascontiguousarray(e, np.int16)
    out = np.zeros(3 * (K + 4), np.int16) if soft is None else np.array(soft, np.int16)
    if lib().or_derate_match(_ptr(e), e.size, K, F, rv, rm_kw(K) if ncb is None else ncb,
                             _ptr(out)):
        raise ValueError("bad de-rate-matching arguments")
    return out


def win_len(K: int, nw: int) -> int:
    """Length of all but the last window (0: the count leaves a window empty)."""
    return int(lib().or_win_len(int(K), int(nw)))


def tb_decode(llr, tbs: int, p: Params):
    return tb_decode_windows(llr, tbs, p, None)


def tb_decode_windows(llr, tbs: int, p: Params, nw_per_cb):
    """tb_decode with a window count per code block (None: p.n_windows)."""
    llr = np.ascontiguousarray(llr, np.int16)
    bits = np.zeros((tbs + 7) // 8, np.uint8)
    res = TbResult()
    nw = None if nw_per_cb is None else np.ascontiguousarray(nw_per_cb, np.int32)
    if lib().or_tb_decode_w(_ptr(llr), tbs, ct.byref(p), _ptr(nw), _ptr(bits), ct.byref(res)):
        raise ValueError("bad tb_decode arguments")
    return bits, {"tb_ok": res.tb_ok, "max_iters_used": res.max_iters_used, "C": res.C,
                  "cb_ok": list(res.cb_ok[:res.C]), "cb_iters": list(res.cb_iters[:res.C])}


def tb_purge_marked(llr, tbs: int, p: Params, nw_per_cb=None):
    """The paper's Algorithm 2 on top of independent block decoding: a
    transport block fails as soon as one of its code blocks fails.  With a
    stopping rule, a block that stops (the rule fires) while its CRC fails is
    known to have failed, so its transport block is marked failed and the
    work of its still-iterating siblings can be dropped.  Returns
    (bits, result, marked): the plain decode of every block with the rule,
    and whether some block stopped failed.  A block that fails at the last
    iteration stopped there iff decoding with one more iteration allowed
    also ends at that iteration (iterations are causal)."""
    bits, res = tb_decode_windows(llr, tbs, p, nw_per_cb)
    if not p.early_stop:
        return bits, res, False
    marked = any(ok == 0 and it < p.max_iters for ok, it in zip(res["cb_ok"], res["cb_iters"]))
    if not marked and p.max_iters < 16 and 0 in res["cb_ok"]:
        p1 = Params(p.max_iters + 1, p.early_stop, p.n_windows, p.win_init, p.mi_eps)
        _, r1 = tb_decode_windows(llr, tbs, p1, nw_per_cb)
        marked = any(ok == 0 and it0 == p.max_iters and it1 == p.max_iters
                     for ok, it0, it1 in zip(res["cb_ok"], res["cb_iters"], r1["cb_iters"]))
    return bits, res, marked
