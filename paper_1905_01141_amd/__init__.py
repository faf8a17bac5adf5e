"""Python binding of libtdec, the MI355X (gfx950) LTE turbo decoder.

Argument marshalling only: every step of the decoding path runs in the HIP
kernels of libtdec.so (see include/tdec.h for the C ABI and its contract).
PyTorch supplies device memory and the stream.  Importing works without a
GPU; any call that needs the library raises if libtdec.so is missing or no
GPU is present -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as ct
import functools
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtdec.so")

CRC_NONE, CRC24A, CRC24B = 0, 1, 2
STATUS = {0: "OK", -1: "EINVAL", -2: "ERANGE", -3: "ENOMEM", -4: "EDEVICE", -5: "EBUSY"}
EXPORTS = ("tdec_segment", "tdec_tb_llr_count", "tdec_k_table", "tdec_qpp", "tdec_create",
           "tdec_destroy", "tdec_pick_windows", "cb_decode_batch", "tb_decode", "tb_decode_batch",
           "cb_encode_batch", "tb_encode")


class TdecError(RuntimeError):
    def __init__(self, fn, code):
        super().__init__(f"{fn} failed: {STATUS.get(code, code)}")
        self.code = code


class Params(ct.Structure):
    _fields_ = [("max_iters", ct.c_int32), ("early_stop", ct.c_int32),
                ("n_windows", ct.c_int32), ("win_init", ct.c_int32)]


class Seg(ct.Structure):
    _fields_ = [(n, ct.c_int32) for n in
                ("B", "C", "L", "Kplus", "Kminus", "Cplus", "Cminus", "F")]


class CbDesc(ct.Structure):
    _fields_ = [("llr_off", ct.c_int64), ("bits_off", ct.c_int64), ("K", ct.c_int32),
                ("F", ct.c_int16), ("crc", ct.c_int8), ("rsv", ct.c_int8)]


# tdec_cb_desc as a numpy record (same layout) for vectorised checks
DESC_DTYPE = np.dtype([("llr_off", "<i8"), ("bits_off", "<i8"), ("K", "<i4"), ("F", "<i2"),
                       ("crc", "i1"), ("rsv", "i1")])

# tdec_tb_result as stored in device memory
TB_RESULT_DTYPE = np.dtype([("tb_ok", "<i4"), ("max_iters_used", "<i4"), ("C", "<i4"),
                            ("rsv", "<i4"), ("cb_ok", "u1", (64,)), ("cb_iters", "u1", (64,))])
TB_RESULT_BYTES = TB_RESULT_DTYPE.itemsize

_lib = None


def lib():
    """Load libtdec.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1905_01141_amd.build`")
        L = ct.CDLL(LIB_PATH)
        P, vp, i32, i64 = ct.POINTER, ct.c_void_p, ct.c_int32, ct.c_int64
        L.tdec_segment.argtypes = [i32, P(Seg)]
        L.tdec_tb_llr_count.restype = i64
        L.tdec_tb_llr_count.argtypes = [i32]
        L.tdec_k_table.argtypes = [vp]
        L.tdec_qpp.argtypes = [i32, vp, vp, vp]
        L.tdec_create.argtypes = [ct.c_int, ct.c_size_t, P(vp)]
        L.tdec_destroy.argtypes = [vp]
        L.tdec_destroy.restype = None
        L.tdec_pick_windows.argtypes = [vp, i32]
        L.cb_decode_batch.argtypes = [vp, i32, vp, vp, P(Params), vp, vp, vp, vp]
        L.tb_decode.argtypes = [vp, vp, i32, P(Params), vp, vp, vp]
        L.tb_decode_batch.argtypes = [vp, i32, vp, vp, vp, vp, P(Params), vp, vp, vp]
        L.cb_encode_batch.argtypes = [vp, i32, vp, vp, vp, vp]
        L.tb_encode.argtypes = [vp, vp, i32, vp, vp]
        _lib = L
    return _lib


def _check(fn, code):
    if code != 0:
        raise TdecError(fn, code)


def _np_ptr(a):
    return None if a is None else a.ctypes.data_as(ct.c_void_p)


def _dptr(t):
    """Device pointer of a torch CUDA tensor (or None)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return ct.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ct.c_void_p(s.cuda_stream)


# ----------------------------------------------------------------------------- helpers
def params(max_iters=6, early_stop=0, n_windows=1, win_init=0) -> Params:
    return Params(max_iters, early_stop, n_windows, win_init)


def segment(tbs: int) -> dict:
    s = Seg()
    _check("tdec_segment", lib().tdec_segment(int(tbs), ct.byref(s)))
    return {n: getattr(s, n) for n, _ in Seg._fields_}


def cb_sizes(tbs: int) -> list[tuple[int, int]]:
    s = segment(tbs)
    return [(s["Kminus"] if r < s["Cminus"] else s["Kplus"], s["F"] if r == 0 else 0)
            for r in range(s["C"])]


@functools.lru_cache(maxsize=4096)
def tb_llr_count(tbs: int) -> int:
    n = lib().tdec_tb_llr_count(int(tbs))
    if n < 0:
        raise TdecError("tdec_tb_llr_count", -2)
    return int(n)


def k_table() -> np.ndarray:
    out = np.zeros(188, np.int32)
    lib().tdec_k_table(_np_ptr(out))
    return out


def qpp(K: int) -> tuple[np.ndarray, int, int]:
    pi = np.zeros(K, np.int32)
    f1, f2 = ct.c_int32(), ct.c_int32()
    _check("tdec_qpp", lib().tdec_qpp(int(K), _np_ptr(pi), ct.byref(f1), ct.byref(f2)))
    return pi, f1.value, f2.value


def make_descs(cbs) -> tuple[ct.Array, int, int]:
    """Descriptor array for (K, F, crc) code blocks laid out back to back.
    Returns (descs, total LLR elements, total payload bytes)."""
    descs = (CbDesc * len(cbs))()
    llr_off = bits_off = 0
    for i, (K, F, crc) in enumerate(cbs):
        descs[i].llr_off, descs[i].bits_off = llr_off, bits_off
        descs[i].K, descs[i].F, descs[i].crc = int(K), int(F), int(crc)
        llr_off += 3 * (K + 4)
        L = 0 if crc == CRC_NONE else 24
        bits_off += (K - F - L + 7) // 8
    return descs, llr_off, bits_off


def _desc_extent(descs):
    """(LLR elements, payload bytes) a descriptor array reaches, vectorised."""
    if len(descs) == 0:
        return 0, 0
    v = np.frombuffer(descs, dtype=DESC_DTYPE, count=len(descs))
    K = v["K"].astype(np.int64)
    L = np.where(v["crc"] == CRC_NONE, 0, 24)
    nb = np.maximum(0, (K - v["F"] - L + 7) // 8)
    return int((v["llr_off"] + 3 * (K + 4)).max()), int((v["bits_off"] + nb).max())


def _need(t, dtype: str, n: int, name: str):
    """Check that device tensor t has the dtype and at least n elements, so
    that no descriptor can make a kernel reach past the buffer."""
    if t is None:
        raise ValueError(f"{name}: tensor required")
    if str(t.dtype) != "torch." + dtype:
        raise ValueError(f"{name}: {dtype} tensor expected, got {t.dtype}")
    if t.numel() < n:
        raise ValueError(f"{name}: {n} elements needed, tensor has {t.numel()}")


# ----------------------------------------------------------------------------- context
class Decoder:
    """A libtdec context on one GPU (owns the device workspace)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self.device = device
        h = ct.c_void_p()
        _check("tdec_create", lib().tdec_create(device, hbm_budget_bytes, ct.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().tdec_destroy(self._h)
            self._h = ct.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def pick_windows(self, K: int) -> int:
        return int(lib().tdec_pick_windows(self._h, int(K)))

    def cb_decode_batch(self, descs, llr, p: Params, bits=None, crc_ok=None, iters=None,
                        stream=None):
        """llr: int16 CUDA tensor; bits: uint8 CUDA tensor or None; crc_ok /
        iters: uint8 CUDA tensors with one entry per code block."""
        n = len(descs)
        n_llr, n_bits = _desc_extent(descs)
        _need(llr, "int16", n_llr, "llr")
        if bits is not None:
            _need(bits, "uint8", n_bits, "bits")
        _need(crc_ok, "uint8", n, "crc_ok")
        _need(iters, "uint8", n, "iters")
        _check("cb_decode_batch",
               lib().cb_decode_batch(self._h, n, ct.cast(descs, ct.c_void_p), _dptr(llr),
                                     ct.byref(p), _dptr(bits), _dptr(crc_ok), _dptr(iters),
                                     _stream(stream)))

    def tb_decode(self, llr, tbs: int, p: Params, bits, res, stream=None):
        """res: uint8 CUDA tensor of TB_RESULT_BYTES bytes."""
        _need(llr, "int16", tb_llr_count(tbs), "llr")
        if bits is not None:
            _need(bits, "uint8", (tbs + 7) // 8, "bits")
        _need(res, "uint8", TB_RESULT_BYTES, "res")
        _check("tb_decode", lib().tb_decode(self._h, _dptr(llr), int(tbs), ct.byref(p),
                                            _dptr(bits), _dptr(res), _stream(stream)))

    def tb_decode_batch(self, tbs, llr_off, bits_off, llr, p: Params, bits, res, stream=None):
        tbs = np.ascontiguousarray(tbs, np.int32)
        llr_off = np.ascontiguousarray(llr_off, np.int64)
        bits_off = None if bits_off is None else np.ascontiguousarray(bits_off, np.int64)
        n = tbs.size
        if n:
            counts = np.array([tb_llr_count(int(t)) for t in tbs], np.int64)
            _need(llr, "int16", int((llr_off + counts).max()), "llr")
            if bits is not None:
                _need(bits, "uint8", int((bits_off + (tbs.astype(np.int64) + 7) // 8).max()), "bits")
        _need(res, "uint8", n * TB_RESULT_BYTES, "res")
        _check("tb_decode_batch",
               lib().tb_decode_batch(self._h, tbs.size, _np_ptr(tbs), _np_ptr(llr_off),
                                     _np_ptr(bits_off), _dptr(llr), ct.byref(p), _dptr(bits),
                                     _dptr(res), _stream(stream)))

    def cb_encode_batch(self, descs, payload, coded, stream=None):
        n_llr, n_bits = _desc_extent(descs)
        _need(payload, "uint8", n_bits, "payload")
        _need(coded, "uint8", n_llr, "coded")
        _check("cb_encode_batch",
               lib().cb_encode_batch(self._h, len(descs), ct.cast(descs, ct.c_void_p),
                                     _dptr(payload), _dptr(coded), _stream(stream)))

    def tb_encode(self, payload, tbs: int, coded, stream=None):
        _need(payload, "uint8", (tbs + 7) // 8, "payload")
        _need(coded, "uint8", tb_llr_count(tbs), "coded")
        _check("tb_encode", lib().tb_encode(self._h, _dptr(payload), int(tbs), _dptr(coded),
                                            _stream(stream)))


def parse_tb_results(raw: np.ndarray) -> list[dict]:
    """Decode the bytes of tdec_tb_result entries copied back to the host."""
    arr = np.frombuffer(np.ascontiguousarray(raw).tobytes(), dtype=TB_RESULT_DTYPE)
    out = []
    for r in arr:
        C = int(r["C"])
        out.append({"tb_ok": int(r["tb_ok"]), "max_iters_used": int(r["max_iters_used"]),
                    "C": C, "cb_ok": [int(x) for x in r["cb_ok"][:C]],
                    "cb_iters": [int(x) for x in r["cb_iters"][:C]]})
    return out
